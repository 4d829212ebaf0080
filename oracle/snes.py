"""Plain reference of the training loop around the fitness evaluation: the
separable natural evolution strategy (SNES) and the NEP loss (Sec. II.A).

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle``): imported by
``tests/`` and never by the product package.

The paper optimises the parameters with SNES (Schaul et al., "High dimensions
and heavy tails for natural evolution strategies", GECCO 2011) on a loss of
energy, force and virial RMSEs plus L1 and L2 regularisation weighted by
lambda_e, lambda_f, lambda_v, lambda_1, lambda_2.  Written here from that
publication's algorithm:

  * sample  z_k = mu + sigma * s_k,  s_k ~ N(0, I),  k = 1..lambda
    (the s_k are inputs: whoever draws them hands the same numbers to both
    sides);
  * rank the samples by loss, best first (ties: lower index first);
  * utilities u_r = max(0, ln(lambda/2 + 1) - ln r) / sum_j max(0, ...) - 1/lambda
    for ranks r = 1..lambda;
  * natural gradients  g_mu = sum_r u_r s_(r),  g_sigma = sum_r u_r (s_(r)^2 - 1);
  * updates  mu <- mu + eta_mu sigma g_mu,  sigma <- sigma exp(eta_sigma/2 g_sigma).

The loss (reading: the published NEP form, the paper gives only its terms):
  L(z) = lambda_e RMSE_E + lambda_f RMSE_F + lambda_v RMSE_W
         + lambda_1 mean|z| + lambda_2 sqrt(mean z^2)
with RMSE_E and RMSE_W per bead (W over xx, yy, zz, xy, yz, xz) and RMSE_F
per force component, over the structures of the training set.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np


def utilities(lam: int) -> np.ndarray:
    """Rank-based fitness shaping of SNES, indexed by rank (best first)."""
    r = np.arange(1, lam + 1, dtype=np.float64)
    raw = np.maximum(0.0, math.log(lam / 2.0 + 1.0) - np.log(r))
    return raw / raw.sum() - 1.0 / lam


def default_rates(dim: int):
    """SNES defaults: eta_mu = 1, eta_sigma = (3 + ln d) / (5 sqrt d)."""
    return 1.0, (3.0 + math.log(dim)) / (5.0 * math.sqrt(dim))


def rank_order(losses: np.ndarray) -> np.ndarray:
    """Indices of the candidates from best (lowest loss) to worst; ties keep
    index order; a non-finite loss ranks after every finite one."""
    L = np.where(np.isfinite(losses), np.asarray(losses, np.float64), np.inf)
    return np.argsort(L, kind="stable")


def generation(mu: np.ndarray, sigma: np.ndarray, s: np.ndarray, losses: np.ndarray, eta_mu: float,
               eta_sigma: float):
    """One SNES update from the samples' standard-normal draws s [lambda, d]
    and their losses; returns the new (mu, sigma)."""
    lam = s.shape[0]
    order = rank_order(losses)
    u = utilities(lam)
    g_mu = np.zeros_like(mu, dtype=np.float64)
    g_sigma = np.zeros_like(mu, dtype=np.float64)
    for r in range(lam):
        k = order[r]
        g_mu += u[r] * s[k]
        g_sigma += u[r] * (s[k] * s[k] - 1.0)
    return mu + eta_mu * sigma * g_mu, sigma * np.exp(0.5 * eta_sigma * g_sigma)


def loss(rmse: np.ndarray, z: np.ndarray, lam_e: float, lam_f: float, lam_v: float, lam_1: float,
         lam_2: float) -> np.ndarray:
    """NEP loss of each candidate: rmse [lambda, 3] (E, F, W), z [lambda, d]."""
    z = np.asarray(z, np.float64)
    reg1 = np.abs(z).mean(axis=1)
    reg2 = np.sqrt((z * z).mean(axis=1))
    return lam_e * rmse[:, 0] + lam_f * rmse[:, 1] + lam_v * rmse[:, 2] + lam_1 * reg1 + lam_2 * reg2


def fitness_rmse(spec, candidates: np.ndarray, systems: Sequence, labels, n_threads: int = 0) -> np.ndarray:
    """RMSE_E, RMSE_F, RMSE_W of every candidate parameter vector against
    reference labels (E [S], F list of [n_s, 3], W [S, 3, 3]) with the FP64
    evaluator."""
    import oracle
    E_ref, F_ref, W_ref = labels
    comp = [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)]
    out = np.zeros((candidates.shape[0], 3))
    for k, p in enumerate(candidates):
        e2 = f2 = w2 = 0.0
        nf = 0
        for s, sysm in enumerate(systems):
            r = oracle.efv(spec, p, sysm.pos_f32().astype(np.float64), sysm.types,
                           sysm.box.astype(np.float32).astype(np.float64), sysm.pbc, n_threads=n_threads)
            N = sysm.n
            e2 += ((r.E - E_ref[s]) / N) ** 2
            f2 += ((r.F - F_ref[s]) ** 2).sum()
            nf += 3 * N
            w2 += sum(((r.Wtot[a, b] - W_ref[s][a, b]) / N) ** 2 for a, b in comp)
        S = len(systems)
        out[k] = [math.sqrt(e2 / S), math.sqrt(f2 / nf), math.sqrt(w2 / (6 * S))]
    return out
