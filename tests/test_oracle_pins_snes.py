"""Pins of the SNES reference (oracle/snes.py) against closed forms, special
cases and its defining property (convergence on a separable quadratic)."""
import math

import numpy as np

import oracle
import workloads as W
from oracle import snes


def test_utilities_closed_form_and_invariants():
    for lam in (2, 4, 10, 16, 64):
        u = snes.utilities(lam)
        assert abs(u.sum()) < 1e-14
        assert np.all(np.diff(u) <= 1e-15)
        # ranks r >= lambda/2 + 1 (0-based index >= lambda/2) get no positive weight: u = -1/lambda
        np.testing.assert_allclose(u[int(math.ceil(lam / 2.0)):], -1.0 / lam, atol=1e-15)
        assert np.all(u[:int(math.ceil(lam / 2.0))] > -1.0 / lam)
    raw = np.array([math.log(3.0), math.log(3.0) - math.log(2.0), 0.0, 0.0])
    np.testing.assert_allclose(snes.utilities(4), raw / raw.sum() - 0.25, atol=1e-15)


def test_update_depends_on_losses_only_through_their_ranks():
    rng = np.random.default_rng(1)
    mu, sigma = rng.normal(size=7), rng.uniform(0.5, 2.0, 7)
    s = rng.normal(size=(12, 7))
    L = rng.normal(size=12)
    a = snes.generation(mu, sigma, s, L, 1.0, 0.2)
    b = snes.generation(mu, sigma, s, np.exp(3 * L) + 5.0, 1.0, 0.2)   # monotone transform
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    # ties rank by index; a non-finite loss ranks last
    assert snes.rank_order(np.array([1.0, np.nan, 1.0, 0.5])).tolist() == [3, 0, 2, 1]


def test_antithetic_pair_moves_the_mean_along_the_better_sample():
    """lambda = 2 with s_2 = -s_1: utilities (1/2, -1/2), so g_mu = s_1 when
    sample 1 is better, g_sigma = 0, and mu' = mu + eta sigma s_1."""
    rng = np.random.default_rng(2)
    mu, sigma = rng.normal(size=5), rng.uniform(0.1, 1.0, 5)
    s1 = rng.normal(size=5)
    m2, s2 = snes.generation(mu, sigma, np.stack([s1, -s1]), np.array([0.1, 0.2]), 0.7, 0.3)
    np.testing.assert_allclose(m2, mu + 0.7 * sigma * s1, rtol=1e-15)
    np.testing.assert_array_equal(s2, sigma)


def test_unit_magnitude_samples_leave_sigma_unchanged():
    rng = np.random.default_rng(3)
    s = rng.choice([-1.0, 1.0], size=(10, 4))
    _, sig = snes.generation(np.zeros(4), np.full(4, 0.3), s, rng.normal(size=10), 1.0, 0.5)
    np.testing.assert_allclose(sig, 0.3, rtol=1e-15)


def test_converges_on_a_separable_quadratic():
    """SNES with its default rates minimises sum_i a_i (z_i - c_i)^2 (d = 10)."""
    d = 10
    rng = np.random.default_rng(4)
    a = rng.uniform(0.5, 5.0, d)
    c = rng.normal(size=d)
    lam = 4 + int(3 * math.log(d))
    eta_mu, eta_sigma = snes.default_rates(d)
    mu, sigma = np.zeros(d), np.ones(d)
    for _ in range(400):
        s = rng.normal(size=(lam, d))
        z = mu + sigma * s
        f = ((z - c) ** 2 * a).sum(axis=1)
        mu, sigma = snes.generation(mu, sigma, s, f, eta_mu, eta_sigma)
    assert np.abs(mu - c).max() < 1e-4, np.abs(mu - c).max()
    assert sigma.max() < 1e-3


def test_loss_terms():
    rmse = np.array([[0.1, 0.2, 0.3], [1.0, 2.0, 3.0]])
    z = np.array([[3.0, -4.0], [0.0, 0.0]])
    L = snes.loss(rmse, z, 1.0, 2.0, 0.5, 0.1, 0.01)
    np.testing.assert_allclose(L, [0.1 + 0.4 + 0.15 + 0.1 * 3.5 + 0.01 * math.sqrt(12.5), 1.0 + 4.0 + 1.5],
                               rtol=1e-15)


def test_fitness_rmse_is_zero_for_the_teacher_and_positive_otherwise():
    spec = W.water_spec(8)
    rng = np.random.default_rng(5)
    teacher = W.draw_params(spec, rng)
    systems = [W.water_random_sites(rng, n, W.WATER_DENSITY) for n in (40, 64)]
    labels = ([], [], [])
    for sysm in systems:
        r = oracle.efv(spec, teacher, sysm.pos_f32().astype(np.float64), sysm.types,
                       sysm.box.astype(np.float32).astype(np.float64), sysm.pbc)
        labels[0].append(r.E)
        labels[1].append(r.F)
        labels[2].append(r.Wtot)
    cands = np.stack([teacher, teacher + 0.05 * rng.normal(size=teacher.size)])
    out = snes.fitness_rmse(spec, cands, systems, labels)
    assert np.all(out[0] == 0.0)
    assert np.all(out[1] > 0.0)
