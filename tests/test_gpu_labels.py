"""Constrained-MD label generation (Sec. II.C.1) through nep_md_step with a
bead constraint, against the FP64 oracle running the same constrained NVE
from the same start (needs an MI355X).  The system is the paper's water
training box in shape: 1536 atoms mapped onto 512 beads, with a synthetic
two-type atomistic model standing in for the missing NEP-AA."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import rel_rms

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PER = np.array([True, True, True])


def _coms(pos, masses, gs, box):
    out = []
    for g in range(gs.size - 1):
        a, b = gs[g], gs[g + 1]
        d = pos[a:b] - pos[a]
        d -= box * np.round(d / box)
        m = masses[a:b]
        out.append(pos[a] + (m[:, None] * d).sum(axis=0) / m.sum())
    return np.array(out)


def test_constrained_labels_track_oracle():
    from paper_2603_01234_amd import engine as E
    spec = W.water_aa_spec(60)
    params = W.draw_params(spec, np.random.default_rng(33))
    sysm, gs = W.water_atomistic(np.random.SeedSequence(34), 8, temperature=300.0)
    assert sysm.n == 1536 and gs.size - 1 == 512
    model = E.Model.from_spec(spec, params)
    rep = E.Replica(model, sysm.pos_f32(), sysm.types, sysm.box, sysm.pbc, skin=0.1, vel=sysm.vel)
    rep.efv(per_bead_virial=False)
    steps, dt, T = 100, 0.5, 300.0
    Ep = torch.zeros(steps, dtype=torch.float64, device="cuda")
    Ek = torch.zeros(steps, dtype=torch.float64, device="cuda")
    F_lab, W_lab, W_tot = rep.constrained_labels(gs, steps, dt, sysm.masses, T, E_pot=Ep, E_kin=Ek)
    p32 = sysm.pos_f32().astype(np.float64)
    r = oracle.md_ens(spec, params.astype(np.float32).astype(np.float64), p32,
                      sysm.vel.astype(np.float32).astype(np.float64), sysm.types, sysm.masses,
                      sysm.box.astype(np.float32).astype(np.float64), PER, dt, steps, group_start=gs)
    n = sysm.n
    dE = np.abs(Ep.cpu().numpy() - r.E_pot).max() / n
    dK = np.abs(Ek.cpu().numpy() - r.E_kin).max() / n
    L = np.asarray(rep.box, np.float64)
    d = rep.positions().astype(np.float64) - r.pos
    d -= L * np.round(d / L)
    # A bead's force and virial are sums over its atoms that largely cancel
    # (the intramolecular forces), so their error is bounded relative to the
    # size of the summands, sum_{i in I} |f_i| and sum_{i in I} |W_i| (taken
    # at the start), as for a total virial
    e0 = oracle.efv(spec, params.astype(np.float32).astype(np.float64), p32, sysm.types,
                    sysm.box.astype(np.float32).astype(np.float64), PER)
    sF = np.add.reduceat(np.linalg.norm(e0.F, axis=1), gs[:-1])
    sW = np.add.reduceat(np.linalg.norm(e0.W.reshape(-1, 9), axis=1), gs[:-1])
    eF = np.linalg.norm(F_lab - r.F_sum / steps) / np.linalg.norm(sF)
    eW = np.linalg.norm((W_lab - r.W_sum / steps).reshape(-1, 9)) / np.linalg.norm(sW)
    print(f"bead F rel to itself {rel_rms(F_lab, r.F_sum / steps):.2e}, bead W rel to itself "
          f"{rel_rms(W_lab, r.W_sum / steps):.2e}", flush=True)
    Wt_ref = oracle.virial_correction(r.W_sum / steps, n, 512, T)
    eWt = rel_rms(W_tot, Wt_ref)
    mb = sysm.masses[sysm.types]
    c0 = _coms(p32, mb, gs, L)
    c1 = _coms(rep.positions().astype(np.float64), mb, gs, L)
    dc = c1 - c0
    dc -= L * np.round(dc / L)
    print(f"labels: |dE_pot|/N {dE:.2e}, |dE_kin|/N {dK:.2e}, max |dx| {np.abs(d).max():.2e} nm, "
          f"bead F err / summands {eF:.2e}, bead W err / summands {eW:.2e}, corrected W_tot rel {eWt:.2e}, COM drift {np.abs(dc).max():.1e} nm",
          flush=True)
    assert dE < 1e-5 and dK < 1e-5 and np.abs(d).max() < 1e-4
    assert eF < 1e-5 and eW < 1e-5 and eWt < 1e-5
    assert np.abs(dc).max() < 1e-5
    model.close()


def test_single_atom_beads_label_the_static_force():
    """Every atom its own bead and at rest: the labels are the static force and
    per-atom virial of the configuration (the oracle's, to the contract's
    tolerances)."""
    from paper_2603_01234_amd import engine as E
    spec = W.water_aa_spec(30)
    params = W.draw_params(spec, np.random.default_rng(35))
    sysm, _ = W.water_atomistic(np.random.SeedSequence(36), 4, temperature=300.0)
    model = E.Model.from_spec(spec, params)
    rep = E.Replica(model, sysm.pos_f32(), sysm.types, sysm.box, sysm.pbc, skin=0.1)
    rep.efv(per_bead_virial=False)
    F_lab, W_lab, _ = rep.constrained_labels(np.arange(sysm.n + 1), 5, 0.5, sysm.masses, 300.0)
    ref = oracle.efv(spec, params.astype(np.float32).astype(np.float64), sysm.pos_f32().astype(np.float64),
                     sysm.types, sysm.box.astype(np.float32).astype(np.float64), PER)
    eF, eW = rel_rms(F_lab, ref.F), rel_rms(W_lab, ref.W)
    print(f"static labels: F rel {eF:.2e}, W rel {eW:.2e}")
    assert eF < 1e-5 and eW < 1e-5
    model.close()
