"""The MD step's virial, strained and compressed trajectories, and list
ownership of the processing order, against the FP64 oracle (needs an MI355X).

Every MD step evaluates the per-bead and total virial (Eqs. 15-16); the
constant strain-rate loading is the nanowire's (Sec. III.C.5).  Trajectories
are compared step by step with the oracle integrating the same equations in
FP64 from the same float32 start; snapshots are compared at the GPU's own
positions.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import TOL_F_RMS, TOL_U, TOL_W, compare_efv, rel_rms

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rep(spec, params, system, skin=0.1, vel=None):
    from paper_2603_01234_amd import engine as E
    model = E.Model.from_spec(spec, params)
    rep = E.Replica(model, system.pos_f32(), system.types, system.box, system.pbc, skin=skin,
                    vel=system.vel if vel is None else vel)
    rep._keep = model
    return rep


def _p64(params):
    return params.astype(np.float32).astype(np.float64)


def _unwrap_diff(a, b, box, pbc):
    d = a - b
    for k in range(3):
        if pbc[k]:
            d[:, k] -= box[k] * np.round(d[:, k] / box[k])
    return d


def test_md_virial_trace_and_per_bead_virial_config0():
    """Config 0, 100 steps: the total virial of every step (W_trace) at steps
    50 and 100, and the per-bead virial after the last step, against the
    oracle at the GPU's own positions (1e-5 relative)."""
    spec, params, system, opts = W.config0()
    rep = _rep(spec, params, system, opts["skin"])
    rep.efv()
    Wt = torch.zeros((100, 9), dtype=torch.float64, device="cuda")
    for half in range(2):
        rep.md(50, opts["dt"], [W.WATER_MASS], rebuild_every=opts["rebuild_every"],
               W_trace=Wt[50 * half:], per_bead_virial=True)
        torch.cuda.synchronize()
        ref = oracle.efv(spec, _p64(params), rep.positions().astype(np.float64), system.types,
                         system.box.astype(np.float32).astype(np.float64), system.pbc)
        got = Wt[50 * half + 49].cpu().numpy().reshape(3, 3)
        e_tot = rel_rms(got, ref.Wtot)
        e_bead = rel_rms(rep.virials(), ref.W)
        print(f"step {50 * (half + 1)}: W_tot rel {e_tot:.2e}, W_i rel RMS {e_bead:.2e}", flush=True)
        assert e_tot <= TOL_W and e_bead <= TOL_W
    assert np.isfinite(Wt.cpu().numpy()).all() and (Wt.cpu().numpy() != 0).any(axis=1).all()


def _wire(n_target=6000, seed=99):
    seq = np.random.SeedSequence(seed)
    return W.gold_nanowire(seq, n_target=n_target, core_radius=0.9, au_cells_z=27)


def _trajectory_against_oracle(spec, params, system, skin, dt, n_steps, rate, rebuild_every, label,
                               tol_e=1e-5, tol_x=1e-4):
    """GPU MD under strain against the oracle's FP64 run: per-step potential
    and kinetic energy per bead, and the final positions."""
    rep = _rep(spec, params, system, skin)
    rep.efv(per_bead_virial=False)
    Ep = torch.zeros(n_steps, dtype=torch.float64, device="cuda")
    Ek = torch.zeros(n_steps, dtype=torch.float64, device="cuda")
    rep.md(n_steps, dt, system.masses, rebuild_every=rebuild_every, strain_rate=rate, E_pot=Ep, E_kin=Ek)
    Ep, Ek = Ep.cpu().numpy(), Ek.cpu().numpy()
    p32 = system.pos_f32().astype(np.float64)
    v32 = system.vel.astype(np.float32).astype(np.float64)
    box0 = np.asarray(system.box, np.float64)
    pos, vel, F, box, Epo, Eko = oracle.md(spec, _p64(params), p32, v32, system.types.astype(np.int32),
                                           system.masses, box0.copy(), system.pbc, dt, n_steps,
                                           strain_rate=np.asarray(rate, np.float64), box0=box0)
    n = system.n
    dE = np.abs(Ep - Epo).max() / n
    dK = np.abs(Ek - Eko).max() / n
    dx = np.abs(_unwrap_diff(rep.positions().astype(np.float64), pos, box, system.pbc)).max()
    db = np.abs(np.asarray(rep.box, np.float64) - box).max() / box.max()
    print(f"{label}: rebuilds {rep.n_rebuilds}, max |dE_pot|/N {dE:.2e}, |dE_kin|/N {dK:.2e}, "
          f"max |dx| {dx:.2e} nm, box rel {db:.1e}", flush=True)
    assert db < 2e-7
    assert dE < tol_e and dK < tol_e
    assert dx < tol_x
    return rep


def test_strained_wire_trajectory_tracks_oracle():
    """A 6,000-site Au/CG wire (two types, pair cutoffs, H = 50, open across
    the axis) under 1e-4 engineering strain per step along z for 25 steps of
    5 fs: per-step energies and the final positions against the oracle's
    strained FP64 trajectory (the nanowire loading, Sec. III.C.5)."""
    spec = W.aacg_gold_spec(50)
    params = W.draw_params(spec, np.random.default_rng(12))
    wire = _wire()
    _trajectory_against_oracle(spec, params, wire, 0.1, 5.0, 25, (0.0, 0.0, 1e-4), 10, "wire +1e-4/step")


def test_compressive_strain_rebuilds_in_time():
    """Compression shrinks every separation affinely: 1.5e-3 per step on all
    three axes for 60 steps (about 9% per axis) with the schedule switched off
    (rebuild_every 10,000).  Only the rebuild test, with its affine-shrink term,
    keeps the lists complete; a missing pair would show as an energy jump far
    above the per-step tolerance."""
    spec, params, system, _ = W.config0()
    system.vel = W.maxwell_velocities(np.random.default_rng(8), np.full(system.n, W.WATER_MASS), 300.0)
    rep = _trajectory_against_oracle(spec, params, system, 0.1, 2.0, 60, (-1.5e-3, -1.5e-3, -1.5e-3), 10_000,
                                     "compress -1.5e-3/step")
    # 60 steps shrink a list reach of 0.9 nm by ~0.08 nm: at least one rebuild
    assert rep.n_rebuilds >= 1


def test_negative_strain_that_collapses_the_box_is_rejected():
    from paper_2603_01234_amd import binding as B
    spec, params, system, _ = W.config0()
    rep = _rep(spec, params, system, 0.1)
    rep.efv()
    with pytest.raises(B.NepError) as e:
        rep.md(20, 2.0, [W.WATER_MASS], strain_rate=(0.0, -0.05, 0.0))
    assert e.value.code == B.NEP_ERR_ARG


def test_evaluation_with_a_fresh_zeroed_workspace_after_a_build():
    """The processing order belongs to the lists: lists built with one
    workspace and evaluated with another, zeroed one give the same results bit
    for bit (and the oracle's)."""
    from paper_2603_01234_amd import binding as B
    spec, params, system, opts = W.config1()
    rep = _rep(spec, params, system, opts["skin"])
    rep.build()
    rep.efv()
    U1, F1, W1 = rep.U.clone(), rep.F.clone(), rep.W.clone()
    ws2 = torch.zeros_like(rep.ws)
    s, nb = rep.c_system(), rep.c_neighbors()
    U2 = torch.zeros_like(rep.U)
    F2 = torch.zeros_like(rep.F)
    W2 = torch.zeros_like(rep.W)
    B.check(B.nep_compute_efv(rep.model.handle, s, nb, U2.data_ptr(), F2.data_ptr(), W2.data_ptr(), None, None,
                              ws2.data_ptr(), rep.ws_bytes, torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert torch.equal(U1, U2) and torch.equal(F1, F2) and torch.equal(W1, W2)
    targets = np.random.default_rng(31).choice(system.n, 100, replace=False)
    ref = oracle.efv(spec, _p64(params), rep.positions().astype(np.float64), system.types,
                     system.box.astype(np.float32).astype(np.float64), system.pbc, targets=targets)
    compare_efv(rep, ref, system.n, targets=targets, label="zeroed second workspace")


def test_lists_without_an_order_use_index_order():
    """order = NULL in nep_neighbors: the build writes none and the kernels
    take beads in index order; the results equal those with the order."""
    from paper_2603_01234_amd import binding as B
    spec, params, system, opts = W.config0()
    rep = _rep(spec, params, system, opts["skin"])
    rep.efv()
    F1, U1 = rep.F.clone(), rep.U.clone()
    s, nb = rep.c_system(), rep.c_neighbors()
    nb.order = None
    st = torch.cuda.current_stream().cuda_stream
    B.check(B.nep_build_neighbors(rep.model.handle, s, nb, 1, rep.ws.data_ptr(), rep.ws_bytes, st))
    F2, U2 = torch.zeros_like(rep.F), torch.zeros_like(rep.U)
    B.check(B.nep_compute_efv(rep.model.handle, s, nb, U2.data_ptr(), F2.data_ptr(), None, None, None,
                              rep.ws.data_ptr(), rep.ws_bytes, st))
    torch.cuda.synchronize()
    assert torch.equal(F1, F2) and torch.equal(U1, U2)


def _random_box_system(rng, n, density, n_types):
    L = (n / density) ** (1.0 / 3.0)
    pos = np.zeros((0, 3))
    while pos.shape[0] < n:
        cand = rng.uniform(0.0, L, (4 * n, 3))
        keep = []
        for c in cand:
            if pos.shape[0] + len(keep) >= n:
                break
            allp = np.concatenate([pos] + [np.asarray(keep).reshape(-1, 3)])
            d = allp - c
            d -= L * np.round(d / L)
            if allp.shape[0] == 0 or np.min(np.sum(d * d, axis=1)) > 0.2 ** 2:
                keep.append(c)
        pos = np.concatenate([pos, np.asarray(keep).reshape(-1, 3)])
    types = rng.integers(0, n_types, n).astype(np.uint8)
    return W.System(pos[:n], types, np.array([L, L, L]), np.array([True, True, True]),
                    np.full(n_types, 18.0))


@pytest.mark.parametrize("n_types,H", [(3, 20), (4, 12)])
def test_efv_parity_three_and_four_types(n_types, H):
    """The fused and gather kernels for n_types = 3 and 4 (per-pair cutoffs as
    arithmetic means of per-type values) against the oracle, every bead."""
    rng = np.random.default_rng(40 + n_types)
    rc = np.array([0.6, 0.7, 0.8, 0.75][:n_types])
    rcR = 0.5 * (rc[:, None] + rc[None, :])
    spec = W.ModelSpec(n_types=n_types, n_hidden=H, rc_R=rcR, rc_A=rcR - 0.1)
    params = W.draw_params(spec, rng)
    system = _random_box_system(rng, 400, 25.0, n_types)
    rep = _rep(spec, params, system, 0.1)
    rep.efv()
    ref = oracle.efv(spec, _p64(params), rep.positions().astype(np.float64), system.types,
                     system.box.astype(np.float32).astype(np.float64), system.pbc)
    compare_efv(rep, ref, system.n, label=f"T={n_types}")


def test_batched_form_rejects_more_than_two_types():
    from paper_2603_01234_amd import binding as B
    from paper_2603_01234_amd import engine as E
    rng = np.random.default_rng(3)
    rc = np.full((3, 3), 0.7)
    spec = W.ModelSpec(n_types=3, n_hidden=8, rc_R=rc, rc_A=rc - 0.1)
    system = _random_box_system(rng, 64, 25.0, 3)
    rep = _rep(spec, W.draw_params(spec, rng), system, 0.0)
    rep.build()
    fb = E.FitnessBatch([rep.model], [rep])
    with pytest.raises(B.NepError) as e:
        fb.evaluate(rmse=False, items=True)
    assert "n_types <= 2" in str(e.value)


@pytest.mark.parametrize("H", [8, 12])
def test_efv_parity_small_hidden_layers(H):
    """Hidden widths padded to 8 and 16 (the smallest built network tiles),
    config 0 positions, every bead against the oracle."""
    spec0, _, system, opts = W.config0()
    spec = W.water_spec(H)
    params = W.draw_params(spec, np.random.default_rng(50 + H))
    rep = _rep(spec, params, system, opts["skin"])
    rep.efv()
    ref = oracle.efv(spec, _p64(params), rep.positions().astype(np.float64), system.types,
                     system.box.astype(np.float32).astype(np.float64), system.pbc)
    compare_efv(rep, ref, system.n, label=f"H={H}")


def test_neighbor_sets_config2_sampled():
    """The 200,000-site wire (open x, y; three pair cutoffs): sampled rows,
    Au core and CG shell alike, equal the float32 brute force as sets."""
    from gpu_helpers import gpu_sets
    from oracle.neighbors_f32 import neighbor_sets
    spec, params, system, opts = W.config2()
    rep = _rep(spec, params, system, opts["skin"])
    rep.build()
    rng = np.random.default_rng(2)
    rows = np.concatenate([rng.choice(np.nonzero(system.types == t)[0], 75, replace=False) for t in (0, 1)])
    rows = rows.tolist()
    pos = rep.positions()
    got = gpu_sets(rep, rows)
    refR = neighbor_sets(pos, system.types, rep.box, system.pbc, spec.rc_R, opts["skin"], rows=rows)
    refA = neighbor_sets(pos, system.types, rep.box, system.pbc, spec.rc_A, opts["skin"], rows=rows)
    sizes = []
    for i in rows:
        assert got[i][0] == refR[i], f"row {i}: radial set differs"
        assert got[i][1] == refA[i], f"row {i}: angular prefix differs"
        sizes.append(len(refR[i]))
    print("config2 row lengths: min", min(sizes), "max", max(sizes))
