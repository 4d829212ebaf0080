"""Thermostats, the per-call barostat and the HNEMD drive of nep_md_step
against the FP64 oracle integrating the same equations (oracle.md_ens) from
the same float32 start (needs an MI355X).  The paper equilibrates in NVT/NPT
(Sec. III.A.1, III.C.3) and measures heat transport by HNEMD (Sec. III.B.3);
the algorithms are the published ones its engine offers (Berendsen, Bussi,
Berendsen barostat, Fan et al.'s many-body HNEMD)."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import rel_rms

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PER = np.array([True, True, True])


def _start(T=300.0, seed=8):
    spec, params, system, opts = W.config0()
    system.vel = W.maxwell_velocities(np.random.default_rng(seed), np.full(system.n, W.WATER_MASS), T)
    return spec, params, system


def _rep(spec, params, system, skin=0.1):
    from paper_2603_01234_amd import engine as E
    model = E.Model.from_spec(spec, params)
    rep = E.Replica(model, system.pos_f32(), system.types, system.box, system.pbc, skin=skin, vel=system.vel)
    rep._keep = model
    rep.efv(per_bead_virial=False)
    return rep


def _oracle_start(params, system):
    return (params.astype(np.float32).astype(np.float64), system.pos_f32().astype(np.float64),
            system.vel.astype(np.float32).astype(np.float64), system.box.astype(np.float32).astype(np.float64))


def _traces(n):
    z = lambda *s: torch.zeros(s, dtype=torch.float64, device="cuda")
    return z(n), z(n), z(n, 9), z(n, 3)


def _compare(rep, r, Ep, Ek, Wt, Jt, system, label, check_J=False):
    n = system.n
    Ep, Ek, Wt, Jt = (t.cpu().numpy() for t in (Ep, Ek, Wt, Jt))
    dE = np.abs(Ep - r.E_pot).max() / n
    dK = np.abs(Ek - r.E_kin).max() / n
    d = rep.positions().astype(np.float64) - r.pos
    L = np.asarray(rep.box, np.float64)
    d -= L * np.round(d / L)
    dW = max(rel_rms(Wt[k], r.W[k].ravel()) for k in range(len(Ep)))
    out = f"{label}: max |dE_pot|/N {dE:.2e}, |dE_kin|/N {dK:.2e}, max |dx| {np.abs(d).max():.2e}, W rel {dW:.2e}"
    if check_J:
        # the heat current is a sum of large terms of both signs: its error is
        # measured against the scale of those terms (the RMS over the run)
        scale = np.sqrt((r.J ** 2).mean())
        dJ = np.abs(Jt - r.J).max() / scale
        out += f", J err / rms(J) {dJ:.2e}"
        assert dJ < 1e-3
    print(out, flush=True)
    assert dE < 1e-5 and dK < 1e-5 and np.abs(d).max() < 1e-4 and dW < 1e-5


@pytest.mark.parametrize("thermostat", [1, 2])
def test_nvt_tracks_oracle(thermostat):
    """Config 0 at 300 K coupled to 600 K (Berendsen, or Bussi with the same
    random numbers on both sides) for 100 steps: per-step energies, virial
    and final positions against the oracle."""
    spec, params, system = _start()
    rep = _rep(spec, params, system)
    steps, T0, tau = 100, 600.0, 40.0
    noise = None
    if thermostat == 2:
        rng = np.random.default_rng(17)
        noise = np.stack([rng.normal(size=steps), rng.chisquare(3 * system.n - 4, size=steps)], axis=1)
    Ep, Ek, Wt, Jt = _traces(steps)
    ens = dict(thermostat=thermostat, T_target=T0, tau_T=tau)
    if noise is not None:
        ens["noise"] = torch.from_numpy(noise).cuda()
    rep.md(steps, 2.0, [W.WATER_MASS], rebuild_every=10, E_pot=Ep, E_kin=Ek, W_trace=Wt, ensemble=ens)
    p64, x, v, box = _oracle_start(params, system)
    r = oracle.md_ens(spec, p64, x, v, system.types, [W.WATER_MASS], box, PER, 2.0, steps, thermostat=thermostat,
                      T_target=T0, tau_T=tau, noise=noise)
    _compare(rep, r, Ep, Ek, Wt, Jt, system, f"NVT thermostat {thermostat}")
    T_end = 2 * Ek[-1].item() / ((3 * system.n - 3) * oracle.KB_EV)
    print(f"T after {steps} steps: {T_end:.0f} K")


def test_npt_calls_track_oracle():
    """Five calls of 10 steps with the Berendsen barostat (0.3 GPa target) and
    a Berendsen thermostat: each call's factor comes from the previous call's
    mean pressure, on both sides.  Box, pressure and energies per call against
    the oracle."""
    spec, params, system = _start(seed=9)
    rep = _rep(spec, params, system)
    P0 = 0.3 * 6.241509
    beta, tauP = 0.05, 200.0
    p64, x, v, box = _oracle_start(params, system)
    P_gpu = P_or = np.full(3, np.nan)
    for c in range(5):
        Ep, Ek, Wt, Jt = _traces(10)
        rep.md(10, 2.0, [W.WATER_MASS], rebuild_every=10, E_pot=Ep, E_kin=Ek, W_trace=Wt,
               ensemble=dict(thermostat=1, T_target=300.0, tau_T=50.0, barostat=1, P_target=(P0,) * 3, tau_P=tauP,
                             beta=beta, P_in=tuple(P_gpu)))
        P_gpu = rep.P_out.copy()
        r = oracle.md_ens(spec, p64, x, v, system.types, [W.WATER_MASS], box, PER, 2.0, 10, step0=10 * c,
                          thermostat=1, T_target=300.0, tau_T=50.0, barostat=1, P_target=(P0,) * 3, tau_P=tauP,
                          beta=beta, P_in=P_or)
        x, v, box, P_or = r.pos, r.vel, r.box, r.P_out
        dP = np.abs(P_gpu - P_or).max() / np.abs(P_or).max()
        db = np.abs(np.asarray(rep.box, np.float64) - box).max() / box.max()
        print(f"call {c}: box {np.asarray(rep.box)} P {P_gpu / 6.241509} GPa, dP rel {dP:.2e}, box rel {db:.1e}")
        assert dP < 1e-5 and db < 1e-6
        _compare(rep, r, Ep, Ek, Wt, Jt, system, f"NPT call {c}")
    assert np.abs(np.asarray(rep.box, np.float64) - system.box).max() > 1e-4   # the box did move


def test_hnemd_drive_and_heat_current_track_oracle():
    """HNEMD on config 0: F_e = 0.4/nm along z with a Berendsen thermostat at
    300 K for 100 steps.  Heat current per step, energies, virial and final
    positions against the oracle; the drive keeps the total momentum at zero."""
    spec, params, system = _start(seed=10)
    rep = _rep(spec, params, system)
    Fe = (0.0, 0.0, 0.4)
    steps = 100
    Ep, Ek, Wt, Jt = _traces(steps)
    rep.md(steps, 2.0, [W.WATER_MASS], rebuild_every=10, E_pot=Ep, E_kin=Ek, W_trace=Wt, J_trace=Jt,
           ensemble=dict(thermostat=1, T_target=300.0, tau_T=100.0, Fe=Fe))
    p64, x, v, box = _oracle_start(params, system)
    r = oracle.md_ens(spec, p64, x, v, system.types, [W.WATER_MASS], box, PER, 2.0, steps, thermostat=1,
                      T_target=300.0, tau_T=100.0, Fe=Fe)
    _compare(rep, r, Ep, Ek, Wt, Jt, system, "HNEMD", check_J=True)
    p = rep.velocities().sum(axis=0)
    assert np.abs(p).max() < 1e-4 * np.abs(rep.velocities()).max()


def test_strained_wire_with_thermostat_tracks_oracle():
    """The wire loading (1e-4 per step along z) under a Bussi thermostat at
    300 K: the strain and the thermostat together against the oracle."""
    spec = W.aacg_gold_spec(50)
    params = W.draw_params(spec, np.random.default_rng(12))
    wire = W.gold_nanowire(np.random.SeedSequence(99), n_target=6000, core_radius=0.9, au_cells_z=27)
    from paper_2603_01234_amd import engine as E
    model = E.Model.from_spec(spec, params)
    rep = E.Replica(model, wire.pos_f32(), wire.types, wire.box, wire.pbc, skin=0.1, vel=wire.vel)
    rep.efv(per_bead_virial=False)
    steps = 25
    rng = np.random.default_rng(5)
    noise = np.stack([rng.normal(size=steps), rng.chisquare(3 * wire.n - 4, size=steps)], axis=1)
    Ep, Ek, Wt, Jt = _traces(steps)
    rate = (0.0, 0.0, 1e-4)
    rep.md(steps, 5.0, wire.masses, rebuild_every=10, strain_rate=rate, E_pot=Ep, E_kin=Ek, W_trace=Wt,
           ensemble=dict(thermostat=2, T_target=300.0, tau_T=100.0, noise=torch.from_numpy(noise).cuda()))
    box0 = np.asarray(wire.box, np.float64)
    r = oracle.md_ens(spec, params.astype(np.float32).astype(np.float64), wire.pos_f32().astype(np.float64),
                      wire.vel.astype(np.float32).astype(np.float64), wire.types, wire.masses, box0.copy(),
                      wire.pbc, 5.0, steps, strain_rate=np.asarray(rate), box0=box0, thermostat=2, T_target=300.0,
                      tau_T=100.0, noise=noise)
    _compare(rep, r, Ep, Ek, Wt, Jt, wire, "wire + Bussi")
