"""Pins of the oracle's ensemble and HNEMD integrator (oracle.md_ens) against
things other than itself: the already pinned NVE integrator, closed forms of
free particles, the canonical distribution of the kinetic energy, the energy
balance of a driven system, and the heat current as the time derivative of
sum_i r_i E_i on an open cluster (Hardy's definition).

Free particles come from an all-zero parameter vector: every site energy and
force vanishes, so the thermostat and barostat act alone.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

PER = np.array([True, True, True])
OPEN = np.array([False, False, False])
KB = oracle.KB_EV


def _free(n=40, L=6.0, T=300.0, seed=1):
    spec = W.water_spec(6)
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, L, (n, 3))
    vel = W.maxwell_velocities(rng, np.full(n, W.WATER_MASS), T)
    return spec, np.zeros(spec.n_params), pos, vel, np.zeros(n, int), np.array([L, L, L])


def test_no_options_equals_the_nve_integrator():
    """With every option off the ensemble integrator is the NVE one: the same
    trajectory bit for bit (the kinetic energy is summed per axis, so equal to
    rounding)."""
    spec, params, system, _ = W.config0()
    sysm = W.water_box(np.random.SeedSequence(5), 4, temperature=500.0)
    pos = sysm.pos_f32().astype(np.float64)
    a = oracle.md(spec, params, pos, sysm.vel, sysm.types, [W.WATER_MASS], sysm.box, PER, 2.0, 15)
    b = oracle.md_ens(spec, params, pos, sysm.vel, sysm.types, [W.WATER_MASS], sysm.box, PER, 2.0, 15)
    np.testing.assert_array_equal(a[0], b.pos)
    np.testing.assert_array_equal(a[1], b.vel)
    np.testing.assert_array_equal(a[4], b.E_pot)
    np.testing.assert_allclose(a[5], b.E_kin, rtol=1e-14)


def test_berendsen_relaxes_free_particles_exponentially():
    """lam^2 = 1 + (dt/tau)(T0/T - 1) on free particles gives
    T_{s+1} = T_s + (dt/tau)(T0 - T_s), so T_s - T0 = (T_init - T0)(1 - dt/tau)^(s+1)."""
    spec, p, pos, vel, ty, box = _free(T=900.0)
    n = pos.shape[0]
    Nf = 3 * n - 3
    K0 = 0.5 * W.WATER_MASS * (vel ** 2).sum() / W.ACCEL_EV_NM_AMU
    T_init = 2 * K0 / (Nf * KB)
    dt, tau, T0 = 2.0, 50.0, 300.0
    r = oracle.md_ens(spec, p, pos, vel, ty, [W.WATER_MASS], box, PER, dt, 40, thermostat=1, T_target=T0,
                      tau_T=tau)
    T = 2 * r.E_kin / (Nf * KB)
    ref = T0 + (T_init - T0) * (1 - dt / tau) ** np.arange(1, 41)
    np.testing.assert_allclose(T, ref, rtol=1e-12)


def test_bussi_samples_the_canonical_kinetic_energy():
    """Stochastic velocity rescaling leaves K gamma-distributed with shape
    N_f/2 and scale k_B T0: mean N_f k_B T0 / 2 and variance 2 Kbar^2 / N_f.
    With tau = dt successive values are nearly independent."""
    spec, p, pos, vel, ty, box = _free(n=20, L=40.0, T=150.0, seed=3)
    n = pos.shape[0]
    Nf = 3 * n - 3
    T0 = 300.0
    steps = 6000
    rng = np.random.default_rng(11)
    noise = np.stack([rng.normal(size=steps), rng.chisquare(Nf - 1, size=steps)], axis=1)
    r = oracle.md_ens(spec, p, pos, vel, ty, [W.WATER_MASS], box, PER, 1.0, steps, thermostat=2, T_target=T0,
                      tau_T=1.0, noise=noise)
    K = r.E_kin[200:]
    Kbar = 0.5 * Nf * KB * T0
    m, v = K.mean(), K.var()
    se_m = math.sqrt(2.0 / Nf) * Kbar / math.sqrt(K.size / 2.0)
    print(f"<K>/Kbar {m / Kbar:.4f} (se {se_m / Kbar:.4f}), var ratio {v / (2 * Kbar ** 2 / Nf):.3f}")
    assert abs(m - Kbar) < 4 * se_m
    assert 0.85 < v / (2 * Kbar ** 2 / Nf) < 1.15


def test_bussi_with_infinite_coupling_time_keeps_the_kinetic_energy():
    spec, p, pos, vel, ty, box = _free(seed=4)
    rng = np.random.default_rng(2)
    noise = np.stack([rng.normal(size=20), rng.chisquare(3 * 40 - 4, size=20)], axis=1)
    r = oracle.md_ens(spec, p, pos, vel, ty, [W.WATER_MASS], box, PER, 2.0, 20, thermostat=2, T_target=300.0,
                      tau_T=1e300, noise=noise)
    K0 = 0.5 * W.WATER_MASS * (vel ** 2).sum() / W.ACCEL_EV_NM_AMU
    np.testing.assert_allclose(r.E_kin, K0, rtol=1e-12)


def test_berendsen_barostat_scales_an_ideal_gas_box():
    """Free particles: W = 0, so P_dd = 2 K_dd / V (ideal gas).  With the call's
    scale factor mu_d = cbrt(1 - beta dt/tau_P (P0_d - P_in_d)) the box after s
    steps is L mu^s, positions scale with it, and the mean pressure follows
    from the constant K_dd over the shrinking volume."""
    spec, p, pos, vel, ty, box = _free(T=300.0, seed=6)
    dt, tauP, beta, steps = 2.0, 400.0, 0.02, 12
    P0 = np.array([0.5, 0.3, 0.1])
    Pin = np.array([0.05, 0.1, 0.2])
    r = oracle.md_ens(spec, p, pos, vel, ty, [W.WATER_MASS], box, PER, dt, steps, barostat=1, P_target=P0,
                      tau_P=tauP, beta=beta, P_in=Pin)
    mu = np.cbrt(1 - beta * dt / tauP * (P0 - Pin))
    np.testing.assert_allclose(r.box, box * mu ** steps, rtol=1e-13)
    x = pos.copy()
    for _ in range(steps):
        x = (x + dt * vel) * mu
    np.testing.assert_allclose(r.pos, x, rtol=1e-12)
    Kd = 0.5 * W.WATER_MASS * (vel ** 2).sum(axis=0) / W.ACCEL_EV_NM_AMU
    V = np.prod(box) * np.prod(mu) ** np.arange(1, steps + 1)
    np.testing.assert_allclose(r.P_out, (2 * Kd[None, :] / V[:, None]).mean(axis=0), rtol=1e-12)
    # the clamp keeps a single call within 1% per step
    r2 = oracle.md_ens(spec, p, pos, vel, ty, [W.WATER_MASS], box, PER, dt, 3, barostat=1, P_target=(50.0,) * 3,
                       tau_P=10.0, beta=1.0, P_in=(0.0,) * 3)
    np.testing.assert_allclose(r2.box, box * 0.99 ** 3, rtol=1e-13)


def _small_water(seed=5, n_side=4, T=600.0):
    spec, params, _, _ = W.config0()
    sysm = W.water_box(np.random.SeedSequence(seed), n_side, temperature=T)
    return spec, params, sysm


def test_zero_driving_force_is_plain_md_and_driving_conserves_momentum():
    spec, params, sysm = _small_water()
    pos = sysm.pos_f32().astype(np.float64)
    a = oracle.md_ens(spec, params, pos, sysm.vel, sysm.types, [W.WATER_MASS], sysm.box, PER, 2.0, 10)
    b = oracle.md_ens(spec, params, pos, sysm.vel, sysm.types, [W.WATER_MASS], sysm.box, PER, 2.0, 10,
                      Fe=(0.0, 0.0, 0.0))
    np.testing.assert_array_equal(a.vel, b.vel)
    c = oracle.md_ens(spec, params, pos, sysm.vel, sysm.types, [W.WATER_MASS], sysm.box, PER, 2.0, 30,
                      Fe=(0.3, -0.2, 0.5))
    assert np.abs(c.vel.sum(axis=0)).max() < 1e-12 * np.abs(c.vel).max() * sysm.n


def test_driving_force_energy_balance():
    """Without a thermostat the driving force does work F_e . J per unit time:
    H(t) - H(0) = int F_e . J dt (with zero total momentum the mean removal
    does no work).  The run starts from the plain potential force, so the
    first half-kick carries no drive: the trapezoid sum loses dt/2 F_e . J(0).
    What remains shrinks like dt^2."""
    spec, params, sysm = _small_water(seed=9, T=400.0)
    pos = sysm.pos_f32().astype(np.float64)
    Fe = np.array([0.0, 0.0, 2.0])
    E0 = oracle.efv(spec, params, pos, sysm.types, sysm.box, PER).E
    K0 = 0.5 * W.WATER_MASS * (sysm.vel ** 2).sum() / W.ACCEL_EV_NM_AMU
    res = []
    for dt, n in ((1.0, 40), (0.5, 80)):
        r = oracle.md_ens(spec, params, pos, sysm.vel, sysm.types, [W.WATER_MASS], sysm.box, PER, dt, n, Fe=Fe)
        H = r.E_pot + r.E_kin
        # J at t = 0 from the starting state
        e0 = oracle.efv(spec, params, pos, sysm.types, sysm.box, PER)
        J0 = np.einsum("iab,ib->a", e0.W, sysm.vel)
        Jt = np.concatenate([J0[None], r.J])
        P = Jt @ Fe
        work = np.concatenate([[0.0], np.cumsum(0.5 * dt * (P[1:] + P[:-1])) - 0.5 * dt * P[0]])
        dH = np.concatenate([[0.0], H - (E0 + K0)])
        res.append(np.abs(dH - work).max())
        print(f"dt {dt}: max |dH| {np.abs(dH).max():.3e} eV, residual {res[-1]:.3e} eV")
        assert res[-1] < 0.01 * np.abs(dH).max()
    assert 3.0 < res[0] / res[1] < 5.5


def test_heat_current_is_the_time_derivative_of_r_times_site_energy():
    """On an open cluster J_pot + sum_i E_i v_i = d/dt sum_i r_i E_i, with
    E_i = m v_i^2/2 + U_i (Hardy).  The time derivative is a central
    difference over two short steps of the oracle's own NVE trajectory."""
    spec = W.water_spec(12)
    params = W.draw_params(spec, np.random.default_rng(23))
    rng = np.random.default_rng(24)
    pos = W.small_cluster(rng, 14, 1.1, 0.22)
    vel = W.maxwell_velocities(rng, np.full(14, W.WATER_MASS), 800.0)
    ty = np.zeros(14, int)
    box = np.array([20.0, 20.0, 20.0])
    h = 0.02
    states = []
    x, v = pos.copy(), vel.copy()
    for k in range(3):
        if k:
            r = oracle.md_ens(spec, params, x, v, ty, [W.WATER_MASS], box, OPEN, h, 1)
            x, v = r.pos, r.vel
            J = r.J[0]
        e = oracle.efv(spec, params, x, ty, box, OPEN)
        Ei = 0.5 * W.WATER_MASS * (v ** 2).sum(axis=1) / W.ACCEL_EV_NM_AMU + e.U
        G = (x * Ei[:, None]).sum(axis=0)
        states.append((G, J if k else None, Ei, v))
    dGdt = (states[2][0] - states[0][0]) / (2 * h)
    _, J1, E1, v1 = states[1]
    J_full = J1 + (v1 * E1[:, None]).sum(axis=0)
    print("dG/dt", dGdt, "J", J_full)
    np.testing.assert_allclose(J_full, dGdt, rtol=2e-4, atol=1e-6 * np.abs(dGdt).max())


# --------------------------------------------------------------------------
# constrained bead centres of mass (Sec. II.C.1, Eqs. 9, 12, 14, 17)
# --------------------------------------------------------------------------
def _aa_water(n_side=3, seed=13, T=300.0):
    spec = W.water_aa_spec(16)
    params = W.draw_params(spec, np.random.default_rng(seed))
    sysm, gs = W.water_atomistic(np.random.SeedSequence(seed), n_side, temperature=T)
    return spec, params, sysm, gs


def _coms(pos, masses, gs, box):
    """Molecule centres of mass with each molecule unwrapped by minimum image
    about its first atom."""
    out = []
    for g in range(gs.size - 1):
        a, b = gs[g], gs[g + 1]
        d = pos[a:b] - pos[a]
        d -= box * np.round(d / box)
        m = masses[a:b]
        out.append(pos[a] + (m[:, None] * d).sum(axis=0) / m.sum())
    return np.array(out)


def test_constraint_holds_every_bead_centre_of_mass():
    spec, params, sysm, gs = _aa_water()
    pos = sysm.pos_f32().astype(np.float64)
    mb = sysm.masses[sysm.types]
    r = oracle.md_ens(spec, params, pos, sysm.vel, sysm.types, sysm.masses, sysm.box, PER, 0.5, 40, group_start=gs)
    c0 = _coms(pos, mb, gs, sysm.box)
    c1 = _coms(r.pos, mb, gs, sysm.box)
    d = c1 - c0
    d -= sysm.box * np.round(d / sysm.box)
    assert np.abs(d).max() < 1e-12
    p = (mb[:, None] * r.vel).reshape(-1, 3, 3).sum(axis=1)
    assert np.abs(p).max() < 1e-12 * np.abs(mb[:, None] * r.vel).max()
    # the atoms did move inside their molecules
    assert np.abs(r.pos - pos).max() > 1e-4
    # the total NEP force vanishes, so the beads' forces sum to zero every step
    assert np.abs(r.F_sum.sum(axis=0)).max() < 1e-9 * np.abs(r.F_sum).max()


def test_constrained_nve_conserves_energy_to_second_order():
    """The constraint forces do no work (the constrained velocities are zero),
    so the constrained run is NVE: the energy error falls ~4x per halving of dt."""
    spec, params, sysm, gs = _aa_water(seed=14, T=500.0)
    pos = sysm.pos_f32().astype(np.float64)
    errs = []
    for dt, n in ((0.5, 40), (0.25, 80)):
        r = oracle.md_ens(spec, params, pos, sysm.vel, sysm.types, sysm.masses, sysm.box, PER, dt, n,
                          group_start=gs)
        E = r.E_pot + r.E_kin
        errs.append(np.abs(E - E[0]).max())
    assert 3.0 < errs[0] / errs[1] < 5.5, errs


def test_single_atom_beads_give_the_static_force_and_virial():
    """Every atom its own bead: the constraint holds every atom in place, so
    the time-averaged bead force and virial are the static force and per-atom
    virial of the starting configuration."""
    spec, params, sysm, _ = _aa_water(n_side=2, seed=15)
    pos = sysm.pos_f32().astype(np.float64)
    n = sysm.n
    gs = np.arange(n + 1)
    r = oracle.md_ens(spec, params, pos, np.zeros((n, 3)), sysm.types, sysm.masses, sysm.box, PER, 0.5, 6,
                      group_start=gs)
    e = oracle.efv(spec, params, pos, sysm.types, sysm.box, PER)
    np.testing.assert_array_equal(r.pos, pos)
    np.testing.assert_allclose(r.F_sum / 6, e.F, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(r.W_sum / 6, e.W, rtol=1e-13, atol=1e-13)


def test_one_bead_holding_every_atom_is_plain_nve():
    spec, params, sysm, _ = _aa_water(n_side=2, seed=16)
    pos = sysm.pos_f32().astype(np.float64)
    v = sysm.vel - (sysm.masses[sysm.types][:, None] * sysm.vel).sum(0) / sysm.masses[sysm.types].sum()
    a = oracle.md_ens(spec, params, pos, v, sysm.types, sysm.masses, sysm.box, PER, 0.5, 20)
    b = oracle.md_ens(spec, params, pos, v, sysm.types, sysm.masses, sysm.box, PER, 0.5, 20,
                      group_start=[0, sysm.n])
    np.testing.assert_allclose(b.pos, a.pos, rtol=0, atol=1e-12)
    np.testing.assert_allclose(b.E_pot, a.E_pot, rtol=1e-12)


def test_virial_correction_adds_the_removed_kinetic_degrees_of_freedom():
    Wb = np.random.default_rng(1).normal(size=(5, 3, 3))
    got = oracle.virial_correction(Wb, 15, 5, 300.0)
    np.testing.assert_allclose(got, Wb.sum(0) + 10 * 8.617333262e-5 * 300.0 * np.eye(3), rtol=1e-15)
