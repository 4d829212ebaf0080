"""Pins of the FP64 oracle against things other than itself.

Each test fixes a part of the oracle by a closed form, a library routine, a
special case, an invariant or a finite difference, chosen so that a plausible
slip (a dropped term, a wrong sign or index, a transposed operand) fails one:

  basis (Eqs. 7-8)        Chebyshev closed form cos(k theta), numpy chebval /
                          chebder, cutoff edge values
  harmonics (Eq. 5)       scipy.special.sph_harm_y (Condon-Shortley), addition
                          theorem, finite-difference gradient
  descriptor (Eqs. 3-5)   two-bead and three-bead closed forms, Legendre double
                          sum on random clusters (scipy eval_legendre)
  network (Eq. 2)         isolated bead, single neuron, identical per-type nets
  forces                  central differences of E, sum F = 0, zero torque
  virial (Eqs. 15-16)     strain derivative of E, per-bead finite differences
                          of U_j, W = sum r_i (x) F_i for open clusters
  invariances             translation, rotation, permutation
  MD                      velocity-Verlet energy error ~ dt^2
"""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as C
from scipy.special import eval_legendre, sph_harm_y

import oracle
import workloads as W

OPEN = np.array([False, False, False])
PER = np.array([True, True, True])


def _basis_lib(K, r, rc):
    """f_k and df_k/dr from numpy's Chebyshev routines (library, not the oracle)."""
    if r > rc:
        return np.zeros(K + 1), np.zeros(K + 1)
    s = r / rc - 1.0
    x = 2 * s * s - 1
    dxdr = 4 * s / rc
    fc = 0.5 * (1 + math.cos(math.pi * r / rc))
    dfc = -0.5 * math.pi / rc * math.sin(math.pi * r / rc)
    f = np.zeros(K + 1)
    df = np.zeros(K + 1)
    for k in range(K + 1):
        e = np.zeros(k + 1)
        e[k] = 1.0
        Tk = C.chebval(x, e)
        dTk = C.chebval(x, C.chebder(e)) if k > 0 else 0.0
        f[k] = 0.5 * (Tk + 1) * fc
        df[k] = 0.5 * dTk * dxdr * fc + 0.5 * (Tk + 1) * dfc
    return f, df


def _ann(spec, parts, t, q):
    w0, b0, w1, b1 = parts["w0"][t], parts["b0"][t], parts["w1"][t], parts["b1"][0]
    z = w0 @ q - b0
    h = np.tanh(z)
    return float(w1 @ h - b1), (w1 * (1 - h * h)) @ w0


# --------------------------------------------------------------------------
# basis
# --------------------------------------------------------------------------
def test_chebyshev_closed_form():
    rc = 0.8
    for r in np.linspace(0.05, 0.79, 23):
        f, _ = oracle.basis(8, r, rc)
        fc = 0.5 * (1 + math.cos(math.pi * r / rc))
        x = 2 * (r / rc - 1) ** 2 - 1
        T = 2 * f / fc - 1
        th = math.acos(x)
        np.testing.assert_allclose(T, [math.cos(k * th) for k in range(9)], atol=1e-12)


def test_basis_matches_numpy_chebyshev():
    for rc in (0.5, 0.8, 2.0):
        for r in np.linspace(0.01, rc * 1.1, 31):
            f, df = oracle.basis(8, r, rc)
            fl, dfl = _basis_lib(8, r, rc)
            np.testing.assert_allclose(f, fl, atol=1e-13)
            np.testing.assert_allclose(df, dfl, atol=1e-11)


def test_basis_edges_and_derivative():
    rc = 0.8
    f, df = oracle.basis(8, rc, rc)
    assert np.abs(f).max() < 1e-15 and np.abs(df).max() < 1e-14
    f, df = oracle.basis(8, rc * 1.0001, rc)
    assert not f.any() and not df.any()
    # derivative against central differences
    h = 1e-6
    for r in (0.11, 0.37, 0.62, 0.79):
        _, df = oracle.basis(8, r, rc)
        fp, _ = oracle.basis(8, r + h, rc)
        fm, _ = oracle.basis(8, r - h, rc)
        np.testing.assert_allclose(df, (fp - fm) / (2 * h), atol=1e-7)


# --------------------------------------------------------------------------
# spherical harmonics
# --------------------------------------------------------------------------
def _dirs(n=40, seed=1):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    d[0] = [0, 0, 1]      # poles and axes
    d[1] = [0, 0, -1]
    d[2] = [1, 0, 0]
    d[3] = [0, -1, 0]
    return d * rng.uniform(0.2, 0.9, (n, 1))


def test_ylm_matches_scipy():
    for d in _dirs():
        r = np.linalg.norm(d)
        theta = math.acos(max(-1.0, min(1.0, d[2] / r)))
        phi = math.atan2(d[1], d[0])
        for l in range(1, 5):
            for m in range(-l, l + 1):
                y, _ = oracle.ylm(l, m, d)
                ref = complex(sph_harm_y(l, m, theta, phi))
                assert abs(y - ref) < 1e-12, (l, m, d, y, ref)


def test_ylm_addition_theorem_and_gradient():
    h = 1e-6
    for d in _dirs(12, 2):
        for l in range(1, 5):
            s = sum(abs(oracle.ylm(l, m, d)[0]) ** 2 for m in range(-l, l + 1))
            assert abs(s - (2 * l + 1) / (4 * math.pi)) < 1e-13
            for m in range(-l, l + 1):
                _, g = oracle.ylm(l, m, d)
                for a in range(3):
                    e = np.zeros(3)
                    e[a] = h
                    fd = (oracle.ylm(l, m, d + e)[0] - oracle.ylm(l, m, d - e)[0]) / (2 * h)
                    assert abs(g[a] - fd) < 1e-7, (l, m, a)


# --------------------------------------------------------------------------
# descriptor closed forms
# --------------------------------------------------------------------------
def _spec1(H=30):
    return W.water_spec(H)


def _params(spec, seed=7, sigma=0.1):
    return W.draw_params(spec, np.random.default_rng(seed), sigma)


def _g(parts, key, t_i, t_j, K, r, rc):
    f, df = _basis_lib(K, r, rc)
    c = parts[key][t_i, t_j]
    return c @ f, c @ df


def test_two_bead_closed_form():
    spec = _spec1()
    p = _params(spec)
    parts = spec.split(p)
    for r in (0.25, 0.45, 0.62):
        pos = np.array([[1.0, 1.0, 1.0], [1.0, 1.0, 1.0]]) + np.array([[0, 0, 0], [0.6, -0.3, 0.7]]) / np.linalg.norm([0.6, -0.3, 0.7]) * np.array([[0], [r]])
        res = oracle.efv(spec, p, pos, [0, 0], [5, 5, 5], OPEN, want_desc=True)
        gR, dgR = _g(parts, "cR", 0, 0, 8, r, 0.8)
        gA, dgA = _g(parts, "cA", 0, 0, 8, r, 0.5)
        q = np.concatenate([gR] + [(2 * l + 1) / (4 * math.pi) * gA ** 2 for l in range(1, 5)])
        dq = np.concatenate([dgR] + [(2 * l + 1) / (4 * math.pi) * 2 * gA * dgA for l in range(1, 5)])
        np.testing.assert_allclose(res.desc[0], q, atol=1e-13)
        np.testing.assert_allclose(res.desc[1], q, atol=1e-13)
        U, dUdq = _ann(spec, parts, 0, q)
        np.testing.assert_allclose(res.U, [U, U], atol=1e-13)
        # E(r) = 2 U(q(r));  F on bead 1 = -dE/dr along the bond
        u = (pos[1] - pos[0]) / r
        F1 = -2 * (dUdq @ dq) * u
        np.testing.assert_allclose(res.F[1], F1, atol=1e-12)
        np.testing.assert_allclose(res.F[0], -F1, atol=1e-12)
        # virial of a pair: W = r_01 (x) F_1 = -r_01 (x) F_0 ... total W = sum_i r_i (x) F_i
        Wt = np.outer(pos[0], res.F[0]) + np.outer(pos[1], res.F[1])
        np.testing.assert_allclose(res.Wtot, Wt, atol=1e-12)


def test_three_bead_legendre_closed_form():
    spec = _spec1()
    p = _params(spec, 11)
    parts = spec.split(p)
    for (r1, r2, th) in ((0.3, 0.42, 0.7), (0.28, 0.31, 2.1), (0.45, 0.33, math.pi - 0.01)):
        o = np.array([2.0, 2.0, 2.0])
        a = np.array([1.0, 0.0, 0.0])
        b = np.array([math.cos(th), math.sin(th), 0.0])
        pos = np.stack([o, o + r1 * a, o + r2 * b])
        res = oracle.efv(spec, p, pos, [0, 0, 0], [6, 6, 6], OPEN, want_desc=True)
        g1, _ = _g(parts, "cA", 0, 0, 8, r1, 0.5)
        g2, _ = _g(parts, "cA", 0, 0, 8, r2, 0.5)
        for l in range(1, 5):
            ref = (2 * l + 1) / (4 * math.pi) * (g1 ** 2 + g2 ** 2 + 2 * g1 * g2 * eval_legendre(l, math.cos(th)))
            got = res.desc[0, 9 + (l - 1) * 7: 9 + l * 7]
            np.testing.assert_allclose(got, ref, atol=1e-13)


def _legendre_descriptor(spec, parts, pos, types, box, pbc, i):
    """q_n and q_nl of bead i by the Legendre double sum (addition theorem)."""
    pairs = oracle.pairs_within(pos, types, spec.n_types, spec.rc_R, box, pbc)
    sel = pairs[pairs[:, 0] == i]
    nR, nA = spec.n_max_R + 1, spec.n_max_A + 1
    qR = np.zeros(nR)
    vecs, gs = [], []
    for (_, j, nx, ny, nz) in sel:
        d = pos[j] + np.array([nx, ny, nz]) * box - pos[i]
        r = np.linalg.norm(d)
        ti, tj = types[i], types[j]
        gR, _ = _g(parts, "cR", ti, tj, spec.basis_R, r, spec.rc_R[ti, tj])
        qR += gR
        if r < spec.rc_A[ti, tj]:
            gA, _ = _g(parts, "cA", ti, tj, spec.basis_A, r, spec.rc_A[ti, tj])
            vecs.append(d / r)
            gs.append(gA)
    qA = np.zeros((spec.l_max, nA))
    if vecs:
        U = np.array(vecs)
        G = np.array(gs)              # (J, nA)
        cos = np.clip(U @ U.T, -1, 1)
        for l in range(1, spec.l_max + 1):
            P = eval_legendre(l, cos)
            qA[l - 1] = (2 * l + 1) / (4 * math.pi) * np.einsum("jn,jk,kn->n", G, P, G)
    return np.concatenate([qR, qA.ravel()])


def test_descriptor_equals_legendre_double_sum_periodic():
    spec, params, system, _ = W.config0()
    parts = spec.split(params)
    pos = system.pos_f32().astype(np.float64)
    res = oracle.efv(spec, params, pos, system.types, system.box, system.pbc, want_desc=True)
    for i in (0, 17, 255, 511):
        ref = _legendre_descriptor(spec, parts, pos, system.types, system.box, system.pbc, i)
        np.testing.assert_allclose(res.desc[i], ref, rtol=1e-11, atol=1e-12)


def test_descriptor_equals_legendre_double_sum_two_types_small_box():
    spec = W.aacg_gold_spec(8)
    params = _params(spec, 5)
    parts = spec.split(params)
    rng = np.random.default_rng(3)
    box = np.array([1.3, 1.45, 1.2])   # smaller than twice the cutoff: self-images
    pos = W.small_cluster(rng, 14, box=1.2, min_dist=0.2) % box
    types = rng.integers(0, 2, 14)
    res = oracle.efv(spec, params, pos, types, box, PER, want_desc=True)
    for i in range(0, 14, 3):
        ref = _legendre_descriptor(spec, parts, pos, types, box, PER, i)
        np.testing.assert_allclose(res.desc[i], ref, rtol=1e-11, atol=1e-12)


# --------------------------------------------------------------------------
# network special cases
# --------------------------------------------------------------------------
def test_isolated_bead():
    spec = _spec1()
    p = _params(spec, 3)
    parts = spec.split(p)
    res = oracle.efv(spec, p, [[1.0, 1.0, 1.0], [3.0, 3.0, 3.0]], [0, 0], [5, 5, 5], OPEN)
    U0 = parts["w1"][0] @ np.tanh(-parts["b0"][0]) - parts["b1"][0]
    np.testing.assert_allclose(res.U, [U0, U0], atol=1e-14)
    assert np.abs(res.F).max() == 0.0 and np.abs(res.W).max() == 0.0


def test_single_neuron():
    spec = W.ModelSpec(n_types=1, n_hidden=1, rc_R=[[0.8]], rc_A=[[0.5]])
    p = _params(spec, 9)
    parts = spec.split(p)
    nu = 13                              # one angular component (l = 1, n = 4)
    w0 = np.zeros_like(parts["w0"])
    w0[0, 0, nu] = 0.7
    parts["w0"] = w0
    p2 = spec.join(parts)
    rng = np.random.default_rng(0)
    pos = W.small_cluster(rng, 6, 0.7, 0.22)
    res = oracle.efv(spec, p2, pos, np.zeros(6, int), [4, 4, 4], OPEN, want_desc=True)
    for i in range(6):
        ref = parts["w1"][0, 0] * math.tanh(0.7 * res.desc[i, nu] - parts["b0"][0, 0]) - parts["b1"][0]
        assert abs(res.U[i] - ref) < 1e-14


def test_identical_per_type_networks_reduce_to_single_network():
    s1 = W.ModelSpec(n_types=1, n_hidden=12, rc_R=[[0.8]], rc_A=[[0.5]])
    s2 = W.ModelSpec(n_types=2, n_hidden=12, rc_R=np.full((2, 2), 0.8), rc_A=np.full((2, 2), 0.5))
    p1 = _params(s1, 21)
    a = s1.split(p1)
    b = {"w0": np.stack([a["w0"][0]] * 2), "b0": np.stack([a["b0"][0]] * 2),
         "w1": np.stack([a["w1"][0]] * 2), "b1": a["b1"],
         "cR": np.broadcast_to(a["cR"][0, 0], (2, 2) + a["cR"].shape[2:]),
         "cA": np.broadcast_to(a["cA"][0, 0], (2, 2) + a["cA"].shape[2:])}
    p2 = s2.join(b)
    spec, params, system, _ = W.config0()
    pos = system.pos_f32().astype(np.float64)
    r1 = oracle.efv(s1, p1, pos, system.types, system.box, PER)
    types2 = np.random.default_rng(1).integers(0, 2, system.n)
    r2 = oracle.efv(s2, p2, pos, types2, system.box, PER)
    np.testing.assert_allclose(r2.U, r1.U, atol=1e-13)
    np.testing.assert_allclose(r2.F, r1.F, atol=1e-12)


# --------------------------------------------------------------------------
# forces and virial by finite differences; invariants
# --------------------------------------------------------------------------
def _rand_box_system(seed, n=20, box=(1.7, 1.9, 1.8)):
    rng = np.random.default_rng(seed)
    box = np.array(box)
    pos = W.small_cluster(rng, n, box=min(box), min_dist=0.21) % box
    return pos, box


@pytest.mark.parametrize("case", ["periodic", "open", "two_types"])
def test_forces_are_minus_energy_gradient(case):
    if case == "two_types":
        spec = W.aacg_gold_spec(10)
    else:
        spec = _spec1(16)
    p = _params(spec, 31)
    pos, box = _rand_box_system(4, 18)
    pbc = OPEN if case == "open" else PER
    types = np.random.default_rng(2).integers(0, spec.n_types, pos.shape[0])
    res = oracle.efv(spec, p, pos, types, box, pbc)
    h = 1e-5
    fd = np.zeros_like(pos)
    for i in range(pos.shape[0]):
        for a in range(3):
            pp = pos.copy(); pp[i, a] += h
            pm = pos.copy(); pm[i, a] -= h
            Ep = oracle.efv(spec, p, pp, types, box, pbc).E
            Em = oracle.efv(spec, p, pm, types, box, pbc).E
            fd[i, a] = -(Ep - Em) / (2 * h)
    scale = np.abs(res.F).max()
    assert np.abs(res.F - fd).max() <= 1e-7 * scale
    assert np.abs(res.F.sum(axis=0)).max() < 1e-12 * max(1.0, scale) * pos.shape[0]


def test_total_virial_is_minus_strain_derivative_open():
    spec = _spec1(16)
    p = _params(spec, 41)
    pos, box = _rand_box_system(5, 16)
    res = oracle.efv(spec, p, pos, np.zeros(16, int), box * 3, OPEN)
    h = 1e-6
    dEde = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            e = np.zeros((3, 3)); e[a, b] = h
            Ep = oracle.efv(spec, p, pos @ (np.eye(3) + e).T, np.zeros(16, int), box * 3, OPEN).E
            Em = oracle.efv(spec, p, pos @ (np.eye(3) - e).T, np.zeros(16, int), box * 3, OPEN).E
            dEde[a, b] = (Ep - Em) / (2 * h)
    # W_{ba} = - dE/d eps_{ab}
    np.testing.assert_allclose(res.Wtot, -dEde.T, atol=1e-7 * np.abs(res.Wtot).max())
    np.testing.assert_allclose(res.Wtot, res.Wtot.T, atol=1e-10 * np.abs(res.Wtot).max())
    # open boundaries: W = sum_i r_i (x) F_i
    np.testing.assert_allclose(res.Wtot, np.einsum("ia,ib->ab", pos, res.F), atol=1e-11)
    # zero total torque
    tq = np.cross(pos, res.F).sum(axis=0)
    assert np.abs(tq).max() < 1e-11


@pytest.mark.parametrize("box", [(1.7, 1.9, 1.8), (1.1, 1.2, 1.05)])
def test_total_virial_diagonal_strain_periodic(box):
    spec = _spec1(16)
    p = _params(spec, 43)
    pos, boxa = _rand_box_system(6, 14, box)
    res = oracle.efv(spec, p, pos, np.zeros(14, int), boxa, PER)
    h = 1e-6
    for a in range(3):
        s = np.ones(3); s[a] += h
        Ep = oracle.efv(spec, p, pos * s, np.zeros(14, int), boxa * s, PER).E
        s = np.ones(3); s[a] -= h
        Em = oracle.efv(spec, p, pos * s, np.zeros(14, int), boxa * s, PER).E
        assert abs(res.Wtot[a, a] + (Ep - Em) / (2 * h)) < 1e-7 * np.abs(res.Wtot).max()
    np.testing.assert_allclose(res.Wtot, res.Wtot.T, atol=1e-10 * np.abs(res.Wtot).max())
    np.testing.assert_allclose(res.W.sum(axis=0), res.Wtot, atol=1e-12)


def test_per_bead_virial_by_finite_differences_of_site_energies():
    """W_i = sum_j r_ij (x) dU_j/dr_ji, and dU_j/dr_ji = dU_j/dr_i on an open cluster."""
    spec = _spec1(16)
    p = _params(spec, 47)
    pos, box = _rand_box_system(8, 12)
    ty = np.zeros(12, int)
    res = oracle.efv(spec, p, pos, ty, box * 3, OPEN)
    h = 1e-6
    for i in (0, 5, 11):
        Wi = np.zeros((3, 3))
        for b in range(3):
            pp = pos.copy(); pp[i, b] += h
            pm = pos.copy(); pm[i, b] -= h
            dU = (oracle.efv(spec, p, pp, ty, box * 3, OPEN).U - oracle.efv(spec, p, pm, ty, box * 3, OPEN).U) / (2 * h)
            for j in range(12):
                if j == i:
                    continue
                Wi[:, b] += (pos[j] - pos[i]) * dU[j]
        np.testing.assert_allclose(res.W[i], Wi, atol=1e-7 * max(1.0, np.abs(Wi).max()))


def test_invariances():
    spec = W.aacg_gold_spec(10)
    p = _params(spec, 51)
    rng = np.random.default_rng(9)
    pos = W.small_cluster(rng, 15, 1.1, 0.2)
    ty = rng.integers(0, 2, 15)
    big = np.array([9.0, 9.0, 9.0])
    base = oracle.efv(spec, p, pos, ty, big, OPEN)
    # translation
    t = oracle.efv(spec, p, pos + [0.31, -0.2, 0.05], ty, big, OPEN)
    np.testing.assert_allclose(t.U, base.U, atol=1e-13)
    np.testing.assert_allclose(t.F, base.F, atol=1e-12)
    # rotation: U invariant, F rotates
    from scipy.spatial.transform import Rotation
    R = Rotation.from_rotvec([0.3, -1.1, 0.7]).as_matrix()
    r = oracle.efv(spec, p, pos @ R.T, ty, big, OPEN)
    np.testing.assert_allclose(r.U, base.U, atol=1e-12)
    np.testing.assert_allclose(r.F, base.F @ R.T, atol=1e-11)
    np.testing.assert_allclose(r.Wtot, R @ base.Wtot @ R.T, atol=1e-11)
    # permutation
    perm = rng.permutation(15)
    q = oracle.efv(spec, p, pos[perm], ty[perm], big, OPEN)
    np.testing.assert_allclose(q.U, base.U[perm], atol=1e-13)
    np.testing.assert_allclose(q.F, base.F[perm], atol=1e-12)
    np.testing.assert_allclose(q.W, base.W[perm], atol=1e-12)
    # periodic translation by a full box vector and by a fraction
    spec1, p1, system, _ = W.config0()
    pos0 = system.pos_f32().astype(np.float64)
    a = oracle.efv(spec1, p1, pos0, system.types, system.box, PER)
    b = oracle.efv(spec1, p1, pos0 + [0.123, 0.77, -0.4], system.types, system.box, PER)
    np.testing.assert_allclose(b.U, a.U, atol=1e-12)
    np.testing.assert_allclose(b.F, a.F, atol=1e-11)


def test_pairs_match_float32_predicate_at_zero_skin():
    from oracle.neighbors_f32 import neighbor_sets
    spec, params, system, _ = W.config0()
    pos32 = system.pos_f32()
    pairs = oracle.pairs_within(pos32.astype(np.float64), system.types, 1, spec.rc_R, system.box.astype(np.float32).astype(np.float64), system.pbc)
    rows = [0, 100, 511]
    sets = neighbor_sets(pos32, system.types, system.box, system.pbc, spec.rc_R, 0.0, rows=rows)
    for i in rows:
        ref = {tuple(x[1:]) for x in pairs[pairs[:, 0] == i].tolist()}
        assert sets[i] == ref


# --------------------------------------------------------------------------
# MD: velocity-Verlet is second order
# --------------------------------------------------------------------------
def test_nve_energy_error_scales_with_dt_squared():
    spec, params, _, _ = W.config0()
    system = W.water_box(np.random.SeedSequence(77), 4, temperature=600.0)
    pos = system.pos_f32().astype(np.float64)
    vel = system.vel
    errs = []
    for dt, n in ((4.0, 25), (2.0, 50)):
        _, _, _, _, Ep, Ek = oracle.md(spec, params, pos, vel, system.types, [W.WATER_MASS], system.box, PER, dt, n)
        E = Ep + Ek
        errs.append(np.abs(E - E[0]).max())
    ratio = errs[0] / errs[1]
    assert 3.0 < ratio < 5.3, (errs, ratio)


# --------------------------------------------------------------------------
# target mode, multi-image pair enumeration, unit constant, strain branch
# --------------------------------------------------------------------------
def test_target_mode_equals_full_evaluation_config0():
    """or_efv with a target subset fills U, F and W of those beads exactly as
    the full evaluation does (it evaluates every bead within reach of a
    target, and sums the same pair terms in the same order)."""
    spec, params, system, _ = W.config0()
    pos = system.pos_f32().astype(np.float64)
    full = oracle.efv(spec, params, pos, system.types, system.box, system.pbc)
    tg = np.random.default_rng(4).choice(system.n, 37, replace=False)
    part = oracle.efv(spec, params, pos, system.types, system.box, system.pbc, targets=tg)
    np.testing.assert_array_equal(part.U[tg], full.U[tg])
    np.testing.assert_array_equal(part.F[tg], full.F[tg])
    np.testing.assert_array_equal(part.W[tg], full.W[tg])
    rest = np.setdiff1d(np.arange(system.n), tg)
    assert np.isnan(part.U[rest]).all() and np.isnan(part.E)


def test_target_mode_equals_full_evaluation_two_types_self_images():
    """The same in a two-type periodic box smaller than twice the cutoff, where
    a bead interacts with several images of a neighbour and of itself."""
    spec = W.aacg_gold_spec(12)
    params = _params(spec, 61)
    rng = np.random.default_rng(62)
    box = np.array([1.25, 1.4, 1.15])
    pos = W.small_cluster(rng, 16, box=1.15, min_dist=0.2) % box
    types = rng.integers(0, 2, 16)
    full = oracle.efv(spec, params, pos, types, box, PER)
    for tg in ([3], [0, 7, 15], list(range(0, 16, 2))):
        part = oracle.efv(spec, params, pos, types, box, PER, targets=tg)
        np.testing.assert_array_equal(part.U[tg], full.U[tg])
        np.testing.assert_array_equal(part.F[tg], full.F[tg])
        np.testing.assert_array_equal(part.W[tg], full.W[tg])


@pytest.mark.parametrize("box", [(0.62, 0.62, 0.62), (0.83, 0.95, 0.7), (1.3, 1.1, 1.25), (0.65, 1.3, 0.9)])
def test_pairs_within_match_brute_force_on_image_boxes(box):
    """The oracle's cell enumeration of periodic images against an independent
    brute force over every image vector in range, on boxes of 0.62-1.3 nm where
    a bead sees several images of the same neighbour (and of itself) inside
    r_c = 0.8 nm.  Every row is compared as a set of (j, image).  No box length
    is a multiple of r_c, where the FP64 and float32 predicates may round a
    self-image pair at exactly r_c differently."""
    from oracle.neighbors_f32 import neighbor_sets
    spec = W.water_spec(8)
    box = np.array(box)
    rng = np.random.default_rng(int(box.sum() * 1000))
    n = 9
    pos = (rng.uniform(0.0, 1.0, (n, 3)) * box).astype(np.float32)
    pairs = oracle.pairs_within(pos.astype(np.float64), np.zeros(n, int), 1, spec.rc_R,
                                box.astype(np.float32).astype(np.float64), PER)
    sets = neighbor_sets(pos, np.zeros(n, int), box, PER, spec.rc_R, 0.0)
    multi = 0
    for i in range(n):
        ref = {tuple(x[1:]) for x in pairs[pairs[:, 0] == i].tolist()}
        assert sets[i] == ref, (i, sorted(sets[i] ^ ref))
        js = [e[0] for e in ref]
        multi += len(js) - len(set(js))
    assert multi > 0, "the box should produce several images of one neighbour"


def test_accel_constant_from_codata():
    """1 eV/nm acting on 1 amu, in nm/fs^2.  The constant is the Faraday
    constant (CODATA 2018, 96485.33212 C/mol) over 1 g/mol, to 1e-12.  From
    the exact elementary charge and the CODATA 2018 atomic mass constant it
    differs by 4e-10 relative (the molar mass constant is 1 g/mol only to
    3.5e-10), far below float32 resolution; a wrong power of ten or an
    inverted ratio fails both checks."""
    faraday = 96485.33212        # C/mol
    a_f = faraday / 1e-3 / 1e-9 * 1e9 / 1e30
    e = 1.602176634e-19          # J per eV (exact)
    u = 1.66053906660e-27        # kg per amu (CODATA 2018)
    a_si = e / 1e-9 / u          # m/s^2
    a = a_si * 1e9 / 1e30        # nm / fs^2
    for c in (oracle.ACCEL, W.ACCEL_EV_NM_AMU):
        assert abs(a_f - c) < 1e-12 * a_f
        assert abs(a - c) < 1e-9 * a


def test_md_strain_branch_with_zero_forces():
    """With every parameter zero the site energies and forces vanish, so a
    strained run is pure kinematics: x_{s+1} = (x_s + dt v) L(s+1)/L(s) along
    the strained axis, the box follows L(s) = L0 (1 + rate s), and velocities
    stay constant.  From rest the positions scale by L(s)/L0 exactly."""
    spec = W.water_spec(6)
    p = np.zeros(spec.n_params)
    rng = np.random.default_rng(71)
    box0 = np.array([3.0, 3.2, 2.9])
    pos0 = rng.uniform(0.1, 2.8, (10, 3))
    rate = np.array([0.0, -2e-3, 5e-3])
    dt, steps, step0 = 2.0, 12, 3
    ty = np.zeros(10, int)
    # from rest: pure affine scaling about the origin
    box_s0 = box0 * (1 + rate * step0)
    pos, vel, F, box, Ep, Ek = oracle.md(spec, p, pos0, np.zeros((10, 3)), ty, [18.0], box_s0, PER, dt, steps,
                                         step0=step0, strain_rate=rate, box0=box0)
    L = box0 * (1 + rate * (step0 + steps))
    np.testing.assert_allclose(box, L, rtol=1e-15)
    np.testing.assert_allclose(pos, pos0 * (L / box_s0), rtol=1e-13)
    assert not F.any() and not Ep.any() and not Ek.any()
    # moving beads: the recurrence in closed form
    v0 = rng.normal(0, 1e-3, (10, 3))
    pos, vel, F, box, Ep, Ek = oracle.md(spec, p, pos0, v0, ty, [18.0], box_s0, PER, dt, steps,
                                         step0=step0, strain_rate=rate, box0=box0)
    x = pos0.copy()
    for s in range(step0, step0 + steps):
        lam = (1 + rate * (s + 1)) / (1 + rate * s)
        x = (x + dt * v0) * lam
    np.testing.assert_allclose(pos, x, rtol=1e-12, atol=1e-14)
    np.testing.assert_array_equal(vel, v0)
    K = 0.5 * 18.0 * (v0 ** 2).sum() / W.ACCEL_EV_NM_AMU
    np.testing.assert_allclose(Ek, K, rtol=1e-13)
