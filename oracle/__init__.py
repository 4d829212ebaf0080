"""FP64 CPU oracle for the NEP energy / force / virial path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product package.  It shares no
code with the HIP library; the two meet only through the seeded generators in
``workloads``.

``nep_oracle.c`` is the evaluator (Sec. II.A, Eqs. 2-8; Eqs. 15-16);
``neighbors_f32`` is the float32 brute-force neighbour-set reference that uses
the exact list predicate of the library contract.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nep_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
ACCEL = 9.648533212e-5  # nm/fs^2 per (eV/nm)/amu
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 -fopenmp (no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_GNU_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Model(ctypes.Structure):
    _fields_ = [("n_types", ctypes.c_int), ("n_max_R", ctypes.c_int), ("n_max_A", ctypes.c_int),
                ("basis_R", ctypes.c_int), ("basis_A", ctypes.c_int), ("l_max", ctypes.c_int),
                ("n_hidden", ctypes.c_int),
                ("rc_R", ctypes.c_double * 64), ("rc_A", ctypes.c_double * 64)]


class _MdOpts(ctypes.Structure):
    _fields_ = [("thermostat", ctypes.c_int), ("T_target", ctypes.c_double), ("tau_T", ctypes.c_double),
                ("noise", ctypes.POINTER(ctypes.c_double)), ("kB", ctypes.c_double),
                ("barostat", ctypes.c_int), ("P_target", ctypes.c_double * 3), ("tau_P", ctypes.c_double),
                ("beta", ctypes.c_double), ("P_in", ctypes.c_double * 3), ("Fe", ctypes.c_double * 3),
                ("n_groups", ctypes.c_int), ("group_start", ctypes.POINTER(ctypes.c_int)),
                ("F_sum", ctypes.POINTER(ctypes.c_double)), ("W_sum", ctypes.POINTER(ctypes.c_double))]


KB_EV = 8.617333262e-5   # Boltzmann constant, eV/K (CODATA, exact since 2019)


def _load():
    global _lib
    if _lib is None:
        path = build()
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        d, i = ctypes.c_double, ctypes.c_int
        lib.or_basis.argtypes = [i, d, d, P(d), P(d)]
        lib.or_basis.restype = i
        lib.or_ylm.argtypes = [i, i, P(d), P(d), P(d), P(d), P(d)]
        lib.or_ylm.restype = None
        lib.or_efv.argtypes = [P(_Model), P(d), i, P(d), P(i), P(d), P(i), i, P(i),
                               P(d), P(d), P(d), P(d), P(d), P(d), i]
        lib.or_efv.restype = ctypes.c_long
        lib.or_pairs_within.argtypes = [i, P(d), P(i), i, P(d), P(d), P(i), ctypes.c_long,
                                        P(ctypes.c_int32)]
        lib.or_pairs_within.restype = ctypes.c_long
        lib.or_md.argtypes = [P(_Model), P(d), i, P(d), P(d), P(i), P(d), P(d), P(d), P(i),
                              d, i, ctypes.c_long, P(d), d, P(d), P(d), P(d), i]
        lib.or_md.restype = i
        lib.or_md_ens.argtypes = [P(_Model), P(d), i, P(d), P(d), P(i), P(d), P(d), P(d), P(i),
                                  d, i, ctypes.c_long, P(d), d, P(_MdOpts), P(d), P(d), P(d), P(d), P(d), P(d), i]
        lib.or_md_ens.restype = i
        lib.or_param_count.argtypes = [P(_Model)]
        lib.or_param_count.restype = ctypes.c_long
        lib.or_max_threads.restype = i
        _lib = lib
    return _lib


def _ptr(a, ct=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ct)) if a is not None else None


def _model(spec) -> _Model:
    m = _Model()
    m.n_types, m.n_max_R, m.n_max_A = spec.n_types, spec.n_max_R, spec.n_max_A
    m.basis_R, m.basis_A, m.l_max, m.n_hidden = spec.basis_R, spec.basis_A, spec.l_max, spec.n_hidden
    T = spec.n_types
    rr = np.asarray(spec.rc_R, np.float64).reshape(T * T)
    ra = np.asarray(spec.rc_A, np.float64).reshape(T * T)
    for k in range(T * T):
        m.rc_R[k] = float(rr[k])
        m.rc_A[k] = float(ra[k])
    return m


def max_threads() -> int:
    return int(_load().or_max_threads())


def param_count(spec) -> int:
    m = _model(spec)
    return int(_load().or_param_count(ctypes.byref(m)))


def basis(n_basis: int, r: float, rc: float):
    """f_k(r) and df_k/dr for k = 0..n_basis (Eqs. 7-8)."""
    f = np.zeros(n_basis + 1)
    df = np.zeros(n_basis + 1)
    _load().or_basis(n_basis, float(r), float(rc), _ptr(f), _ptr(df))
    return f, df


def ylm(l: int, m: int, d: Sequence[float]):
    """Complex Y_lm (Condon-Shortley) at direction d and its gradient w.r.t. d."""
    dv = np.ascontiguousarray(d, dtype=np.float64)
    re, im = ctypes.c_double(), ctypes.c_double()
    gr, gi = np.zeros(3), np.zeros(3)
    _load().or_ylm(l, m, _ptr(dv), ctypes.byref(re), ctypes.byref(im), _ptr(gr), _ptr(gi))
    return complex(re.value, im.value), gr + 1j * gi


class EFV:
    def __init__(self, U, F, W, E, Wtot, desc, n_pairs):
        self.U, self.F, self.W, self.E, self.Wtot, self.desc, self.n_pairs = U, F, W, E, Wtot, desc, n_pairs


def efv(spec, params, pos, types, box, pbc, targets: Optional[Sequence[int]] = None,
        want_desc: bool = False, n_threads: int = 0) -> EFV:
    """Per-bead U, forces F (n,3), per-bead virial W (n,3,3), totals.

    With ``targets`` only those beads' outputs are computed (others are NaN);
    E and Wtot are then NaN."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    n = pos.shape[0]
    types = np.ascontiguousarray(types, dtype=np.int32)
    params = np.ascontiguousarray(params, dtype=np.float64)
    box = np.ascontiguousarray(box, dtype=np.float64)
    pbc_a = np.ascontiguousarray(np.asarray(pbc).astype(np.int32))
    if params.size != spec.n_params:
        raise ValueError("parameter vector has the wrong length")
    U = np.full(n, np.nan)
    F = np.full((n, 3), np.nan)
    W = np.full((n, 9), np.nan)
    E = ctypes.c_double(np.nan)
    Wt = np.full(9, np.nan)
    desc = np.zeros((n, spec.n_desc)) if want_desc else None
    if targets is None:
        nt, tg = 0, None
    else:
        tg = np.ascontiguousarray(targets, dtype=np.int32)
        nt = tg.size
    m = _model(spec)
    npairs = lib.or_efv(ctypes.byref(m), _ptr(params), n, _ptr(pos), _ptr(types, ctypes.c_int),
                        _ptr(box), _ptr(pbc_a, ctypes.c_int), nt,
                        _ptr(tg, ctypes.c_int) if tg is not None else None,
                        _ptr(U), _ptr(F), _ptr(W), ctypes.byref(E), _ptr(Wt),
                        _ptr(desc) if desc is not None else None, int(n_threads))
    if npairs < 0:
        raise ValueError("oracle rejected the input")
    return EFV(U, F, W.reshape(n, 3, 3), E.value, Wt.reshape(3, 3), desc, npairs)


def pairs_within(pos, types, n_types, rc_table, box, pbc) -> np.ndarray:
    """(i, j, nx, ny, nz) for every ordered pair with |r_ij| < rc(t_i, t_j), FP64."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    types = np.ascontiguousarray(types, dtype=np.int32)
    rc = np.ascontiguousarray(rc_table, dtype=np.float64).reshape(-1)
    box = np.ascontiguousarray(box, dtype=np.float64)
    pbc_a = np.ascontiguousarray(np.asarray(pbc).astype(np.int32))
    cnt = lib.or_pairs_within(pos.shape[0], _ptr(pos), _ptr(types, ctypes.c_int), n_types, _ptr(rc),
                              _ptr(box), _ptr(pbc_a, ctypes.c_int), 0, None)
    out = np.zeros((max(cnt, 1), 5), dtype=np.int32)
    lib.or_pairs_within(pos.shape[0], _ptr(pos), _ptr(types, ctypes.c_int), n_types, _ptr(rc),
                        _ptr(box), _ptr(pbc_a, ctypes.c_int), cnt, _ptr(out, ctypes.c_int32))
    return out[:cnt]


def md(spec, params, pos, vel, types, masses, box, pbc, dt, n_steps, step0=0,
       strain_rate=None, box0=None, n_threads: int = 0):
    """FP64 velocity-Verlet NVE; returns (pos, vel, F, box, E_pot[n_steps], E_kin[n_steps])."""
    lib = _load()
    pos = np.array(pos, dtype=np.float64).reshape(-1, 3).copy()
    vel = np.array(vel, dtype=np.float64).reshape(-1, 3).copy()
    n = pos.shape[0]
    types = np.ascontiguousarray(types, dtype=np.int32)
    masses = np.ascontiguousarray(masses, dtype=np.float64)
    box = np.array(box, dtype=np.float64).copy()
    box0 = np.array(box if box0 is None else box0, dtype=np.float64)
    pbc_a = np.ascontiguousarray(np.asarray(pbc).astype(np.int32))
    params = np.ascontiguousarray(params, dtype=np.float64)
    F = np.zeros((n, 3))
    Ep = np.zeros(max(n_steps, 1))
    Ek = np.zeros(max(n_steps, 1))
    sr = None if strain_rate is None else np.ascontiguousarray(strain_rate, dtype=np.float64)
    m = _model(spec)
    rc = lib.or_md(ctypes.byref(m), _ptr(params), n, _ptr(pos), _ptr(vel), _ptr(types, ctypes.c_int),
                   _ptr(masses), _ptr(box), _ptr(box0), _ptr(pbc_a, ctypes.c_int), float(dt),
                   int(n_steps), int(step0), _ptr(sr) if sr is not None else None, ACCEL,
                   _ptr(F), _ptr(Ep), _ptr(Ek), int(n_threads))
    if rc != 0:
        raise ValueError("oracle md failed")
    return pos, vel, F, box, Ep[:n_steps], Ek[:n_steps]


class MDRun:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def md_ens(spec, params, pos, vel, types, masses, box, pbc, dt, n_steps, step0=0, strain_rate=None, box0=None,
           thermostat=0, T_target=300.0, tau_T=100.0, noise=None, barostat=0, P_target=(0.0, 0.0, 0.0),
           tau_P=1000.0, beta=0.0, P_in=(np.nan, np.nan, np.nan), Fe=(0.0, 0.0, 0.0), group_start=None,
           n_threads: int = 0) -> MDRun:
    """FP64 velocity Verlet with a thermostat (1 Berendsen, 2 Bussi: noise
    [n_steps, 2] of (R, S)), a per-call Berendsen barostat (scale factor from
    P_in, eV/nm^3) and the HNEMD driving force F_e (1/nm).  Returns pos, vel,
    F, box and per-step E_pot, E_kin, W [n_steps, 3, 3], J [n_steps, 3]
    and the mean diagonal pressure P_out (eV/nm^3).  group_start [N_CG + 1]:
    the centre of mass of the atoms of each bead (contiguous ranges) is held
    fixed, and F_sum [N_CG, 3] / W_sum [N_CG, 3, 3] accumulate the beads'
    total atomic forces and virials over the steps (Eqs. 12, 14)."""
    lib = _load()
    pos = np.array(pos, dtype=np.float64).reshape(-1, 3).copy()
    vel = np.array(vel, dtype=np.float64).reshape(-1, 3).copy()
    n = pos.shape[0]
    types = np.ascontiguousarray(types, dtype=np.int32)
    masses = np.ascontiguousarray(masses, dtype=np.float64)
    box = np.array(box, dtype=np.float64).copy()
    box0 = np.array(box if box0 is None else box0, dtype=np.float64)
    pbc_a = np.ascontiguousarray(np.asarray(pbc).astype(np.int32))
    params = np.ascontiguousarray(params, dtype=np.float64)
    F = np.zeros((n, 3))
    k = max(n_steps, 1)
    Ep, Ek, Wt, Jt = np.zeros(k), np.zeros(k), np.zeros((k, 9)), np.zeros((k, 3))
    Pout = np.zeros(3)
    sr = None if strain_rate is None else np.ascontiguousarray(strain_rate, dtype=np.float64)
    o = _MdOpts()
    o.thermostat, o.T_target, o.tau_T, o.kB = int(thermostat), float(T_target), float(tau_T), KB_EV
    nz = None
    if noise is not None:
        nz = np.ascontiguousarray(noise, dtype=np.float64).reshape(-1)
        o.noise = nz.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    o.barostat, o.tau_P, o.beta = int(barostat), float(tau_P), float(beta)
    for d in range(3):
        o.P_target[d] = float(P_target[d])
        o.P_in[d] = float(P_in[d])
        o.Fe[d] = float(Fe[d])
    gs = Fs = Ws = None
    if group_start is not None:
        gs = np.ascontiguousarray(group_start, dtype=np.int32)
        ng = gs.size - 1
        Fs, Ws = np.zeros((ng, 3)), np.zeros((ng, 9))
        o.n_groups = ng
        o.group_start = gs.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        o.F_sum = Fs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        o.W_sum = Ws.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    m = _model(spec)
    rc = lib.or_md_ens(ctypes.byref(m), _ptr(params), n, _ptr(pos), _ptr(vel), _ptr(types, ctypes.c_int),
                       _ptr(masses), _ptr(box), _ptr(box0), _ptr(pbc_a, ctypes.c_int), float(dt), int(n_steps),
                       int(step0), _ptr(sr) if sr is not None else None, ACCEL, ctypes.byref(o), _ptr(F), _ptr(Ep),
                       _ptr(Ek), _ptr(Wt), _ptr(Jt), _ptr(Pout), int(n_threads))
    if rc != 0:
        raise ValueError("oracle md_ens failed")
    return MDRun(pos=pos, vel=vel, F=F, box=box, E_pot=Ep[:n_steps], E_kin=Ek[:n_steps],
                 W=Wt[:n_steps].reshape(-1, 3, 3), J=Jt[:n_steps], P_out=Pout,
                 F_sum=Fs, W_sum=None if Ws is None else Ws.reshape(-1, 3, 3))


def virial_correction(W_bead_mean, n_atoms: int, n_beads: int, T: float):
    """The virial correction of the CG labels (Eq. 17): the total virial
    gains (N_AA - N_CG) k_B T I for the kinetic contribution of the degrees of
    freedom the coarse-graining removes.  W_bead_mean [N_CG, 3, 3]; returns
    the corrected total (3, 3)."""
    return np.asarray(W_bead_mean).sum(axis=0) + (n_atoms - n_beads) * KB_EV * T * np.eye(3)
