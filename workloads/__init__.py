"""Seeded synthetic inputs for the NEP energy/force/virial path.

This module is shared by the FP64 oracle and the HIP path and therefore holds
none of the method's arithmetic: it only draws positions, types, boxes,
velocities, parameter vectors and request traces from seeded generators, and
describes the flat parameter layout that both sides consume.

Units throughout: nm, eV, amu, fs.

Workload shapes follow the paper's systems:
  * the 512-bead water box of the water example (Sec. III.A),
  * the two-type quasi-hexagonal C60 monolayer (Sec. III.B),
  * the gold AACG model with four atoms per bead and type-pair cutoffs (Sec. III.C),
with random N(0, 0.1^2) parameters standing in for the trained models, which
are not available.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# ---------------------------------------------------------------------------
# unit constants (nm, eV, amu, fs)
# ---------------------------------------------------------------------------
#: acceleration of 1 eV/nm acting on 1 amu, in nm/fs^2
ACCEL_EV_NM_AMU = 9.648533212e-5
#: Boltzmann constant in eV/K
KB_EV = 8.617333262e-5

WATER_DENSITY = 33.4  # beads / nm^3
WATER_MASS = 18.0     # amu
AU_MASS = 196.967     # amu
AU_LATTICE = 0.408    # nm, fcc
BEAD_LATTICE = 0.65   # nm, fcc lattice of 4-atom beads

BASE_SEED = 2603_01234


# ---------------------------------------------------------------------------
# model specification and flat parameter layout
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class ModelSpec:
    """Hyperparameters of one NEP model (Sec. II.A notation).

    ``rc_R`` / ``rc_A`` are [n_types][n_types] symmetric cutoff tables in nm.
    """
    n_types: int = 1
    n_max_R: int = 8
    n_max_A: int = 6
    basis_R: int = 8
    basis_A: int = 8
    l_max: int = 4
    n_hidden: int = 30
    rc_R: np.ndarray = dataclasses.field(default_factory=lambda: np.array([[0.8]]))
    rc_A: np.ndarray = dataclasses.field(default_factory=lambda: np.array([[0.5]]))

    def __post_init__(self):
        self.rc_R = np.asarray(self.rc_R, dtype=np.float64).reshape(self.n_types, self.n_types)
        self.rc_A = np.asarray(self.rc_A, dtype=np.float64).reshape(self.n_types, self.n_types)

    @property
    def n_desc(self) -> int:
        return (self.n_max_R + 1) + (self.n_max_A + 1) * self.l_max

    def layout(self) -> dict:
        """Offsets of the flat parameter vector.

        Order: w0[t][mu][nu], b0[t][mu], w1[t][mu], b1, cR[ti][tj][n][k],
        cA[ti][tj][n][k].  Descriptor index nu: radial n first, then angular
        (l, n) as nu = (n_max_R+1) + (l-1)*(n_max_A+1) + n.
        """
        T, H, D = self.n_types, self.n_hidden, self.n_desc
        sizes = [
            ("w0", T * H * D), ("b0", T * H), ("w1", T * H), ("b1", 1),
            ("cR", T * T * (self.n_max_R + 1) * (self.basis_R + 1)),
            ("cA", T * T * (self.n_max_A + 1) * (self.basis_A + 1)),
        ]
        out, off = {}, 0
        for name, sz in sizes:
            out[name] = (off, sz)
            off += sz
        out["total"] = (0, off)
        return out

    @property
    def n_params(self) -> int:
        return self.layout()["total"][1]

    def split(self, params: np.ndarray) -> dict:
        """Views of the flat vector with their natural shapes."""
        T, H, D = self.n_types, self.n_hidden, self.n_desc
        lay = self.layout()
        p = np.asarray(params)
        shapes = {
            "w0": (T, H, D), "b0": (T, H), "w1": (T, H), "b1": (1,),
            "cR": (T, T, self.n_max_R + 1, self.basis_R + 1),
            "cA": (T, T, self.n_max_A + 1, self.basis_A + 1),
        }
        return {k: p[o:o + s].reshape(shapes[k]) for k, (o, s) in lay.items() if k != "total"}

    def join(self, parts: dict) -> np.ndarray:
        return np.concatenate([np.asarray(parts[k], dtype=np.float64).ravel()
                               for k in ("w0", "b0", "w1", "b1", "cR", "cA")])


def draw_params(spec: ModelSpec, rng: np.random.Generator, sigma: float = 0.1) -> np.ndarray:
    """Every trainable array ~ N(0, sigma^2), drawn in the flat layout order."""
    return rng.normal(0.0, sigma, spec.n_params)


def water_spec(n_hidden: int = 30) -> ModelSpec:
    return ModelSpec(n_types=1, n_hidden=n_hidden, rc_R=[[0.8]], rc_A=[[0.5]])


def aacg_gold_spec(n_hidden: int = 50) -> ModelSpec:
    """Two types (0 = Au atom, 1 = CG bead); mixed cutoffs are arithmetic means,
    and each angular cutoff is 0.1 nm below the radial one (Sec. III.C.2)."""
    rR = np.array([[0.6, 0.8], [0.8, 1.0]])
    return ModelSpec(n_types=2, n_hidden=n_hidden, rc_R=rR, rc_A=rR - 0.1)


def c60_spec(n_hidden: int = 30) -> ModelSpec:
    """Two crystallographically distinct bead types, same radial and angular cutoff."""
    r = np.full((2, 2), 2.0)
    return ModelSpec(n_types=2, n_hidden=n_hidden, rc_R=r, rc_A=r.copy())


# ---------------------------------------------------------------------------
# structures
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class System:
    pos: np.ndarray          # (N, 3) float64, wrapped into [0, L) on periodic dims
    types: np.ndarray        # (N,) uint8
    box: np.ndarray          # (3,) float64
    pbc: np.ndarray          # (3,) bool
    masses: np.ndarray       # (n_types,) amu
    vel: Optional[np.ndarray] = None  # (N, 3) nm/fs
    name: str = ""

    @property
    def n(self) -> int:
        return self.pos.shape[0]

    def pos_f32(self) -> np.ndarray:
        """Float32 copy with every periodic coordinate in [0, L) after rounding."""
        p = wrap_f32(self.pos, self.box, self.pbc)
        return p


def wrap_f32(pos: np.ndarray, box, pbc) -> np.ndarray:
    p = np.array(pos, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    for d in range(3):
        if pbc[d]:
            p[:, d] = np.mod(p[:, d], box[d])
    p32 = p.astype(np.float32)
    L32 = np.asarray(box, dtype=np.float32)
    for d in range(3):
        if pbc[d]:
            col = p32[:, d]
            col[col >= L32[d]] = np.float32(0.0)
            col[col < 0] = np.float32(0.0)
    return p32


def _jittered_sc(rng, n_side: int, spacing: float, jitter: float) -> np.ndarray:
    g = np.arange(n_side, dtype=np.float64) * spacing
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    pos += rng.uniform(-jitter, jitter, pos.shape)
    return pos


def maxwell_velocities(rng, masses_per_bead: np.ndarray, temperature: float) -> np.ndarray:
    """Maxwell-Boltzmann velocities (nm/fs) with the centre-of-mass momentum removed."""
    sigma = np.sqrt(KB_EV * temperature * ACCEL_EV_NM_AMU / masses_per_bead)
    v = rng.normal(size=(masses_per_bead.size, 3)) * sigma[:, None]
    m = masses_per_bead[:, None]
    v -= (m * v).sum(axis=0) / m.sum()
    return v


def water_box(seed_seq: np.random.SeedSequence, n_side: int, density: float = WATER_DENSITY,
              jitter: float = 0.05, temperature: Optional[float] = None) -> System:
    s_pos, s_vel = seed_seq.spawn(2)
    rng = np.random.default_rng(s_pos)
    a = density ** (-1.0 / 3.0)
    L = n_side * a
    pos = _jittered_sc(rng, n_side, a, jitter)
    box = np.array([L, L, L])
    pbc = np.array([True, True, True])
    pos = np.mod(pos, L)
    n = pos.shape[0]
    types = np.zeros(n, dtype=np.uint8)
    masses = np.array([WATER_MASS])
    vel = None
    if temperature is not None:
        vel = maxwell_velocities(np.random.default_rng(s_vel), np.full(n, WATER_MASS), temperature)
    else:
        vel = np.zeros((n, 3))
    return System(pos, types, box, pbc, masses, vel, name=f"water_sc{n_side}")


def water_random_sites(rng, n: int, density: float, jitter: float = 0.05) -> System:
    """n beads on a seeded subset of the smallest simple-cubic lattice with >= n sites."""
    n_side = int(math.ceil(n ** (1.0 / 3.0) - 1e-9))
    while n_side ** 3 < n:
        n_side += 1
    L = (n / density) ** (1.0 / 3.0)
    a = L / n_side
    g = np.arange(n_side) * a
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    sites = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    pick = np.sort(rng.choice(sites.shape[0], size=n, replace=False))
    pos = sites[pick] + rng.uniform(-jitter, jitter, (n, 3))
    box = np.array([L, L, L])
    pos = np.mod(pos, L)
    return System(pos, np.zeros(n, dtype=np.uint8), box, np.array([True, True, True]),
                  np.array([WATER_MASS]), None, name=f"water_rand{n}")


def c60_monolayer(rng, n_target: int, jitter: float = 0.05, a: float = 1.0) -> System:
    """Centred-rectangular cell (a, sqrt(3) a) with type 0 at (0,0) and type 1 at
    (a/2, b/2); periodic in x and y, open in z.  Beads are emitted grouped by type."""
    b = math.sqrt(3.0) * a
    cells = max(1, int(round(n_target / 2)))
    nx = max(1, int(round(math.sqrt(cells * math.sqrt(3.0)))))
    ny = max(1, int(round(cells / nx)))
    Lx, Ly, Lz = nx * a, ny * b, 8.0
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    base = np.stack([i.ravel() * a, j.ravel() * b, np.full(i.size, Lz / 2)], axis=1)
    p0 = base
    p1 = base + np.array([a / 2, b / 2, 0.0])
    pos = np.concatenate([p0, p1], axis=0)
    types = np.concatenate([np.zeros(len(p0), np.uint8), np.ones(len(p1), np.uint8)])
    pos = pos + rng.uniform(-jitter, jitter, pos.shape)
    box = np.array([Lx, Ly, Lz])
    pos[:, 0] = np.mod(pos[:, 0], Lx)
    pos[:, 1] = np.mod(pos[:, 1], Ly)
    return System(pos, types, box, np.array([True, True, False]),
                  np.array([720.0, 720.0]), None, name=f"c60_{nx}x{ny}")


def _fcc(a_xy: float, a_z: float, nxy: int, nz: int) -> np.ndarray:
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    i = np.arange(-nxy, nxy + 1)
    k = np.arange(nz)
    I, J, K = np.meshgrid(i, i, k, indexing="ij")
    cells = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1).astype(np.float64)
    pts = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    pts[:, 0] *= a_xy
    pts[:, 1] *= a_xy
    pts[:, 2] *= a_z
    return pts


def gold_nanowire(seed_seq: np.random.SeedSequence, n_target: int = 200_000,
                  core_radius: float = 1.5, gap: float = 0.2, jitter: float = 0.02,
                  temperature: float = 300.0, au_cells_z: int = 170) -> System:
    """Cylinder along z (periodic, L_z = 170 fcc Au cells); fcc Au core (type 0)
    inside ``core_radius``, fcc CG beads (type 1, lattice 0.65 nm, 107 cells along
    z so the bead lattice is commensurate) outside ``core_radius + gap`` up to the
    radius that brings the total to ``n_target`` sites.  x and y are open.
    ``au_cells_z`` shortens the wire for small test systems (bead cells along z
    are scaled by 107/170 and rounded)."""
    s_pos, s_vel = seed_seq.spawn(2)
    rng = np.random.default_rng(s_pos)
    Lz = au_cells_z * AU_LATTICE
    bead_cells_z = max(1, int(round(au_cells_z * 107 / 170)))
    au = _fcc(AU_LATTICE, AU_LATTICE, int(core_radius / AU_LATTICE) + 2, au_cells_z)
    rho_au = np.hypot(au[:, 0], au[:, 1])
    au = au[rho_au < core_radius]
    a_bz = Lz / bead_cells_z
    n_beads_target = n_target - au.shape[0]
    # outer radius from the bead density 4 / (a^2 a_z)
    dens = 4.0 / (BEAD_LATTICE ** 2 * a_bz)
    r_in = core_radius + gap
    r_out = math.sqrt(n_beads_target / (dens * math.pi * Lz) + r_in ** 2)
    beads = _fcc(BEAD_LATTICE, a_bz, int(r_out / BEAD_LATTICE) + 2, bead_cells_z)
    rho_b = np.hypot(beads[:, 0], beads[:, 1])
    order = np.argsort(rho_b, kind="stable")
    beads, rho_b = beads[order], rho_b[order]
    beads = beads[rho_b >= r_in][:n_beads_target]
    pos = np.concatenate([au, beads], axis=0)
    types = np.concatenate([np.zeros(len(au), np.uint8), np.ones(len(beads), np.uint8)])
    pos = pos + rng.uniform(-jitter, jitter, pos.shape)
    margin = 2.0
    Lxy = 2 * (r_out + margin)
    pos[:, 0] += Lxy / 2
    pos[:, 1] += Lxy / 2
    pos[:, 2] = np.mod(pos[:, 2], Lz)
    # spatial order along z then type keeps neighbours close in memory
    masses = np.array([AU_MASS, 4 * AU_MASS])
    m = masses[types]
    vel = maxwell_velocities(np.random.default_rng(s_vel), m, temperature)
    return System(pos, types, np.array([Lxy, Lxy, Lz]), np.array([False, False, True]),
                  masses, vel, name="au_aacg_wire")


O_MASS, H_MASS = 15.999, 1.008   # amu
OH_BOND, HOH_ANGLE = 0.09572, 104.52   # nm, degrees


def water_aa_spec(n_hidden: int = 60) -> ModelSpec:
    """A two-type atomistic water model (0 = O, 1 = H) standing in for the
    paper's NEP-AA water, whose trained weights are not available: radial
    cutoff 0.5 nm, angular 0.4 nm, 60 neurons."""
    return ModelSpec(n_types=2, n_hidden=n_hidden, rc_R=np.full((2, 2), 0.5), rc_A=np.full((2, 2), 0.4))


def water_atomistic(seed_seq: np.random.SeedSequence, n_side: int, density: float = WATER_DENSITY,
                    jitter: float = 0.03, temperature: float = 300.0):
    """n_side^3 rigid-geometry water molecules (O, H, H, contiguous) with random
    orientations on a jittered simple-cubic lattice of molecule centres, in a
    periodic cube at `density` molecules per nm^3.  Velocities are Maxwell at
    `temperature` with every molecule's centre-of-mass velocity removed.
    Returns (System of 3 n_side^3 atoms, group_start [n_mol + 1])."""
    s_pos, s_rot, s_vel = seed_seq.spawn(3)
    rng = np.random.default_rng(s_pos)
    a = density ** (-1.0 / 3.0)
    L = n_side * a
    centres = _jittered_sc(rng, n_side, a, jitter)
    nm = centres.shape[0]
    half = math.radians(HOH_ANGLE) / 2.0
    local = np.array([[0.0, 0.0, 0.0],
                      [OH_BOND * math.sin(half), 0.0, OH_BOND * math.cos(half)],
                      [-OH_BOND * math.sin(half), 0.0, OH_BOND * math.cos(half)]])
    m = np.array([O_MASS, H_MASS, H_MASS])
    local -= (m[:, None] * local).sum(axis=0) / m.sum()
    rr = np.random.default_rng(s_rot)
    q = rr.normal(size=(nm, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
                  np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
                  np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], 1)
    pos = (centres[:, None, :] + np.einsum("mab,kb->mka", R, local)).reshape(-1, 3)
    pos = np.mod(pos, L)
    types = np.tile(np.array([0, 1, 1], np.uint8), nm)
    masses = np.array([O_MASS, H_MASS])
    mb = masses[types]
    v = maxwell_velocities(np.random.default_rng(s_vel), mb, temperature)
    v = v.reshape(nm, 3, 3)
    mm = mb.reshape(nm, 3)
    v -= (mm[:, :, None] * v).sum(axis=1, keepdims=True) / mm.sum(axis=1)[:, None, None]
    sysm = System(pos, types, np.array([L, L, L]), np.array([True, True, True]), masses, v.reshape(-1, 3),
                  name=f"water_aa_{nm}")
    return sysm, np.arange(0, 3 * nm + 1, 3, dtype=np.int32)


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------
def seeds(config: int) -> np.random.SeedSequence:
    return np.random.SeedSequence(BASE_SEED + config)


def config0():
    """512 water-like beads, one EFV plus 100 NVE steps at dt = 2 fs, v0 = 0."""
    s_sys, s_par = seeds(0).spawn(2)
    spec = water_spec(30)
    system = water_box(s_sys, 8)
    params = draw_params(spec, np.random.default_rng(s_par))
    return spec, params, system, dict(dt=2.0, steps=100, skin=0.1, rebuild_every=10)


def config1():
    """216,000 water-like beads (60^3), Maxwell 300 K, rebuild every 10 steps."""
    s_sys, s_par = seeds(1).spawn(2)
    spec = water_spec(30)
    system = water_box(s_sys, 60, temperature=300.0)
    params = draw_params(spec, np.random.default_rng(s_par))
    return spec, params, system, dict(dt=2.0, steps=1000, skin=0.1, rebuild_every=10)


def config2():
    """200,000-site Au/CG nanowire, H = 50, strain 1e-4 per step along z."""
    s_sys, s_par = seeds(2).spawn(2)
    spec = aacg_gold_spec(50)
    system = gold_nanowire(s_sys)
    params = draw_params(spec, np.random.default_rng(s_par))
    return spec, params, system, dict(dt=5.0, steps=500, skin=0.1, rebuild_every=10,
                                      strain_per_step=(0.0, 0.0, 1e-4))


@dataclasses.dataclass
class FitnessWorkload:
    specs: List[ModelSpec]           # one per family: [water-like, C60-like]
    base_params: List[np.ndarray]    # one per family
    candidates: List[np.ndarray]     # per family: (n_cand, n_params); row 0 = base
    systems: List[System]
    family: np.ndarray               # (n_structures,) 0 = water-like, 1 = C60-like


def config3(n_candidates: int = 64, n_structures: int = 2000, sigma_perturb: float = 0.05,
            size_range=(32, 1024)) -> FitnessWorkload:
    """64 perturbed candidate sets x 2000 periodic structures, sizes log-uniform."""
    s_sz, s_water, s_c60, s_pw, s_pc, s_zw, s_zc = seeds(3).spawn(7)
    rng_sz = np.random.default_rng(s_sz)
    lo, hi = size_range
    n_half = n_structures // 2
    sizes = np.exp(rng_sz.uniform(math.log(lo), math.log(hi), n_structures)).astype(int)
    sizes = np.clip(sizes, lo, hi)
    rw = np.random.default_rng(s_water)
    rc = np.random.default_rng(s_c60)
    systems, fam = [], []
    for s in range(n_structures):
        if s < n_half:
            scale = rw.uniform(0.8, 1.2)
            systems.append(water_random_sites(rw, int(sizes[s]), WATER_DENSITY * scale))
            fam.append(0)
        else:
            systems.append(c60_monolayer(rc, int(sizes[s])))
            fam.append(1)
    specs = [water_spec(30), c60_spec(30)]
    bases = [draw_params(specs[0], np.random.default_rng(s_pw)),
             draw_params(specs[1], np.random.default_rng(s_pc))]
    cands = []
    for f, sz in enumerate((s_zw, s_zc)):
        z = np.random.default_rng(sz).normal(size=(n_candidates, specs[f].n_params))
        c = bases[f][None, :] + sigma_perturb * z
        c[0] = bases[f]
        cands.append(c)
    return FitnessWorkload(specs, bases, cands, systems, np.array(fam))


@dataclasses.dataclass
class ServeWorkload:
    spec: ModelSpec
    params: np.ndarray
    replicas: List[System]
    arrivals_s: np.ndarray   # (n_req,) seconds from start
    replica_of: np.ndarray   # (n_req,) target replica
    steps_per_request: int
    warmup_requests: int


def config4(n_replicas: int = 256, n_requests: int = 20_000, rate_hz: float = 2000.0,
            size_range=(500, 20_000), steps_per_request: int = 10,
            warmup_requests: int = 1000) -> ServeWorkload:
    """Independent water-like replicas at density scale U(1.00, 1.25) with
    config-0 weights; Poisson request trace, each request = 10 MD steps."""
    s_sz, s_sys, s_vel, s_arr, s_tgt = seeds(4).spawn(5)
    spec, params, _, _ = config0()
    rs = np.random.default_rng(s_sz)
    sizes = rs.integers(size_range[0], size_range[1] + 1, n_replicas)
    scales = rs.uniform(1.00, 1.25, n_replicas)
    rp = np.random.default_rng(s_sys)
    rv = np.random.default_rng(s_vel)
    reps = []
    for r in range(n_replicas):
        sysr = water_random_sites(rp, int(sizes[r]), WATER_DENSITY * scales[r])
        sysr.vel = maxwell_velocities(rv, np.full(sysr.n, WATER_MASS), 300.0)
        sysr.name = f"replica{r}"
        reps.append(sysr)
    ra = np.random.default_rng(s_arr)
    gaps = ra.exponential(1.0 / rate_hz, n_requests)
    arrivals = np.cumsum(gaps)
    tgt = np.random.default_rng(s_tgt).integers(0, n_replicas, n_requests)
    return ServeWorkload(spec, params, reps, arrivals, tgt, steps_per_request, warmup_requests)


def small_cluster(rng, n: int, box: float = 1.6, min_dist: float = 0.22) -> np.ndarray:
    """A random open cluster of n points with pairwise distance >= min_dist."""
    pts = []
    while len(pts) < n:
        p = rng.uniform(0.0, box, 3)
        if all(np.linalg.norm(p - q) >= min_dist for q in pts):
            pts.append(p)
    return np.array(pts)


__all__ = [n for n in dir() if not n.startswith("_")]
