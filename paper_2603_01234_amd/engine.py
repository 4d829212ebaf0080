"""Device-resident systems on top of the C-ABI.

PyTorch is used only to own device memory and to hand the current HIP stream to
libnep; every step of the NEP evaluation, the neighbour build and the
integrator runs in the library's kernels.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional, Sequence

import numpy as np
import torch

from . import binding as B


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


class Model:
    """An immutable NEP model on the current device."""

    def __init__(self, n_types: int, n_hidden: int, rc_R, rc_A, params: np.ndarray):
        self.n_types = int(n_types)
        self.n_hidden = int(n_hidden)
        self.rc_R = np.asarray(rc_R, dtype=np.float32).reshape(n_types, n_types)
        self.rc_A = np.asarray(rc_A, dtype=np.float32).reshape(n_types, n_types)
        self.hyper = B.make_hyper(n_types, n_hidden, self.rc_R, self.rc_A)
        self.params = np.ascontiguousarray(params, dtype=np.float32)
        self.handle = B.nep_model_create(self.hyper, self.params)

    @classmethod
    def from_spec(cls, spec, params):
        return cls(spec.n_types, spec.n_hidden, spec.rc_R, spec.rc_A, params)

    def set_network(self, engine: str) -> "Model":
        """'valu' (default) or 'mfma': the network of the single-system fused
        kernel on the vector ALUs or on the FP32 matrix cores."""
        code = B.nep_model_set_network(self.handle, {"valu": B.NEP_NETWORK_VALU, "mfma": B.NEP_NETWORK_MFMA}[engine])
        B.check(code)
        return self

    def close(self):
        if self.handle:
            B.nep_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MAX_CAP = 4096      # row capacity limit of the library
MAX_CAP_A = 255     # angular-prefix capacity limit (the build keeps the in-cutoff angular count in a byte)


def estimate_caps(n, box, pbc, rc_max, rcA_max, skin, pos=None):
    """Row capacities from the mean density with head-room; overflow grows them."""
    vol = float(np.prod(box))
    if pos is not None and not all(pbc):
        ext = np.ptp(pos, axis=0) + 1e-3
        for d in range(3):
            if not pbc[d]:
                vol = vol / box[d] * max(ext[d], 1.0)
    rho = n / max(vol, 1e-9)
    cap = int(1.6 * rho * 4.0 / 3.0 * math.pi * (rc_max + skin) ** 3) + 16
    cap_A = int(1.6 * rho * 4.0 / 3.0 * math.pi * (rcA_max + skin) ** 3) + 16
    cap = min(max(cap, 8), MAX_CAP)
    return cap, max(min(cap_A, cap, MAX_CAP_A), 4)


class Replica:
    """One system resident on the device: positions, velocities, forces, lists, workspace."""

    def __init__(self, model: Model, pos: np.ndarray, types: np.ndarray, box, pbc, skin: float = 0.1,
                 vel: Optional[np.ndarray] = None, cap: Optional[int] = None, cap_A: Optional[int] = None,
                 device: str = "cuda"):
        self.model = model
        self.device = torch.device(device)
        pos = np.asarray(pos, dtype=np.float32).reshape(-1, 3)
        self.n = pos.shape[0]
        self.box0 = np.asarray(box, dtype=np.float64).copy()
        self.box = np.asarray(box, dtype=np.float32).copy()
        self.pbc = [int(bool(p)) for p in pbc]
        self.skin = float(skin)
        dev = self.device
        n = max(self.n, 1)
        self.xyz = torch.zeros((3, n), dtype=torch.float32, device=dev)
        if self.n:
            self.xyz[:, :self.n] = torch.from_numpy(np.ascontiguousarray(pos.T)).to(dev)
        self.type = torch.zeros(n, dtype=torch.uint8, device=dev)
        if self.n:
            self.type[:self.n] = torch.from_numpy(np.asarray(types, dtype=np.uint8)).to(dev)
        self.v = torch.zeros((3, n), dtype=torch.float32, device=dev)
        if vel is not None and self.n:
            self.v[:, :self.n] = torch.from_numpy(np.ascontiguousarray(np.asarray(vel, np.float32).T)).to(dev)
        self.F = torch.zeros((3, n), dtype=torch.float32, device=dev)
        self.U = torch.zeros(n, dtype=torch.float32, device=dev)
        self.W = None
        self.E_tot = torch.zeros(1, dtype=torch.float64, device=dev)
        self.W_tot = torch.zeros(9, dtype=torch.float64, device=dev)
        self.status = torch.zeros(4, dtype=torch.int32, device=dev)
        self.ref = torch.zeros((3, n), dtype=torch.float32, device=dev)
        self.cnt = torch.zeros((2, n), dtype=torch.int32, device=dev)
        self.order = torch.zeros(n, dtype=torch.int32, device=dev)   # processing order written by the builds
        if cap is None or cap_A is None:
            c, ca = estimate_caps(self.n, self.box, self.pbc, float(model.rc_R.max()), float(model.rc_A.max()),
                                  self.skin, pos)
            cap = cap or c
            cap_A = cap_A or ca
        self._alloc_lists(cap, cap_A)
        self.step = 0
        self.n_rebuilds = 0
        self.lists_valid = False
        self.perm = None   # after sort(): original index of the bead at each position
        self.P_out = None  # mean diagonal pressure of the last ensemble call (eV/nm^3)
        self.pair_test = True  # MD rebuild gate: the pair test (False: the two-largest test alone)

    # -- buffers ----------------------------------------------------------------
    def _alloc_lists(self, cap, cap_A):
        n = max(self.n, 1)
        self.cap = int(min(cap, MAX_CAP))
        self.cap_A = int(min(cap_A, self.cap, MAX_CAP_A))
        self.nbr = torch.zeros((self.cap, n), dtype=torch.int32, device=self.device)
        self.rev = torch.zeros((self.cap_A, n), dtype=torch.int32, device=self.device)
        self.ws_bytes = B.nep_workspace_bytes(self.model.handle, self.n, self.cap, self.cap_A)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self._cstruct = None

    def c_system(self) -> B.System:
        s = B.System()
        s.n = self.n
        s.x, s.y, s.z = self.xyz[0].data_ptr(), self.xyz[1].data_ptr(), self.xyz[2].data_ptr()
        s.type = self.type.data_ptr()
        for d in range(3):
            s.box[d] = float(self.box[d])
            s.pbc[d] = self.pbc[d]
        return s

    def c_replica(self) -> B.Replica:
        """nep_replica view of this system (cached until the lists are reallocated;
        the box must not change meanwhile)."""
        if self._cstruct is None:
            s, nb = self.c_system(), self.c_neighbors()
            rp = B.Replica(ctypes.pointer(s), self.v.data_ptr(), self.F.data_ptr(), self.U.data_ptr(),
                           ctypes.pointer(nb), self.ws.data_ptr(), self.ws_bytes, 0, 0, 0)
            self._cstruct = (rp, s, nb)
        return self._cstruct[0]

    def c_neighbors(self) -> B.Neighbors:
        nb = B.Neighbors()
        nb.cap, nb.cap_A = self.cap, self.cap_A
        nb.nbr, nb.rev, nb.cnt, nb.ref = (self.nbr.data_ptr(), self.rev.data_ptr(), self.cnt.data_ptr(),
                                          self.ref.data_ptr())
        nb.skin = self.skin
        nb.status = self.status.data_ptr()
        nb.order = self.order.data_ptr()
        return nb

    # -- calls ------------------------------------------------------------------
    def build(self, max_tries: int = 4, wrap: bool = True):
        """nep_build_neighbors (periodic coordinates wrapped in place unless
        wrap=False), growing the row capacities after an overflow."""
        for _ in range(max_tries):
            s, nb = self.c_system(), self.c_neighbors()
            code = B.nep_build_neighbors(self.model.handle, s, nb, int(wrap), self.ws.data_ptr(), self.ws_bytes,
                                         _stream())
            if code == B.NEP_ERR_NEIGHBOR_OVERFLOW:
                st = self.status.cpu().tolist()
                self._alloc_lists(max(self.cap, int(st[1] * 1.2) + 8), max(self.cap_A, int(st[2] * 1.2) + 8))
                continue
            B.check(code)
            self.lists_valid = True
            return
        raise B.NepError(B.NEP_ERR_NEIGHBOR_OVERFLOW, "capacity growth did not converge")

    def efv(self, per_bead_virial: bool = True):
        if not self.lists_valid:
            self.build()
        if per_bead_virial and self.W is None:
            self.W = torch.zeros((9, max(self.n, 1)), dtype=torch.float32, device=self.device)
        s, nb = self.c_system(), self.c_neighbors()
        B.check(B.nep_compute_efv(self.model.handle, s, nb, _ptr(self.U), _ptr(self.F),
                                  _ptr(self.W) if per_bead_virial else None, _ptr(self.E_tot), _ptr(self.W_tot),
                                  self.ws.data_ptr(), self.ws_bytes, _stream()))
        return self

    def sort(self):
        """nep_sort_system: beads back into cell order (with v, F, U and the
        permutation); the host views below keep the original numbering."""
        if self.n == 0:
            return self
        if self.perm is None:
            self.perm = torch.arange(self.n, dtype=torch.int32, device=self.device)
        for _ in range(4):
            s, nb = self.c_system(), self.c_neighbors()
            code = B.nep_sort_system(self.model.handle, s, _ptr(self.v), _ptr(self.F), _ptr(self.U),
                                     _ptr(self.perm), nb, self.ws.data_ptr(), self.ws_bytes, _stream())
            if code == B.NEP_ERR_NEIGHBOR_OVERFLOW:
                st = self.status.cpu().tolist()
                self._alloc_lists(max(self.cap, int(st[1] * 1.2) + 8), max(self.cap_A, int(st[2] * 1.2) + 8))
                self.build(wrap=False)
                return self
            B.check(code)
            self.lists_valid = True
            return self
        return self

    def md(self, n_steps: int, dt: float, masses: Sequence[float], rebuild_every: int = 10,
           strain_rate=(0.0, 0.0, 0.0), E_pot: Optional[torch.Tensor] = None,
           E_kin: Optional[torch.Tensor] = None,
           pair_counts: Optional[torch.Tensor] = None, regrow: bool = True, sort_every: int = 0,
           W_trace: Optional[torch.Tensor] = None, per_bead_virial: bool = False, ensemble: Optional[dict] = None,
           J_trace: Optional[torch.Tensor] = None):
        """nep_md_step; after a rebuild overflow the rows are regrown and the
        remaining steps resumed with a forced rebuild (x, v, F are those of the
        last completed step, so the trajectory continues unchanged).  With
        sort_every > 0 the beads are put back into cell order (sort()) every
        sort_every steps.  W_trace: float64 [n_steps, 9] total virial per step;
        per_bead_virial: self.W holds the per-bead virial at the final step.
        ensemble: nep_md_params ensemble fields (thermostat, T_target, tau_T,
        noise: float64 device tensor [n_steps, 2], barostat, P_target, tau_P,
        beta, P_in, Fe); J_trace: float64 [n_steps, 3] heat current per step.
        The call's mean diagonal pressure is left in self.P_out."""
        if per_bead_virial and self.W is None:
            self.W = torch.zeros((9, max(self.n, 1)), dtype=torch.float32, device=self.device)
        if sort_every and sort_every > 0:
            done = 0
            while done < n_steps:
                k = min(int(sort_every), n_steps - done)
                ens = None
                if ensemble is not None:
                    ens = dict(ensemble)
                    if ens.get("noise") is not None:
                        ens["noise"] = ens["noise"][done:]
                self.md(k, dt, masses, rebuild_every, strain_rate,
                        None if E_pot is None else E_pot[done:], None if E_kin is None else E_kin[done:],
                        pair_counts, regrow, 0, None if W_trace is None else W_trace[done:], per_bead_virial,
                        ens, None if J_trace is None else J_trace[done:])
                done += k
                if done < n_steps:
                    self.sort()
            return self
        if not self.lists_valid:
            self.build()
        remaining = int(n_steps)
        done_total = 0
        force = False
        while True:
            mp = B.MdParams()
            mp.dt_fs = float(dt)
            mp.n_steps = remaining
            mp.rebuild_every = int(rebuild_every)
            mp.force_rebuild = int(force)
            for t in range(4):
                mp.mass[t] = float(masses[t]) if t < len(masses) else 1.0
            for d in range(3):
                mp.strain_rate[d] = float(strain_rate[d])
                mp.box0[d] = float(self.box0[d])
            mp.step = int(self.step)
            mp.pair_counts = _ptr(pair_counts)
            mp.W_trace = None if W_trace is None else W_trace.data_ptr() + 72 * done_total
            mp.W = _ptr(self.W) if per_bead_virial else None
            mp.J_trace = None if J_trace is None else J_trace.data_ptr() + 24 * done_total
            con = None if ensemble is None else ensemble.get("constraint")
            mp.constraint = None if con is None else ctypes.pointer(con)
            mp.plain_skin_test = 0 if self.pair_test else 1
            for d in range(3):
                mp.P_in[d] = float("nan")
            if ensemble:
                e = ensemble
                mp.thermostat = int(e.get("thermostat", 0))
                mp.T_target = float(e.get("T_target", 0.0))
                mp.tau_T = float(e.get("tau_T", 0.0))
                noise = e.get("noise")
                mp.noise = None if noise is None else noise.data_ptr() + 16 * done_total
                mp.barostat = int(e.get("barostat", 0))
                mp.tau_P = float(e.get("tau_P", 0.0))
                mp.beta = float(e.get("beta", 0.0))
                for d in range(3):
                    mp.P_target[d] = float(e.get("P_target", (0.0, 0.0, 0.0))[d])
                    mp.P_in[d] = float(e.get("P_in", (float("nan"),) * 3)[d])
                    mp.Fe[d] = float(e.get("Fe", (0.0, 0.0, 0.0))[d])
            s, nb = self.c_system(), self.c_neighbors()
            ep = None if E_pot is None else E_pot.data_ptr() + 8 * done_total
            ek = None if E_kin is None else E_kin.data_ptr() + 8 * done_total
            code = B.nep_md_step(self.model.handle, s, _ptr(self.v), mp, nb, _ptr(self.F), _ptr(self.U),
                                 ep, ek, self.ws.data_ptr(), self.ws_bytes, _stream())
            done = int(mp.step) - self.step
            self.step = int(mp.step)
            self.n_rebuilds += int(mp.n_rebuilds)
            for d in range(3):
                self.box[d] = s.box[d]
            self.P_out = np.array([mp.P_out[d] for d in range(3)])
            done_total += done
            remaining -= done
            if code == B.NEP_ERR_NEIGHBOR_OVERFLOW and regrow:
                st = self.status.cpu().tolist()
                self._alloc_lists(max(self.cap, int(st[1] * 1.25) + 8), max(self.cap_A, int(st[2] * 1.25) + 8))
                if remaining > 0:
                    force = True
                    continue
                self.build()
                return self
            B.check(code)
            return self

    def npt(self, n_calls: int, steps_per_call: int, dt: float, masses: Sequence[float], P_target, tau_P: float,
            beta: float, thermostat: int = 1, T_target: float = 300.0, tau_T: float = 100.0, rebuild_every: int = 10,
            noise: Optional[torch.Tensor] = None, E_pot=None, E_kin=None, P_in=None):
        """NPT as a sequence of nep_md_step calls: the barostat factor of a
        call comes from the mean pressure of the call before (P_in of the
        first call, non-finite: unscaled).  Returns the per-call boxes and mean
        pressures (eV/nm^3)."""
        P = np.full(3, np.nan) if P_in is None else np.asarray(P_in, np.float64)
        boxes, pressures = [], []
        for c in range(n_calls):
            ens = dict(thermostat=thermostat, T_target=T_target, tau_T=tau_T, barostat=1, P_target=P_target,
                       tau_P=tau_P, beta=beta, P_in=tuple(P))
            if noise is not None:
                ens["noise"] = noise[c * steps_per_call:]
            k0 = c * steps_per_call
            self.md(steps_per_call, dt, masses, rebuild_every,
                    E_pot=None if E_pot is None else E_pot[k0:], E_kin=None if E_kin is None else E_kin[k0:],
                    ensemble=ens)
            P = self.P_out.copy()
            boxes.append(np.asarray(self.box, np.float64).copy())
            pressures.append(P.copy())
        return np.array(boxes), np.array(pressures)

    def constrained_labels(self, group_start: np.ndarray, n_steps: int, dt: float, masses: Sequence[float],
                           T_label: float, rebuild_every: int = 10, E_pot=None, E_kin=None):
        """CG training labels by constrained MD (Sec. II.C.1): NVE with the
        centre of mass of each bead's atoms (contiguous ranges given by
        group_start) held fixed, accumulating the beads' total atomic force
        and virial every step.  Returns the time-averaged bead forces
        [N_CG, 3] (Eq. 12), bead virials [N_CG, 3, 3] (Eq. 14) and the total
        virial with the correction (N_AA - N_CG) k_B T_label I (Eqs. 16-17);
        the accumulation runs in the library's kernels.  The atoms must stay
        in the given order (no sort)."""
        gs = torch.as_tensor(np.asarray(group_start, np.int32), device=self.device).contiguous()
        G = gs.numel() - 1
        Fs = torch.zeros((3, G), dtype=torch.float64, device=self.device)
        Ws = torch.zeros((9, G), dtype=torch.float64, device=self.device)
        con = B.Constraint(G, gs.data_ptr(), Fs.data_ptr(), Ws.data_ptr())
        self.md(n_steps, dt, masses, rebuild_every, E_pot=E_pot, E_kin=E_kin, ensemble=dict(constraint=con))
        F = (Fs / n_steps).T.cpu().numpy()
        Wb = (Ws / n_steps).T.cpu().numpy().reshape(G, 3, 3)
        kB = 8.617333262e-5
        Wtot = Wb.sum(axis=0) + (self.n - G) * kB * T_label * np.eye(3)
        return F, Wb, Wtot

    def device_bytes(self) -> int:
        """Device memory this replica holds (state, lists, workspace)."""
        ts = [self.xyz, self.type, self.v, self.F, self.U, self.E_tot, self.W_tot, self.status, self.ref, self.cnt,
              self.order, self.nbr, self.rev, self.ws]
        if self.W is not None:
            ts.append(self.W)
        if self.perm is not None:
            ts.append(self.perm)
        return int(sum(t.numel() * t.element_size() for t in ts))

    # -- eviction (served form) -------------------------------------------------
    _SNAP = ("xyz", "type", "v", "F", "U", "status", "ref", "cnt", "order", "nbr", "rev")

    def snapshot(self) -> dict:
        """Every device array of the replica (state, lists and their order,
        the numbering map) copied to pinned host memory, so that restore()
        continues the same trajectory bit for bit.  Only the list slots in use
        (up to the longest row) are copied; the host buffers are kept with the
        snapshot and reused by the next one of this replica."""
        cnt_max = self.cnt.amax(dim=1).cpu().tolist() if self.n else [0, 0]
        rows, rows_A = max(int(cnt_max[0]), 1), max(int(cnt_max[1]), 1)
        parts = {k: getattr(self, k) for k in self._SNAP if k not in ("nbr", "rev")}
        parts["nbr"] = self.nbr[:rows]
        parts["rev"] = self.rev[:rows_A]
        if self.perm is not None:
            parts["perm"] = self.perm
        pool = getattr(self, "_pinned", None) or {}
        snap = {}
        for k, t in parts.items():
            buf = pool.get(k)
            if buf is None or buf.numel() < t.numel():
                buf = torch.empty(t.numel(), dtype=t.dtype, pin_memory=True)
                pool[k] = buf
            dst = buf[:t.numel()].view(t.shape)
            dst.copy_(t, non_blocking=True)
            snap[k] = dst
        torch.cuda.current_stream().synchronize()
        self._pinned = pool
        snap.setdefault("perm", None)
        snap.update(step=self.step, n_rebuilds=self.n_rebuilds, box=self.box.copy(), cap=self.cap,
                    cap_A=self.cap_A, lists_valid=self.lists_valid, pool=pool)
        return snap

    def restore(self, snap: dict):
        """The inverse of snapshot() on a replica of the same system."""
        if (self.cap, self.cap_A) != (snap["cap"], snap["cap_A"]):
            self._alloc_lists(snap["cap"], snap["cap_A"])
        for k in self._SNAP:
            src = snap[k]
            getattr(self, k)[:src.shape[0]].copy_(src, non_blocking=True)
        self.perm = None if snap["perm"] is None else snap["perm"].to(self.device, non_blocking=True)
        torch.cuda.current_stream().synchronize()
        self._pinned = snap["pool"]
        self.step, self.n_rebuilds = snap["step"], snap["n_rebuilds"]
        self.box = snap["box"].copy()
        self.lists_valid = snap["lists_valid"]
        self._cstruct = None
        return self

    # -- host views (original numbering unless internal=True) ---------------------
    def _unperm(self, a: np.ndarray, internal: bool) -> np.ndarray:
        if internal or self.perm is None:
            return a
        out = np.empty_like(a)
        out[self.perm.cpu().numpy()] = a
        return out

    def positions(self, internal: bool = False) -> np.ndarray:
        return self._unperm(self.xyz[:, :self.n].T.contiguous().cpu().numpy(), internal)

    def forces(self, internal: bool = False) -> np.ndarray:
        return self._unperm(self.F[:, :self.n].T.contiguous().cpu().numpy(), internal)

    def velocities(self, internal: bool = False) -> np.ndarray:
        return self._unperm(self.v[:, :self.n].T.contiguous().cpu().numpy(), internal)

    def site_energies(self, internal: bool = False) -> np.ndarray:
        return self._unperm(self.U[:self.n].cpu().numpy(), internal)

    def virials(self, internal: bool = False) -> np.ndarray:
        return self._unperm(self.W[:, :self.n].T.contiguous().cpu().numpy().reshape(-1, 3, 3), internal)

    def neighbor_rows(self):
        """Host copy of the lists: (entries [cap, n] uint32, counts [2, n])."""
        return (self.nbr.cpu().numpy().view(np.uint32), self.cnt.cpu().numpy())


def decode_row(entries: np.ndarray):
    e = entries.astype(np.uint64)
    j = (e & 0x1FFFFFF).astype(np.int64)
    code = (e >> 25).astype(np.int64)
    nx = code % 5 - 2
    ny = (code // 5) % 5 - 2
    nz = code // 25 - 2
    return j, nx, ny, nz


class FitnessBatch:
    """Candidates of one model family scored on many structures in one
    persistent launch (nep_compute_efv_batch).  The structures stay resident
    with their lists, built once and shared by every candidate."""

    def __init__(self, models: Sequence[Model], replicas: Sequence[Replica]):
        if not models:
            raise ValueError("need at least one model")
        self.models = list(models)
        self.replicas = list(replicas)
        for r in self.replicas:
            if not r.lists_valid:
                r.build()
        self.device = self.replicas[0].device if self.replicas else torch.device("cuda")
        self.labels = None
        self._ws = None
        self._ws_key = None

    def _c(self):
        return ([m.handle for m in self.models], [r.c_system() for r in self.replicas],
                [r.c_neighbors() for r in self.replicas])

    def all_pairs(self):
        """Every (candidate, structure) pair, candidate-major."""
        return [(m, s) for m in range(len(self.models)) for s in range(len(self.replicas))]

    def set_labels(self, E, F, W):
        """E: [S] eV; F: [sum_s n_s, 3] eV/nm in structure order; W: [S, 9] eV."""
        dev = self.device
        self.labels = (torch.as_tensor(np.asarray(E, np.float64), device=dev).contiguous(),
                       torch.as_tensor(np.asarray(F, np.float64).reshape(-1, 3), device=dev).contiguous(),
                       torch.as_tensor(np.asarray(W, np.float64).reshape(-1, 9), device=dev).contiguous())

    def _workspace(self, n_items: int):
        key = n_items
        if self._ws is None or self._ws_key != key:
            models, systems, lists = self._c()
            nbytes = B.nep_batch_workspace_bytes(models, systems, lists, n_items, None)
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self._ws_key = key
        base = self._ws.data_ptr()
        off = (-base) % 256
        return base + off, self._ws.numel() - off

    def autotune(self, work=None):
        work = self.all_pairs() if work is None else work
        ws, nbytes = self._workspace(len(work))
        models, systems, lists = self._c()
        return B.nep_batch_autotune(models, systems, lists, work, ws, nbytes, _stream())

    def evaluate(self, work=None, cfg: Optional[B.BatchConfig] = None, rmse: bool = True,
                 items: bool = False, forces: bool = False):
        """Returns dict with 'rmse' [n_models, 3] (RMSE_E eV/bead, RMSE_F eV/nm,
        RMSE_W eV/bead), 'items' [n_items, 10] (E, W) and 'forces' [rows, 3]."""
        work = self.all_pairs() if work is None else work
        n_items = len(work)
        ws, nbytes = self._workspace(n_items)
        models, systems, lists = self._c()
        dev = self.device
        out = {}
        lab = None
        if rmse:
            if self.labels is None:
                raise ValueError("labels are not set")
            lab = B.Labels(self.labels[0].data_ptr(), self.labels[1].data_ptr(), self.labels[2].data_ptr())
            out["rmse"] = torch.zeros((len(self.models), 3), dtype=torch.float64, device=dev)
        if items:
            out["items"] = torch.zeros((max(n_items, 1), 10), dtype=torch.float64, device=dev)
        if forces:
            rows = sum(self.replicas[s].n for _, s in work)
            out["forces"] = torch.zeros((max(rows, 1), 3), dtype=torch.float32, device=dev)
        B.check(B.nep_compute_efv_batch(models, systems, lists, work, lab, _ptr(out.get("rmse")),
                                        _ptr(out.get("items")), _ptr(out.get("forces")), cfg, ws, nbytes,
                                        _stream()))
        return out


class SnesTrainer:
    """The training loop of the paper (Sec. II.A) on the device: SNES over a
    population of candidate parameter vectors, each scored by the persistent
    fitness kernel against reference labels.  mu and sigma stay on the device;
    a generation is four stream-ordered library calls (sample, load the
    candidates into the population's models, batched RMSEs, update), with the
    standard normal draws either given or drawn with torch on the device."""

    def __init__(self, spec, mu0: np.ndarray, sigma0, pop: int, replicas: Sequence[Replica], labels,
                 weights=(1.0, 1.0, 0.1, 0.0, 0.0), eta=None, seed: int = 0, device: str = "cuda"):
        self.pop = int(pop)
        self.dim = int(mu0.size)
        self.device = torch.device(device)
        self.models = [Model.from_spec(spec, mu0.astype(np.float32)) for _ in range(self.pop)]
        self.batch = FitnessBatch(self.models, replicas)
        self.batch.set_labels(*labels)
        dev = self.device
        self.mu = torch.as_tensor(np.asarray(mu0, np.float32), device=dev).contiguous()
        sig = np.broadcast_to(np.asarray(sigma0, np.float32), (self.dim,)).copy()
        self.sigma = torch.as_tensor(sig, device=dev).contiguous()
        self.z = torch.empty((self.pop, self.dim), dtype=torch.float32, device=dev)
        self.loss = torch.empty(self.pop, dtype=torch.float64, device=dev)
        self.order = torch.empty(self.pop, dtype=torch.int32, device=dev)
        if eta is None:
            eta = (1.0, (3.0 + math.log(self.dim)) / (5.0 * math.sqrt(self.dim)))
        self.h = B.SnesParams(*[float(x) for x in weights], float(eta[0]), float(eta[1]))
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(int(seed))
        self.rmse = None

    def generation(self, s: Optional[torch.Tensor] = None, cfg: Optional[B.BatchConfig] = None):
        """One generation; s: float32 [pop, dim] standard normals on the
        device (drawn here when None).  Returns s."""
        if s is None:
            s = torch.randn((self.pop, self.dim), generator=self.gen, device=self.device, dtype=torch.float32)
        s = s.contiguous()
        st = _stream()
        B.check(B.nep_snes_sample(self.pop, self.dim, self.mu.data_ptr(), self.sigma.data_ptr(), s.data_ptr(),
                                  self.z.data_ptr(), st))
        B.check(B.nep_models_load_params([m.handle for m in self.models], self.z.data_ptr(), st))
        res = self.batch.evaluate(cfg=cfg, rmse=True)
        self.rmse = res["rmse"]
        B.check(B.nep_snes_update(self.pop, self.dim, s.data_ptr(), self.z.data_ptr(), self.rmse.data_ptr(), self.h,
                                  self.mu.data_ptr(), self.sigma.data_ptr(), self.loss.data_ptr(),
                                  self.order.data_ptr(), st))
        return s

    def close(self):
        for m in self.models:
            m.close()


def replica_footprint(model: Model, n: int, box, pbc, skin: float, pos=None) -> int:
    """Device bytes a Replica of n beads holds: state, lists and workspace."""
    cap, cap_A = estimate_caps(n, np.asarray(box, np.float32), pbc, float(model.rc_R.max()),
                               float(model.rc_A.max()), skin, pos)
    n1 = max(n, 1)
    state = n1 * (4 * 3 * 5 + 4 + 1 + 4 * 2)          # xyz, v, F, ref, vh-less state, U, type, cnt
    lists = 4 * n1 * (cap + cap_A)
    return state + lists + B.nep_workspace_bytes(model.handle, n, cap, cap_A)


class MdStepBatch:
    """One velocity-Verlet step for many resident replicas per call
    (nep_md_step_batch)."""

    def __init__(self, model: Model, dt: float, masses: Sequence[float], rebuild_every: int = 10,
                 max_active: int = 256, device: str = "cuda"):
        self.model = model
        self.dt = float(dt)
        self.masses = list(masses)
        self.rebuild_every = int(rebuild_every)
        self.max_active = int(max_active)
        nbytes = B.nep_md_batch_workspace_bytes(self.max_active)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self._ws.data_ptr()
        self._ws_ptr = base + (-base) % 256
        self._ws_bytes = self._ws.numel() - (-base) % 256
        self.E_pot = torch.zeros(self.max_active, dtype=torch.float64, device=device)
        self.E_kin = torch.zeros(self.max_active, dtype=torch.float64, device=device)

    def step(self, reps: Sequence[Replica]):
        """Advances every replica by one step; returns the per-replica status
        codes (a replica whose rebuild overflowed is regrown, rebuilt and left
        at its last step, its code NEP_ERR_NEIGHBOR_OVERFLOW)."""
        if len(reps) > self.max_active:
            raise ValueError("more replicas than max_active")
        if not reps:
            return []
        arr = (B.Replica * len(reps))()
        for k, r in enumerate(reps):
            if not r.lists_valid:
                r.build()
            arr[k] = r.c_replica()
            arr[k].step = r.step
        B.check(B.nep_md_step_batch(self.model.handle, arr, self.dt,
                                    self.masses, self.rebuild_every, self.E_pot.data_ptr(), self.E_kin.data_ptr(),
                                    self._ws_ptr, self._ws_bytes, _stream()))
        codes = []
        for k, r in enumerate(reps):
            r.step = int(arr[k].step)
            r.n_rebuilds += int(arr[k].rebuilt)
            code = int(arr[k].status)
            if code == B.NEP_ERR_NEIGHBOR_OVERFLOW:
                st = r.status.cpu().tolist()
                r._alloc_lists(max(r.cap, int(st[1] * 1.25) + 8), max(r.cap_A, int(st[2] * 1.25) + 8))
                r.build()
            elif code != B.NEP_OK:
                raise B.NepError(code, f"replica {k}: step failed")
            codes.append(code)
        return codes


class Server:
    """Continuous batching of MD requests over independent replicas.

    A request advances one replica by a number of steps; requests for a busy
    replica wait in order.  Replicas stay on the host until a request needs
    them, are admitted to the device when their footprint fits the HBM budget
    (idle resident replicas are evicted least recently used to make room), and
    then stay resident with their lists.  Every tick advances each replica
    with an active request by one step in one nep_md_step_batch call; requests
    that arrived meanwhile join at the next tick and finished ones leave.
    A replica is put into cell order (Replica.sort) when it is admitted and
    every sort_every of its steps (0: never), which keeps the neighbour
    gathers of its workgroups local as the beads diffuse."""

    def __init__(self, model: Model, systems, skin: float, dt: float, masses: Sequence[float],
                 rebuild_every: int = 10, hbm_budget: Optional[int] = None, max_active: int = 256,
                 clock=None, sort_every: int = 100):
        import collections
        import time
        self.model = model
        self.skin = float(skin)
        self.masses = list(masses)
        self.host = [dict(pos=np.asarray(s.pos_f32()), vel=np.asarray(s.vel, np.float32), types=s.types,
                          box=np.asarray(s.box, np.float64), pbc=s.pbc, step=0) for s in systems]
        self.footprint = [replica_footprint(model, h["pos"].shape[0], h["box"], h["pbc"], self.skin, h["pos"])
                          for h in self.host]
        self.budget = hbm_budget if hbm_budget is not None else sum(self.footprint)
        self.stepper = MdStepBatch(model, dt, masses, rebuild_every, max_active)
        self.max_active = int(max_active)
        self.resident = collections.OrderedDict()   # replica id -> Replica, least recently used first
        self.used = 0
        self.pending = collections.OrderedDict()    # replica id -> deque of [req, steps_left, t_arrival, steps]
        self.active = collections.OrderedDict()     # replica id -> [req, steps_left, t_arrival, steps]
        self.done = []                              # (req, replica, t_arrival, t_done, bead-steps)
        self.ticks = 0
        self.evictions = 0
        self.admissions = 0
        self.clock = clock or time.perf_counter
        self.sort_every = int(sort_every)

    # -- residency ------------------------------------------------------------
    def _admit(self, rid: int) -> bool:
        need = self.footprint[rid]
        if need > self.budget:
            raise ValueError(f"replica {rid} alone exceeds the HBM budget")
        while self.used + need > self.budget:
            victim = next((k for k in self.resident if k not in self.active), None)
            if victim is None:
                return False
            self._evict(victim)
        h = self.host[rid]
        r = Replica(self.model, h["pos"], h["types"], h["box"], h["pbc"], skin=self.skin, vel=h["vel"],
                    cap=h["snap"]["cap"] if "snap" in h else None, cap_A=h["snap"]["cap_A"] if "snap" in h else None)
        if "snap" in h:
            r.restore(h["snap"])                    # the state it was evicted with, lists included
        else:
            r.step = h["step"]
            if self.sort_every > 0:
                r.sort()                            # cell order, lists built
            r.efv(per_bead_virial=False)            # lists and forces at the stored positions
        self.resident[rid] = r
        self.footprint[rid] = r.device_bytes()      # the estimate replaced by what the replica holds
        self.used += self.footprint[rid]
        self.admissions += 1
        return True

    def _evict(self, rid: int):
        r = self.resident.pop(rid)
        h = self.host[rid]
        h["pos"], h["vel"], h["step"] = r.positions(), r.velocities(), r.step
        h["snap"] = r.snapshot()
        self.used -= self.footprint[rid]
        self.evictions += 1
        del r

    def replica(self, rid: int) -> Optional[Replica]:
        return self.resident.get(rid)

    # -- requests -------------------------------------------------------------
    def submit(self, req: int, rid: int, n_steps: int, t_arrival: float):
        import collections
        self.pending.setdefault(rid, collections.deque()).append([req, int(n_steps), float(t_arrival), int(n_steps)])

    def idle(self) -> bool:
        return not self.active and not self.pending

    def tick(self) -> int:
        """Admits waiting requests, runs one batched step; returns requests completed."""
        for rid in list(self.pending.keys()):
            if len(self.active) >= self.max_active:
                break
            if rid in self.active:
                continue
            if rid not in self.resident and not self._admit(rid):
                continue
            q = self.pending[rid]
            self.active[rid] = q.popleft()
            if not q:
                del self.pending[rid]
        if not self.active:
            return 0
        rids = list(self.active.keys())
        reps = [self.resident[k] for k in rids]
        codes = self.stepper.step(reps)
        self.ticks += 1
        t = self.clock()
        finished = 0
        for rid, r, code in zip(rids, reps, codes):
            self.resident.move_to_end(rid)
            if code != B.NEP_OK:
                continue                            # lists regrown; the step runs again next tick
            if self.sort_every > 0 and r.step % self.sort_every == 0:
                r.sort()
            a = self.active[rid]
            a[1] -= 1
            if a[1] == 0:
                del self.active[rid]
                self.done.append((a[0], rid, a[2], t, r.n * a[3]))
                finished += 1
        return finished
