"""ctypes binding of libnep (include/nep.h): argument marshalling only.

Every step of the computation runs in the HIP library; PyTorch supplies device
memory (tensor storage) and the current HIP stream.  If libnep.so is missing
the import fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int, c_int32, c_int64, c_size_t, c_void_p
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnep.so")

NEP_OK = 0
NEP_ERR_ARG = -1
NEP_ERR_HIP = -2
NEP_ERR_NEIGHBOR_OVERFLOW = -3
NEP_ERR_SKIN_VIOLATION = -4
NEP_ERR_NONFINITE = -5
NEP_ERR_OVERLAP = -6
NEP_ERR_UNSUPPORTED = -7
NEP_ERR_OUTSIDE_BOX = -8
# bits of status[0]
NEP_FLAG_OVERFLOW_R = 1
NEP_FLAG_OVERFLOW_A = 2
NEP_FLAG_SKIN = 4
NEP_FLAG_NONFINITE = 8
NEP_FLAG_OUTSIDE_BOX = 16
NEP_FLAG_OVERLAP = 32
NEP_FLAG_IMAGE_RANGE = 64
NEP_FLAG_BAD_TYPE = 128

FLAG_OVERFLOW_R, FLAG_OVERFLOW_A, FLAG_SKIN = 1, 2, 4
FLAG_NONFINITE, FLAG_OUTSIDE_BOX, FLAG_OVERLAP, FLAG_IMAGE_RANGE = 8, 16, 32, 64

EXPORTS = ["nep_param_count", "nep_model_create", "nep_model_destroy", "nep_workspace_bytes",
           "nep_build_neighbors", "nep_compute_efv", "nep_md_step", "nep_check_status",
           "nep_last_error", "nep_timing_begin", "nep_timing_end", "nep_batch_workspace_bytes",
           "nep_compute_efv_batch", "nep_batch_autotune", "nep_md_batch_workspace_bytes", "nep_md_step_batch",
           "nep_sort_system", "nep_compute_efv_noalloc", "nep_models_load_params", "nep_snes_sample",
           "nep_snes_update", "nep_model_set_network"]

NEP_NOALLOC_SCRATCH_BYTES = 64 << 20
NEP_NETWORK_VALU = 0
NEP_NETWORK_MFMA = 1


class NepError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libnep error {code}: {msg}")
        self.code = code


class Hyper(ctypes.Structure):
    _fields_ = [("n_types", c_int), ("n_max_R", c_int), ("n_max_A", c_int), ("basis_R", c_int),
                ("basis_A", c_int), ("l_max", c_int), ("n_hidden", c_int),
                ("rc_R", POINTER(c_float)), ("rc_A", POINTER(c_float))]


class System(ctypes.Structure):
    _fields_ = [("n", c_int), ("x", c_void_p), ("y", c_void_p), ("z", c_void_p), ("type", c_void_p),
                ("box", c_float * 3), ("pbc", c_int * 3)]


class Neighbors(ctypes.Structure):
    _fields_ = [("cap", c_int), ("cap_A", c_int), ("nbr", c_void_p), ("rev", c_void_p),
                ("cnt", c_void_p), ("ref", c_void_p), ("skin", c_float), ("status", c_void_p),
                ("order", c_void_p)]


class Replica(ctypes.Structure):
    _fields_ = [("sys", POINTER(System)), ("v", c_void_p), ("F", c_void_p), ("U", c_void_p),
                ("nbrs", POINTER(Neighbors)), ("ws", c_void_p), ("ws_bytes", c_size_t), ("step", c_int64),
                ("rebuilt", c_int), ("status", c_int)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("block", c_int), ("order", c_int), ("wg_per_cu", c_int), ("schedule", c_int)]


NEP_BATCH_TUNE_CONFIGS = 36


class Labels(ctypes.Structure):
    _fields_ = [("E", c_void_p), ("F", c_void_p), ("W", c_void_p)]


class SnesParams(ctypes.Structure):
    _fields_ = [("lambda_e", c_double), ("lambda_f", c_double), ("lambda_v", c_double), ("lambda_1", c_double),
                ("lambda_2", c_double), ("eta_mu", c_double), ("eta_sigma", c_double)]


class Constraint(ctypes.Structure):
    _fields_ = [("n_groups", c_int), ("group_start", c_void_p), ("F_sum", c_void_p), ("W_sum", c_void_p)]


class MdParams(ctypes.Structure):
    _fields_ = [("dt_fs", c_float), ("n_steps", c_int), ("rebuild_every", c_int), ("force_rebuild", c_int),
                ("mass", c_float * 4),
                ("strain_rate", c_double * 3), ("box0", c_double * 3), ("step", c_int64),
                ("n_rebuilds", c_int), ("pair_counts", c_void_p), ("W_trace", c_void_p), ("W", c_void_p),
                ("thermostat", c_int), ("T_target", c_float), ("tau_T", c_float), ("noise", c_void_p),
                ("barostat", c_int), ("P_target", c_double * 3), ("tau_P", c_double), ("beta", c_double),
                ("P_in", c_double * 3), ("P_out", c_double * 3), ("Fe", c_float * 3), ("J_trace", c_void_p),
                ("constraint", POINTER(Constraint)), ("plain_skin_test", c_int)]


_lib = None


def lib():
    """Loads libnep.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_01234_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.nep_param_count.argtypes = [POINTER(Hyper)]
        L.nep_param_count.restype = c_size_t
        L.nep_model_create.argtypes = [POINTER(Hyper), POINTER(c_float), c_size_t, POINTER(c_void_p)]
        L.nep_model_create.restype = c_int
        L.nep_model_destroy.argtypes = [c_void_p]
        L.nep_model_destroy.restype = c_int
        L.nep_model_set_network.argtypes = [c_void_p, c_int]
        L.nep_model_set_network.restype = c_int
        L.nep_workspace_bytes.argtypes = [c_void_p, c_int, c_int, c_int]
        L.nep_workspace_bytes.restype = c_size_t
        L.nep_build_neighbors.argtypes = [c_void_p, POINTER(System), POINTER(Neighbors), c_int, c_void_p, c_size_t,
                                          c_void_p]
        L.nep_build_neighbors.restype = c_int
        L.nep_compute_efv.argtypes = [c_void_p, POINTER(System), POINTER(Neighbors), c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
        L.nep_compute_efv.restype = c_int
        L.nep_md_step.argtypes = [c_void_p, POINTER(System), c_void_p, POINTER(MdParams), POINTER(Neighbors),
                                  c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
        L.nep_md_step.restype = c_int
        L.nep_check_status.argtypes = [POINTER(Neighbors), POINTER(c_int32), c_void_p]
        L.nep_check_status.restype = c_int
        L.nep_timing_begin.argtypes = [c_int, ctypes.c_uint]
        L.nep_timing_begin.restype = c_int
        L.nep_timing_end.argtypes = [POINTER(c_double), POINTER(c_int)]
        L.nep_timing_end.restype = c_int
        L.nep_batch_workspace_bytes.argtypes = [c_void_p, c_int, c_void_p, c_void_p, c_int, c_int,
                                                POINTER(BatchConfig)]
        L.nep_batch_workspace_bytes.restype = c_size_t
        L.nep_compute_efv_batch.argtypes = [c_void_p, c_int, c_void_p, c_void_p, c_int, c_void_p, c_int,
                                            POINTER(Labels), c_void_p, c_void_p, c_void_p, POINTER(BatchConfig),
                                            c_void_p, c_size_t, c_void_p]
        L.nep_compute_efv_batch.restype = c_int
        L.nep_batch_autotune.argtypes = [c_void_p, c_int, c_void_p, c_void_p, c_int, c_void_p, c_int, c_void_p,
                                         c_size_t, c_void_p, POINTER(BatchConfig), POINTER(c_float),
                                         POINTER(BatchConfig), POINTER(c_int)]
        L.nep_batch_autotune.restype = c_int
        L.nep_md_batch_workspace_bytes.argtypes = [c_int]
        L.nep_md_batch_workspace_bytes.restype = c_size_t
        L.nep_md_step_batch.argtypes = [c_void_p, POINTER(Replica), c_int, c_float, POINTER(c_float), c_int,
                                        c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
        L.nep_md_step_batch.restype = c_int
        L.nep_sort_system.argtypes = [c_void_p, POINTER(System), c_void_p, c_void_p, c_void_p, c_void_p,
                                      POINTER(Neighbors), c_void_p, c_size_t, c_void_p]
        L.nep_sort_system.restype = c_int
        L.nep_compute_efv_noalloc.argtypes = [c_void_p, POINTER(System), POINTER(Neighbors), c_void_p, c_void_p,
                                              c_void_p, c_void_p, c_void_p, c_void_p]
        L.nep_compute_efv_noalloc.restype = c_int
        L.nep_models_load_params.argtypes = [c_void_p, c_int, c_void_p, c_void_p]
        L.nep_models_load_params.restype = c_int
        L.nep_snes_sample.argtypes = [c_int, c_size_t, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
        L.nep_snes_sample.restype = c_int
        L.nep_snes_update.argtypes = [c_int, c_size_t, c_void_p, c_void_p, c_void_p, POINTER(SnesParams), c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_void_p]
        L.nep_snes_update.restype = c_int
        L.nep_last_error.argtypes = []
        L.nep_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def last_error() -> str:
    return lib().nep_last_error().decode()


def check(code: int):
    if code != NEP_OK:
        raise NepError(code, last_error())
    return code


def make_hyper(n_types, n_hidden, rc_R, rc_A, n_max_R=8, n_max_A=6, basis_R=8, basis_A=8, l_max=4):
    rr = np.ascontiguousarray(np.asarray(rc_R, dtype=np.float32).reshape(-1))
    ra = np.ascontiguousarray(np.asarray(rc_A, dtype=np.float32).reshape(-1))
    h = Hyper(n_types, n_max_R, n_max_A, basis_R, basis_A, l_max, n_hidden,
              rr.ctypes.data_as(POINTER(c_float)), ra.ctypes.data_as(POINTER(c_float)))
    h._keep = (rr, ra)  # keep the host tables alive with the struct
    return h


def nep_param_count(h: Hyper) -> int:
    return int(lib().nep_param_count(ctypes.byref(h)))


def nep_model_create(h: Hyper, params: np.ndarray) -> int:
    p = np.ascontiguousarray(params, dtype=np.float32)
    out = c_void_p()
    check(lib().nep_model_create(ctypes.byref(h), p.ctypes.data_as(POINTER(c_float)), p.size, ctypes.byref(out)))
    return out.value


def nep_model_destroy(model: int) -> None:
    check(lib().nep_model_destroy(model))


def nep_model_set_network(model: int, engine: int) -> int:
    """Returns the library's code (NEP_ERR_UNSUPPORTED for a model the
    matrix-core network does not take)."""
    return int(lib().nep_model_set_network(model, engine))


def nep_workspace_bytes(model: int, n: int, cap: int, cap_A: int) -> int:
    return int(lib().nep_workspace_bytes(model, n, cap, cap_A))


def nep_build_neighbors(model, sys: System, nb: Neighbors, wrap: int, ws_ptr, ws_bytes, stream) -> int:
    return lib().nep_build_neighbors(model, ctypes.byref(sys), ctypes.byref(nb), int(wrap), ws_ptr, ws_bytes, stream)


def nep_compute_efv(model, sys: System, nb: Neighbors, U, F, W, E_tot, W_tot, ws_ptr, ws_bytes, stream) -> int:
    return lib().nep_compute_efv(model, ctypes.byref(sys), ctypes.byref(nb), U, F, W, E_tot, W_tot,
                                 ws_ptr, ws_bytes, stream)


def nep_compute_efv_noalloc(model, sys: System, nb: Neighbors, U, F, W, E_tot, W_tot, stream) -> int:
    return lib().nep_compute_efv_noalloc(model, ctypes.byref(sys), ctypes.byref(nb), U, F, W, E_tot, W_tot, stream)


def nep_md_step(model, sys: System, v, mp: MdParams, nb: Neighbors, F, U, E_pot, E_kin, ws_ptr, ws_bytes,
                stream) -> int:
    return lib().nep_md_step(model, ctypes.byref(sys), v, ctypes.byref(mp), ctypes.byref(nb), F, U, E_pot,
                             E_kin, ws_ptr, ws_bytes, stream)


def nep_check_status(nb: Neighbors, stream):
    out = (c_int32 * 4)()
    code = lib().nep_check_status(ctypes.byref(nb), out, stream)
    return code, list(out)


def nep_timing_begin(max_launches: int, class_mask: int = 0xF) -> None:
    """Kernel classes: bit 0 main, 1 gather, 2 build, 3 kick-drift."""
    check(lib().nep_timing_begin(int(max_launches), int(class_mask)))


def nep_timing_end():
    """Returns (ms[4], launches[4]) per kernel class (main, gather, build, kick-drift)."""
    ms = (c_double * 4)()
    cnt = (c_int * 4)()
    check(lib().nep_timing_end(ms, cnt))
    return list(ms), list(cnt)


def _batch_arrays(models, systems, lists, work):
    """Host arrays for the batched calls (kept alive by the caller)."""
    m = (c_void_p * len(models))(*models)
    sy = (System * max(len(systems), 1))(*systems)
    li = (Neighbors * max(len(lists), 1))(*lists)
    w = np.ascontiguousarray(np.asarray(work, dtype=np.int32).reshape(-1, 2))
    return m, sy, li, w


def nep_batch_workspace_bytes(models, systems, lists, n_items: int, cfg: Optional[BatchConfig]) -> int:
    m, sy, li, _ = _batch_arrays(models, systems, lists, np.zeros((0, 2)))
    n = lib().nep_batch_workspace_bytes(m, len(models), sy, li, len(systems), int(n_items),
                                        ctypes.byref(cfg) if cfg is not None else None)
    if n == 0:
        raise NepError(NEP_ERR_ARG, last_error())
    return int(n)


def nep_compute_efv_batch(models, systems, lists, work, labels: Optional[Labels], rmse, item_out, F_out,
                          cfg: Optional[BatchConfig], ws_ptr, ws_bytes, stream) -> int:
    m, sy, li, w = _batch_arrays(models, systems, lists, work)
    return lib().nep_compute_efv_batch(m, len(models), sy, li, len(systems), w.ctypes.data, w.shape[0],
                                       ctypes.byref(labels) if labels is not None else None, rmse, item_out,
                                       F_out, ctypes.byref(cfg) if cfg is not None else None, ws_ptr, ws_bytes,
                                       stream)


def nep_batch_autotune(models, systems, lists, work, ws_ptr, ws_bytes, stream):
    """Returns (best BatchConfig, [ms] per tried configuration, [tried
    BatchConfig], from_cache)."""
    m, sy, li, w = _batch_arrays(models, systems, lists, work)
    best = BatchConfig()
    ms = (c_float * NEP_BATCH_TUNE_CONFIGS)()
    tried = (BatchConfig * NEP_BATCH_TUNE_CONFIGS)()
    hit = c_int(0)
    check(lib().nep_batch_autotune(m, len(models), sy, li, len(systems), w.ctypes.data, w.shape[0], ws_ptr,
                                   ws_bytes, stream, ctypes.byref(best), ms, tried, ctypes.byref(hit)))
    return best, list(ms), list(tried), bool(hit.value)


def nep_md_batch_workspace_bytes(max_active: int) -> int:
    return int(lib().nep_md_batch_workspace_bytes(int(max_active)))


def nep_md_step_batch(model, reps, dt: float, masses, rebuild_every: int, E_pot, E_kin, ws_ptr, ws_bytes,
                      stream) -> int:
    """reps: ctypes array of Replica (its sys / nbrs pointers kept alive by the caller)."""
    m = (c_float * 4)(*[float(masses[t]) if t < len(masses) else 1.0 for t in range(4)])
    return lib().nep_md_step_batch(model, reps, len(reps), float(dt), m, int(rebuild_every), E_pot, E_kin,
                                   ws_ptr, ws_bytes, stream)


def nep_sort_system(model, sys: System, v, F, U, perm, nb: Neighbors, ws_ptr, ws_bytes, stream) -> int:
    return lib().nep_sort_system(model, ctypes.byref(sys), v, F, U, perm, ctypes.byref(nb), ws_ptr, ws_bytes, stream)


def nep_models_load_params(models, params_ptr, stream) -> int:
    m = (c_void_p * len(models))(*models)
    return lib().nep_models_load_params(m, len(models), params_ptr, stream)


def nep_snes_sample(pop: int, dim: int, mu, sigma, s, z, stream) -> int:
    return lib().nep_snes_sample(int(pop), int(dim), mu, sigma, s, z, stream)


def nep_snes_update(pop: int, dim: int, s, z, rmse, h: SnesParams, mu, sigma, loss, order, stream) -> int:
    return lib().nep_snes_update(int(pop), int(dim), s, z, rmse, ctypes.byref(h), mu, sigma, loss, order, stream)
