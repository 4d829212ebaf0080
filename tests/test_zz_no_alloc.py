"""The allocation-free evaluation (nep_compute_efv_noalloc) through the C-ABI
against nep_compute_efv on the same lists: identical results, bit for bit,
on two calls in a row (the second on a smaller system, so stale contents of
the shared static scratch must not leak into it), and a clear error for an
evaluation that does not fit the static scratch (needs an MI355X)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _replica(system, spec, params, skin=0.1):
    from paper_2603_01234_amd import engine as E
    model = E.Model.from_spec(spec, params)
    rep = E.Replica(model, system.pos_f32(), system.types, system.box, system.pbc, skin=skin)
    rep._keep = model
    rep.build()
    return rep


def _both(rep):
    """(U, F, W, E, W_tot) from nep_compute_efv and from the allocation-free call."""
    from paper_2603_01234_amd import binding as B
    st = torch.cuda.current_stream().cuda_stream
    outs = []
    for noalloc in (False, True):
        n = max(rep.n, 1)
        U = torch.full((n,), np.nan, dtype=torch.float32, device="cuda")
        F = torch.full((3, n), np.nan, dtype=torch.float32, device="cuda")
        Wb = torch.full((9, n), np.nan, dtype=torch.float32, device="cuda")
        E = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
        Wt = torch.full((9,), np.nan, dtype=torch.float64, device="cuda")
        s, nb = rep.c_system(), rep.c_neighbors()
        if noalloc:
            code = B.nep_compute_efv_noalloc(rep.model.handle, s, nb, U.data_ptr(), F.data_ptr(), Wb.data_ptr(),
                                             E.data_ptr(), Wt.data_ptr(), st)
        else:
            code = B.nep_compute_efv(rep.model.handle, s, nb, U.data_ptr(), F.data_ptr(), Wb.data_ptr(),
                                     E.data_ptr(), Wt.data_ptr(), rep.ws.data_ptr(), rep.ws_bytes, st)
        B.check(code)
        torch.cuda.synchronize()
        outs.append((U, F, Wb, E, Wt))
    return outs


def test_noalloc_equals_workspace_call_twice_second_smaller():
    spec, params, system, opts = W.config1()
    # a 13,824-bead box of the config-1 model (fits the static scratch), then config 0 (512 beads)
    big = W.water_box(np.random.SeedSequence(11), 24, temperature=300.0)
    for sysm in (big, system if False else W.config0()[2]):
        rep = _replica(sysm, spec, params, opts["skin"])
        ref, got = _both(rep)
        print(f"n={rep.n}: comparing {len(ref)} outputs", flush=True)
        for a, b in zip(ref, got):
            assert torch.isfinite(a).all()
            assert torch.equal(a, b)


def test_noalloc_rejects_an_evaluation_beyond_the_static_scratch():
    from paper_2603_01234_amd import binding as B
    spec, params, system, opts = W.config1()
    rep = _replica(system, spec, params, opts["skin"])   # 216,000 beads: far beyond 64 MiB of scratch
    s, nb = rep.c_system(), rep.c_neighbors()
    code = B.nep_compute_efv_noalloc(rep.model.handle, s, nb, rep.U.data_ptr(), rep.F.data_ptr(), None, None,
                                     None, torch.cuda.current_stream().cuda_stream)
    assert code == B.NEP_ERR_ARG
    assert "static array" in B.last_error()
