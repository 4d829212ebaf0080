"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nep.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(nep_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2603_01234_amd import binding as B
    L = B.lib()
    names = _declared()
    assert "nep_compute_efv" in names and "nep_md_step" in names and "nep_build_neighbors" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(B.EXPORTS) == set(names)


def test_param_count_matches_layout():
    from paper_2603_01234_amd import binding as B
    import workloads as W
    for spec in (W.water_spec(30), W.aacg_gold_spec(50), W.c60_spec(30)):
        h = B.make_hyper(spec.n_types, spec.n_hidden, spec.rc_R, spec.rc_A)
        assert B.nep_param_count(h) == spec.n_params
    assert B.nep_param_count(B.make_hyper(0, 30, [0.8], [0.5])) == 0


def test_model_create_rejects_bad_hyperparameters_without_device_work():
    from paper_2603_01234_amd import binding as B
    import workloads as W
    spec = W.water_spec(30)
    p = np.zeros(spec.n_params, np.float32)
    bad = [
        (B.make_hyper(1, 30, [0.8], [0.5], l_max=3), B.NEP_ERR_UNSUPPORTED),
        (B.make_hyper(5, 30, np.ones(25), np.ones(25)), B.NEP_ERR_UNSUPPORTED),
        (B.make_hyper(1, 65, [0.8], [0.5]), B.NEP_ERR_UNSUPPORTED),
        (B.make_hyper(1, 30, [0.5], [0.8]), B.NEP_ERR_UNSUPPORTED),   # angular above radial
        (B.make_hyper(1, 30, [-0.8], [0.5]), B.NEP_ERR_ARG),
        (B.make_hyper(2, 30, [0.8, 0.7, 0.6, 0.8], [0.5] * 4), B.NEP_ERR_ARG),  # asymmetric
    ]
    for h, code in bad:
        out = ctypes.c_void_p()
        n = B.nep_param_count(h)
        q = np.zeros(max(n, 1), np.float32)
        rc = B.lib().nep_model_create(ctypes.byref(h), q.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n,
                                      ctypes.byref(out))
        assert rc == code, (rc, B.last_error())
        assert out.value is None
    h = B.make_hyper(1, 30, [0.8], [0.5])
    out = ctypes.c_void_p()
    rc = B.lib().nep_model_create(ctypes.byref(h), p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), p.size - 1,
                                  ctypes.byref(out))
    assert rc == B.NEP_ERR_ARG and "expected" in B.last_error()
    p2 = p.copy()
    p2[3] = np.nan
    rc = B.lib().nep_model_create(ctypes.byref(h), p2.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), p2.size,
                                  ctypes.byref(out))
    assert rc == B.NEP_ERR_ARG and "non-finite" in B.last_error()


def test_calls_reject_null_model_and_bad_structs():
    from paper_2603_01234_amd import binding as B
    s = B.System()
    nb = B.Neighbors()
    assert B.nep_build_neighbors(None, s, nb, 0, None, 0, None) == B.NEP_ERR_ARG
    assert B.nep_compute_efv(None, s, nb, None, None, None, None, None, None, 0, None) == B.NEP_ERR_ARG
    mp = B.MdParams()
    assert B.nep_md_step(None, s, None, mp, nb, None, None, None, None, None, 0, None) == B.NEP_ERR_ARG
    code, _ = B.nep_check_status(nb, None)
    assert code == B.NEP_ERR_ARG
    assert B.lib().nep_workspace_bytes(None, 10, 8, 4) == 0


def test_binding_constants_match_header():
    """Status codes and flag bits in the binding equal the header's values."""
    from paper_2603_01234_amd import binding as B
    txt = open(HEADER).read()
    flags = dict((k, int(v)) for k, v in re.findall(r"#define\s+(NEP_FLAG_[A-Z_]+)\s+(\d+)", txt))
    codes = dict((k, int(v)) for k, v in re.findall(r"\b(NEP_(?:OK|ERR_[A-Z_]+))\s*=\s*(-?\d+)", txt))
    assert len(flags) == 8 and len(codes) >= 9
    for k, v in list(flags.items()) + list(codes.items()):
        assert getattr(B, k) == v, k


def test_md_params_layout_matches_header():
    """Field order of nep_md_params in the binding follows the header."""
    from paper_2603_01234_amd import binding as B
    txt = open(HEADER).read()
    body = txt[txt.index("typedef struct {\n    float dt_fs;"):txt.index("} nep_md_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"\b([A-Za-z_0-9]+)(?:\[\d+\])?;", body)
    assert names == [f[0] for f in B.MdParams._fields_]


def _struct_fields(txt, name):
    """Field names of a typedef struct in the header, in order."""
    end = txt.index("} " + name + ";")
    start = txt.rindex("typedef struct {", 0, end)
    body = re.sub(r"/\*.*?\*/", "", txt[start + len("typedef struct {"):end], flags=re.S)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        # "float *x, *y, *z" declares three fields
        for part in decl.split(","):
            m = re.search(r"([A-Za-z_0-9]+)\s*(?:\[[^\]]*\])?\s*$", part.strip())
            out.append(m.group(1))
    return out


@pytest.mark.parametrize("cname,pyname", [("nep_neighbors", "Neighbors"), ("nep_system", "System"),
                                          ("nep_replica", "Replica"), ("nep_batch_config", "BatchConfig"),
                                          ("nep_labels", "Labels"), ("nep_md_params", "MdParams")])
def test_struct_layouts_match_header(cname, pyname):
    """Every C-ABI struct of the header and its ctypes mirror in the binding
    have the same fields in the same order."""
    from paper_2603_01234_amd import binding as B
    txt = open(HEADER).read()
    assert _struct_fields(txt, cname) == [f[0] for f in getattr(B, pyname)._fields_]


def test_library_unit_constant_matches_codata():
    """The library's acceleration unit (1 eV/nm on 1 amu in nm/fs^2) is the
    Faraday constant over 1 g/mol, the value the oracle is pinned to."""
    src = open(os.path.join(ROOT, "paper_2603_01234_amd", "csrc", "nep_internal.h")).read()
    val = float(re.search(r"ACCEL\s*=\s*([0-9.eE+-]+)f", src).group(1))
    assert abs(val - 96485.33212 / 1e-3 / 1e-9 * 1e9 / 1e30) < 1e-12 * val
