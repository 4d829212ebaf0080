"""Regression pin: the oracle still reproduces its stored config-0 result."""
import json
import os

import numpy as np

import oracle
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_matches_stored_config0():
    with open(os.path.join(HERE, "golden", "config0_oracle.json")) as f:
        g = json.load(f)
    spec, params, system, _ = W.config0()
    pos = system.pos_f32().astype(np.float64)
    box = system.box.astype(np.float32).astype(np.float64)
    r = oracle.efv(spec, params, pos, system.types, box, system.pbc, want_desc=True)
    assert abs(r.E - g["E_tot"]) < 1e-9
    np.testing.assert_allclose(r.Wtot, g["W_tot"], atol=1e-9)
    np.testing.assert_allclose(r.U[:8], g["U_first8"], atol=1e-12)
    np.testing.assert_allclose(r.F[:8], g["F_first8"], atol=1e-11)
    np.testing.assert_allclose(r.W[0], g["W_bead0"], atol=1e-11)
    np.testing.assert_allclose(r.desc[0], g["desc_bead0"], atol=1e-12)
    assert r.n_pairs == g["n_pairs_within_0.8nm"]
