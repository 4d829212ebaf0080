"""Writes tests/golden/config0_oracle.json from the FP64 oracle alone.

The paper prints no worked NEP evaluation, so the stored values here are the
oracle's own result on the seeded 512-bead water-like box; they guard the
oracle's arithmetic against silent change (any intended change must rerun
this script and name the passage that justifies it).

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def main():
    spec, params, system, _ = W.config0()
    pos = system.pos_f32().astype(np.float64)
    box = system.box.astype(np.float32).astype(np.float64)
    r = oracle.efv(spec, params, pos, system.types, box, system.pbc, want_desc=True)
    out = {
        "what": "FP64 oracle on the seeded 512-bead water-like box (config 0 inputs), float32-rounded positions",
        "E_tot": r.E,
        "W_tot": r.Wtot.tolist(),
        "U_first8": r.U[:8].tolist(),
        "F_first8": r.F[:8].tolist(),
        "W_bead0": r.W[0].tolist(),
        "desc_bead0": r.desc[0].tolist(),
        "n_pairs_within_0.8nm": int(r.n_pairs),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config0_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
