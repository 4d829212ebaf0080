"""Float32 brute-force neighbour-set reference (test infrastructure only).

The library promises neighbour lists that equal, as sets, the pairs selected by
this predicate, evaluated in float32 with every operation rounded on its own
(no fused multiply-add):

    s_d  = fl(n_d * L_d)                       n_d an integer image index
    dx_d = fl(fl(x_j,d + s_d) - x_i,d)
    d2   = fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz))
    keep (j, n) != (i, 0) iff d2 < fl32((r_c(t_i, t_j) + skin)^2)

with (r_c + skin)^2 formed in double from the float32 inputs and rounded once.
The paper only says "within a cutoff distance" (Sec. II.A); fixing the
rounding makes the set comparison exact.  numpy evaluates each float32
operation separately, so it never contracts.
"""
from __future__ import annotations

import itertools
import math
from typing import Dict, Iterable, Optional, Set, Tuple

import numpy as np


def cutoff_sq_table(rc_table, skin) -> np.ndarray:
    rc = np.asarray(rc_table, dtype=np.float32).astype(np.float64)
    s = float(np.float32(skin))
    t = rc + s
    return (t * t).astype(np.float32)


def neighbor_sets(pos, types, box, pbc, rc_table, skin, rows: Optional[Iterable[int]] = None,
                  chunk: int = 256) -> Dict[int, Set[Tuple[int, int, int, int]]]:
    """{i: {(j, nx, ny, nz), ...}} for the requested rows (all rows by default)."""
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    n = pos.shape[0]
    types = np.asarray(types).astype(np.int64)
    box32 = np.asarray(box, dtype=np.float32)
    rc2 = cutoff_sq_table(rc_table, skin)
    rcmax = float(np.asarray(rc_table, dtype=np.float32).max()) + float(np.float32(skin))
    rows = np.arange(n) if rows is None else np.asarray(list(rows), dtype=np.int64)
    # per dimension: "single" = one candidate image per pair (box wider than
    # twice the reach), else an explicit range of images.
    mode = []
    for d in range(3):
        if not pbc[d]:
            mode.append(("fixed", [0]))
        elif float(box32[d]) > 2.0 * rcmax + 1e-3:
            mode.append(("single", None))
        else:
            m = int(math.ceil(rcmax / float(box32[d]))) + 1
            mode.append(("fixed", list(range(-m, m + 1))))
    out: Dict[int, Set[Tuple[int, int, int, int]]] = {int(i): set() for i in rows}
    jj = np.arange(n)
    fixed_lists = [mode[d][1] if mode[d][0] == "fixed" else [None] for d in range(3)]
    for c0 in range(0, rows.size, chunk):
        ri = rows[c0:c0 + chunk]
        xi = pos[ri]                     # (c, 3)
        ti = types[ri]
        cut = rc2[ti[:, None], types[None, :]]  # (c, n)
        for combo in itertools.product(*fixed_lists):
            dxs, imgs = [], []
            for d in range(3):
                if combo[d] is None:
                    img = np.rint((xi[:, d, None].astype(np.float64) - pos[None, :, d].astype(np.float64))
                                  / float(box32[d])).astype(np.int64)
                else:
                    img = np.full((ri.size, n), combo[d], dtype=np.int64)
                s = img.astype(np.float32) * box32[d]
                dx = (pos[None, :, d] + s) - xi[:, d, None]
                dxs.append(dx.astype(np.float32))
                imgs.append(img)
            d2 = (dxs[0] * dxs[0] + dxs[1] * dxs[1]) + dxs[2] * dxs[2]
            keep = d2 < cut
            self_zero = (jj[None, :] == ri[:, None]) & (imgs[0] == 0) & (imgs[1] == 0) & (imgs[2] == 0)
            keep &= ~self_zero
            a, b = np.nonzero(keep)
            for r_, j_ in zip(a.tolist(), b.tolist()):
                out[int(ri[r_])].add((j_, int(imgs[0][r_, j_]), int(imgs[1][r_, j_]), int(imgs[2][r_, j_])))
    return out
