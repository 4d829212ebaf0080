"""The generator of the fused-predicate regression test (CPU): its pairs sit
where separate rounding and a multiply-add disagree, and the float32
brute-force reference follows the separately rounded predicate on them."""
import numpy as np

from gpu_helpers import predicate_edge_pairs
from oracle.neighbors_f32 import cutoff_sq_table, neighbor_sets


def test_edge_pairs_separate_rounding_from_fused():
    rc2 = cutoff_sq_table([[0.8]], 0.1)[0, 0]
    xi, xj = predicate_edge_pairs(np.random.default_rng(1), rc2, 12)
    assert xi.shape == (12, 3)
    d = xj - xi
    sep = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    assert np.all(np.abs(sep.astype(np.float64) / np.float64(rc2) - 1.0) < 1e-6)   # at the cutoff
    # the reference keeps exactly the pairs the separately rounded d2 keeps
    for k in range(12):
        pos = np.stack([xi[k], xj[k]])
        ref = neighbor_sets(pos, np.zeros(2, np.uint8), (50.0, 50.0, 50.0), [False] * 3, [[0.8]], 0.1)
        assert (ref[0] == {(1, 0, 0, 0)}) == bool(sep[k] < rc2)
