"""Property shared by the GPU tests: between rebuilds, the kept Verlet lists
must still hold every pair within r_cut at the current positions (the skin
criterion guarantees it).  Checked with a k-d tree on the current positions,
with a relative margin of 1e-5 below r_cut so that the FP32 predicate's
rounding cannot matter."""
import numpy as np
from scipy.spatial import cKDTree


def assert_lists_cover(counts, cols, pos, L, rc, rows=None, offset=0, n=None):
    """counts, cols: the lists in caller indices (whole context); pos: current
    caller-order positions of the whole context; the system occupies rows
    offset .. offset + n with box L (periodic on every axis)."""
    n = len(pos) - offset if n is None else n
    p = np.asarray(pos[offset:offset + n], np.float64)
    L = np.asarray(L, np.float64)
    p = np.mod(p, L)
    p = np.where(p >= L, p - L, p)
    tree = cKDTree(p, boxsize=L)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    found = tree.query_ball_point(p[rows], rc * (1 - 1e-5))
    checked = 0
    for i, nb in zip(rows, found):
        have = set(cols[offset + i, :counts[offset + i]].tolist())
        for j in nb:
            if j != i:
                assert offset + j in have, (offset, int(i), int(j))
                checked += 1
    assert checked > 0
    return checked
