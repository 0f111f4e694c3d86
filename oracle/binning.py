"""Integer index build reported by the GPU plan, recomputed for bit-exact checks.

The plan reports its binning parameters (x0, y0, inv_c, ncx, ncy, nsub, ntx).
Fine cell indices are fx = clamp(floor((x - x0) * inv_c), 0, ncx - 1) (and the
same in y) in FP64 with one subtraction and one multiplication; the tile of a
cell is (fx // nsub, fy // nsub) and the sort key orders points by tile, then
by fine cell inside the tile.  A stable sort by key gives the permutation;
CSR rows are the sorted points, columns the sorted positions of their
neighbours (Section 1, fixed-radius neighbour search) in ascending order.
"""
import numpy as np

from .nearfield import near_pairs


def bin_keys(z, x0, y0, inv_c, ncx, ncy, nsub, ntx):
    z = np.asarray(z, dtype=np.float64)
    fx = np.floor((z[:, 0] - x0) * inv_c)
    fy = np.floor((z[:, 1] - y0) * inv_c)
    fx = np.clip(fx, 0, ncx - 1).astype(np.int64)
    fy = np.clip(fy, 0, ncy - 1).astype(np.int64)
    tile = (fy // nsub) * ntx + (fx // nsub)
    return tile * (nsub * nsub) + (fy % nsub) * nsub + (fx % nsub)


def stable_perm(keys):
    """Sorted position -> original index, stable in the original index."""
    return np.argsort(keys, kind="stable")


def csr_from_perm(z, perm, delta_min):
    """row_ptr [N+1] and col (sorted positions, ascending per row), diagonal included."""
    zs = np.asarray(z, dtype=np.float64)[perm]
    k, l = near_pairs(zs, delta_min)
    n = len(zs)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, k + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr, l.astype(np.int64)
