"""Order-independent fingerprints of sets of (row, neighbour) pairs.

A NeighborList row set is compared with the oracle's at full size without
storing the oracle's 10^7-10^8 pairs: every pair (key built from frame, row
and neighbour index) is passed through the splitmix64 finaliser (Steele,
Lea and Flood, "Fast splittable pseudorandom number generators", 2014) and
the 64-bit results are summed modulo 2^64 per block of rows.  A missing,
extra or duplicated pair changes its block's sum unless other errors cancel
it exactly, which for unrelated mistakes happens with probability ~2^-64.
This is test infrastructure: it holds none of the analysis arithmetic.
"""
import numpy as np

_C0 = np.uint64(0x9E3779B97F4A7C15)
_C1 = np.uint64(0xBF58476D1CE4E5B9)
_C2 = np.uint64(0x94D049BB133111EB)


def mix(x):
    """splitmix64 output function of uint64 array x (wrapping arithmetic)."""
    x = np.asarray(x, np.uint64) + _C0
    x = (x ^ (x >> np.uint64(30))) * _C1
    x = (x ^ (x >> np.uint64(27))) * _C2
    return x ^ (x >> np.uint64(31))


def keys(rows, nbrs, frame=None):
    """uint64 keys (frame << 44) | (row << 22) | nbr for rows, nbrs < 2^22."""
    k = (np.asarray(rows, np.uint64) << np.uint64(22)) | np.asarray(nbrs, np.uint64)
    if frame is not None:
        k |= np.asarray(frame, np.uint64) << np.uint64(44)
    return k


def block_sums(row_of_pair, h, n_rows, block):
    """Per block of `block` rows: (pair counts int64, wrapping sums of h uint64).
    row_of_pair must be non-decreasing (pairs stored row by row)."""
    nb = (n_rows + block - 1) // block
    b = np.asarray(row_of_pair, np.int64) // block
    edges = np.searchsorted(b, np.arange(nb + 1), side="left")
    cs = np.concatenate([np.zeros(1, np.uint64), np.cumsum(h, dtype=np.uint64)])
    sums = cs[edges[1:]] - cs[edges[:-1]]
    return np.diff(edges).astype(np.int64), sums
