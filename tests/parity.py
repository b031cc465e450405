"""Ambiguity-aware comparison of GPU results with the FP64 oracle.

A pair is ambiguous when its oracle r^2 lies within REL (relative) of
r_max^2 or of a histogram edge; the GPU may decide it either way.  Every
other pair must agree exactly.
"""
import numpy as np

REL = 1e-5


def gpu_rows(nl, rows):
    """{query: (point indices, distances)} for the listed queries, on the host."""
    off = nl.offsets.cpu().numpy()
    cnt = nl.counts.cpu().numpy()
    pidx = nl.point_idx.cpu().numpy()
    dist = nl.dist.cpu().numpy() if nl.dist is not None else None
    out = {}
    for q in rows:
        a, c = int(off[q]), int(cnt[q])
        out[int(q)] = (pidx[a:a + c], None if dist is None else dist[a:a + c])
    return out


def check_rows(nl, oracle_csr, rows, r_max, dist_atol=4e-6, dist_rtol=2e-6):
    """Checks GPU rows against oracle rows (oracle_csr computed for exactly `rows`,
    in that order, with r2 limit r_max^2 (1 + REL)).  Returns (n_certain, n_ambiguous)."""
    o_off, o_idx, o_r2 = oracle_csr
    g = gpu_rows(nl, rows)
    lo, hi = r_max ** 2 * (1 - REL), r_max ** 2 * (1 + REL)
    n_cert = n_amb = 0
    for k, q in enumerate(rows):
        oi = o_idx[o_off[k]:o_off[k + 1]]
        orr = o_r2[o_off[k]:o_off[k + 1]]
        certain = oi[orr < lo]
        amb = oi[(orr >= lo) & (orr < hi)]
        gi, gd = g[int(q)]
        assert len(np.unique(gi)) == len(gi), f"duplicate neighbours in row {q}"
        gs = set(gi.tolist())
        cs = set(certain.tolist())
        missing = cs - gs
        extra = gs - cs - set(amb.tolist())
        assert not missing and not extra, (
            f"row {q}: missing {sorted(missing)[:10]} extra {sorted(extra)[:10]}")
        if gd is not None and len(gi):
            ref = dict(zip(oi.tolist(), np.sqrt(orr).tolist()))
            r = np.array([ref[j] for j in gi.tolist()])
            err = np.abs(gd.astype(np.float64) - r)
            assert np.all(err <= dist_atol + dist_rtol * r), f"row {q}: max dist error {err.max()}"
        n_cert += len(certain)
        n_amb += len(amb)
    return n_cert, n_amb


def check_hist(gpu_counts, lo, hi):
    g = np.asarray(gpu_counts, dtype=np.int64)
    lo = lo.astype(np.int64)
    hi = hi.astype(np.int64)
    bad = np.nonzero((g < lo) | (g > hi))[0]
    assert bad.size == 0, f"bins outside [lo, hi]: {bad[:10]} gpu={g[bad[:10]]} lo={lo[bad[:10]]} hi={hi[bad[:10]]}"
