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


def check_knn_rows(nl, o_idx, o_r2, o_len, rows, k, r_guard=0.0, dist_atol=4e-6, dist_rtol=2e-6):
    """Checks GPU k-nearest rows against oracle rows.

    o_idx/o_r2/o_len: oracle output for exactly `rows` (row t of the oracle is
    query rows[t]), k + extra entries each in (r^2, j) order; with r_guard the
    oracle must have been run with the guard widened by the band.  A neighbour
    is ambiguous when its r^2 lies within REL of the k-th r^2 (or of
    r_guard^2).  Returns (n_certain, n_ambiguous)."""
    g = gpu_rows(nl, rows)
    m = o_idx.shape[1]
    g2 = r_guard * r_guard
    n_cert = n_amb = 0
    for t, q in enumerate(rows):
        ln = int(o_len[t])
        oi = o_idx[t, :ln]
        orr = o_r2[t, :ln]
        gi, gd = g[int(q)]
        assert len(np.unique(gi)) == len(gi), f"duplicate neighbours in row {q}"
        in_guard = np.ones(ln, bool) if r_guard <= 0 else orr < g2 * (1 + REL)
        sure_guard = np.ones(ln, bool) if r_guard <= 0 else orr < g2 * (1 - REL)
        if len(gi) == k:
            r2k = orr[k - 1] if ln >= k else np.inf
            allowed = (orr <= r2k * (1 + REL)) & in_guard
            certain = (orr < r2k * (1 - REL)) & sure_guard
            # the oracle's extra entries must reach past the band
            assert ln < m or orr[-1] > r2k * (1 + REL), f"row {q}: oracle needs more extra entries"
        else:
            assert len(gi) < k
            allowed = in_guard
            certain = sure_guard
            assert ln < m or (r_guard > 0 and orr[-1] >= g2 * (1 + REL)), f"row {q}: short row"
            assert int(certain.sum()) <= len(gi) <= int(allowed.sum()), (
                f"row {q}: {len(gi)} neighbours, oracle certain {certain.sum()} allowed {allowed.sum()}")
        gs = set(gi.tolist())
        cs = set(oi[certain].tolist())
        al = set(oi[allowed].tolist())
        missing = cs - gs
        extra = gs - al
        assert not missing and not extra, (
            f"row {q}: missing {sorted(missing)[:10]} extra {sorted(extra)[:10]}")
        if len(gi):
            ref = dict(zip(oi.tolist(), orr.tolist()))
            r2 = np.array([ref[j] for j in gi.tolist()])
            if gd is not None:
                r = np.sqrt(r2)
                err = np.abs(gd.astype(np.float64) - r)
                assert np.all(err <= dist_atol + dist_rtol * r), f"row {q}: max dist error {err.max()}"
                assert np.all(np.diff(gd) >= 0), f"row {q}: distances not sorted"
            # sorted by r^2 up to near-ties
            assert np.all(r2[:-1] <= r2[1:] * (1 + 2 * REL) + 1e-12), f"row {q}: order"
        n_cert += len(cs)
        n_amb += len(al) - len(cs)
    return n_cert, n_amb
