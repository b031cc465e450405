#!/usr/bin/env python3
"""Writes the full-size expected values of the GPU parity tests.

Calls only the FP64 oracle (`oracle/`, brute force over every (query,
point) pair) and the seeded input generators; nothing here comes from the
GPU library.  One run takes a few hours on 8 host cores.  Outputs (numpy
.npz, compressed), one per workload:

  fluid2d_pmft200.npz  2D fluid N = 262,144: 200 x 200 PMFT count bounds on
                       [-3, 3)^2, bonds within r_max = 3 (self-query).
  fcc1M_ball_rdf.npz   noisy FCC N = 1,048,576, tilts (0.5, 0.2, 0.1): ball
                       query r_max = 2.5 (self-query) and its 256-bin RDF on
                       [0, 2.5): RDF bounds, and per block of 4096 rows the
                       count and pair-hash sum of the certain pairs (r^2 below
                       r_max^2 (1 - 1e-5)); the pairs in the cutoff band are
                       listed explicitly.
  traj256_ball_rdf.npz the 256-frame trajectory: per frame the 128-bin RDF
                       bounds on [0, 2.5) and the count and hash sum of its
                       certain ball pairs (r_max = 2.5), plus the band pairs.
  fcc1M_knn12.npz      the FCC system's k = 12 nearest rows: per block of
                       4096 rows the count and hash sum over rows whose 12th
                       and 13th neighbours are farther apart than the band;
                       rows with a near-tie at rank 12 are stored in full
                       (their first 16 candidates and squared distances).

Usage: python tests/golden/make_golden.py [names...]   (default: all)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import oracle  # noqa: E402
import pairhash  # noqa: E402
from paper_1906_06317_amd import workloads  # noqa: E402

REL = oracle.REL_BAND
BLOCK = 4096
CHUNK = 16384
T0 = time.time()


def log(msg):
    print(f"[{time.time() - T0:8.1f} s] {msg}", file=sys.stderr, flush=True)


def meta(**kw):
    kw["generated_by"] = "tests/golden/make_golden.py (FP64 brute-force oracle)"
    kw["oracle_threads"] = oracle.num_threads()
    return np.array(json.dumps(kw))


def ball_sweep(sysm, r_max, bins, cap, frame=None, label=""):
    """All self-query rows of sysm: RDF bounds, per-block certain counts and
    hash sums, and the band pairs (rows, nbrs)."""
    ob = oracle.make_box(sysm.L, sysm.tilt, sysm.dim)
    n = sysm.points.shape[0]
    lo = np.zeros(bins, np.uint64)
    hi = np.zeros(bins, np.uint64)
    namb = np.zeros(1, np.uint64)
    r2_sure = r_max * r_max * (1.0 - REL)
    nb = (n + BLOCK - 1) // BLOCK
    bcount = np.zeros(nb, np.int64)
    bsum = np.zeros(nb, np.uint64)
    amb_r, amb_j, amb_r2 = [], [], []
    for a in range(0, n, CHUNK):
        b = min(n, a + CHUNK)
        cnt, idx, r2, lo, hi, namb = oracle.ball_rdf_rows(ob, sysm.points, r_max, bins, rows=(a, b),
                                                          cap=cap, lo=lo, hi=hi, n_amb=namb)
        valid = np.arange(cap)[None, :] < cnt[:, None]
        rows = np.broadcast_to(np.arange(a, b)[:, None], idx.shape)
        sure = valid & (r2 < r2_sure)
        band = valid & ~(r2 < r2_sure)
        amb_r.append(rows[band])
        amb_j.append(idx[band])
        amb_r2.append(r2[band])
        rr, jj = rows[sure], idx[sure]  # row-major: rows non-decreasing
        h = pairhash.mix(pairhash.keys(rr, jj, frame))
        c, s = pairhash.block_sums(rr - a, h, b - a, BLOCK)
        k0 = a // BLOCK
        bcount[k0:k0 + len(c)] += c
        bsum[k0:k0 + len(s)] += s
        if (a // CHUNK) % 8 == 0:
            log(f"{label} rows {b}/{n}")
    return dict(hist_lo=lo, hist_hi=hi, n_amb_hist=namb, block_count=bcount, block_hash=bsum,
                band_rows=np.concatenate(amb_r).astype(np.int32),
                band_nbrs=np.concatenate(amb_j).astype(np.int32),
                band_r2=np.concatenate(amb_r2))


def make_pmft(out):
    s = workloads.fluid_2d()
    ob = oracle.make_box(s.L, s.tilt, s.dim)
    log("2D fluid PMFT 200x200: start")
    lo, hi, namb = oracle.pmft2d_counts(ob, s.points, None, s.theta, 200, 200, 3.0, 3.0, 3.0)
    log(f"2D fluid PMFT done: {int(lo.sum())} certain pairs, {namb} ambiguous")
    np.savez_compressed(out, lo=lo.astype(np.uint32), hi_minus_lo=(hi - lo).astype(np.uint16),
                        n_amb=np.array(namb),
                        meta=meta(workload="fluid_2d(seed=1003): N=262144, density 0.7",
                                  nbx=200, nby=200, x_max=3.0, y_max=3.0, r_max=3.0,
                                  exclude_ii=True, rel_band=REL, abs_band=REL * 3.0))


def make_fcc_ball(out):
    s = workloads.large_fcc()
    log("FCC 2^20 ball + RDF: start")
    d = ball_sweep(s, 2.5, 256, 160, label="FCC ball")
    log(f"FCC ball done: {int(d['block_count'].sum())} certain pairs, "
        f"{len(d['band_rows'])} band pairs")
    np.savez_compressed(out, block=np.array(BLOCK), **d,
                        meta=meta(workload="large_fcc(seed=1002): 64^3 FCC cells, a=4^(1/3), "
                                           "noise 0.05a, tilts (0.5,0.2,0.1), N=1048576",
                                  r_max=2.5, bins=256, r_min=0.0, exclude_ii=True, rel_band=REL,
                                  hash="pairhash.mix(pairhash.keys(row, nbr))"))


def make_traj(out):
    frames = workloads.trajectory()
    F = len(frames)
    lo = np.zeros((F, 128), np.uint64)
    hi = np.zeros((F, 128), np.uint64)
    fcount = np.zeros(F, np.int64)
    fsum = np.zeros(F, np.uint64)
    band = {"frame": [], "rows": [], "nbrs": [], "r2": []}
    log("trajectory: start")
    for f, s in enumerate(frames):
        d = ball_sweep(s, 2.5, 128, 192, frame=f, label=f"frame {f}")
        lo[f], hi[f] = d["hist_lo"], d["hist_hi"]
        fcount[f] = d["block_count"].sum()
        fsum[f] = np.sum(d["block_hash"], dtype=np.uint64)
        band["frame"].append(np.full(len(d["band_rows"]), f, np.int32))
        band["rows"].append(d["band_rows"])
        band["nbrs"].append(d["band_nbrs"])
        band["r2"].append(d["band_r2"])
        log(f"trajectory frame {f}/{F} (N={s.points.shape[0]}) done")
    np.savez_compressed(out, hist_lo=lo.astype(np.uint32),
                        hist_hi_minus_lo=(hi - lo).astype(np.uint16),
                        frame_count=fcount, frame_hash=fsum,
                        band_frame=np.concatenate(band["frame"]),
                        band_rows=np.concatenate(band["rows"]),
                        band_nbrs=np.concatenate(band["nbrs"]),
                        band_r2=np.concatenate(band["r2"]),
                        meta=meta(workload="trajectory(seed=1004): 256 frames", r_max=2.5,
                                  bins=128, r_min=0.0, exclude_ii=True, rel_band=REL,
                                  hash="pairhash.mix(pairhash.keys(local row, nbr, frame))"))


def make_knn(out):
    s = workloads.large_fcc()
    ob = oracle.make_box(s.L, s.tilt, s.dim)
    n = s.points.shape[0]
    k, m = 12, 16
    nb = (n + BLOCK - 1) // BLOCK
    bcount = np.zeros(nb, np.int64)
    bsum = np.zeros(nb, np.uint64)
    tie_rows, tie_idx, tie_r2 = [], [], []
    log("FCC k=12: start")
    for a in range(0, n, CHUNK):
        b = min(n, a + CHUNK)
        # each row's own point is its nearest entry (r = 0): ask for one more
        # and drop it, which is the k nearest with the self pair excluded
        idx, r2, ln = oracle.knn(ob, s.points, k + 1, query_points=s.points[a:b],
                                 exclude_ii=False, extra=m - k)
        rows = np.arange(a, b)
        own = idx == rows[:, None]
        assert np.all(own.sum(1) == 1)
        keep = ~own
        idx = idx[keep].reshape(b - a, m)
        r2 = r2[keep].reshape(b - a, m)
        assert np.all(ln == m + 1)
        tie = r2[:, k] <= r2[:, k - 1] * (1.0 + REL)
        # the stored candidates must reach past the band of every tie row
        assert np.all(r2[tie, m - 1] > r2[tie, k - 1] * (1.0 + REL))
        tie_rows.append(rows[tie])
        tie_idx.append(idx[tie])
        tie_r2.append(r2[tie])
        sure = ~tie
        rr = np.repeat(rows[sure], k)
        jj = idx[sure, :k].ravel()
        h = pairhash.mix(pairhash.keys(rr, jj))
        c, sm = pairhash.block_sums(rr - a, h, b - a, BLOCK)
        k0 = a // BLOCK
        bcount[k0:k0 + len(c)] += c
        bsum[k0:k0 + len(sm)] += sm
        if (a // CHUNK) % 8 == 0:
            log(f"FCC k=12 rows {b}/{n}")
    tie_rows = np.concatenate(tie_rows).astype(np.int32)
    log(f"FCC k=12 done: {len(tie_rows)} rows with a near-tie at rank 12")
    np.savez_compressed(out, block=np.array(BLOCK), k=np.array(k), block_count=bcount,
                        block_hash=bsum, tie_rows=tie_rows,
                        tie_idx=np.concatenate(tie_idx).astype(np.int32),
                        tie_r2=np.concatenate(tie_r2),
                        meta=meta(workload="large_fcc(seed=1002), N=1048576", k=k,
                                  exclude_ii=True, rel_band=REL,
                                  hash="pairhash.mix(pairhash.keys(row, nbr)) over the 12 "
                                       "neighbours of rows without a near-tie at rank 12"))


JOBS = {"fluid2d_pmft200": make_pmft, "fcc1M_ball_rdf": make_fcc_ball,
        "traj256_ball_rdf": make_traj, "fcc1M_knn12": make_knn}


def main():
    names = sys.argv[1:] or list(JOBS)
    for name in names:
        out = os.path.join(HERE, name + ".npz")
        tmp = out + ".tmp.npz"
        JOBS[name](tmp)
        os.replace(tmp, out)
        log(f"wrote {out}")


if __name__ == "__main__":
    main()
