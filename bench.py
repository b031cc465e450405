#!/usr/bin/env python3
"""Benchmark: periodic neighbour queries and pair histograms on one MI355X.

Headline step (the large configuration): 64^3 FCC cells (N = 1,048,576)
with Gaussian noise 0.05 a, a = 4^(1/3) (density 1), in a triclinic box
with tilts (0.5, 0.2, 0.1).  One step, from positions resident in HBM:
cell-list build, the ball query r_max = 2.5 writing the NeighborList (point
index + distance per pair) with the 256-bin RDF on [0, 2.5) binned in the
same pass, and the k = 12 nearest-neighbour query (its own cell list).
`value` counts the ordered ball pairs found, listed and binned per second
of the whole step.  The fill kernel (the dominant one) is timed with HIP
events on its stream inside the timed region for the roofline entry.

The other hot-path steps are measured on their own workloads and reported
under "rows": the 2D PMFT (N = 262,144 fluid, 200 x 200 bins), the batched
trajectory (256 frames of uneven size, each with its own box; one HIP-graph
launch against a loop of per-frame calls) and the Gaussian-smoothed RDF
forward and adjoint (N = 131,072).

The FP64 oracle is timed on the host on a bounded sample of query rows of
the headline system (cpu_baseline); it is the brute-force checker, not a
tuned CPU code.
"""
import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "fill_kernel_fcc1M_traffic.md")
# sources the fill kernel is compiled from: a recorded traffic figure is
# reported only while they are unchanged
FILL_SOURCES = ["paper_1906_06317_amd/csrc/pairs.hip", "paper_1906_06317_amd/csrc/pair_common.hpp",
                "paper_1906_06317_amd/csrc/internal.hpp"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=24.0,
                    help="target CPU time for the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rows", action="store_true", help="headline step only")
    ap.add_argument("--source-hash", action="store_true",
                    help="print the fill kernel's source hash (for the traffic record) and exit")
    ap.add_argument("--only", choices=["pmft2d", "pmft3", "correlation", "steinhardt", "clusters",
                                       "batched", "smooth_rdf", "small"],
                    help="run one row alone and print its JSON (for profiling that row)")
    ap.add_argument("--batch-config", type=int, default=None,
                    help="batched row: after the autotuner has run, use this launch "
                         "configuration instead of its pick (for counter runs, whose "
                         "serialised dispatches can change the pick)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (a known-size reference for "
                         "memory-traffic counters)")
    return ap.parse_args()


class Hip:
    """HIP events through the process's HIP runtime (the one torch loaded)."""

    def __init__(self):
        import torch  # noqa: F401
        L = ctypes.CDLL("libamdhip64.so.7")
        L.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        L.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                          ctypes.c_void_p]
        L.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.L = L

    def events(self, n):
        out = [ctypes.c_void_p() for _ in range(n)]
        for e in out:
            assert self.L.hipEventCreate(ctypes.byref(e)) == 0
        return out

    def ms(self, a, b):
        f = ctypes.c_float()
        assert self.L.hipEventElapsedTime(ctypes.byref(f), a, b) == 0
        return f.value

    def destroy(self, evs):
        for e in evs:
            self.L.hipEventDestroy(e)


def fill_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in FILL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    """HBM bytes per fill-kernel launch from the committed counter record
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known size), or None
    when the record is missing or the kernel's sources changed since."""
    if not os.path.exists(TRAFFIC_RECORD):
        return None
    vals = {}
    for line in open(TRAFFIC_RECORD):
        if ":" in line and line.strip().startswith(("traffic_bytes_per_launch", "source_sha256")):
            k, v = line.strip().strip("`").split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != fill_source_hash():
        return None
    return int(vals["traffic_bytes_per_launch"])


def timed(fn, reps, warmup=1):
    """Mean ms per call of fn() on the current stream (torch events)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        fn()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / reps


def cpu_baseline(sysm, target_s):
    import numpy as np

    import oracle
    ob = oracle.make_box(sysm.L, sysm.tilt, sysm.dim)
    n = sysm.points.shape[0]
    rng = np.random.default_rng(99)

    def run(nq):
        rows = np.sort(rng.choice(n, nq, replace=False))
        q = sysm.points[rows]
        t = time.perf_counter()
        # per query row: the neighbour list (count + fill) and the RDF pass
        _, idx, _ = oracle.ball_query(ob, sysm.points, 2.5, query_points=q, exclude_ii=False)
        oracle.rdf_counts(ob, sysm.points, 256, 2.5, query_points=q, exclude_ii=False)
        dt = time.perf_counter() - t
        return dt, int(idx.shape[0]) - nq  # drop each row's self pair at r = 0

    run(32)  # thread start-up
    dt, _ = run(128)
    nq = int(min(n, max(128, 128 * target_s / max(dt, 1e-3))))
    dt, pairs = run(nq)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": pairs / dt, "unit": "pairs/s", "cores": oracle.num_threads(),
            "cpu_model": model, "kind": "oracle",
            "sample": f"{nq} random query rows of the same N=1,048,576 system (brute force over "
                      f"all points, FP64), ball list + RDF, {dt:.1f} s"}


def headline(args, ppa, hip):
    import numpy as np
    import torch

    from paper_1906_06317_amd import workloads
    L = ppa.lib()
    sysm = workloads.large_fcc()
    n = sysm.points.shape[0]
    r_max, bins, k = 2.5, 256, 12
    box = ppa.Box(sysm.L, sysm.tilt, sysm.dim)
    pts = torch.as_tensor(sysm.points).cuda()

    # size the outputs exactly from one pass
    counts0, nl0 = ppa.rdf_counts(box, pts, bins, r_max, neighbor_list=True)
    P = nl0.n_pairs
    hist1 = counts0.cpu().numpy()
    del nl0

    ws = ppa.Workspace()
    wptr, wlen = ws.get(ppa.workspace_bytes(box, n, 0, r_max, ppa.PPA_WS_NLIST))
    wsk = ppa.Workspace()
    kptr, klen = wsk.get(ppa.knn_workspace_bytes(box, n, 0, k))
    offsets = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    rowc = torch.empty(n, dtype=torch.int32, device="cuda")
    pidx = torch.empty(P, dtype=torch.int32, device="cuda")
    dist = torch.empty(P, dtype=torch.float32, device="cuda")
    npairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    hist = torch.zeros(bins, dtype=torch.int64, device="cuda")
    koff = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    kidx = torch.empty(n * k, dtype=torch.int32, device="cuda")
    kdist = torch.empty(n * k, dtype=torch.float32, device="cuda")
    knp = torch.zeros(1, dtype=torch.int64, device="cuda")
    cb = box.c()
    sptr = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())

    def step(ev=None):
        if ev:
            L.ppa_profile_next(ev[0], ev[1], ev[2], ev[3])
        rc = L.ppa_rdf(ctypes.byref(cb), p(pts), n, None, n, bins, 0.0, r_max, 1, 0, wptr, wlen,
                       p(hist), p(offsets), p(rowc), p(pidx), p(dist), P, p(npairs), sptr)
        if rc != 0:
            raise RuntimeError(L.ppa_last_error().decode())
        if ev:
            L.ppa_profile_next(None, None, ev[4], ev[5])
        rc = L.ppa_query_knn(ctypes.byref(cb), p(pts), n, None, n, k, 0.0, 1, 0, kptr, klen,
                             p(koff), None, p(kidx), p(kdist), p(knp), sptr)
        if rc != 0:
            raise RuntimeError(L.ppa_last_error().decode())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if ws.status() != 0 or wsk.status() != 0:
        raise RuntimeError("device status after warmup: " + L.ppa_last_error().decode())

    ev = [hip.events(6) for _ in range(args.steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for i in range(args.steps):
        step(ev[i])
    t1.record()
    torch.cuda.synchronize()
    ms_step = t0.elapsed_time(t1) / args.steps
    count_all = [hip.ms(e[0], e[1]) for e in ev]
    fill_all = [hip.ms(e[2], e[3]) for e in ev]
    count_ms = float(np.mean(count_all))
    fill_ms = float(np.mean(fill_all))
    knn_ms = float(np.mean([hip.ms(e[4], e[5]) for e in ev]))
    for e in ev:
        hip.destroy(e)
    if ws.status() != 0 or wsk.status() != 0:
        raise RuntimeError("device status: " + L.ppa_last_error().decode())
    # the histogram accumulates over calls: every step must add the same counts
    h = hist.cpu().numpy()
    assert np.array_equal(h, hist1 * (args.warmup + args.steps)), "histogram drifted across steps"
    assert int(npairs.item()) == P and int(knp.item()) == n * k

    # ball + RDF alone, for the row table
    def ball_only():
        L.ppa_rdf(ctypes.byref(cb), p(pts), n, None, n, bins, 0.0, r_max, 1, 0, wptr, wlen,
                  p(hist), p(offsets), p(rowc), p(pidx), p(dist), P, p(npairs), sptr)
    ball_ms = timed(ball_only, max(5, args.steps // 2))

    # the same call with every row ordered by neighbour index (PPA_SORT_ROWS)
    def ball_sorted():
        L.ppa_rdf(ctypes.byref(cb), p(pts), n, None, n, bins, 0.0, r_max, 1, ppa.PPA_SORT_ROWS,
                  wptr, wlen, p(hist), p(offsets), p(rowc), p(pidx), p(dist), P, p(npairs), sptr)
    sorted_ms = timed(ball_sorted, max(5, args.steps // 2))
    srt = pidx[:P]
    starts = offsets[:-1][offsets[:-1] < P]  # first entry of every non-empty row
    new_row = torch.zeros(P, dtype=torch.bool, device="cuda").index_fill_(0, starts, True)
    rows_ok = bool(torch.all((srt[1:] > srt[:-1]) | new_row[1:]).item())
    if ws.status() != 0 or not rows_ok:
        raise RuntimeError("sorted rows: device status or order check failed")

    # algorithmic bytes of the fill kernel per launch: positions read (12 B per
    # point), row offsets read (8 B per query), neighbour list written (4 B
    # index + 4 B distance per pair), histogram (8 B per bin)
    alg_bytes = 12 * n + 8 * n + 8 * P + 8 * bins
    achieved = alg_bytes / (fill_ms * 1e-3) / 1e9
    line = {
        "metric": "pair evaluations/s for periodic ball query+RDF at N=1M; batched vs per-frame",
        "value": P / (ms_step * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "noisy FCC N=1,048,576 (a=4^(1/3), sigma=0.05a), triclinic box "
                               "tilts (0.5,0.2,0.1); ball r_max=2.5 -> NeighborList + RDF 256 bins, "
                               "plus k=12 nearest query",
                   "n_points": n, "r_max": r_max, "bins": bins, "k": k, "n_pairs": P,
                   "rows": "CSR in query order (count, scan, fill)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(),
                     "kernel": "fill_kernel (ball list + RDF)", "kernel_ms": fill_ms,
                     "algorithmic_bytes": alg_bytes, "count_kernel_ms": count_ms,
                     "kernel_ms_median": float(np.median(fill_all)),
                     "kernel_ms_min": float(np.min(fill_all)),
                     "count_kernel_ms_median": float(np.median(count_all)),
                     "valu_diagnostic": valu_diagnostic(ppa, box, n, r_max, count_ms, fill_ms)},
    }
    rows = {
        "ball_rdf": {"ms": ball_ms, "pairs_per_s": P / (ball_ms * 1e-3),
                     "note": "cell build + count + scan + fill with fused RDF",
                     "end_to_end_achieved_GBps": alg_bytes / (ball_ms * 1e-3) / 1e9,
                     "end_to_end_frac": alg_bytes / (ball_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "fill_kernel_frac": achieved / HBM_PEAK_GBS,
                     "sorted_rows_ms": sorted_ms,
                     "sort_rows_ms": sorted_ms - ball_ms},
        "knn": {"workload": "same system, k=12 (own cell list)", "ms_in_step": None,
                "select_kernels_ms": knn_ms, "pairs": n * k},
    }
    knn_call = timed(lambda: L.ppa_query_knn(ctypes.byref(cb), p(pts), n, None, n, k, 0.0, 1, 0,
                                             kptr, klen, p(koff), None, p(kidx), p(kdist), p(knp),
                                             sptr), 10)
    rows["knn"]["ms_in_step"] = knn_call
    rows["knn"]["pairs_per_s"] = n * k / (knn_call * 1e-3)
    return line, rows, sysm


def copy_bandwidth():
    """Device-to-device copy rate (GB/s, bytes read + written) of a 1 GiB buffer."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    ms = timed(lambda: dst.copy_(src), 10, warmup=2)
    del src, dst
    return 2 * (1 << 30) / (ms * 1e-3) / 1e9


def paper_context(ppa):
    """The paper's two performance statements, re-measured here as context:
    the 2D PMFT against the RDF on its workload shape (10 frames x 20,000
    points, density 3.82, r = 1; the paper gives no bin counts: 100 RDF bins,
    100 x 100 PMFT bins here), which it found about 3x slower on an Intel Xeon
    E5-2680 v2; and neighbour finding on random 3D points with about 12
    neighbours within r = 1 (density 2.865) as N grows."""
    import numpy as np
    import torch

    from paper_1906_06317_amd import workloads
    rng = np.random.default_rng(77)
    frames = []
    for f in range(10):
        s = workloads.uniform(20000, 3.82, seed=700 + f, dim=2)
        frames.append((s, rng.uniform(0, 2 * math.pi, 20000).astype(np.float32)))
    boxes = [ppa.Box(s.L, s.tilt, s.dim) for s, _ in frames]
    pts = [torch.as_tensor(s.points).cuda() for s, _ in frames]
    ths = [torch.as_tensor(t).cuda() for _, t in frames]
    h = torch.zeros(100, dtype=torch.int64, device="cuda")
    c = torch.zeros((100, 100), dtype=torch.uint32, device="cuda")
    rdf_ms = timed(lambda: [ppa.rdf_counts(b, p, 100, 1.0, counts=h, check=False)
                            for b, p in zip(boxes, pts)], 5)
    pmft_ms = timed(lambda: [ppa.pmft2d_counts(b, p, t, 100, 100, 1.0, 1.0, 1.0, counts=c,
                                               check=False)
                             for b, p, t in zip(boxes, pts, ths)], 5)
    scaling = {}
    for n in (1000, 10000, 100000, 1000000):
        s = workloads.uniform(n, 2.865, seed=800)
        b = ppa.Box(s.L, s.tilt, s.dim)
        p = torch.as_tensor(s.points).cuda()
        nl = ppa.query_ball(b, p, 1.0)
        ms = timed(lambda: ppa.query_ball(b, p, 1.0, capacity=nl.n_pairs + 1024, check=False), 5)
        scaling[str(n)] = {"ms": ms, "pairs": nl.n_pairs, "pairs_per_s": nl.n_pairs / (ms * 1e-3)}
    return {"pmft_over_rdf_2d": pmft_ms / rdf_ms, "rdf_ms": rdf_ms, "pmft_ms": pmft_ms,
            "paper_pmft_over_rdf": "about 3 (Intel Xeon E5-2680 v2, CPU threads)",
            "workload": "10 frames x 20,000 2D points, density 3.82, r=1; 100 RDF bins, "
                        "100x100 PMFT bins",
            "neighbor_scaling_3d_uniform_density_2.865_r1": scaling,
            "note": "the paper prints no absolute numbers; these are context, not a target"}


# Non-packed FP32 lane operations per second of the device: 256 CUs x 64
# lanes x 2.4 GHz (the packed and dual-issue forms behind the 157.3 TFLOP/s
# figure are not used by this build's device code).
VALU_LANE_OPS = 256 * 64 * 2.4e9
# v_exp_f32 is a quarter-rate transcendental: 16 lanes per CU per clock.
EXP_PEAK = 256 * 16 * 2.4e9
ADJOINT_TERM_OPS = 7


def valu_diagnostic(ppa, box, n, r_max, count_ms, fill_ms):
    """Candidate evaluations of one pass of the 27-cell stencil (cells of
    width >= r_max per axis, n / ncells points each), and the lane-operation
    rate at 4 operations per candidate (three FMAs and a compare of the
    expanded test) against the non-packed VALU peak."""
    w = box.widths()
    cells = 1
    for k in range(3):
        cells *= max(1, int(w[k] // (r_max * (1 + 1e-5))))
    per_query = 27.0 * n / cells
    evals = per_query * n
    return {"cells": cells, "candidates_per_query": per_query, "candidate_evaluations": evals,
            "count_lane_ops_frac": 4 * evals / (count_ms * 1e-3) / VALU_LANE_OPS,
            "fill_lane_ops_frac": 4 * evals / (fill_ms * 1e-3) / VALU_LANE_OPS,
            "valu_lane_ops_peak": VALU_LANE_OPS}


def lds_atomic_peak(ppa):
    """LDS atomic adds per second of the device (microbenchmark, random bins)."""
    import torch
    L = ppa.lib()
    out = torch.zeros(1, dtype=torch.int32, device="cuda")
    sptr = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    res = {}
    for lb in (8, 14):
        blocks, iters = 2048, 256
        ms = timed(lambda: L.ppa_probe_lds_atomics(lb, iters, blocks, ctypes.c_void_p(out.data_ptr()),
                                                   sptr), 5)
        res[f"{1 << lb}_bins_per_s"] = blocks * 256 * 8 * iters / (ms * 1e-3)
    return res


def global_atomic_peak(ppa):
    """Global-memory atomic adds per second of the device (microbenchmark,
    random words of a histogram of 2^17 and 2^19 words)."""
    import torch
    L = ppa.lib()
    sptr = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    res = {}
    for lw in (17, 19):
        hist = torch.zeros(1 << lw, dtype=torch.int32, device="cuda")
        blocks, iters = 2048, 16
        ms = timed(lambda: L.ppa_probe_global_atomics(lw, iters, blocks,
                                                      ctypes.c_void_p(hist.data_ptr()), sptr), 5)
        res[f"{1 << lw}_words_per_s"] = blocks * 256 * 8 * iters / (ms * 1e-3)
    return res


def row_pmft3(ppa, hip, peak):
    """PMFT over three pair coordinates: XYT on the 2D fluid, XYZ on a 3D fluid."""
    import numpy as np
    import torch

    from paper_1906_06317_amd import workloads
    L = ppa.lib()
    out = {}
    s = workloads.fluid_2d()
    s3 = workloads.fluid_3d()
    cases = {
        "xyt": (s, (100, 100, 36), "2D fluid N=262,144, density 0.7, orientations uniform; "
                "r_max=3, 100x100x36 bins over (x', y') in [-3,3)^2 and t in [0, 2 pi)"),
        "xyz": (s3, (50, 50, 50), "3D fluid N=262,144, density 0.9, unit quaternions uniform "
                "over rotations; r_max=2, 50^3 bins on [-2,2)^3"),
    }
    for name, (sys_, nb, desc) in cases.items():
        box = ppa.Box(sys_.L, sys_.tilt, sys_.dim)
        n = sys_.points.shape[0]
        pts = torch.as_tensor(sys_.points).cuda()
        counts = torch.zeros(nb, dtype=torch.uint32, device="cuda")
        if name == "xyt":
            th = torch.as_tensor(sys_.theta).cuda()
            fn = lambda: ppa.pmft_xyt_counts(box, pts, th, *nb, 3.0, 3.0, 3.0, counts=counts,
                                             check=False)
            r_max = 3.0
        else:
            qq = torch.as_tensor(sys_.quat).cuda()
            fn = lambda: ppa.pmft_xyz_counts(box, pts, qq, *nb, 2.0, 2.0, 2.0, 2.0, counts=counts,
                                             check=False)
            r_max = 2.0
        evs = []

        def call():
            e = hip.events(2)
            evs.append(e)
            L.ppa_profile_next(None, None, e[0], e[1])
            fn()
        ms = timed(call, 10, warmup=2)
        kern = float(np.mean([hip.ms(e[0], e[1]) for e in evs[2:]]))
        for e in evs:
            hip.destroy(e)
        if ppa.default_workspace().status() != 0:
            raise RuntimeError(L.ppa_last_error().decode())
        pairs = ppa.query_ball(box, pts, r_max, with_dist=False).n_pairs
        ref = peak["131072_words_per_s"] if name == "xyz" else peak["524288_words_per_s"]
        out[name] = {"workload": desc, "ms": ms, "binning_kernel_ms": kern, "pairs": pairs,
                     "pairs_per_s": pairs / (ms * 1e-3),
                     "binning_global_atomics_per_s": pairs / (kern * 1e-3),
                     "frac_of_global_atomic_probe": pairs / (kern * 1e-3) / ref}
    return out


def row_pmft(ppa, hip):
    import numpy as np
    import torch

    from paper_1906_06317_amd import workloads
    L = ppa.lib()
    s = workloads.fluid_2d()
    n = s.points.shape[0]
    box = ppa.Box(s.L, s.tilt, s.dim)
    pts = torch.as_tensor(s.points).cuda()
    th = torch.as_tensor(s.theta).cuda()
    ws = ppa.Workspace()
    wptr, wlen = ws.get(ppa.pmft2d_workspace_bytes(box, n, 0, 200, 200, 3.0, 3.0, 3.0))
    counts = torch.zeros(200 * 200, dtype=torch.int32, device="cuda")
    cb = box.c()
    sptr = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    evs = []

    def call():
        e = hip.events(2)
        evs.append(e)
        L.ppa_profile_next(None, None, e[0], e[1])
        rc = L.ppa_pmft2d(ctypes.byref(cb), p(pts), n, None, p(th), n, 200, 200, 3.0, 3.0, 3.0, 1,
                          0, wptr, wlen, p(counts), sptr)
        if rc != 0:
            raise RuntimeError(L.ppa_last_error().decode())
    ms = timed(call, 10, warmup=2)
    kern = float(np.mean([hip.ms(e[0], e[1]) for e in evs[2:]]))
    for e in evs:
        hip.destroy(e)
    if ws.status() != 0:
        raise RuntimeError(L.ppa_last_error().decode())
    pairs = int(counts.to(torch.int64).sum().item()) // 12
    # the same call at other bin counts: the LDS window with 32-bit counters
    # (100), with two 16-bit counters per word (256), global atomics (300)
    by_bins = {}
    for nb in (100, 256, 300):
        wp, wl = ws.get(ppa.pmft2d_workspace_bytes(box, n, 0, nb, nb, 3.0, 3.0, 3.0))
        c = torch.zeros(nb * nb, dtype=torch.int32, device="cuda")

        def call_nb():
            rc = L.ppa_pmft2d(ctypes.byref(cb), p(pts), n, None, p(th), n, nb, nb, 3.0, 3.0, 3.0,
                              1, 0, wp, wl, p(c), sptr)
            if rc != 0:
                raise RuntimeError(L.ppa_last_error().decode())
        by_bins[f"{nb}x{nb}"] = timed(call_nb, 5, warmup=1)
    if ws.status() != 0:
        raise RuntimeError(L.ppa_last_error().decode())
    return {"workload": "2D fluid N=262,144, density 0.7, r_max=3, 200x200 bins on [-3,3)^2",
            "ms": ms, "binning_kernels_ms": kern, "pairs": pairs,
            "pairs_per_s": pairs / (ms * 1e-3), "ms_by_bins": by_bins}


def row_correlation(ppa, hip):
    """Spatial correlation of psi_6-like values on the 2D fluid."""
    import numpy as np
    import torch

    from paper_1906_06317_amd import workloads
    L = ppa.lib()
    s = workloads.fluid_2d()
    box = ppa.Box(s.L, s.tilt, s.dim)
    pts = torch.as_tensor(s.points).cuda()
    psi = np.exp(6j * s.theta.astype(np.float64)).astype(np.complex64)
    vals = torch.as_tensor(np.stack([psi.real, psi.imag], 1)).cuda()
    bins, r_max = 120, 6.0
    sums = torch.zeros((bins, 2), dtype=torch.float64, device="cuda")
    counts = torch.zeros(bins, dtype=torch.uint64, device="cuda")
    evs = []

    def call():
        e = hip.events(2)
        evs.append(e)
        L.ppa_profile_next(None, None, e[0], e[1])
        ppa.correlation_sums(box, pts, vals, bins, r_max, sums=sums, counts=counts, check=False)
    ms = timed(call, 10, warmup=2)
    kern = float(np.mean([hip.ms(e[0], e[1]) for e in evs[2:]]))
    for e in evs:
        hip.destroy(e)
    if ppa.default_workspace().status() != 0:
        raise RuntimeError(L.ppa_last_error().decode())
    pairs = int(counts.cpu().numpy().astype(np.int64).sum()) // 12
    return {"workload": "2D fluid N=262,144, density 0.7, values exp(6i theta) (theta uniform), "
                        "r_max=6, 120 bins; sums of conj(f_i) g_j in float64",
            "ms": ms, "kernels_ms": kern, "pairs": pairs, "pairs_per_s": pairs / (ms * 1e-3),
            "lds_atomics_per_pair": 3,
            "lds_atomics_per_s": 3 * pairs / (kern * 1e-3)}


def row_steinhardt(ppa, hip):
    """Q6 and W6 on the k = 12 list of the headline system (the paper's
    Steinhardt example)."""
    import numpy as np
    import torch

    from paper_1906_06317_amd import workloads
    L = ppa.lib()
    s = workloads.large_fcc()
    box = ppa.Box(s.L, s.tilt, s.dim)
    pts = torch.as_tensor(s.points).cuda()
    nl = ppa.query_knn(box, pts, 12)
    out = {"workload": "noisy FCC N=1,048,576 (the headline system), its k=12 NeighborList; "
                       "Q_l and normalised W_l per particle in float64"}
    for l, with_w in ((6, False), (6, True), (12, True)):
        evs = []

        def call():
            e = hip.events(2)
            evs.append(e)
            L.ppa_profile_next(None, None, e[0], e[1])
            ppa.steinhardt(box, pts, nl, l, with_w=with_w, check=False)
        timed(call, 10, warmup=2)
        kern = float(np.mean([hip.ms(e[0], e[1]) for e in evs[2:]]))
        for e in evs:
            hip.destroy(e)
        out[f"l{l}{'_w' if with_w else ''}_kernel_ms"] = kern
    ql, wl = ppa.steinhardt(box, pts, nl, 6, with_w=True)
    out["mean_q6"] = float(ql.mean().item())
    out["mean_w6"] = float(wl.mean().item())
    out["bonds"] = nl.n_pairs
    out["bonds_per_s_q6"] = nl.n_pairs / (out["l6_kernel_ms"] * 1e-3)
    return out


def row_clusters(ppa, hip):
    """Clusters of a 1M-point uniform fluid from its ball list, below and
    above the percolation threshold."""
    import numpy as np
    import torch

    from paper_1906_06317_amd import workloads
    L = ppa.lib()
    s = workloads.uniform(1 << 20, 1.0, seed=640)
    box = ppa.Box(s.L, s.tilt, s.dim)
    pts = torch.as_tensor(s.points).cuda()
    out = {"workload": "uniform N=1,048,576, density 1; bonds within r_cut from the ball query "
                       "(r_cut 0.8: about 2.1 bonds per point, below percolation; 1.2: about 7.2, "
                       "one spanning cluster); the ball list is symmetric, so the calls pass "
                       "PPA_CLUSTER_SYMMETRIC"}
    for r_cut in (0.8, 1.2):
        nl = ppa.query_ball(box, pts, r_cut)
        evs = []

        def call():
            e = hip.events(2)
            evs.append(e)
            L.ppa_profile_next(None, None, e[0], e[1])
            ppa.clusters(nl, 1 << 20, check=False, symmetric=True)
        timed(call, 10, warmup=2)
        kern = float(np.mean([hip.ms(e[0], e[1]) for e in evs[2:]]))
        for e in evs:
            hip.destroy(e)
        labels, cidx, sizes, k = ppa.clusters(nl, 1 << 20, symmetric=True)
        out[f"r{r_cut}"] = {"bonds": nl.n_pairs, "clusters": k,
                            "largest": int(sizes.max().item()), "kernels_ms": kern,
                            "bonds_per_s": nl.n_pairs / (kern * 1e-3)}
    return out


def row_batched(ppa, hip, force_config=None):
    import numpy as np
    import torch

    from paper_1906_06317_amd import workloads
    L = ppa.lib()
    frames = workloads.trajectory()
    F = len(frames)
    sizes = [f.points.shape[0] for f in frames]
    boxes = [ppa.Box(f.L, f.tilt, f.dim) for f in frames]
    bins, r_max = 128, 2.5
    pts = torch.as_tensor(np.concatenate([f.points for f in frames])).cuda()
    plan = ppa.BatchPlan(boxes, sizes, bins, r_max)
    hist0, nl0 = plan.run(pts)  # sizes the per-frame outputs below
    total_pairs = nl0.n_pairs
    tune_ms, cfg = plan.autotune(pts, reps=2)
    if force_config is not None:
        cfg = plan.config(force_config)
    hist = torch.zeros((F, bins), dtype=torch.int64, device="cuda")
    launch = plan.graph(pts, hist)
    batched_ms = timed(launch, 5, warmup=1)
    torch.cuda.synchronize()
    if plan.ws.status() != 0:
        raise RuntimeError(L.ppa_last_error().decode())

    # per-frame baseline: one eager ppa_rdf call (own cell list, list + RDF)
    # per frame on the same stream, outputs in per-frame slices
    off = nl0.offsets.cpu().numpy()
    pb = plan.offsets_host
    ws = ppa.Workspace()
    need = max(ppa.workspace_bytes(b, m, 0, r_max, ppa.PPA_WS_NLIST) for b, m in zip(boxes, sizes))
    wptr, wlen = ws.get(need)
    pf_hist = torch.zeros((F, bins), dtype=torch.int64, device="cuda")
    pf_off = torch.empty(int(pb[-1]) + F, dtype=torch.int64, device="cuda")
    pf_cnt = torch.empty(int(pb[-1]), dtype=torch.int32, device="cuda")
    cap = [int(off[pb[f + 1]] - off[pb[f]]) + 1024 for f in range(F)]
    cbase = np.concatenate([[0], np.cumsum(cap)])
    pf_idx = torch.empty(int(cbase[-1]), dtype=torch.int32, device="cuda")
    pf_dist = torch.empty(int(cbase[-1]), dtype=torch.float32, device="cuda")
    pf_np = torch.zeros(F, dtype=torch.int64, device="cuda")
    cboxes = [b.c() for b in boxes]
    sptr = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    base = pts.data_ptr()
    es = pf_idx.element_size()

    def per_frame():
        for f in range(F):
            m = sizes[f]
            rc = L.ppa_rdf(ctypes.byref(cboxes[f]), ctypes.c_void_p(base + 12 * int(pb[f])), m, None,
                           m, bins, 0.0, r_max, 1, 0, wptr, wlen,
                           ctypes.c_void_p(pf_hist.data_ptr() + 8 * bins * f),
                           ctypes.c_void_p(pf_off.data_ptr() + 8 * (int(pb[f]) + f)),
                           ctypes.c_void_p(pf_cnt.data_ptr() + 4 * int(pb[f])),
                           ctypes.c_void_p(pf_idx.data_ptr() + es * int(cbase[f])),
                           ctypes.c_void_p(pf_dist.data_ptr() + 4 * int(cbase[f])), cap[f],
                           ctypes.c_void_p(pf_np.data_ptr() + 8 * f), sptr)
            if rc != 0:
                raise RuntimeError(L.ppa_last_error().decode())
    per_frame_ms = timed(per_frame, 3, warmup=1)
    if ws.status() != 0:
        raise RuntimeError(L.ppa_last_error().decode())
    assert int(pf_np.sum().item()) == total_pairs
    return {"workload": "256 frames, N_f log-uniform in [1e3, 2e5] (total %d), own triclinic boxes, "
                        "ball r_max=2.5 -> NeighborList + per-frame RDF 128 bins" % int(pb[-1]),
            "frames": F, "points": int(pb[-1]), "pairs": total_pairs,
            "batched_ms": batched_ms, "batched_frames_per_s": F / (batched_ms * 1e-3),
            "batched_pairs_per_s": total_pairs / (batched_ms * 1e-3),
            "per_frame_ms": per_frame_ms, "per_frame_frames_per_s": F / (per_frame_ms * 1e-3),
            "speedup": per_frame_ms / batched_ms,
            "autotuned": cfg, "autotune_ms": tune_ms, "config_forced": force_config,
            "note": "batched = one HIP-graph launch of the autotuned plan; per-frame = 256 eager "
                    "ppa_rdf calls with list, each building its own cell list"}


def row_smooth(ppa, hip):
    import numpy as np
    import torch

    from paper_1906_06317_amd import workloads
    L = ppa.lib()
    s, _ = workloads.smooth_target_pair()
    n = s.points.shape[0]
    box = ppa.Box(s.L, s.tilt, s.dim)
    pts = torch.as_tensor(s.points).cuda()
    bins, r_max, sigma = 200, 3.0, 0.02
    ws = ppa.Workspace()
    wptr, wlen = ws.get(ppa.smooth_rdf_workspace_bytes(box, n, bins, r_max, sigma))
    h = torch.zeros(bins, dtype=torch.float64, device="cuda")
    gh = torch.as_tensor(np.random.default_rng(0).normal(size=bins)).cuda()
    grad = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    cb = box.c()
    sptr = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())

    def fwd():
        rc = L.ppa_smooth_rdf_fwd(ctypes.byref(cb), p(pts), n, bins, r_max, sigma, 0, wptr, wlen,
                                  p(h), sptr)
        if rc != 0:
            raise RuntimeError(L.ppa_last_error().decode())

    def bwd():
        rc = L.ppa_smooth_rdf_bwd(ctypes.byref(cb), p(pts), n, bins, r_max, sigma, p(gh), 0, wptr,
                                  wlen, p(grad), sptr)
        if rc != 0:
            raise RuntimeError(L.ppa_last_error().decode())
    fwd_ms = timed(fwd, 5, warmup=2)
    bwd_ms = timed(bwd, 5, warmup=2)
    if ws.status() != 0:
        raise RuntimeError(L.ppa_last_error().decode())
    nl = ppa.query_ball(box, pts, r_max + 8 * sigma)
    # window terms: bins b with |c_b - r| <= 8 sigma, c_b = (b + 1/2) dr, per pair
    r = nl.dist.double()
    dr = r_max / bins
    lo = torch.clamp(torch.ceil((r - 8 * sigma) / dr - 0.5), min=0)
    hi = torch.clamp(torch.floor((r + 8 * sigma) / dr - 0.5), max=bins - 1)
    terms = float(torch.clamp(hi - lo + 1, min=0).sum().item())
    return {"workload": "perturbed simple-cubic N=131,072, density 0.9, sigma 0.02, 200 bins on "
                        "[0,3), pairs within 3.16",
            "pairs": nl.n_pairs, "forward_ms": fwd_ms, "adjoint_ms": bwd_ms,
            "forward_pairs_per_s": nl.n_pairs / (fwd_ms * 1e-3),
            "adjoint_pairs_per_s": nl.n_pairs / (bwd_ms * 1e-3),
            "window_terms": terms,
            "roofline": {"bound": "alu", "unit": "exp/s", "peak": EXP_PEAK,
                         "forward_achieved": terms / (fwd_ms * 1e-3),
                         "forward_frac": terms / (fwd_ms * 1e-3) / EXP_PEAK,
                         "note": "forward: one exp2 per window term (quarter-rate "
                                 "transcendental peak)",
                         "adjoint": {"bound": "alu", "unit": "lane-op/s",
                                     "peak": VALU_LANE_OPS, "ops_per_term": ADJOINT_TERM_OPS,
                                     "achieved": ADJOINT_TERM_OPS * terms / (bwd_ms * 1e-3),
                                     "frac": ADJOINT_TERM_OPS * terms / (bwd_ms * 1e-3)
                                     / VALU_LANE_OPS,
                                     "note": "adjoint: Gaussians by recurrence, 7 lane "
                                             "operations per window term (4 float32 "
                                             "multiplies, an add, a conversion and a "
                                             "float64 add)"}}}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def row_small(ppa, hip):
    """The small configuration (N = 4096 uniform, density 0.8, cubic): ball
    r_max = 3 writing the list with the 100-bin RDF in the same call, and
    the oracle over every row (brute force, FP64, all host threads)."""
    import numpy as np
    import torch

    import oracle
    from paper_1906_06317_amd import workloads
    L = ppa.lib()
    s = workloads.small_uniform()
    n = s.points.shape[0]
    box = ppa.Box(s.L, s.tilt, s.dim)
    pts = torch.as_tensor(s.points).cuda()
    counts0, nl0 = ppa.rdf_counts(box, pts, 100, 3.0, neighbor_list=True)
    P = nl0.n_pairs
    ws = ppa.Workspace()
    wptr, wlen = ws.get(ppa.workspace_bytes(box, n, 0, 3.0, ppa.PPA_WS_NLIST))
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    rc_ = torch.empty(n, dtype=torch.int32, device="cuda")
    pidx = torch.empty(P, dtype=torch.int32, device="cuda")
    dist = torch.empty(P, dtype=torch.float32, device="cuda")
    npairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    hist = torch.zeros(100, dtype=torch.int64, device="cuda")
    cb = box.c()
    sptr = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    ms = timed(lambda: L.ppa_rdf(ctypes.byref(cb), p(pts), n, None, n, 100, 0.0, 3.0, 1, 0, wptr,
                                 wlen, p(hist), p(off), p(rc_), p(pidx), p(dist), P, p(npairs),
                                 sptr), 50, warmup=3)
    if ws.status() != 0:
        raise RuntimeError(L.ppa_last_error().decode())
    ob = oracle.make_box(s.L, s.tilt, s.dim)
    t = time.perf_counter()
    _, idx, _ = oracle.ball_query(ob, s.points, 3.0)
    oracle.rdf_counts(ob, s.points, 100, 3.0)
    cpu_s = time.perf_counter() - t
    return {"workload": "uniform N=4096, density 0.8, cubic; ball r_max=3 -> NeighborList + RDF "
                        "100 bins on [0,3) in one call", "pairs": P, "ms": ms,
            "pairs_per_s": P / (ms * 1e-3), "note": "latency-bound: a few microseconds of work",
            "oracle": {"value": int(idx.shape[0]) / cpu_s, "unit": "pairs/s",
                       "cores": oracle.num_threads(), "kind": "oracle",
                       "sample": f"every row (brute force, FP64), ball list + RDF, {cpu_s:.2f} s"}}


def oracle_rows(budget_s=4.0):
    """The oracle timed on bounded samples of the other configurations
    (brute force, FP64, all host threads): the 2D PMFT's query rows, the
    batched trajectory's rows from every 16th frame, and the smoothed RDF's
    rows (forward) and gradient rows."""
    import numpy as np

    import oracle
    from paper_1906_06317_amd import workloads
    rng = np.random.default_rng(7)
    out = {"cores": oracle.num_threads(), "cpu_model": _cpu_model()}

    def scaled(fn, nq0):
        """Runs fn(nq) at nq0 rows, then at a size that fills the budget."""
        dt, w = fn(nq0)
        nq = int(max(nq0, nq0 * budget_s / max(dt, 1e-3)))
        dt, w = fn(nq)
        return nq, dt, w

    s = workloads.fluid_2d()
    ob = oracle.make_box(s.L, s.tilt, s.dim)

    def pmft(nq):
        rows = rng.choice(s.points.shape[0], nq, replace=False)
        t = time.perf_counter()
        lo, _, _ = oracle.pmft2d_counts(ob, s.points, s.points[rows], s.theta[rows], 200, 200,
                                        3.0, 3.0, 3.0, exclude_ii=False)
        return time.perf_counter() - t, int(lo.sum()) - nq  # own entries at r = 0
    nq, dt, w = scaled(pmft, 64)
    out["pmft2d"] = {"value": w / dt, "unit": "pairs/s", "kind": "oracle",
                     "sample": f"{nq} random query rows of the 2D fluid (200x200 PMFT counts), "
                               f"{dt:.1f} s"}

    frames = workloads.trajectory()

    def traj(nq):
        pairs, t = 0, time.perf_counter()
        for f in range(0, len(frames), 16):
            fs = frames[f]
            m = min(nq, fs.points.shape[0])
            rows = rng.choice(fs.points.shape[0], m, replace=False)
            fb = oracle.make_box(fs.L, fs.tilt, fs.dim)
            _, idx, _ = oracle.ball_query(fb, fs.points, 2.5, query_points=fs.points[rows],
                                          exclude_ii=False)
            oracle.rdf_counts(fb, fs.points, 128, 2.5, query_points=fs.points[rows],
                              exclude_ii=False)
            pairs += int(idx.shape[0]) - m
        return time.perf_counter() - t, pairs
    nq, dt, w = scaled(traj, 16)
    out["batched"] = {"value": w / dt, "unit": "pairs/s", "kind": "oracle",
                      "sample": f"{nq} random rows of each of 16 frames (every 16th), ball list + "
                                f"RDF per frame, {dt:.1f} s"}

    sc, _ = workloads.smooth_target_pair()
    sb = oracle.make_box(sc.L, sc.tilt, sc.dim)
    pts64 = sc.points.astype(np.float64)

    def smooth(nq):
        rows = rng.choice(sc.points.shape[0], nq, replace=False)
        t = time.perf_counter()
        for k in rows:
            oracle.smooth_rdf_row(sb, sc.points, int(k), pts64[k], 200, 3.0, 0.02)
        oracle.smooth_rdf_grad(sb, sc.points, 200, 3.0, 0.02, np.ones(200), rows=rows)
        dt = time.perf_counter() - t
        # the rows' pairs within r_max + 8 sigma (counted after the timing)
        _, idx, _ = oracle.ball_query(sb, sc.points, 3.16, query_points=sc.points[rows],
                                      exclude_ii=False)
        return dt, int(idx.shape[0]) - nq
    nq, dt, w = scaled(smooth, 16)
    out["smooth_rdf"] = {"value": w / dt, "unit": "pairs/s (forward row + gradient row)",
                         "kind": "oracle",
                         "sample": f"{nq} random rows of the perturbed simple-cubic system, one "
                                   f"forward row and one gradient row each, {dt:.1f} s"}
    return out


def main():
    args = parse()
    if args.source_hash:
        print(fill_source_hash())
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1906_06317_amd as ppa
    torch.cuda.set_device(0)
    hip = Hip()
    ppa.lib()
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only:
        fns = {"pmft2d": lambda: row_pmft(ppa, hip),
               "pmft3": lambda: row_pmft3(ppa, hip, global_atomic_peak(ppa)),
               "correlation": lambda: row_correlation(ppa, hip),
               "steinhardt": lambda: row_steinhardt(ppa, hip),
               "clusters": lambda: row_clusters(ppa, hip),
               "batched": lambda: row_batched(ppa, hip, args.batch_config),
               "smooth_rdf": lambda: row_smooth(ppa, hip),
               "small": lambda: row_small(ppa, hip)}
        print(json.dumps({"row": args.only, **fns[args.only]()}), flush=True)
        return
    line, rows, sysm = headline(args, ppa, hip)
    copy_gbs = copy_bandwidth()
    line["roofline"]["measured_copy_GBps"] = copy_gbs
    line["roofline"]["frac_of_measured_copy"] = line["roofline"]["achieved"] / copy_gbs
    peak = lds_atomic_peak(ppa)
    rows["lds_atomic_probe"] = peak
    rows["ball_rdf"]["fill_lds_atomics_per_s"] = line["config"]["n_pairs"] / (
        line["roofline"]["kernel_ms"] * 1e-3)
    rows["ball_rdf"]["fill_frac_of_lds_atomic_probe"] = (
        rows["ball_rdf"]["fill_lds_atomics_per_s"] / peak["256_bins_per_s"])
    if not args.no_rows:
        rows["pmft2d"] = row_pmft(ppa, hip)
        rows["pmft2d"]["binning_lds_atomics_per_s"] = rows["pmft2d"]["pairs"] / (
            rows["pmft2d"]["binning_kernels_ms"] * 1e-3)
        rows["pmft2d"]["frac_of_lds_atomic_probe"] = (
            rows["pmft2d"]["binning_lds_atomics_per_s"] / peak["16384_bins_per_s"])
        gpeak = global_atomic_peak(ppa)
        rows["global_atomic_probe"] = gpeak
        rows["pmft3"] = row_pmft3(ppa, hip, gpeak)
        rows["correlation"] = row_correlation(ppa, hip)
        rows["correlation"]["frac_of_lds_atomic_probe"] = (
            rows["correlation"]["lds_atomics_per_s"] / peak["256_bins_per_s"])
        rows["steinhardt"] = row_steinhardt(ppa, hip)
        rows["clusters"] = row_clusters(ppa, hip)
        rows["batched"] = row_batched(ppa, hip, args.batch_config)
        rows["smooth_rdf"] = row_smooth(ppa, hip)
        rows["small"] = row_small(ppa, hip)
        rows["paper_context"] = paper_context(ppa)
        if not args.no_cpu_baseline:
            rows["oracle"] = oracle_rows()
    line["rows"] = rows
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(sysm, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
