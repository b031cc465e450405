#!/usr/bin/env python3
"""Benchmark: periodic ball query + RDF at N = 1,048,576 on one MI355X.

Workload: 64^3 FCC cells (N = 1,048,576) with Gaussian noise 0.05 a,
a = 4^(1/3) (density 1), in a triclinic box with tilts (0.5, 0.2, 0.1);
ball query r_max = 2.5 into a NeighborList (point index + distance per
pair) with a 256-bin RDF on [0, 2.5) binned in the same pass.

A step is one full pass from positions resident in HBM: cell-list build
(cell index, counting sort, scans), the ball query writing the list, and the
RDF histogram.  `value` counts ordered pairs found (and written, and binned)
per second.  The dominant kernel (the pair kernel) is timed with HIP events
on its own stream inside the timed region for the roofline entry.

The FP64 oracle is timed on the host on a bounded sample of query rows
(cpu_baseline); it is the brute-force checker, not a tuned CPU code.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time for the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def hip_runtime():
    import torch  # noqa: F401  (loads the process's HIP runtime first)
    L = ctypes.CDLL("libamdhip64.so.7")
    L.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    L.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                      ctypes.c_void_p]
    L.hipEventDestroy.argtypes = [ctypes.c_void_p]
    return L


def cpu_baseline(sysm, n_pairs_total, target_s):
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
        lo, hi, _ = oracle.rdf_counts(ob, sysm.points, 256, 2.5, query_points=q, exclude_ii=False)
        dt = time.perf_counter() - t
        return dt, int(idx.shape[0]) - nq  # drop each row's self pair at r = 0

    dt, _ = run(128)
    nq = int(min(n, max(128, 128 * target_s / max(dt, 1e-3))))
    dt, pairs = run(nq)
    return {"value": pairs / dt, "unit": "pairs/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{nq} random query rows of the same N=1,048,576 system (brute force over "
                      f"all points, FP64), ball list + RDF, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1906_06317_amd as ppa
    from paper_1906_06317_amd import workloads

    torch.cuda.set_device(0)
    hip = hip_runtime()
    L = ppa.lib()
    sysm = workloads.large_fcc()
    n = sysm.points.shape[0]
    r_max, bins = 2.5, 256
    box = ppa.Box(sysm.L, sysm.tilt, sysm.dim)
    pts = torch.as_tensor(sysm.points).cuda()

    # size the outputs exactly from one pass
    counts0, nl0 = ppa.rdf_counts(box, pts, bins, r_max, neighbor_list=True)
    P = nl0.n_pairs
    hist1 = counts0.cpu().numpy()
    del nl0

    ws = ppa.Workspace()
    wptr, wlen = ws.get(ppa.workspace_bytes(box, n, 0, r_max, ppa.PPA_WS_NLIST))
    offsets = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    rowc = torch.empty(n, dtype=torch.int32, device="cuda")
    pidx = torch.empty(P, dtype=torch.int32, device="cuda")
    dist = torch.empty(P, dtype=torch.float32, device="cuda")
    npairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    hist = torch.zeros(bins, dtype=torch.int64, device="cuda")
    cb = box.c()
    stream = torch.cuda.current_stream()
    sptr = ctypes.c_void_p(stream.cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())

    def step():
        rc = L.ppa_rdf(ctypes.byref(cb), p(pts), n, None, n, bins, 0.0, r_max, 1, 0, wptr, wlen,
                       p(hist), p(offsets), p(rowc), p(pidx), p(dist), P, p(npairs), sptr)
        if rc != 0:
            raise RuntimeError(L.ppa_last_error().decode())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if ws.status() != 0:
        raise RuntimeError("device status after warmup: " + L.ppa_last_error().decode())

    ev = []
    for _ in range(args.steps):
        e4 = [ctypes.c_void_p() for _ in range(4)]
        for e in e4:
            assert hip.hipEventCreate(ctypes.byref(e)) == 0
        ev.append(e4)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for i in range(args.steps):
        L.ppa_profile_next(*ev[i])
        step()
    t1.record()
    torch.cuda.synchronize()
    ms_step = t0.elapsed_time(t1) / args.steps
    count_ms, fill_ms = [], []
    for e4 in ev:
        f = ctypes.c_float()
        assert hip.hipEventElapsedTime(ctypes.byref(f), e4[0], e4[1]) == 0
        count_ms.append(f.value)
        assert hip.hipEventElapsedTime(ctypes.byref(f), e4[2], e4[3]) == 0
        fill_ms.append(f.value)
        for e in e4:
            hip.hipEventDestroy(e)
    st = ws.status()
    if st != 0:
        raise RuntimeError("device status: " + L.ppa_last_error().decode())
    # the histogram accumulates over calls: every step must add the same counts
    h = hist.cpu().numpy()
    assert np.array_equal(h, hist1 * (args.warmup + args.steps)), "histogram drifted across steps"
    assert int(npairs.item()) == P

    kernel_ms = float(np.mean(fill_ms))
    # algorithmic bytes of the fill kernel per launch: positions read (12 B per
    # point), row offsets read (8 B per query), neighbour list written (4 B
    # index + 4 B distance per pair), histogram (8 B per bin)
    alg_bytes = 12 * n + 8 * n + 8 * P + 8 * bins
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    out = {
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
                               "tilts (0.5,0.2,0.1); ball r_max=2.5 -> NeighborList + RDF 256 bins",
                   "n_points": n, "r_max": r_max, "bins": bins, "n_pairs": P,
                   "rows": "CSR in query order (count, scan, fill)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "fill_kernel (ball list + RDF)", "kernel_ms": kernel_ms,
                     "algorithmic_bytes": alg_bytes,
                     "count_kernel_ms": float(np.mean(count_ms)),
                     "step_effective_GBps": (12 * n + 8 * P + 8 * n + 8 * bins) / (ms_step * 1e-3) / 1e9},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sysm, P, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
