#!/usr/bin/env python
"""Benchmark of the AdANNS-IVF search hot path on one MI355X.

One step = one ``adanns_search`` over the whole query batch: coarse
assignment on the d_c prefix (MFMA tile kernel + selection), probe
bucketing, the list scan on the d_s prefix (MFMA tile kernel) and the
per-query top-k merge with exact re-measurement (Algorithm 1, inference).

Workload (default): the ImageNet-1K shape of the paper's retrieval
experiments (Section 3 "Datasets", Appendix C): N = 1,281,167 vectors of
d = 2048, 50,000 queries, nlist = 1024, d_s = 2048, k = 10, searched at
d_c = 64, nprobe = 8 (one point of the d_c x nprobe grid). Inputs are
seeded synthetic mixtures (``synth``), resident in HBM before timing.

The index is the oracle's: FP64 Lloyd (10 iterations on 64 * nlist seeded
training rows, then one assignment of every row), imported into the library,
so that the timed batch's own output can be checked against the oracle. The
library's GPU construction of the same index (adanns_build_ivf) is run and its
time reported.

The CPU-baseline leg (before any GPU work) times the FP64 oracle's IVF search
of queries spread evenly over the batch (default 512), its query loop split
over forked worker processes on the host's cores, mean of 3 runs, and
computes exact FP64 ground truth for them. The timed batch's output for those
queries is then checked against the oracle (tie-aware ids, distances to
1e-5) and recall@10 of both reported.

Prints one JSON line (rank 0, N = 1 only).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "QPS at recall@10 parity with FP64 oracle; p50/p99 latency; % HBM roofline"
MFMA_FP32_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="imagenet1k")
    ap.add_argument("--n", type=int, default=None, help="database rows (default: workload)")
    ap.add_argument("--nq", type=int, default=None)
    ap.add_argument("--dc", type=int, default=None)
    ap.add_argument("--nprobe", type=int, default=None)
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--cpu-sample", type=int, default=512,
                    help="queries of the batch the oracle searches (timed) and checks")
    ap.add_argument("--cpu-runs", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB device-to-device copy first (HBM counter calibration)")
    ap.add_argument("--form", default="ivf",
                    choices=["ivf", "precision", "batching", "pq", "serving", "diagnostics",
                             "sweep", "latency"],
                    help="ivf: the headline FP32 search; the others measure the other forms")
    ap.add_argument("--no-tune", action="store_true", help="skip the tile-shape autotuner")
    ap.add_argument("--no-filtered", action="store_true",
                    help="skip the exact search with a quantised first pass")
    ap.add_argument("--row-copy", action="store_true",
                    help="add the row-major copy of the vectors that the exact re-measures read")
    ap.add_argument("--rerank", type=int, default=256, help="precision form shortlist")
    ap.add_argument("--widths", default=None,
                    help="sweep form: comma-separated d_c values (default: the whole grid)")
    ap.add_argument("--probes", default=None,
                    help="sweep form: comma-separated nprobe values (default: the whole grid)")
    ap.add_argument("--pq-rotation", default="opq", choices=["opq", "random"],
                    help="IVF-PQ forms: learned OPQ rotation or a seeded random one")
    return ap.parse_args()


SCAN_SOURCE_END = b"// ---- per-query selection and exact re-measurement"


def kernel_source_digest() -> str:
    """Digest of the FP32 tile kernels' source: internal.h and kernels.hip up
    to the start of the selection code (the tile kernels and every helper
    they use are defined above it), so that changes elsewhere keep the
    committed traffic figures valid."""
    import hashlib
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2305_19435_amd", "csrc", "internal.h"), "rb") as fh:
        h.update(fh.read())
    with open(os.path.join(ROOT, "paper_2305_19435_amd", "csrc", "kernels.hip"), "rb") as fh:
        src = fh.read()
    cut = src.find(SCAN_SOURCE_END)
    if cut < 0:
        raise RuntimeError("kernels.hip: the selection-code marker is missing")
    h.update(src[:cut])
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, shape):
    """HBM bytes per launch of ``kernel`` at tile shape ``shape`` (tq, tv, grid)
    from the committed counter summary, if it was taken on the current kernel
    source; otherwise None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path) or shape is None:
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_digest") != kernel_source_digest():
        return None
    return t.get("hbm_bytes_per_launch_by_shape", {}).get("%dx%dx%d" % tuple(shape))


def host_info():
    """Core count and CPU model of the host the oracle runs on."""
    import platform
    import subprocess
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
            "machine": platform.machine()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            key, _, val = line.partition(":")
            if key.strip() in ("Model name", "Socket(s)", "Core(s) per socket",
                               "Thread(s) per core", "CPU max MHz"):
                info[key.strip()] = val.strip()
    except Exception:  # lscpu missing: fall back to /proc/cpuinfo
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    info["Model name"] = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return info


# The oracle's query loop is run by a pool of forked workers; these globals
# are set before the fork, so the workers share the arrays copy-on-write.
_ORACLE = {}


def _oracle_chunk(qs):
    from oracle import ivf
    g = _ORACLE
    return ivf.ivf_search64(g["X"], g["Q"][qs], g["C"], g["off"], g["ids"], g["d_c"], g["d_s"],
                            g["nprobe"], g["k"], return_candidates=True)


def oracle_search_timed(X, Q, qs, C64, off, ids, d_c, d_s, nprobe, k, workers, runs):
    """FP64 oracle IVF search of queries ``qs`` on ``workers`` processes (the
    oracle as it stands, its query loop split over the pool), ``runs`` times.
    Returns (dist, ids, probes, candidates, seconds per run)."""
    import multiprocessing as mp
    _ORACLE.update(X=X, Q=Q, C=C64, off=off, ids=ids, d_c=d_c, d_s=d_s, nprobe=nprobe, k=k)
    parts = [qs[i::workers] for i in range(workers)]
    times = []
    res = None
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        for _ in range(runs):
            t0 = time.perf_counter()
            res = pool.map(_oracle_chunk, parts)
            times.append(time.perf_counter() - t0)
    n = len(qs)
    D = np.empty((n, k))
    I = np.empty((n, k), dtype=np.int64)
    P = np.empty((n, nprobe), dtype=np.int64)
    cands = [None] * n
    for w_, (d_, i_, p_, c_) in enumerate(res):
        pos = np.arange(w_, n, workers)
        D[pos], I[pos], P[pos] = d_, i_, p_
        for j, c in zip(pos, c_):
            cands[j] = c
    return D, I, P, cands, times


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this library runs on one GPU only (multi-GPU sharding is "
                                   "designed, not built); --gpus must be 1"}), flush=True)
        sys.exit(2)

    import synth

    if args.form != "ivf":
        import torch
        import paper_2305_19435_amd as lib
        torch.cuda.set_device(0)
        import bench_forms
        bench_forms.run(args, lib, torch, log)
        return
    w = synth.WORKLOADS[args.workload]
    n = args.n or w.n
    nq = args.nq or w.nq
    d_c = args.dc or w.d_c
    nprobe = args.nprobe or w.nprobe
    d_s, k, nlist = w.d_s, w.k, w.nlist
    mix = w.mixture()

    t0 = time.time()
    X = mix.database(n)
    Q = mix.queries(nq)
    log(f"generated X {X.shape} Q {Q.shape} in {time.time() - t0:.1f}s")

    # ---- CPU side first (before the GPU is touched, so that the oracle's
    # worker processes fork from a process without a GPU context) ----
    from oracle import exact, kmeans, metrics
    n_train = min(n, 64 * nlist)
    train_rows = synth.subsample_rows(n, n_train, w.seed)
    init = synth.init_rows(n_train, nlist, w.seed)
    t0 = time.time()
    C64, _, _ = kmeans.kmeans64(X[train_rows, :d_c], nlist, args.iters, init)
    C32 = C64.astype(np.float32)
    assign = kmeans.assign64(X[:, :d_c], C32.astype(np.float64))
    off, ids_o = kmeans.build_lists(assign, nlist)
    oracle_build_s = time.time() - t0
    log(f"oracle index (Lloyd, {args.iters} iters on {n_train} rows) in {oracle_build_s:.1f}s")
    # queries spread over the whole batch: the oracle's timed sample and the
    # parity check of the timed batch
    sample = max(1, min(args.cpu_sample, nq))
    qs = np.unique(np.linspace(0, nq - 1, sample).round().astype(np.int64))
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.time()
        rd, ri, rp, rcand, times = oracle_search_timed(
            X, Q, qs, C32.astype(np.float64), off, ids_o, d_c, d_s, nprobe, k, workers,
            args.cpu_runs)
        log(f"oracle search of {len(qs)} queries x {args.cpu_runs} runs on {workers} processes: "
            f"{['%.2f' % t for t in times]} s")
        t0 = time.time()
        De, Ie = exact.exact_knn64(X, Q[qs], k)
        log(f"exact FP64 ground truth of the sample in {time.time() - t0:.1f}s")
        cpu = {"value": round(len(qs) / float(np.mean(times)), 3), "unit": "queries/s",
               "cores": workers, "kind": "oracle",
               "sample": f"{len(qs)} queries spread evenly over the {nq}-query batch, FP64 IVF "
                         f"search (NumPy, the oracle's query loop split over {workers} forked "
                         f"processes) on the oracle-built index; mean of {args.cpu_runs} runs",
               "runs_s": [round(t, 3) for t in times], "host": host_info()}

    # ---- GPU ----
    import torch
    import paper_2305_19435_amd as lib
    torch.cuda.set_device(0)
    t0 = time.time()
    Xd = torch.from_numpy(X).cuda()
    Qd = torch.from_numpy(Q).cuda()
    torch.cuda.synchronize()
    log(f"uploaded in {time.time() - t0:.1f}s")
    # the library's own index construction on the GPU (reported, not timed
    # below): Lloyd on the same training rows from the same initial rows
    t0 = time.time()
    gidx, obj = lib.IvfIndex.build_ivf(Xd, nlist, d_c, args.iters, init, train_rows=train_rows,
                                        return_objective=True)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    log(f"GPU index built in {build_s:.1f}s; objective {obj[0]:.1f} -> {obj[-1]:.1f}")
    gidx.free()
    # the timed search runs on the oracle-built index, so that its output can
    # be checked against the oracle query by query
    index = lib.IvfIndex.import_ivf(Xd, C32, assign.astype(np.int32))
    del Xd
    torch.cuda.empty_cache()
    if args.row_copy:
        index.add_row_copy()

    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("calibration copy: 1 GiB read, 1 GiB written")

    stream = torch.cuda.current_stream()
    dist = torch.empty((nq, k), dtype=torch.float32, device="cuda")
    ids = torch.empty((nq, k), dtype=torch.int64, device="cuda")
    shape = None
    if not args.no_tune:
        # the library's autotuner picks the scan tile shape for this search
        # shape and caches it; adanns_search then uses the cached choice
        t0 = time.time()
        tb = lib.Batch([(index, nq, d_c, d_s, nprobe, k)], ldq=w.d, ldk=k)
        shape = tb.autotune(Qd, out=(dist, ids), reps=1)
        tb.free()
        log(f"autotuned scan shape (tq, tv, grid) = {shape} in {time.time() - t0:.1f}s")
    for _ in range(args.warmup):
        index.search(Qd, d_c, d_s, nprobe, k, out=(dist, ids))
    torch.cuda.synchronize()

    lib.selection_stats(reset=True)
    lib.timing_reset()
    lib.timing_enable(True)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        index.search(Qd, d_c, d_s, nprobe, k, out=(dist, ids))
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    lib.timing_enable(False)
    reselected, uncertified = lib.selection_stats(reset=True)
    step_ms = np.array([a.elapsed_time(b) for a, b in evs])
    # per step (a search split into query chunks launches a kernel once per
    # chunk; at the headline each launches once per step)
    kern, launches = {}, {}
    for name in ("stage_queries", "tile_dist_coarse", "select_coarse", "bucketing",
                 "tile_dist_scan", "select_scan", "select_redo"):
        cnt, ms = lib.timing_read(name)
        if cnt:
            kern[name] = ms / args.steps
            launches[name] = cnt / args.steps
    ms_per_step = wall * 1000.0 / args.steps
    qps = nq * args.steps / wall
    log(f"{args.steps} steps: {ms_per_step:.3f} ms/step, {qps:,.0f} QPS; kernels {kern}; "
        f"re-selected {reselected}, uncertified {uncertified}")
    timed_d = dist.cpu().numpy()
    timed_i = ids.cpu().numpy()
    filtered = None if args.no_filtered else filtered_leg(lib, torch, index, Qd, d_c, d_s, nprobe, k,
                                                          args.steps, args.warmup, timed_d, timed_i)

    # the same steps with the queries handed over in pinned host memory: the
    # PCIe-inclusive rate (context only; ``value`` keeps inputs resident)
    Qh = torch.from_numpy(Q).pin_memory()
    Qstage = torch.empty_like(Qd)
    torch.cuda.synchronize()
    t_h = time.perf_counter()
    for _ in range(args.steps):
        Qstage.copy_(Qh, non_blocking=True)
        index.search(Qstage, d_c, d_s, nprobe, k, out=(dist, ids))
    torch.cuda.synchronize()
    qps_h2d = nq * args.steps / (time.perf_counter() - t_h)
    del Qh, Qstage

    # probes of the timed batch: one more search with probes out, which must
    # repeat the timed output bit for bit
    d2, i2, probes = index.search(Qd, d_c, d_s, nprobe, k, return_probes=True)
    torch.cuda.synchronize()
    probes = probes.cpu().numpy()
    repeat_bitwise = bool(np.array_equal(d2.cpu().numpy(), timed_d) and
                          np.array_equal(i2.cpu().numpy(), timed_i))
    lens = np.diff(off)
    cand = int(lens[probes.astype(np.int64)].sum())
    flops = {
        "tile_dist_scan": 2.0 * cand * d_s,
        "tile_dist_coarse": 2.0 * nq * nlist * d_c,
    }
    dominant = max(kern, key=kern.get)
    if dominant in flops:
        ach = flops[dominant] / (kern[dominant] * 1e-3) / 1e12
        roof = {"kernel": dominant, "bound": "mfma", "achieved": round(ach, 2),
                "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / MFMA_FP32_PEAK_TFLOPS, 4),
                "traffic": measured_traffic(dominant, w.name, shape),
                "algorithmic_flops_per_launch": flops[dominant] / launches[dominant],
                "flop_count": "2 per (query, candidate, coordinate): one multiply-add of the "
                              "expanded form |x|^2 - 2 q.x on the matrix cores",
                "avg_launch_ms": round(kern[dominant] / launches[dominant], 4),
                "launches_per_step": launches[dominant]}
    else:
        roof = {"kernel": dominant, "bound": "alu", "achieved": None, "peak": None,
                "unit": None, "frac": None, "traffic": None}
    scan_bytes = 4.0 * n * d_s  # one read of the d_s prefix of every vector
    roof["scan_hbm_floor_frac"] = round(scan_bytes / (kern.get("tile_dist_scan", 1e9) * 1e-3)
                                        / 1e9 / HBM_PEAK_GBS, 4)
    # measured bandwidth of this GPU beside the published 8 TB/s: a device
    # copy (1 GiB read + 1 GiB written) and the library's read-only probe
    a_ = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b_ = torch.empty_like(a_)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b_.copy_(a_)
    e0.record()
    for _ in range(5):
        b_.copy_(a_)
    e1.record()
    torch.cuda.synchronize()
    roof["stream_copy_gbs"] = round(5 * 2 * (1 << 30) / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del b_
    roof["stream_read_gbs"] = stream_read_gbs(lib, torch, a_)
    del a_
    # every other kernel of the step against its own bound (algorithmic work)
    # first-pass values + the k rows every query must re-measure (the
    # error-bounded shortlist re-measures the band's rows, at least k; the
    # count is data-dependent, so the achieved rate is a lower bound)
    sel_bytes = 4.0 * cand + nq * k * d_s * 4.0
    others = {}
    if "tile_dist_coarse" in kern:
        t_ = flops["tile_dist_coarse"] / (kern["tile_dist_coarse"] * 1e-3) / 1e12
        others["tile_dist_coarse"] = {"bound": "mfma", "achieved": round(t_, 2),
                                      "unit": "TFLOP/s",
                                      "frac": round(t_ / MFMA_FP32_PEAK_TFLOPS, 4)}
    if "select_scan" in kern:
        g_ = sel_bytes / (kern["select_scan"] * 1e-3) / 1e9
        others["select_scan"] = {"bound": "hbm", "achieved": round(g_, 1), "unit": "GB/s",
                                 "frac": round(g_ / HBM_PEAK_GBS, 4),
                                 "algorithmic_bytes_per_launch": sel_bytes}
    roof["other_kernels"] = others

    out = {
        "metric": METRIC,
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: seeded Gaussian mixture, decaying spectrum, L2-normalised",
        "config": {"workload": f"{w.name}: N={n} d={w.d} nq={nq} nlist={nlist} d_c={d_c} "
                               f"d_s={d_s} nprobe={nprobe} k={k}",
                   "n": n, "d": w.d, "nq": nq, "nlist": nlist, "d_c": d_c, "d_s": d_s,
                   "nprobe": nprobe, "k": k, "candidates_per_query": cand / nq,
                   "index": f"oracle Lloyd (FP64), {args.iters} iters on {n_train} seeded rows, "
                            f"imported; the library's GPU build of the same took "
                            f"{round(build_s, 2)} s",
                   "scan_shape": {"tq": shape[0], "tv": shape[1], "grid": shape[2]} if shape else "default",
                   "remeasure_from": "row-major copy of the vectors" if args.row_copy else
                                     "slab layout",
                   "index_device_bytes": index.device_bytes()},
        "latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 4),
                       "p99": round(float(np.percentile(step_ms, 99)), 4),
                       "note": "whole-batch latency per step"},
        "kernels_ms_per_step": {k_: round(v, 4) for k_, v in kern.items()},
        "shortlists": {"reselected_per_step": reselected / args.steps,
                       "uncertified": uncertified},
        "qps_including_h2d": round(qps_h2d, 1),
        "exact_with_quantised_first_pass": filtered,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if cpu is not None:
        out["recall_at_10"], out["oracle_parity"] = parity_leg(
            X, Q, qs, C32, off, ids_o, d_c, d_s, nprobe, k, timed_d, timed_i, probes, rd, ri,
            rp, rcand, Ie, repeat_bitwise)
    index.free()
    print(json.dumps(out), flush=True)


def filtered_leg(lib, torch, index, Qd, d_c, d_s, nprobe, k, steps, warmup, timed_d, timed_i):
    """The same search's exact FP32 result from a quantised first pass
    (adanns_search_filtered: BF16 / e4m3 list scan, FP32 re-measure of the
    candidates whose quantisation bound reaches the k-th): its rate and
    whether its output equals the timed FP32 path's bit for bit."""
    out = {}
    nq = Qd.shape[0]
    for fmt in ("bf16", "fp8"):
        index.set_precision(fmt)
        d_ = torch.empty((nq, k), dtype=torch.float32, device="cuda")
        i_ = torch.empty((nq, k), dtype=torch.int64, device="cuda")
        for _ in range(warmup):
            index.search_filtered(Qd, d_c, d_s, nprobe, k, fmt, out=(d_, i_))
        torch.cuda.synchronize()
        lib.filtered_stats(reset=True)
        lib.timing_reset()
        lib.timing_enable(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            index.search_filtered(Qd, d_c, d_s, nprobe, k, fmt, out=(d_, i_))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lib.timing_enable(False)
        measured, windowed = lib.filtered_stats(reset=True)
        kern = {}
        for name in ("tile_dist_coarse", "select_coarse", "bucketing", "tile_q_scan",
                     "select_filtered"):
            cnt, ms = lib.timing_read(name)
            if cnt:
                kern[name] = round(ms / steps, 4)  # per step
        same = bool(np.array_equal(d_.cpu().numpy(), timed_d) and
                    np.array_equal(i_.cpu().numpy(), timed_i))
        out[fmt] = {"qps": round(nq * steps / wall, 1), "ms_per_step": round(wall * 1e3 / steps, 4),
                    "kernels_ms_per_step": kern, "output_bitwise_equal_to_fp32_path": same,
                    "exact_measures_per_query": round(measured / (nq * steps), 2),
                    "queries_windowed_frac": round(windowed / (nq * steps), 5)}
        log(f"exact search with a {fmt} first pass: {out[fmt]}")
    return out


def stream_read_gbs(lib, torch, buf):
    """Read bandwidth of the library's read-only probe over ``buf`` (1 GiB)."""
    grid = 32768
    part = torch.empty(grid, dtype=torch.float32, device="cuda")
    nbytes = buf.numel() * 4
    lib.check(lib.lib.adanns_stream_read(buf.data_ptr(), nbytes, part.data_ptr(), grid,
                                         torch.cuda.current_stream().cuda_stream))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        lib.check(lib.lib.adanns_stream_read(buf.data_ptr(), nbytes, part.data_ptr(), grid,
                                             torch.cuda.current_stream().cuda_stream))
    e1.record()
    torch.cuda.synchronize()
    return round(5 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)


def parity_leg(X, Q, qs, C32, off, ids_o, d_c, d_s, nprobe, k, gd_all, gi_all, gp_all, rd, ri,
               rp, rcand, Ie, repeat_bitwise):
    """The timed batch's output for the sampled queries against the oracle
    (tie-aware ids, distances to 1e-5; probes within the tie band, the
    oracle re-run on the library's probes where they differ)."""
    from oracle import check, ivf, metrics
    t0 = time.time()
    gd, gi, gp = gd_all[qs], gi_all[qs], gp_all[qs]
    Cf = C32.astype(np.float64)
    probe_ok = all(check.probes_valid(ivf.coarse64(Q[q], Cf, d_c), gp[j], nprobe)
                   for j, q in enumerate(qs))
    differ = [j for j in range(len(qs)) if not np.array_equal(gp[j], rp[j])]
    rep = check.Report()
    if probe_ok:
        if differ:
            sub = np.asarray(differ)
            d2, i2, _, c2 = ivf.ivf_search64(X, Q[qs[sub]], Cf, off, ids_o, d_c, d_s, nprobe, k,
                                             forced_probes=gp[sub], return_candidates=True)
            for t, j in enumerate(differ):
                rd[j], ri[j], rcand[j] = d2[t], i2[t], c2[t]
        for j, q in enumerate(qs):
            check.compare_knn(Q[q], X, rcand[j], gd[j], gi[j], rd[j], ri[j], d_s, report=rep,
                              tag=f"q{q}")
    rec = {"gpu": metrics.k_recall_at_n(gi, Ie, k), "oracle": metrics.k_recall_at_n(ri, Ie, k),
           "queries": int(len(qs)), "ground_truth": "exact FP64 k-NN at full d"}
    parity = {"queries": int(len(qs)), "of_timed_batch": True,
              "timed_output_repeats_bitwise": repeat_bitwise,
              "probes_valid": bool(probe_ok), "probe_sets_differing": len(differ),
              "ok": bool(rep.ok and probe_ok and repeat_bitwise),
              "id_ties": rep.id_mismatch_ties, "max_rel_dist_err": rep.max_rel_dist_err,
              "problems": rep.problems[:3]}
    log(f"oracle parity of the timed batch {parity} in {time.time() - t0:.1f}s")
    return rec, parity


if __name__ == "__main__":
    main()
