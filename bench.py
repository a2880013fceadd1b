"""Benchmark: sparse triangular solves on one MI355X.

Workload (default): lower and upper triangles (diagonal included) of the 3-D
7-point Laplacian on a 128^3 grid, natural order, FP64 CSR, one right-hand
side.  One step is the paper's experiment (Sec. 5, eq. (3)): the lower solve
followed by the upper solve, y = U^{-1} (L^{-1} b), with the self-scheduled
solver (the schedule under test) -- and the same step is timed with the
level-scheduled solver for the speedup.

Metric: effective HBM GB/s = algorithmic bytes / time, with the bytes lower
bound of one solve nnz*(vb+4) + (n+1)*4 + 3*n*vb (matrix values and indices
once, row pointers once, b read, x written, x read once by dependents),
summed over the two triangles of a step; also solves/s.  Inputs are resident
in HBM before the timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  Its "per_config" object holds the other workloads
(2-D 64x64 lower, the random power-law triangle in FP64 and FP32, the batch
of 256 ILU(0) factors, 16 right-hand sides, the forward solve plus adjoint),
each under the same protocol with its full-size oracle error, roofline
fraction, critical-path bound and setup break-even (Sec. 5.3, Table 7).
--suite also writes per-configuration lines (with the block schedule and
graph replays) to bench_suite.jsonl in the output folder (--out-dir).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
METRIC = "SpTRSV effective HBM GB/s + solves/s (FP64, 1e-12 rel) vs level-scheduled"


def lb_bytes(n, nnz, vb=8, k=1):
    return nnz * (vb + 4) + (n + 1) * 4 + 3 * n * vb * k


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--side", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--epl", type=int, default=None, help="fixed entries per lane (with --no-tune)")
    ap.add_argument("--grid", type=int, default=None, help="fixed persistent grid (with --no-tune)")
    ap.add_argument("--assign", type=int, default=None, help="fixed chunk assignment (with --no-tune)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    ap.add_argument("--no-per-config", action="store_true",
                    help="skip the other workloads (C1, C3, C4a, C4b, C5) in the JSON line")
    ap.add_argument("--configs", default="all",
                    help="comma-separated per-configuration records to run (default all)")
    ap.add_argument("--poll", type=int, default=None, help="fixed polling mode (with --no-tune)")
    ap.add_argument("--xp-stride", type=int, default=None, help="fixed slot width (with --no-tune)")
    ap.add_argument("--suite", action="store_true")
    ap.add_argument("--setup", action="store_true",
                    help="also time the host and device setup routes (bench_setup.jsonl)")
    ap.add_argument("--table2", action="store_true",
                    help="also run the Table 2 grid sweep (bench_table2.jsonl)")
    ap.add_argument("--out-dir", default="bench_results",
                    help="folder (relative to this file) for the extra JSON lines")
    return ap.parse_args()


def committed_traffic(kernel, schedule):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None unless that summary covers this kernel under this
    schedule (lanes rule, grid, assignment, polling, slot width) with the
    current kernels.hip."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "k_self_static_lap3d128_hbm_counters.md")
    try:
        rec = None
        with open(path) as f:
            for line in f:
                if line.startswith("traffic_json:"):
                    rec = json.loads(line.split(":", 1)[1])
        src = os.path.join(root, "paper_1710_04985_amd", "csrc", "kernels.hip")
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernels_hip_sha256_16") != h or rec.get("kernel") != kernel:
        return None
    if rec.get("schedule") != schedule:
        return None
    return rec["bytes_per_launch"]


SCHED_KEYS = ("entries_per_lane", "grid", "assign", "poll", "xp_stride")


def cpu_info():
    """(CPU model, logical CPUs visible, current clock in MHz or None)."""
    model = platform.processor()
    mhz = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and model == platform.processor():
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("cpu MHz") and mhz is None:
                    mhz = float(line.split(":", 1)[1])
    except (OSError, ValueError):
        pass
    return model, os.cpu_count(), mhz


def cpu_baseline(TL, TU, bL, seconds):
    """The oracle (plain C, FP64, one thread) on the same L+U step, repeated
    for about `seconds` of CPU time."""
    import oracle
    o = oracle.get()
    t0 = time.perf_counter()
    reps = 0
    while True:
        y = o.solve(TL.row_ptr, TL.col_idx, TL.vals, bL, False)
        o.solve(TU.row_ptr, TU.col_idx, TU.vals, y, True)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return el / reps, reps


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    import paper_1710_04985_amd as sp

    dev = "cuda:0"
    torch.cuda.set_device(0)
    side = args.side
    TL, xsL, bL = W.c2_lap3d(side=side, upper=False)
    TU = W.laplacian_triangle((side,) * 3, upper=True, diag=6.0)

    def to_dev(T):
        return (torch.from_numpy(T.row_ptr).to(dev), torch.from_numpy(T.col_idx).to(dev),
                torch.from_numpy(T.vals).to(dev))

    dL, dU = to_dev(TL), to_dev(TU)
    b = torch.from_numpy(bL).to(dev)
    torch.cuda.synchronize()

    # analysis on the device (the faster of the two setup routes; both give
    # the same plan bit for bit); the host route is timed for reference.  A
    # first device setup loads the setup kernels and is not timed.
    sp.Handle(*dL, uplo="L", setup="device").close()
    t0 = time.perf_counter()
    hL = sp.Handle(*dL, uplo="L", setup="device")
    analysis_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    sp.Handle(*dL, uplo="L", setup="host").close()
    analysis_ms_host = (time.perf_counter() - t0) * 1e3
    hU = sp.Handle(*dU, uplo="U", setup="device")
    lvL = sp.Handle(*dL, uplo="L").configure(algo=sp.ALGO_LEVEL)
    lvU = sp.Handle(*dU, uplo="U").configure(algo=sp.ALGO_LEVEL)
    nlev = hL.info()["nlev"]

    # the self-scheduled solver: the library's autotuner picks lanes per row
    # and the readiness signal among the self-scheduled candidates; the
    # level-scheduled baseline is tuned the same way among its own
    tuned = {}
    if not args.no_tune:
        for name, h in (("L", hL), ("U", hU), ("L_level", lvL), ("U_level", lvU)):
            if h in (hL, hU):
                h.set_option("algo", sp.ALGO_SELF)
            tuned[name] = h.tune(b)
    else:
        for h in (hL, hU):
            h.set_option("algo", sp.ALGO_SELF)
            if args.epl is not None:
                h.set_option("entries_per_lane", args.epl)
            if args.grid is not None:
                h.set_option("grid", args.grid)
            if args.assign is not None:
                h.set_option("assign", args.assign)
            if args.poll is not None:
                h.set_option("poll", args.poll)
            if args.xp_stride is not None:
                h.set_option("xp_stride", args.xp_stride)
        tuned = {"L": hL.info(), "U": hU.info()}

    def step(hl, hu, out1, out2):
        hl.solve(b, out=out1)
        hu.solve(out1, out=out2)

    y1 = torch.empty_like(b)
    y2 = torch.empty_like(b)

    # parity of the timed configuration against the oracle at full size
    import oracle
    o = oracle.get()
    step(hL, hU, y1, y2)
    hL.status()
    hU.status()
    xo1 = o.solve(TL.row_ptr, TL.col_idx, TL.vals, bL, False)
    xo2 = o.solve(TU.row_ptr, TU.col_idx, TU.vals, xo1, True)
    r1 = y1.cpu().numpy()
    r2 = y2.cpu().numpy()
    err = max(np.abs(r1 - xo1).max() / np.abs(xo1).max(), np.abs(r2 - xo2).max() / np.abs(xo2).max())
    step(lvL, lvU, y1, y2)
    err_level = max(np.abs(y1.cpu().numpy() - xo1).max() / np.abs(xo1).max(),
                    np.abs(y2.cpu().numpy() - xo2).max() / np.abs(xo2).max())
    if err > 1e-12 or err_level > 1e-12:
        print("parity failure: self %.3e level %.3e" % (err, err_level), file=sys.stderr)
        sys.exit(1)

    def timed(hl, hu, steps, warmup):
        for _ in range(warmup):
            step(hl, hu, y1, y2)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            step(hl, hu, y1, y2)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_self = timed(hL, hU, args.steps, args.warmup)
    ms_level = timed(lvL, lvU, args.steps, args.warmup)

    # the same step replayed from HIP graphs (one per triangle): the
    # level-scheduled solve's per-level launches become graph nodes
    def timed_graph(hl, hu, steps, warmup):
        gs = torch.cuda.Stream()
        with torch.cuda.stream(gs):
            g1 = hl.capture(b, y1, stream=gs)
            g2 = hu.capture(y1, y2, stream=gs)
            for _ in range(warmup):
                g1.launch(gs)
                g2.launch(gs)
            gs.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(gs)
            for _ in range(steps):
                g1.launch(gs)
                g2.launch(gs)
            e1.record(gs)
            e1.synchronize()
        hl.status()
        hu.status()
        g1.close()
        g2.close()
        return e0.elapsed_time(e1) / steps

    ms_self_graph = timed_graph(hL, hU, args.steps, args.warmup)
    ms_level_graph = timed_graph(lvL, lvU, args.steps, args.warmup)

    # cold steps: a 1 GiB write evicts the L2s and the last-level cache first
    flush = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    cold = []
    for k in range(5):
        flush.fill_(float(k))
        torch.cuda.synchronize()
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        step(hL, hU, y1, y2)
        c1.record()
        c1.synchronize()
        cold.append(c0.elapsed_time(c1))
    # measured device copy bandwidth (read + write bytes over time), the
    # practical ceiling the HBM fraction is also given against
    src, dst = flush[: 1 << 26], flush[1 << 26:]
    for _ in range(3):
        dst.copy_(src)
    k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    k0.record()
    for _ in range(10):
        dst.copy_(src)
    k1.record()
    k1.synchronize()
    copy_gbs = 2 * src.numel() * 8 * 10 / (k0.elapsed_time(k1) * 1e-3) / 1e9
    del src, dst, flush
    ms_cold = float(np.median(cold))

    # critical-path bound: one producer-to-consumer hop per level
    hop_same = min(sp.probe_hop(same_xcd=True) for _ in range(3))
    hop_cross = min(sp.probe_hop(same_xcd=False) for _ in range(3))

    # per-kernel durations of the self-scheduled solve kernel (HIP events the
    # library records on the solve stream around the kernel launch)
    for h in (hL, hU):
        h.set_option("timing", 1)
        h.kernel_time(reset=True)
    timed(hL, hU, args.steps, 2)
    kmsL, kcL = hL.kernel_time()
    kmsU, kcU = hU.kernel_time()
    for h in (hL, hU):
        h.set_option("timing", 0)
    kernel_ms = (kmsL + kmsU) / max(1, kcL + kcU)

    infoL = hL.info()
    schedule = {k: infoL[k] for k in SCHED_KEYS}
    if infoL["sync"] == sp.SYNC_FLAG:
        kernel_name = "k_self_flag<double>"
    elif infoL["assign"] in (sp.ASSIGN_STATIC, sp.ASSIGN_XCD):
        kernel_name = "k_self_static<double, %d, false>" % infoL["xp_stride"]
    else:
        kernel_name = "k_self_value<double, false>"
    lbL = lb_bytes(TL.n, TL.nnz)
    lbU = lb_bytes(TU.n, TU.nnz)
    nnz_a = TL.nnz + TU.nnz - TL.n
    step_bytes = lbL + lbU
    gbs = step_bytes / (ms_self * 1e-3) / 1e9
    gbs_level = step_bytes / (ms_level * 1e-3) / 1e9
    achieved = lbL / (kernel_ms * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": round(gbs, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_self, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: 3-D 7-point Laplacian triangles (diag 6, off-diag -1), b = L x*, x* ~ U[-1,1] seed 2",
        "config": {"workload": "lap3d_7pt_%d^3_lower_then_upper" % side, "n": TL.n,
                   "nnz_per_triangle": TL.nnz, "nlev": nlev, "rhs": 1,
                   "solver": "self-scheduled", "tuned": tuned},
        "solves_per_s": round(2.0 / (ms_self * 1e-3), 2),
        "level_scheduled": {"ms_per_step": round(ms_level, 5), "gbs": round(gbs_level, 3),
                            "solves_per_s": round(2.0 / (ms_level * 1e-3), 2),
                            "graph_ms_per_step": round(ms_level_graph, 5)},
        "self_graph_ms_per_step": round(ms_self_graph, 5),
        "self_cold_ms_per_step": round(ms_cold, 5),
        "speedup_self_vs_level": round(ms_level / ms_self, 3),
        # the paper's rate for the L-then-U step, eq. (4): 2 nnz(A) / t with
        # A = L + U - D, the matrix both triangles come from
        "gflops_paper": {"self": round(2 * nnz_a / (ms_self * 1e-3) / 1e9, 3),
                         "level": round(2 * nnz_a / (ms_level * 1e-3) / 1e9, 3),
                         "nnz_A": nnz_a},
        "max_rel_err_vs_oracle": float("%.3e" % err),
        "analysis_ms": round(analysis_ms, 2),
        "analysis_ms_host_route": round(analysis_ms_host, 2),
        "bytes_per_step": step_bytes,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": committed_traffic(kernel_name, schedule),
                     "kernel": kernel_name, "schedule": schedule,
                     "kernel_ms": round(kernel_ms, 5), "bytes_per_launch": lbL,
                     "copy_gbs": round(copy_gbs, 1),
                     "frac_of_copy": round(achieved / copy_gbs, 5)},
        "critical_path": {"nlev": nlev, "hop_ns_same_xcd": round(hop_same, 1),
                          "hop_ns_cross_xcd": round(hop_cross, 1),
                          "bound_ms_per_triangle": round(nlev * hop_same * 1e-6, 5),
                          "kernel_over_bound": round(kernel_ms / (nlev * hop_same * 1e-6), 3)},
    }
    # setup amortisation (Sec. 5.3, Table 7) on the lower triangle: solves
    # after which the self-scheduled solver with the device analysis has cost
    # less in total than the level-scheduled one with the host analysis, and
    # than itself with the host analysis (same plan, same solve time)
    import bench_suite
    out["setup"] = {
        "self_device_route_ms": round(analysis_ms, 2), "level_host_route_ms": round(analysis_ms_host, 2),
        "n_s_self_device_vs_level_host": bench_suite.break_even(
            analysis_ms, ms_self / 2, analysis_ms_host, ms_level / 2),
        "n_s_device_vs_host_route": bench_suite.break_even(
            analysis_ms, ms_self / 2, analysis_ms_host, ms_self / 2)}
    if not args.no_per_config:
        for h in (hL, hU, lvL, lvU):
            h.close()
        torch.cuda.synchronize()
        names = bench_suite.CONFIGS if args.configs == "all" else tuple(args.configs.split(","))
        out["per_config"] = bench_suite.per_config(sp, torch, args.steps, args.warmup, hop_same,
                                                   names=names, tune=not args.no_tune)
    if not args.no_cpu_baseline:
        t_cpu, reps = cpu_baseline(TL, TU, bL, args.cpu_seconds)
        model, ncpu, mhz = cpu_info()
        out["cpu_baseline"] = {"value": round(step_bytes / t_cpu / 1e9, 4), "unit": "GB/s",
                               "cores": 1, "kind": "oracle",
                               "sample": "%d full L+U steps of the same workload (%.1f ms each) on %s, "
                                         "%d host CPUs visible%s" % (
                                             reps, t_cpu * 1e3, model, ncpu,
                                             ", %.0f MHz" % mhz if mhz else "")}
    if args.copy_probe_mb:
        nbytes = args.copy_probe_mb << 20
        src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nbytes
    out_dir = os.path.join(os.path.dirname(os.path.abspath(__file__)), args.out_dir)
    if args.suite or args.setup or args.table2:
        os.makedirs(out_dir, exist_ok=True)
    if args.suite:
        import bench_suite
        bench_suite.run(sp, torch, out_path=os.path.join(out_dir, "bench_suite.jsonl"))
    if args.setup:
        import bench_suite
        bench_suite.setup_routes(sp, torch, out_path=os.path.join(out_dir, "bench_setup.jsonl"))
    if args.table2:
        import bench_suite
        bench_suite.table2(sp, torch, out_path=os.path.join(out_dir, "bench_table2.jsonl"))
    # release every handle while the runtime is fully up (not at interpreter exit)
    for h in (hL, hU, lvL, lvU):
        h.close()
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
