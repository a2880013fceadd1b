"""Per-configuration measurements (bench.py --suite).

For each workload: parity of the level- and self-scheduled solves against
the oracle at full size, then the mean time of repeated solves of each
(warm, inputs resident in HBM), effective GB/s over the bytes lower bound,
and the self-over-level speedup.  One JSON line per workload goes to the
output file; progress goes to stderr.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np

import oracle
import workloads as W

DEV = "cuda:0"


def lb_bytes(n, nnz, vb=8, k=1):
    return nnz * (vb + 4) + (n + 1) * 4 + 3 * n * vb * k


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _relerr(x, ref):
    return float(np.abs(np.asarray(x, np.float64) - ref).max() / max(np.abs(ref).max(), 1e-300))


def _time(torch, fn, reps, warm=3):
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def _tri(torch, T, dtype=None):
    dtype = dtype or torch.float64
    return (torch.from_numpy(T.row_ptr).to(DEV), torch.from_numpy(T.col_idx).to(DEV),
            torch.from_numpy(T.vals).to(DEV).to(dtype))


def _single(sp, torch, name, T, b, reps, dtype=None, tol=1e-12):
    """Level vs self on one triangle with one right-hand side."""
    dtype = dtype or torch.float64
    o = oracle.get()
    vals64 = T.vals if dtype == torch.float64 else T.vals.astype(np.float32).astype(np.float64)
    b64 = b if dtype == torch.float64 else b.astype(np.float32).astype(np.float64)
    xo = o.solve(T.row_ptr, T.col_idx, vals64, b64, T.upper)
    d = _tri(torch, T, dtype)
    bd = torch.from_numpy(b).to(DEV).to(dtype)
    x = torch.empty_like(bd)
    uplo = "U" if T.upper else "L"
    res = {"config": name, "n": T.n, "nnz": T.nnz, "dtype": "f64" if dtype == torch.float64 else "f32"}
    t0 = time.perf_counter()
    hs = sp.Handle(*d, uplo=uplo)
    res["analysis_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    res["nlev"] = hs.info()["nlev"]
    hl = sp.Handle(*d, uplo=uplo).configure(algo=sp.ALGO_LEVEL)
    hs.set_option("algo", sp.ALGO_SELF)
    res["tuned_self"] = hs.tune(bd, x)
    res["tuned_level"] = hl.tune(bd, x)
    hb = sp.Handle(*d, uplo=uplo).configure(algo=sp.ALGO_BLOCK)
    for tag, h in (("self", hs), ("level", hl), ("block", hb)):
        h.solve(bd, out=x)
        h.status()
        err = _relerr(x.cpu().numpy(), xo)
        res["rel_err_" + tag] = float("%.3e" % err)
        if err > tol:
            res["parity"] = "FAIL"
        res[tag + "_ms"] = round(_time(torch, lambda: h.solve(bd, out=x), reps), 5)
    vb = 8 if dtype == torch.float64 else 4
    lb = lb_bytes(T.n, T.nnz, vb)
    res["lb_bytes"] = lb
    res["gbs_self"] = round(lb / (res["self_ms"] * 1e-3) / 1e9, 3)
    res["gbs_level"] = round(lb / (res["level_ms"] * 1e-3) / 1e9, 3)
    res["gbs_block"] = round(lb / (res["block_ms"] * 1e-3) / 1e9, 3)
    res["solves_per_s_self"] = round(1e3 / res["self_ms"], 2)
    res["speedup_self_vs_level"] = round(res["level_ms"] / res["self_ms"], 3)
    res.setdefault("parity", "ok")
    return res


def _batched(sp, torch, reps):
    o = oracle.get()
    tris, xs, bs = W.c4a_batch()
    devs = [_tri(torch, t) for t in tris]
    bcat = np.concatenate(bs)
    bd = torch.from_numpy(bcat).to(DEV)
    x = torch.empty_like(bd)
    n = sum(t.n for t in tris)
    nnz = sum(t.nnz for t in tris)
    res = {"config": "c4a_batched_256_ilu0_2d", "n": n, "nnz": nnz, "systems": len(tris),
           "dtype": "f64"}
    t0 = time.perf_counter()
    hs = sp.BatchedHandle([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs])
    res["analysis_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    res["nlev"] = hs.info()["nlev"]
    hl = sp.BatchedHandle([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs])
    hl.set_option("algo", sp.ALGO_LEVEL)
    hs.set_option("algo", sp.ALGO_SELF)
    hb = sp.BatchedHandle([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs])
    hb.set_option("algo", sp.ALGO_BLOCK)
    res["tuned_self"] = hs.tune(bd, x)
    res["tuned_level"] = hl.tune(bd, x)
    xo = np.concatenate([o.solve(t.row_ptr, t.col_idx, t.vals, b) for t, b in zip(tris, bs)])
    for tag, h in (("self", hs), ("level", hl), ("block", hb)):
        h.solve(bd, out=x)
        h.status()
        res["rel_err_" + tag] = float("%.3e" % _relerr(x.cpu().numpy(), xo))
        res[tag + "_ms"] = round(_time(torch, lambda: h.solve(bd, out=x), reps), 5)
    # one HIP graph per solve, replayed
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for tag, h in (("self", hs), ("level", hl), ("block", hb)):
            g = h.capture(bd, x, stream=s)
            g.launch(s)
            s.synchronize()
            res["rel_err_graph_" + tag] = float("%.3e" % _relerr(x.cpu().numpy(), xo))
            res["graph_" + tag + "_ms"] = round(_time(torch, lambda: g.launch(s), reps), 5)
            g.close()
    lb = lb_bytes(n, nnz)
    res["lb_bytes"] = lb
    res["gbs_self"] = round(lb / (res["self_ms"] * 1e-3) / 1e9, 3)
    res["gbs_level"] = round(lb / (res["level_ms"] * 1e-3) / 1e9, 3)
    res["speedup_self_vs_level"] = round(res["level_ms"] / res["self_ms"], 3)
    res["gbs_block"] = round(lb / (res["block_ms"] * 1e-3) / 1e9, 3)
    res["parity"] = "ok" if max(v for k, v in res.items() if k.startswith("rel_err")) <= 1e-12 else "FAIL"
    return res


def _multi(sp, torch, reps, nrhs=16):
    o = oracle.get()
    T, X, B = W.c4b_multi(nrhs=nrhs)
    d = _tri(torch, T)
    Bd = torch.from_numpy(np.ascontiguousarray(B.T)).to(DEV)        # (nrhs, n): column-major n x nrhs
    Xd = torch.empty_like(Bd)
    res = {"config": "c4b_lap3d_128_lower_%drhs" % nrhs, "n": T.n, "nnz": T.nnz, "nrhs": nrhs,
           "dtype": "f64"}
    hs = sp.Handle(*d).configure(algo=sp.ALGO_SELF)
    hl = sp.Handle(*d).configure(algo=sp.ALGO_LEVEL)
    res["nlev"] = hs.info()["nlev"]
    Xo = o.solve_multi(T.row_ptr, T.col_idx, T.vals, B)
    hs.tune_multi(Bd)
    res["tuned_self"] = hs.info()
    for tag, h in (("self", hs), ("level", hl)):
        h.solve_multi(Bd, out=Xd)
        h.status()
        res["rel_err_" + tag] = float("%.3e" % _relerr(Xd.cpu().numpy().T, Xo))
        res[tag + "_ms"] = round(_time(torch, lambda: h.solve_multi(Bd, out=Xd), reps), 5)
    lb = lb_bytes(T.n, T.nnz, 8, nrhs)
    res["lb_bytes"] = lb
    res["gbs_self"] = round(lb / (res["self_ms"] * 1e-3) / 1e9, 3)
    res["gbs_level"] = round(lb / (res["level_ms"] * 1e-3) / 1e9, 3)
    res["rhs_solves_per_s_self"] = round(nrhs * 1e3 / res["self_ms"], 2)
    res["speedup_self_vs_level"] = round(res["level_ms"] / res["self_ms"], 3)
    res["parity"] = "ok" if max(res["rel_err_self"], res["rel_err_level"]) <= 1e-12 else "FAIL"
    return res


def _adjoint(sp, torch, reps, side=96):
    o = oracle.get()
    T, b, w = W.c5_ilu3d(side=side)
    d = _tri(torch, T)
    res = {"config": "c5_ilu0_3d_%d_fwd_adjoint" % side, "n": T.n, "nnz": T.nnz, "dtype": "f64"}
    xo, gbo, gvo = o.adjoint(T.row_ptr, T.col_idx, T.vals, b, w)
    wd = torch.from_numpy(w).to(DEV)
    bd0 = torch.from_numpy(b).to(DEV)
    for tag, algo in (("self", sp.ALGO_SELF), ("level", sp.ALGO_LEVEL)):
        h = sp.Handle(*d).configure(algo=algo)
        h.prepare_transpose()
        res["nlev"] = h.info()["nlev"]
        vals = d[2].clone().requires_grad_(True)
        bd = bd0.clone().requires_grad_(True)

        def step():
            vals.grad = None
            bd.grad = None
            x = sp.sptrsv(vals, bd, h)
            x.backward(wd)
            return x

        x = step()
        h.status()
        err = max(_relerr(x.detach().cpu().numpy(), xo), _relerr(bd.grad.cpu().numpy(), gbo),
                  _relerr(vals.grad.cpu().numpy(), gvo))
        res["rel_err_" + tag] = float("%.3e" % err)
        res[tag + "_ms"] = round(_time(torch, step, reps), 5)
    # forward + adjoint traffic: value gather (read vals, write copy), forward
    # solve, transposed solve, gradient on the pattern (row_ptr, col, x gather,
    # grad_b, grad_vals)
    lb_solve = lb_bytes(T.n, T.nnz)
    gather = T.nnz * 8 * 2 + T.nnz * 4
    grad = (T.n + 1) * 4 + T.nnz * 4 + T.n * 8 * 2 + T.nnz * 8
    lb = 2 * lb_solve + gather + grad
    res["lb_bytes"] = lb
    res["gbs_self"] = round(lb / (res["self_ms"] * 1e-3) / 1e9, 3)
    res["gbs_level"] = round(lb / (res["level_ms"] * 1e-3) / 1e9, 3)
    res["speedup_self_vs_level"] = round(res["level_ms"] / res["self_ms"], 3)
    res["parity"] = "ok" if max(res["rel_err_self"], res["rel_err_level"]) <= 1e-12 else "FAIL"
    return res


def run(sp, torch, out_path, reps=20):
    lines = []

    def emit(r):
        lines.append(r)
        _log(json.dumps(r))
        with open(out_path, "a") as f:
            f.write(json.dumps(r) + "\n")

    T, xs, b = W.c1_lap2d_64()
    emit(_single(sp, torch, "c1_lap2d_64_lower", T, b, reps))
    for upper in (False, True):
        T, xs, b = W.c2_lap3d(upper=upper)
        emit(_single(sp, torch, "c2_lap3d_128_" + ("upper" if upper else "lower"), T, b, reps))
    T, xs, b = W.c3_powerlaw()
    emit(_single(sp, torch, "c3_powerlaw_1M_f64", T, b, reps))
    emit(_single(sp, torch, "c3_powerlaw_1M_f32", T, b, reps, dtype=torch.float32, tol=1e-5))
    emit(_batched(sp, torch, reps))
    emit(_multi(sp, torch, reps))
    emit(_adjoint(sp, torch, reps))
    return lines


def table2(sp, torch, out_path, reps=10):
    """The paper's Sec. 5.1 experiment on its Table 2 grids: lower then upper
    solve (eq. (3)) of the 5/9-point (2-D, n = 2^20) and 7/27-point (3-D,
    n = 2^21) operators, self- vs level-scheduled, against nlev."""
    o = oracle.get()
    rows = []
    for dims_list, stencils in ((W.TABLE2_2D, (5, 9)), (W.TABLE2_3D, (7, 27))):
        for dims in dims_list:
            for pts in stencils:
                L = W.stencil_triangle(dims, pts)
                U = W.stencil_triangle(dims, pts, upper=True)
                b = W.uniform_vector(L.n, 7)
                y1 = o.solve(L.row_ptr, L.col_idx, L.vals, b, False)
                yo = o.solve(U.row_ptr, U.col_idx, U.vals, y1, True)
                dL, dU = _tri(torch, L), _tri(torch, U)
                bd = torch.from_numpy(b).to(DEV)
                t1 = torch.empty_like(bd)
                t2 = torch.empty_like(bd)
                res = {"config": "table2_%dpt_%s" % (pts, "x".join(map(str, dims))), "n": L.n,
                       "nnz_lower": L.nnz, "points": pts}
                for tag, algo in (("self", sp.ALGO_SELF), ("level", sp.ALGO_LEVEL)):
                    hl = sp.Handle(*dL, uplo="L").configure(algo=algo)
                    hu = sp.Handle(*dU, uplo="U").configure(algo=algo)
                    res["nlev"] = hl.info()["nlev"]
                    hl.tune(bd, t1)
                    hu.tune(bd, t1)

                    def step():
                        hl.solve(bd, out=t1)
                        hu.solve(t1, out=t2)

                    step()
                    hl.status()
                    hu.status()
                    res["rel_err_" + tag] = float("%.3e" % _relerr(t2.cpu().numpy(), yo))
                    res[tag + "_ms"] = round(_time(torch, step, reps), 5)
                lb = lb_bytes(L.n, L.nnz) + lb_bytes(U.n, U.nnz)
                res["lb_bytes_step"] = lb
                # the paper's GFLOPS of eq. (4): 2 nnz(A) / t, A = L + D + U
                nnzA = L.nnz + U.nnz - L.n
                res["gflops_self"] = round(2 * nnzA / (res["self_ms"] * 1e-3) / 1e9, 3)
                res["gflops_level"] = round(2 * nnzA / (res["level_ms"] * 1e-3) / 1e9, 3)
                res["gbs_self"] = round(lb / (res["self_ms"] * 1e-3) / 1e9, 3)
                res["speedup_self_vs_level"] = round(res["level_ms"] / res["self_ms"], 3)
                res["parity"] = "ok" if max(res["rel_err_self"], res["rel_err_level"]) <= 1e-12 else "FAIL"
                rows.append(res)
                _log(json.dumps(res))
                with open(out_path, "a") as f:
                    f.write(json.dumps(res) + "\n")
    return rows


def setup_routes(sp, torch, out_path, reps=3):
    """Setup phase (Sec. 4.4, Table 1 routes): wall time of the analysis on
    the host route and on the device route, the oracle's analysis on one
    host core, and the tuned self-scheduled solve time, whose ratio to the
    setup time is the number of solves that pay for one analysis."""
    o = oracle.get()
    rows = []
    work = [("c2_lap3d_128_lower", W.c2_lap3d(upper=False)[0]),
            ("c2_lap3d_128_upper", W.c2_lap3d(upper=True)[0]),
            ("c3_powerlaw_1M", W.c3_powerlaw()[0]),
            ("c5_ilu0_96", W.c5_ilu3d()[0])]
    for name, T in work:
        d = _tri(torch, T)
        uplo = "U" if T.upper else "L"
        res = {"config": "setup_" + name, "n": T.n, "nnz": T.nnz}
        t0 = time.perf_counter()
        lv, nlev, _, _, _ = o.analyze(T.row_ptr, T.col_idx, T.upper)
        res["oracle_analysis_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
        res["nlev"] = int(nlev)
        for route in ("host", "device"):
            ts = []
            for _ in range(reps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                h = sp.Handle(*d, uplo=uplo, setup=route)
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t0) * 1e3)
                got_route, lib_ms = h.setup_info()
                assert got_route == route
                if route == "device":
                    level = h.export_analysis()[0]
                    res["device_levels_equal_oracle"] = bool(np.array_equal(level, lv))
                h.close()
            res[route + "_setup_ms"] = round(float(np.median(ts[1:])), 3)
        h = sp.Handle(*d, uplo=uplo, setup="device")
        bd = torch.from_numpy(W.uniform_vector(T.n, 7)).to(DEV)
        xd = torch.empty_like(bd)
        h.tune(bd, xd)
        res["solve_ms"] = round(_time(torch, lambda: h.solve(bd, out=xd), 20), 5)
        res["device_setup_speedup"] = round(res["host_setup_ms"] / res["device_setup_ms"], 3)
        res["solves_per_device_setup"] = round(res["device_setup_ms"] / res["solve_ms"], 1)
        h.close()
        rows.append(res)
        _log(json.dumps(res))
        with open(out_path, "a") as f:
            f.write(json.dumps(res) + "\n")
    return rows


# ------------------------------------------------------------------------
# Per-configuration records of the default bench line: every workload other
# than the headline one, under the headline's protocol (the paper's Sec. 5:
# mean of back-to-back solves, warm, inputs resident in HBM), with the
# roofline fraction, the critical-path bound, the full-size oracle error and
# the setup amortisation of Table 7.

def break_even(setup_a, solve_a, setup_b, solve_b):
    """Smallest n_s >= 0 with setup_a + n_s*solve_a < setup_b + n_s*solve_b
    (the paper's Sec. 5.3 criterion for Table 7); None if never."""
    if setup_a < setup_b and solve_a <= solve_b:
        return 0
    if solve_a >= solve_b:
        return None
    return int(np.floor((setup_a - setup_b) / (solve_b - solve_a))) + 1


def _kernel_ms(torch, h, fn, steps):
    """Mean duration of the library's main solve kernel (HIP events the
    library records on the solve stream around it)."""
    h.set_option("timing", 1)
    h.kernel_time(reset=True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    ms, cnt = h.kernel_time(reset=True)
    h.set_option("timing", 0)
    return ms / max(cnt, 1)


def _schedule(info):
    keys = ("algo", "entries_per_lane", "sync", "rows_per_lane", "grid", "assign", "poll",
            "xp_stride")
    return {k: info[k] for k in keys}


def _finish(res, lb, hop_ns, hops, setup_self_ms=None, setup_level_host_ms=None,
            setup_host_ms=None):
    res["lb_bytes"] = lb
    res["gbs_self"] = round(lb / (res["self_ms"] * 1e-3) / 1e9, 3)
    res["gbs_level"] = round(lb / (res["level_ms"] * 1e-3) / 1e9, 3)
    res["frac_hbm_self"] = round(res["gbs_self"] / 8000.0, 5)
    if res.get("self_kernel_ms"):
        res["frac_hbm_self_kernel"] = round(lb / (res["self_kernel_ms"] * 1e-3) / 1e9 / 8000.0, 5)
    res["speedup_self_vs_level"] = round(res["level_ms"] / res["self_ms"], 3)
    bound = hops * hop_ns * 1e-6
    res["critical_path"] = {"hops": hops, "hop_ns": round(hop_ns, 1),
                            "bound_ms": round(bound, 5),
                            "self_over_bound": round(res["self_ms"] / bound, 3)}
    if setup_self_ms is not None:
        res["setup"] = {"self_device_route_ms": round(setup_self_ms, 2)}
        if setup_level_host_ms is not None:
            res["setup"]["level_host_route_ms"] = round(setup_level_host_ms, 2)
            res["setup"]["n_s_self_device_vs_level_host"] = break_even(
                setup_self_ms, res["self_ms"], setup_level_host_ms, res["level_ms"])
        if setup_host_ms is not None:
            res["setup"]["self_host_route_ms"] = round(setup_host_ms, 2)
            res["setup"]["n_s_device_vs_host_route"] = break_even(
                setup_self_ms, res["self_ms"], setup_host_ms, res["self_ms"])
    errs = [v for k, v in res.items() if k.startswith("rel_err")]
    tol = res.pop("_tol")
    res["parity"] = "ok" if errs and max(errs) <= tol else "FAIL"
    return res


def _timed_handle(torch, make):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = make()
    torch.cuda.synchronize()
    return h, (time.perf_counter() - t0) * 1e3


# The schedules the autotuner usually picks for each workload (used instead
# of tuning when the bench runs with --no-tune, e.g. under a profiler)
FIXED_SCHEDULES = {
    "c1_lap2d_64_lower": dict(algo=2, grid=256, assign=1),
    "c3_powerlaw_1M_f64": dict(algo=2, grid=512, assign=2, poll=1, xp_stride=4),
    "c3_powerlaw_1M_f32": dict(algo=2, grid=512, assign=2, poll=1, xp_stride=16),
    "c4a_batched_256_ilu0_2d": dict(algo=2, grid=512, assign=2, poll=1),
    "c4b_lap3d_128_lower_16rhs": dict(algo=2, grid=2048, assign=0, poll=1, multi_rows=1),
    "c5_ilu0_3d_96_fwd_adjoint": dict(algo=2, assign=0, grid=0, xp_stride=1),
}


def pc_single(sp, torch, T, b, steps, warmup, hop_ns, dtype=None, tol=1e-12, block=False,
              schedule=None):
    """One triangle, one right-hand side: self (tuned, or `schedule`) vs
    level (tuned, or its default)."""
    dtype = dtype or torch.float64
    o = oracle.get()
    vals64 = T.vals if dtype == torch.float64 else T.vals.astype(np.float32).astype(np.float64)
    b64 = b if dtype == torch.float64 else b.astype(np.float32).astype(np.float64)
    xo = o.solve(T.row_ptr, T.col_idx, vals64, b64, T.upper)
    d = _tri(torch, T, dtype)
    bd = torch.from_numpy(b).to(DEV).to(dtype)
    x = torch.empty_like(bd)
    uplo = "U" if T.upper else "L"
    res = {"n": T.n, "nnz": T.nnz, "dtype": "f64" if dtype == torch.float64 else "f32",
           "_tol": tol}
    hs, setup_dev = _timed_handle(torch, lambda: sp.Handle(*d, uplo=uplo, setup="device"))
    hh, setup_host = _timed_handle(torch, lambda: sp.Handle(*d, uplo=uplo, setup="host"))
    hh.close()
    hl = sp.Handle(*d, uplo=uplo).configure(algo=sp.ALGO_LEVEL)
    res["nlev"] = hs.info()["nlev"]
    hs.set_option("algo", sp.ALGO_SELF)
    if schedule is None:
        t0 = time.perf_counter()
        hs.tune(bd, x)
        res["tune_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
        hl.tune(bd, x)
    else:
        hs.configure(**schedule)
    res["schedule_self"] = _schedule(hs.info())
    hands = [("self", hs), ("level", hl)]
    if block:
        hands.append(("block", sp.Handle(*d, uplo=uplo).configure(algo=sp.ALGO_BLOCK)))
    for tag, h in hands:
        h.solve(bd, out=x)
        h.status()
        res["rel_err_" + tag] = float("%.3e" % _relerr(x.cpu().numpy(), xo))
        res[tag + "_ms"] = round(_time(torch, lambda: h.solve(bd, out=x), steps, warmup), 5)
    res["self_kernel_ms"] = round(_kernel_ms(torch, hs, lambda: hs.solve(bd, out=x), steps), 5)
    for _, h in hands:
        h.close()
    vb = 8 if dtype == torch.float64 else 4
    return _finish(res, lb_bytes(T.n, T.nnz, vb), hop_ns, res["nlev"], setup_dev, setup_host,
                   setup_host)


def pc_batched(sp, torch, steps, warmup, hop_ns, schedule=None):
    o = oracle.get()
    tris, xs, bs = W.c4a_batch()
    devs = [_tri(torch, t) for t in tris]
    bd = torch.from_numpy(np.concatenate(bs)).to(DEV)
    x = torch.empty_like(bd)
    n = sum(t.n for t in tris)
    nnz = sum(t.nnz for t in tris)
    res = {"n": n, "nnz": nnz, "systems": len(tris), "dtype": "f64", "_tol": 1e-12}
    parts = ([dv[0] for dv in devs], [dv[1] for dv in devs], [dv[2] for dv in devs])
    hs, setup_ms = _timed_handle(torch, lambda: sp.BatchedHandle(*parts, setup="device"))
    hl, setup_host = _timed_handle(torch, lambda: sp.BatchedHandle(*parts, setup="host"))
    hl.configure(algo=sp.ALGO_LEVEL)
    hb = sp.BatchedHandle(*parts).configure(algo=sp.ALGO_BLOCK)
    res["nlev"] = hs.info()["nlev"]
    hs.set_option("algo", sp.ALGO_SELF)
    if schedule is None:
        hs.tune(bd, x)
        hl.tune(bd, x)
    else:
        hs.configure(**schedule)
    res["schedule_self"] = _schedule(hs.info())
    xo = np.concatenate([o.solve(t.row_ptr, t.col_idx, t.vals, b) for t, b in zip(tris, bs)])
    for tag, h in (("self", hs), ("level", hl), ("block", hb)):
        h.solve(bd, out=x)
        h.status()
        res["rel_err_" + tag] = float("%.3e" % _relerr(x.cpu().numpy(), xo))
        res[tag + "_ms"] = round(_time(torch, lambda: h.solve(bd, out=x), steps, warmup), 5)
    res["self_kernel_ms"] = round(_kernel_ms(torch, hs, lambda: hs.solve(bd, out=x), steps), 5)
    # the whole batch from one HIP graph, replayed
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = hs.capture(bd, x, stream=s)
        g.launch(s)
        s.synchronize()
        res["rel_err_graph_self"] = float("%.3e" % _relerr(x.cpu().numpy(), xo))
        res["graph_self_ms"] = round(_time(torch, lambda: g.launch(s), steps, warmup), 5)
        g.close()
    for h in (hs, hl, hb):
        h.close()
    return _finish(res, lb_bytes(n, nnz), hop_ns, res["nlev"], setup_ms, setup_host, setup_host)


def pc_multi(sp, torch, steps, warmup, hop_ns, nrhs=16, schedule=None):
    o = oracle.get()
    T, X, B = W.c4b_multi(nrhs=nrhs)
    d = _tri(torch, T)
    Bd = torch.from_numpy(np.ascontiguousarray(B.T)).to(DEV)        # (nrhs, n): column-major
    Xd = torch.empty_like(Bd)
    res = {"n": T.n, "nnz": T.nnz, "nrhs": nrhs, "dtype": "f64", "_tol": 1e-12}
    hs, setup_ms = _timed_handle(torch, lambda: sp.Handle(*d, setup="device"))
    hs.set_option("algo", sp.ALGO_SELF)
    hl = sp.Handle(*d).configure(algo=sp.ALGO_LEVEL)
    res["nlev"] = hs.info()["nlev"]
    Xo = o.solve_multi(T.row_ptr, T.col_idx, T.vals, B)
    if schedule is None:
        hs.tune_multi(Bd)
    else:
        hs.configure(**schedule)
    for tag, h in (("self", hs), ("level", hl)):
        h.solve_multi(Bd, out=Xd)
        h.status()
        res["rel_err_" + tag] = float("%.3e" % _relerr(Xd.cpu().numpy().T, Xo))
        res[tag + "_ms"] = round(_time(torch, lambda: h.solve_multi(Bd, out=Xd), steps, warmup), 5)
    res["self_kernel_ms"] = round(
        _kernel_ms(torch, hs, lambda: hs.solve_multi(Bd, out=Xd), steps), 5)
    res["rhs_solves_per_s_self"] = round(nrhs * 1e3 / res["self_ms"], 2)
    for h in (hs, hl):
        h.close()
    return _finish(res, lb_bytes(T.n, T.nnz, 8, nrhs), hop_ns, res["nlev"], setup_ms)


def pc_adjoint(sp, torch, steps, warmup, hop_ns, side=96, schedule=None):
    """Forward solve plus adjoint (transposed solve and gradient on the
    pattern) through torch.autograd, self vs level."""
    o = oracle.get()
    T, b, w = W.c5_ilu3d(side=side)
    d = _tri(torch, T)
    res = {"n": T.n, "nnz": T.nnz, "dtype": "f64", "_tol": 1e-12}
    xo, gbo, gvo = o.adjoint(T.row_ptr, T.col_idx, T.vals, b, w)
    wd = torch.from_numpy(w).to(DEV)
    bd0 = torch.from_numpy(b).to(DEV)
    setup_ms = {}
    for tag, algo in (("self", sp.ALGO_SELF), ("level", sp.ALGO_LEVEL)):
        def make(route):
            h = sp.Handle(*d, setup=route).configure(algo=algo)
            h.prepare_transpose()
            return h
        if tag == "self":
            hh, setup_ms["host"] = _timed_handle(torch, lambda: make("host"))
            hh.close()
        h, setup_ms[tag] = _timed_handle(torch, lambda: make("device" if tag == "self" else "host"))
        res["nlev"] = h.info()["nlev"]
        # the forward direction's schedule (tuned, or the fixed one) serves
        # the adjoint's transposed solve too
        if schedule is None:
            h.tune(bd0, torch.empty_like(bd0))
        elif tag == "self":
            h.configure(**schedule)
        if tag == "self":
            res["schedule_self"] = _schedule(h.info())
        vals = d[2].clone().requires_grad_(True)
        bd = bd0.clone().requires_grad_(True)

        def step():
            vals.grad = None
            bd.grad = None
            x = sp.sptrsv(vals, bd, h)
            x.backward(wd)
            return x

        x = step()
        h.status()
        err = max(_relerr(x.detach().cpu().numpy(), xo), _relerr(bd.grad.cpu().numpy(), gbo),
                  _relerr(vals.grad.cpu().numpy(), gvo))
        res["rel_err_" + tag] = float("%.3e" % err)
        res[tag + "_ms"] = round(_time(torch, step, steps, warmup), 5)
        h.close()
    lb_solve = lb_bytes(T.n, T.nnz)
    gather = T.nnz * 8 * 2 + T.nnz * 4
    grad = (T.n + 1) * 4 + T.nnz * 4 + T.n * 8 * 2 + T.nnz * 8
    # setup of the forward solve and of the adjoint's transposed analysis
    return _finish(res, 2 * lb_solve + gather + grad, hop_ns, 2 * res["nlev"], setup_ms["self"],
                   setup_ms["level"], setup_ms["host"])


CONFIGS = ("c1_lap2d_64_lower", "c3_powerlaw_1M_f64", "c3_powerlaw_1M_f32",
           "c4a_batched_256_ilu0_2d", "c4b_lap3d_128_lower_16rhs", "c5_ilu0_3d_96_fwd_adjoint")


def per_config(sp, torch, steps, warmup, hop_ns, names=CONFIGS, tune=True):
    """{config name: record} for C1, C3 (FP64, FP32), C4a, C4b and C5 (or the
    subset `names`); tune=False uses FIXED_SCHEDULES instead of the tuner."""
    out = {}
    c3 = None
    for name in names:
        if name not in CONFIGS:
            raise ValueError("unknown configuration %r (one of %s)" % (name, ", ".join(CONFIGS)))
        sched = None if tune else FIXED_SCHEDULES[name]
        _log("per-config:", name)
        if name == "c1_lap2d_64_lower":
            T, _, b = W.c1_lap2d_64()
            out[name] = pc_single(sp, torch, T, b, steps, warmup, hop_ns, block=True, schedule=sched)
        elif name.startswith("c3_"):
            if c3 is None:
                c3 = W.c3_powerlaw()
            T, _, b = c3
            f32 = name.endswith("f32")
            out[name] = pc_single(sp, torch, T, b, steps, warmup, hop_ns,
                                  dtype=torch.float32 if f32 else None, tol=1e-5 if f32 else 1e-12,
                                  schedule=sched)
        elif name.startswith("c4a"):
            out[name] = pc_batched(sp, torch, steps, warmup, hop_ns, schedule=sched)
        elif name.startswith("c4b"):
            out[name] = pc_multi(sp, torch, steps, warmup, hop_ns, schedule=sched)
        else:
            out[name] = pc_adjoint(sp, torch, steps, warmup, hop_ns, schedule=sched)
    return out
