"""Sparse triangular solves on MI355X (gfx950): Python binding of libsptrsv.

The method is Li, "On Parallel Solution of Sparse Triangular Linear Systems
in CUDA" (arXiv:1710.04985): a level-set analysis (Sec. 4.1, 4.4) followed by
a level-scheduled (Sec. 4.1) or self-scheduled (Sec. 4.2) solve.  Every step
runs in the HIP library ``libsptrsv.so`` through its C ABI
(include/sptrsv.h); this module only marshals arguments.  PyTorch supplies
device memory and streams.  There is no fallback: if the library is missing
the import of the binding fails.
"""
from __future__ import annotations

import ctypes
import os
import sys
import weakref

import numpy as np
import torch

from . import _lib as L
from ._lib import SpTRSVError, check, lib

__all__ = ["Handle", "BatchedHandle", "SpTRSVFunction", "sptrsv", "SpTRSVError",
           "ALGO_AUTO", "ALGO_LEVEL", "ALGO_SELF", "SYNC_VALUE", "SYNC_FLAG"]

ALGO_AUTO, ALGO_LEVEL, ALGO_SELF, ALGO_BLOCK, ALGO_COLUMN_LEVEL, ALGO_COLUMN_SELF = 0, 1, 2, 3, 4, 5
SYNC_VALUE, SYNC_FLAG = 0, 1
OPT = {"algo": 0, "group": 1, "entries_per_lane": 2, "sync": 3, "spin_limit": 4,
       "grid": 5, "timing": 6, "wg": 7, "rows_per_lane": 8, "assign": 9, "poll": 10,
       "xp_stride": 11, "multi_rows": 12, "residency_limit": 13,
       "block_resident": 14, "cooperative": 15}
ASSIGN_STATIC, ASSIGN_TICKET, ASSIGN_XCD = 0, 1, 2
SETUP = {"host": 0, "device": 1}

_DT = {torch.float64: 0, torch.float32: 1}


def _stream(stream=None) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _need_cuda(t, name, dtype=None, dense=True):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if dense and not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def _need_vec(t, name, dtype, numel):
    """A contiguous CUDA tensor of `dtype` with exactly `numel` elements (the
    kernels read or write that many: a shorter buffer would be overrun)."""
    _need_cuda(t, name, dtype)
    if t.numel() != numel:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), numel))


class _Base:
    _h = None
    _graphs = None
    n = 0
    dtype = torch.float64
    _value_gen = 0      # bumped by every update_values (the adjoint checks it)

    def _solve(self, fn, b, out, stream):
        _need_vec(b, "b", self.dtype, self.n)
        x = torch.empty_like(b) if out is None else out
        _need_vec(x, "out", self.dtype, self.n)
        check(fn(self._h, _ptr(b), _ptr(x), _stream(stream)))
        return x

    def solve(self, b, out=None, stream=None):
        """x = T^{-1} b (forward substitution for lower, backward for upper)."""
        return self._solve(lib.sptrsv_solve, b, out, stream)

    def solve_t(self, b, out=None, stream=None):
        """x = T^{-T} b."""
        return self._solve(lib.sptrsv_solve_transpose, b, out, stream)

    def solve_multi(self, B, out=None, transpose=False, stream=None):
        """Column-major multi-RHS solve: B is (nrhs, n), column r = B[r], with
        unit stride along a column and column stride ld = B.stride(0) >= n
        (a row-slice of a wider buffer is accepted); out, if given, has the
        same strides."""
        _need_cuda(B, "B", self.dtype, dense=False)
        if B.dim() != 2 or B.shape[1] != self.n:
            raise ValueError("B must be (nrhs, n)")
        ld = B.stride(0) if B.shape[0] > 1 else self.n
        if (self.n > 1 and B.stride(1) != 1) or ld < self.n:
            raise ValueError("B must have unit stride along a column and column stride >= n")
        if out is None:
            X = torch.empty_strided(B.shape, (ld, 1), dtype=B.dtype, device=B.device)
        else:
            X = out
            _need_cuda(X, "out", self.dtype, dense=False)
            if X.shape != B.shape or (B.shape[0] > 1 and X.stride(0) != ld) or \
                    (self.n > 1 and X.stride(1) != 1):
                raise ValueError("out must have the shape and strides of B")
        check(lib.sptrsv_solve_multi(self._h, B.shape[0], max(ld, 1), _ptr(B), _ptr(X),
                                     int(transpose), _stream(stream)))
        return X

    def prepare_transpose(self, stream=None):
        check(lib.sptrsv_prepare_transpose(self._h, _stream(stream)))

    def set_option(self, key, value):
        check(lib.sptrsv_set_option(self._h, OPT[key], int(value)))
        return self

    def get_option(self, key):
        v = ctypes.c_int64()
        check(lib.sptrsv_get_option(self._h, OPT[key], ctypes.byref(v)))
        return v.value

    def configure(self, **kw):
        for k, v in kw.items():
            self.set_option(k, v)
        return self

    def tune(self, b, x=None, stream=None):
        """Times the candidate schedules on b (x is scratch output, not b)."""
        _need_vec(b, "b", self.dtype, self.n)
        x = torch.empty_like(b) if x is None else x
        _need_vec(x, "x", self.dtype, self.n)
        check(lib.sptrsv_tune(self._h, _ptr(b), _ptr(x), _stream(stream)))
        return self.info()

    def tune_multi(self, B, X=None, stream=None):
        """Tunes the schedule of solve_multi for B's number of columns (B is
        (nrhs, n), the column-major n x nrhs matrix); X is scratch output."""
        _need_cuda(B, "B", self.dtype)
        if B.dim() != 2 or B.shape[1] != self.n or B.shape[0] < 2:
            raise ValueError("B must be (nrhs >= 2, n)")
        X = torch.empty_like(B) if X is None else X
        _need_vec(X, "X", self.dtype, B.numel())
        check(lib.sptrsv_tune_multi(self._h, B.shape[0], self.n, _ptr(B), _ptr(X), _stream(stream)))

    def info(self):
        n, nlev, algo, group = (ctypes.c_int32() for _ in range(4))
        nnz = ctypes.c_int64()
        check(lib.sptrsv_get_info(self._h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(nlev),
                                  ctypes.byref(algo), ctypes.byref(group)))
        epl, sync, rpl, grid, assign, poll = (ctypes.c_int32() for _ in range(6))
        check(lib.sptrsv_get_schedule(self._h, None, None, ctypes.byref(epl), ctypes.byref(sync),
                                      ctypes.byref(rpl), ctypes.byref(grid), ctypes.byref(assign),
                                      ctypes.byref(poll)))
        stride = ctypes.c_int32()
        check(lib.sptrsv_get_xp_stride(self._h, ctypes.byref(stride)))
        return {"n": n.value, "nnz": nnz.value, "nlev": nlev.value, "algo": algo.value,
                "group": group.value, "entries_per_lane": epl.value, "sync": sync.value,
                "rows_per_lane": rpl.value, "grid": grid.value, "assign": assign.value,
                "poll": poll.value, "xp_stride": stride.value}

    def export_analysis(self, transpose=False):
        """(level, ilev, jlev, depcnt) as numpy int32 arrays (host copies)."""
        level = np.zeros(self.n, np.int32)
        jlev = np.zeros(self.n, np.int32)
        depcnt = np.zeros(self.n, np.int32)
        ilev_cap = np.zeros(self.n + 1, np.int32)
        p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        check(lib.sptrsv_export_analysis(self._h, int(transpose), p(level), p(ilev_cap), p(jlev),
                                         p(depcnt)))
        nlev = int(level.max()) + 1 if self.n else 0
        return level, ilev_cap[:nlev + 1].copy(), jlev, depcnt

    def status(self):
        """Device-side status of the last solves (synchronises); raises on error."""
        check(lib.sptrsv_get_status(self._h))

    def kernel_time(self, reset=True):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        check(lib.sptrsv_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(cnt), int(reset)))
        return ms.value, cnt.value

    def capture(self, b, x, transpose=False, stream=None):
        """HIP graph of one solve on fixed b/x (stream must not be the default)."""
        _need_vec(b, "b", self.dtype, self.n)
        _need_vec(x, "x", self.dtype, self.n)
        s = torch.cuda.current_stream() if stream is None else stream
        g = ctypes.c_void_p()
        check(lib.sptrsv_graph_capture(self._h, _ptr(b), _ptr(x), int(transpose),
                                       ctypes.c_void_p(s.cuda_stream), ctypes.byref(g)))
        graph = Graph(g, self, b, x)
        if self._graphs is None:
            self._graphs = weakref.WeakSet()
        self._graphs.add(graph)
        return graph

    def close(self):
        """Destroys the handle (and first every graph captured from it)."""
        if self._h:
            for g in list(self._graphs or ()):
                g.close()
            check(lib.sptrsv_destroy(self._h))
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # no HIP calls while the interpreter shuts down (the runtime, or a
        # profiler wrapped around it, may already be tearing down; module
        # globals such as `sys` may already be gone)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A captured solve.  Holds its handle and its b/x tensors, so neither
    can be freed (or their memory reused) while the graph can be launched."""

    def __init__(self, g, owner, b, x):
        self._g = g
        self._keep = (owner, b, x)

    def launch(self, stream=None):
        if not self._g:
            raise RuntimeError("graph is closed")
        check(lib.sptrsv_graph_launch(self._g, _stream(stream)))

    def close(self):
        if self._g:
            lib.sptrsv_graph_destroy(self._g)
            self._g = None
            self._keep = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def probe_hop(same_xcd=False, iters=2000):
    """Nanoseconds for one value to travel from a publishing wavefront to a
    polling one on another CU (same XCD or the next one)."""
    ns = ctypes.c_double()
    check(lib.sptrsv_probe_hop(int(bool(same_xcd)), int(iters), ctypes.byref(ns)))
    return ns.value


class Handle(_Base):
    """Analysis of one CSR triangle (diagonal stored inside the rows).

    row_ptr, col_idx: int32 CUDA tensors; vals: float64/float32 CUDA tensor.
    The handle keeps references to the three tensors (their device memory is
    read by analysis, update_values and grad_vals)."""

    def __init__(self, row_ptr, col_idx, vals, uplo="L", unit_diag=False, stream=None,
                 setup="host"):
        _need_cuda(row_ptr, "row_ptr", torch.int32)
        _need_cuda(col_idx, "col_idx", torch.int32)
        _need_cuda(vals, "vals")
        if vals.dtype not in _DT:
            raise TypeError("vals must be float64 or float32")
        if setup not in SETUP:
            raise ValueError("setup must be one of %s" % sorted(SETUP))
        if vals.numel() != col_idx.numel():
            raise ValueError("vals has %d entries, col_idx %d" % (vals.numel(), col_idx.numel()))
        self.n = row_ptr.numel() - 1
        self.nnz = col_idx.numel()
        self.dtype = vals.dtype
        self.upper = uplo.upper() == "U"
        self.unit_diag = bool(unit_diag)
        self.row_ptr, self.col_idx, self.vals = row_ptr, col_idx, vals
        h = ctypes.c_void_p()
        check(lib.sptrsv_analyze_ex(self.n, self.nnz, _ptr(row_ptr), _ptr(col_idx), _ptr(vals),
                                    _DT[vals.dtype], int(self.upper), int(self.unit_diag),
                                    SETUP[setup], _stream(stream), ctypes.byref(h)))
        self._h = h

    def setup_info(self):
        """(route, milliseconds): where the analysis ran ('host' or 'device',
        the device route hands invalid or unsorted patterns to the host one)
        and its wall time."""
        route = ctypes.c_int32()
        ms = ctypes.c_double()
        check(lib.sptrsv_get_setup(self._h, ctypes.byref(route), ctypes.byref(ms)))
        return {v: k for k, v in SETUP.items()}[route.value], ms.value

    def update_values(self, vals, stream=None):
        _need_vec(vals, "vals", self.dtype, self.nnz)
        check(lib.sptrsv_update_values(self._h, _ptr(vals), _stream(stream)))
        self.vals = vals
        self._value_gen += 1

    def grad_vals(self, grad_b, x, out=None, stream=None):
        """-grad_b[i] * x[j] for each stored entry (i, j), in CSR entry order."""
        _need_vec(grad_b, "grad_b", self.dtype, self.n)
        _need_vec(x, "x", self.dtype, self.n)
        gv = torch.empty(self.nnz, dtype=self.dtype, device=grad_b.device) if out is None else out
        _need_vec(gv, "out", self.dtype, self.nnz)
        check(lib.sptrsv_grad_vals(self._h, _ptr(self.row_ptr), _ptr(self.col_idx), _ptr(grad_b),
                                   _ptr(x), _ptr(gv), _stream(stream)))
        return gv


class BatchedHandle(_Base):
    """Independent triangles solved as one block-diagonal system; b and x are
    the concatenations of the systems' vectors."""

    def __init__(self, row_ptrs, col_idxs, valss, uplo="L", unit_diag=False, stream=None,
                 setup="host"):
        if setup not in SETUP:
            raise ValueError("setup must be one of %s" % sorted(SETUP))
        count = len(row_ptrs)
        if not (count == len(col_idxs) == len(valss)) or count == 0:
            raise ValueError("need the same positive number of row_ptrs, col_idxs, vals")
        dt = valss[0].dtype
        if dt not in _DT:
            raise TypeError("vals must be float64 or float32")
        for i in range(count):
            _need_cuda(row_ptrs[i], "row_ptr", torch.int32)
            _need_cuda(col_idxs[i], "col_idx", torch.int32)
            _need_vec(valss[i], "vals", dt, col_idxs[i].numel())
        self.count = count
        self.sizes = [r.numel() - 1 for r in row_ptrs]
        self.nnzs = [c.numel() for c in col_idxs]
        self.n = sum(self.sizes)
        self.nnz = sum(self.nnzs)
        self.dtype = dt
        self.unit_diag = bool(unit_diag)
        self._keep = (list(row_ptrs), list(col_idxs), list(valss))
        I32 = ctypes.c_int32 * count
        P = ctypes.c_void_p * count
        h = ctypes.c_void_p()
        arr = lambda ts: ctypes.cast(P(*[t.data_ptr() for t in ts]), ctypes.c_void_p)
        check(lib.sptrsv_analyze_batched_ex(
            count, I32(*self.sizes), I32(*self.nnzs), arr(row_ptrs), arr(col_idxs), arr(valss),
            _DT[dt], int(uplo.upper() == "U"), int(unit_diag), SETUP[setup], _stream(stream),
            ctypes.byref(h)))
        self._h = h

    def setup_info(self):
        """(route, milliseconds) of the analysis, as for Handle."""
        route = ctypes.c_int32()
        ms = ctypes.c_double()
        check(lib.sptrsv_get_setup(self._h, ctypes.byref(route), ctypes.byref(ms)))
        return {v: k for k, v in SETUP.items()}[route.value], ms.value

    def update_values(self, valss, stream=None):
        if len(valss) != self.count:
            raise ValueError("need %d value tensors, got %d" % (self.count, len(valss)))
        for v, nz in zip(valss, self.nnzs):
            _need_vec(v, "vals", self.dtype, nz)
        P = ctypes.c_void_p * self.count
        ptrs = P(*[v.data_ptr() for v in valss])
        check(lib.sptrsv_update_values_batched(self._h, ctypes.cast(ptrs, ctypes.c_void_p),
                                               _stream(stream)))
        self._keep = (self._keep[0], self._keep[1], list(valss))
        self._value_gen += 1

    def grad_vals(self, grad_b, x, out=None, stream=None):
        _need_vec(grad_b, "grad_b", self.dtype, self.n)
        _need_vec(x, "x", self.dtype, self.n)
        gv = torch.empty(self.nnz, dtype=self.dtype, device=grad_b.device) if out is None else out
        _need_vec(gv, "out", self.dtype, self.nnz)
        check(lib.sptrsv_grad_vals(self._h, None, None, _ptr(grad_b), _ptr(x), _ptr(gv),
                                   _stream(stream)))
        return gv


class SpTRSVFunction(torch.autograd.Function):
    """x = T^{-1} b with T = (pattern of `handle`, values `vals`).

    Forward gathers `vals` into the handle (one streaming kernel) unless
    `values_current` says the handle already holds exactly these values --
    tensor identity or version counters cannot tell (in-place writes through
    .data do not bump the version).
    Backward (the adjoint): grad_b = T^{-T} grad_x by the transposed solve,
    grad_vals[k] = -grad_b[i] * x[j] for each stored entry k = (i, j).  If
    the handle was given other values between this forward and its backward
    (another forward on the same handle), backward gathers this forward's
    values again first, so the transposed solve uses the matrix that
    produced x."""

    @staticmethod
    def forward(ctx, vals, b, handle, values_current=False):
        if not values_current:
            handle.update_values(vals.detach().contiguous())
        x = handle.solve(b.contiguous())
        ctx.handle = handle
        ctx.value_gen = handle._value_gen
        ctx.save_for_backward(x, vals)
        return x

    @staticmethod
    def backward(ctx, gx):
        x, vals = ctx.saved_tensors
        h = ctx.handle
        if h._value_gen != ctx.value_gen:
            h.update_values(vals.detach().contiguous())
        gb = h.solve_t(gx.contiguous())
        gv = h.grad_vals(gb, x) if ctx.needs_input_grad[0] else None
        return gv, (gb if ctx.needs_input_grad[1] else None), None, None


def sptrsv(vals, b, handle, values_current=False):
    """Differentiable x = T^{-1} b (see SpTRSVFunction)."""
    return SpTRSVFunction.apply(vals, b, handle, values_current)


def analyze_host(row_ptr, col_idx, upper=False, unit_diag=False):
    """Host-only analysis (no GPU): validation status, level, ilev, jlev, depcnt."""
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col_idx, np.int32)
    n = rp.size - 1
    level = np.zeros(n, np.int32)
    jlev = np.zeros(n, np.int32)
    dep = np.zeros(n, np.int32)
    ilev = np.zeros(n + 1, np.int32)
    nlev = ctypes.c_int32(0)
    p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    st = lib.sptrsv_analyze_host(n, ci.size, p(rp), p(ci), int(upper), int(unit_diag), p(level),
                                 p(ilev), p(jlev), p(dep), ctypes.byref(nlev))
    return st, level, ilev[:nlev.value + 1].copy(), jlev, dep
