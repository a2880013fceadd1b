"""Lifetimes around captured graphs: a graph keeps the position-ordered
buffer it was captured with when later calls replace the handle's (several
right-hand sides, the autotuner's wider slots), keeps its handle and b/x
tensors alive, and the handle refuses destruction while graphs live."""
import ctypes
import gc

import numpy as np
import pytest
import torch

import workloads as W
from gpuhelp import bits_equal, dev, dev_tri, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import paper_1710_04985_amd as sp
    assert torch.cuda.is_available()
    return sp


def test_graph_survives_buffer_growth(sp):
    T = W.laplacian_triangle((24, 22, 20))
    h = sp.Handle(*dev_tri(T)).configure(algo=sp.ALGO_SELF)
    s = torch.cuda.Stream()
    b = dev(W.uniform_vector(T.n, 31))
    x = torch.empty_like(b)
    with torch.cuda.stream(s):
        ref = h.solve(b)
        g = h.capture(b, x, stream=s)
        B = dev(np.stack([W.uniform_vector(T.n, 40 + r) for r in range(16)]))
        h.solve_multi(B)                 # grows the handle's buffer to 16 values a row
        h.set_option("xp_stride", 8)     # 64-byte slots: grows it again
        h.solve(b)
        h.tune(b)
        s.synchronize()
        for rep in range(3):
            x.zero_()
            g.launch(s)
            s.synchronize()
            assert bits_equal(x, ref), rep
            h.solve_multi(B)             # eager work between replays
            s.synchronize()
    h.status()
    g.close()
    h.close()


def test_destroy_refused_while_graph_lives(sp):
    T = W.laplacian_triangle((12, 12, 12))
    h = sp.Handle(*dev_tri(T))
    s = torch.cuda.Stream()
    b = dev(W.uniform_vector(T.n, 32))
    x = torch.empty_like(b)
    with torch.cuda.stream(s):
        g = h.capture(b, x, stream=s)
    assert sp.lib.sptrsv_destroy(h._h) == -12          # SPTRSV_ERR_BUSY
    with torch.cuda.stream(s):
        g.launch(s)
    s.synchronize()
    h.status()
    h.close()                                         # closes the graph first
    assert g._g is None and h._h is None


def test_graph_keeps_handle_and_vectors(sp):
    T = W.laplacian_triangle((16, 15, 14))
    b_np = W.uniform_vector(T.n, 33)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        h = sp.Handle(*dev_tri(T))
        ref = h.solve(dev(b_np))
        g = h.capture(dev(b_np), torch.empty(T.n, dtype=torch.float64, device="cuda:0"), stream=s)
        del h
        gc.collect()
        junk = [torch.full((T.n,), 7.0, dtype=torch.float64, device="cuda:0") for _ in range(4)]
        g.launch(s)
        s.synchronize()
    assert bits_equal(g._keep[2], ref)
    g.close()
