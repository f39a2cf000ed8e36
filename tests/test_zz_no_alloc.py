"""The no-allocation propagation entry point against gcr_propagate, through
the C ABI: bitwise-equal rounds on two calls in a row, the second with a
smaller graph (the shared per-GPU scratch keeps the first call's contents),
with and without cameras, and the size limit refused on the host."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2306_08792_amd import _lib as L
from paper_2306_08792_amd import datagen
from paper_2306_08792_amd.gcr import BF16, Context, GcrError, Params

pytestmark = pytest.mark.gpu


def _round_pair(ctx, X, p, cam=None):
    Xd = torch.from_numpy(X).cuda()
    camd = torch.from_numpy(cam).cuda() if cam is not None else None
    Xn = ctx.normalize_rows(Xd)
    g = ctx.build_graph(Xn, p, camd)
    ref = ctx.propagate(g, Xn)
    out = torch.full_like(Xn, float("nan"))
    ctx.propagate_noalloc(g, Xn, out)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_noalloc_propagate_matches_propagate():
    print("no-alloc propagate", flush=True)
    ctx = Context(0)
    try:
        # first call: 9,000 nodes with cameras (two graphs blended)
        X1, _ = datagen.clustered(300, 30, 96, 0.5, seed=61)
        cam = (np.arange(X1.shape[0]) % 5).astype(np.int32)
        p1 = Params(k=12, gamma=0.2, rounds=1, alpha=0.6, precision=BF16)
        a, b = _round_pair(ctx, X1, p1, cam)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        # second call, smaller: 1,000 nodes, one graph, another width
        X2, _ = datagen.clustered(50, 20, 256, 0.5, seed=62)
        p2 = Params(k=20, gamma=0.2, rounds=1, precision=BF16)
        a, b = _round_pair(ctx, X2, p2)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        # and the larger one again after the smaller
        a, b = _round_pair(ctx, X1, p1, cam)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    finally:
        ctx.close()


def test_noalloc_size_limit_is_refused_on_the_host():
    print("no-alloc size limit", flush=True)
    ctx = Context(0)
    try:
        lib = L.load()
        nmax = int(lib.gcr_propagate_noalloc_max_nodes())
        assert nmax > 1_000_000
        # a graph descriptor of nmax + 1 nodes: refused before any launch
        g = L.GcrGraph()
        n = nmax + 1
        g.n, g.k = n, 4
        fake = C.c_void_p(256)
        g.idx = g.self_ = fake
        st = lib.gcr_propagate_noalloc(ctx.h, C.byref(g), fake, C.c_void_p(512), n, 64, None)
        assert st == -4, st
        assert "scratch" in lib.gcr_last_error(ctx.h).decode()
    finally:
        ctx.close()
