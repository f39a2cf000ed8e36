"""Capture of a whole re-ranking into a HIP graph (torch.cuda.CUDAGraph over
the library's stream argument).  The context is created with the workspace
gcr_workspace_size reports and never grows it, so the very first call on it
is the captured one: a batch call enqueues only kernels and device copies
(no allocation, no memset node, no host synchronisation).  Replays are
interleaved with eager calls and synchronisations and every replay is
compared bitwise with the eager result of an independent context."""
import numpy as np
import pytest
import torch

from paper_2306_08792_amd import datagen
from paper_2306_08792_amd.gcr import BF16, Context, GcrError, Params

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("local", [False, True])
def test_rerank_captured_on_first_call(local):
    print(f"graph capture local={local}", flush=True)
    X, ids = datagen.clustered(60, 20, 128, 0.5, seed=51)
    nq = 200
    n, d = X.shape
    cams = (np.arange(n) % 3).astype(np.int32)
    Xd = torch.from_numpy(X).cuda()
    camd = torch.from_numpy(cams).cuda()
    p = Params(k=10, gamma=0.2, rounds=2, alpha=0.7, precision=BF16, topk_out=20)

    def run(c, out):
        if local:
            return c.rerank_local(Xd, nq, p, dense=True, topk=True, keep_features=True, out=out)
        return c.rerank(Xd, nq, p, camd, dense=True, topk=True, keep_features=True, out=out)

    ref_ctx = Context(0)
    ws = Context.workspace_size(p, nq, n - nq, d, with_cameras=True)
    assert ws > 0
    ctx = Context(0, workspace_bytes=ws, auto_reserve=False)
    try:
        eager = run(ref_ctx, {})
        torch.cuda.synchronize()
        ref = {k: v.clone() for k, v in eager.items()}
        out = {k: torch.empty_like(v) for k, v in ref.items()}
        torch.cuda.synchronize()
        held = ctx.workspace_bytes()
        assert held >= ws
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            run(ctx, out)  # the context's first call
        assert ctx.workspace_bytes() == held
        for rep in range(4):
            for v in out.values():
                v.zero_()
            g.replay()
            torch.cuda.synchronize()
            for name, v in ref.items():
                a, b = out[name].cpu().numpy(), v.cpu().numpy()
                assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (rep, name)
            run(ctx, {})  # eager work on the same context between the replays
            torch.cuda.synchronize()
    finally:
        ctx.close()
        ref_ctx.close()


def test_short_workspace_is_nomem_and_allocates_nothing():
    print("short workspace", flush=True)
    X = datagen.random_unit(300, 64, 3)
    p = Params(k=8, rounds=1, precision=BF16, topk_out=10)
    ws = Context.workspace_size(p, 100, 200, 64)
    ctx = Context(0, workspace_bytes=ws // 2, auto_reserve=False)
    try:
        before = ctx.workspace_bytes()
        with pytest.raises(GcrError, match="NOMEM"):
            ctx.rerank(torch.from_numpy(X).cuda(), 100, p, dense=True)
        assert ctx.workspace_bytes() == before
        ctx.reserve(ws)
        out = ctx.rerank(torch.from_numpy(X).cuda(), 100, p, dense=True, topk=True)
        torch.cuda.synchronize()
        assert out["dist"].shape == (100, 200)
    finally:
        ctx.close()
