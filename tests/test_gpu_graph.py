"""Capture of a whole re-ranking into a HIP graph (torch.cuda.CUDAGraph over
the library's stream argument): once the workspace has its size, a call
enqueues only kernels and device copies, so the captured graph replays the
same results.  Replays are interleaved with eager calls and synchronisations
and every replay is compared bitwise with the eager result."""
import numpy as np
import pytest
import torch

from paper_2306_08792_amd import datagen
from paper_2306_08792_amd.gcr import BF16, Context, Params

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("local", [False, True])
def test_rerank_replays_from_a_graph(local):
    print(f"graph capture local={local}", flush=True)
    ctx = Context(0)
    try:
        X, ids = datagen.clustered(60, 20, 128, 0.5, seed=51)
        nq = 200
        cams = (np.arange(X.shape[0]) % 3).astype(np.int32)
        Xd = torch.from_numpy(X).cuda()
        camd = torch.from_numpy(cams).cuda()
        p = Params(k=10, gamma=0.2, rounds=2, alpha=0.7, precision=BF16, topk_out=20)

        def run(out):
            if local:
                return ctx.rerank_local(Xd, nq, p, dense=True, topk=True, keep_features=True, out=out)
            return ctx.rerank(Xd, nq, p, camd, dense=True, topk=True, keep_features=True, out=out)

        eager = run({})
        torch.cuda.synchronize()
        ref = {k: v.clone() for k, v in eager.items()}
        out = {k: torch.empty_like(v) for k, v in ref.items()}
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            run(out)  # warm-up on the capture stream: the workspace keeps its size
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            run(out)
        for rep in range(4):
            for v in out.values():
                v.zero_()
            g.replay()
            torch.cuda.synchronize()
            for name, v in ref.items():
                a, b = out[name].cpu().numpy(), v.cpu().numpy()
                assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (rep, name)
            run({})  # eager work between the replays
            torch.cuda.synchronize()
    finally:
        ctx.close()
