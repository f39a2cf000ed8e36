"""Parity of the 256-row similarity tiles with the FP64 oracle.

Sweeps of one list over many row blocks in float32 or BF16 run 256 x 256
workgroup tiles (waves of 128 x 128, 64-byte chunks, candidate buffers
that keep room for a whole tile instead of re-screening lost entries).
The sizes here (22,300 rows) are the smallest that select them on a
256-unit GPU; the rows checked include the first and the ragged last row
blocks."""
import numpy as np
import pytest
import torch

from oracle import gcr_oracle as O
from paper_2306_08792_amd import datagen
from paper_2306_08792_amd.gcr import BF16, FP32, Context, Params

from parity import chain_compare, check_knn_rows

pytestmark = pytest.mark.gpu

N = 22300  # 88 row blocks of 256, the last one 28 rows short


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def full_chip():
    return torch.cuda.get_device_properties(0).multi_processor_count == 256


def rows_to_check(n, m, seed):
    rng = np.random.default_rng(seed)
    edge = np.concatenate([np.arange(0, 256), np.arange(n - 300, n)])
    return np.union1d(edge, rng.choice(n, size=m, replace=False))


def corpus(seed):
    w = datagen.large_retrieval(seed=seed, nq=2000, ng=N - 2000, d=64, n_ids=500, sigma=0.6)
    return w, O.row_normalize(w.X).astype(np.float32)


@pytest.mark.parametrize("prec", [FP32, BF16])
def test_knn_256_row_tiles(ctx, prec):
    print(f"256-row tiles knn prec={prec}", flush=True)
    _, X = corpus(21)
    ctx.reset_stats()
    idx, dist = ctx.knn(dev(X), Params(k=20, precision=prec))
    st = ctx.stats()
    if full_chip():
        assert st["tile_rows"] == 256, st
    rows = rows_to_check(N, 1500, 1)
    check_knn_rows(host(idx)[rows], host(dist)[rows], X, rows, 20)


def test_knn_256_row_tiles_duplicate_groups(ctx):
    """Groups of 300 identical rows: every row has 299 items at distance 0,
    more than the 256 a buffer keeps after a compaction, so the kernel cuts
    its buffers and the exact step finishes the lists (ties by index)."""
    print("256-row tiles with duplicate groups", flush=True)
    base = datagen.random_unit(75, 64, 5)
    perm = np.random.default_rng(6).permutation(75 * 300)[:N]
    X = np.repeat(base, 300, axis=0)[perm]
    ctx.reset_stats()
    idx, dist = ctx.knn(dev(X), Params(k=20, precision=BF16))
    st = ctx.stats()
    if full_chip():
        assert st["tile_rows"] == 256, st
    rows = rows_to_check(N, 600, 2)
    gi, gd = host(idx), host(dist)
    check_knn_rows(gi[rows], gd[rows], X, rows, 20)
    # exact ties resolve by index: the 20 smallest indices of the row's group
    for r in rows[:200]:
        mates = np.nonzero(perm // 300 == perm[r] // 300)[0]
        mates = mates[mates != r][:20]
        assert np.array_equal(gi[r], mates), (r, gi[r][:5], mates[:5])


def test_rerank_256_row_tiles_chain(ctx):
    """Two rebuilt rounds (the second sweep seeded by the first round's
    lists) on every row against the oracle chain."""
    print("256-row tiles rerank chain", flush=True)
    w, _ = corpus(22)
    p = Params(k=20, gamma=0.2, rounds=2, precision=BF16, rebuild_each_round=True)
    op = O.Params(k=20, gamma=0.2, rounds=2, alpha=1.0)
    ctx.reset_stats()
    chain_compare(ctx, w, p, op, None, "256-row tiles", dense_last=False)
    st = ctx.stats()
    if full_chip():
        assert st["tile_rows"] == 256, st
