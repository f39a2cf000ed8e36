"""Python binding of the GCR / GCRV library (argument marshalling only).

Every function takes torch tensors that live on the GPU, checks dtype,
device and contiguity, and calls the C ABI of libgcr.so on the current
torch stream.  All computation happens in the library's HIP kernels; there
is no CPU path.

Operations (Graph Convolution Based Efficient Re-Ranking, Sec. III):
  knn               neighbour lists of Eq. (4) / Eq. (8)
  build_graph       sparse symmetric graph of Eq. (4)-(9)
  propagate         one round of Eq. (2) / (9) with row re-normalisation
  final_distances   distances between updated query and gallery features
  rerank            the whole method (Eq. (3) rounds, graph rebuilt per round)
  profile_vectors   tracklet profiles, Eq. (10) / Eq. (16)
  gcrv              Alg. 2: profiles, then rerank on them
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Optional

import torch

from . import _lib as L

FP32, BF16, FP8, BF16_RAW, FP8_RAW = 0, 1, 2, 3, 4
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp8": FP8, "bf16_raw": BF16_RAW, "fp8_raw": FP8_RAW}


@dataclasses.dataclass
class Params:
    """Mirror of gcr_params.  Paper defaults: gamma 0.2, k 15, T 3,
    lambda 10 (Sec. IV-B); alpha 1 unless cameras are used."""

    k: int = 15
    cross_k: int = -1
    rounds: int = 3
    rebuild_each_round: bool = True
    normalize_input: bool = True
    precision: int = FP32
    topk_out: int = 100
    gamma: float = 0.2
    alpha: float = 1.0
    beta_same: float = 1.0
    beta_cross: float = 1.0
    lam: float = 10.0
    symmetric: bool = True

    def c(self) -> L.GcrParams:
        p = L.GcrParams()
        p.k, p.cross_k, p.rounds = self.k, self.cross_k, self.rounds
        p.rebuild_each_round = int(self.rebuild_each_round)
        p.normalize_input = int(self.normalize_input)
        p.precision = int(self.precision)
        p.topk_out = self.topk_out
        p.symmetric = int(self.symmetric)
        p.gamma, p.alpha = self.gamma, self.alpha
        p.beta_same, p.beta_cross, p.lambda_ = self.beta_same, self.beta_cross, self.lam
        return p


class GcrError(RuntimeError):
    pass


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(t: torch.Tensor, dtype, name: str, device: torch.device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Graph:
    """A propagation graph held in one device buffer (gcr_graph)."""

    def __init__(self, n: int, k: int, cross_k: int, has_cross: bool, device):
        lib = L.load()
        nbytes = lib.gcr_graph_bytes(n, k, cross_k, int(has_cross))
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = (self.buf.data_ptr() + 255) // 256 * 256
        self.g = L.GcrGraph()
        st = lib.gcr_graph_bind(C.byref(self.g), C.c_void_p(base), n, k, cross_k, int(has_cross))
        if st != L.GCR_OK:
            raise GcrError(f"gcr_graph_bind failed ({st})")
        self.n, self.k, self.has_cross = n, k, has_cross
        self.cross_k = self.g.cross_k
        self.device = device

    def _view(self, ptr, shape, dtype):
        n = 1
        for s in shape:
            n *= s
        esz = torch.empty((), dtype=dtype).element_size()
        off = ptr - self.buf.data_ptr()
        return self.buf[off: off + n * esz].view(dtype).view(*shape)

    def field(self, name: str) -> torch.Tensor:
        """Tensor view of one field (see gcr_graph in include/gcr.h)."""
        g = self.g
        n, k, ck = self.n, self.k, self.cross_k
        ptr = getattr(g, name if name != "self" else "self_")
        if ptr is None:
            raise KeyError(name)
        shapes = {
            "idx": ((n, k), torch.int32), "dist": ((n, k), torch.float32), "w": ((n, k), torch.float32),
            "pf": ((n, k), torch.float32), "rev_ptr": ((n + 1,), torch.int32),
            "rev_src": ((n * k,), torch.int32), "rev_w": ((n * k,), torch.float32),
            "pr": ((n * k,), torch.float32), "deg": ((n,), torch.float32), "self": ((n,), torch.float32),
            "cr_idx": ((n, ck), torch.int32), "cr_dist": ((n, ck), torch.float32),
            "cr_w": ((n, ck), torch.float32), "cr_pf": ((n, ck), torch.float32),
            "cr_rev_ptr": ((n + 1,), torch.int32), "cr_rev_src": ((n * ck,), torch.int32),
            "cr_rev_w": ((n * ck,), torch.float32), "cr_pr": ((n * ck,), torch.float32),
            "cr_deg": ((n,), torch.float32),
        }
        shape, dt = shapes[name]
        return self._view(ptr, shape, dt)


class Context:
    """A library context bound to one GPU (gcr_ctx).

    workspace_bytes: the context's workspace at creation (see
    workspace_size()).  auto_reserve: before each call, grow the workspace
    to what gcr_workspace_size reports for the call's sizes (gcr_reserve,
    which synchronises the device); with False a call that needs more fails
    with NOMEM, and nothing allocates after creation (capture-safe use)."""

    def __init__(self, device: int = 0, workspace_bytes: int = 0, auto_reserve: bool = True):
        if not torch.cuda.is_available():
            raise GcrError("no GPU visible: the GCR library has no CPU path")
        self.lib = L.load()
        self.device = torch.device("cuda", device)
        self.auto_reserve = auto_reserve
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            st = self.lib.gcr_create(C.byref(h), device, int(workspace_bytes))
        if st != L.GCR_OK:
            raise GcrError(f"gcr_create failed ({L.STATUS_NAMES.get(st, st)})")
        self.h = h

    @staticmethod
    def workspace_size(p: "Params", nq: int, ng: int, d: int, with_cameras: bool = False) -> int:
        """Workspace bytes every batch call needs at these sizes (0: unsupported)."""
        lib = L.load()
        pc = p.c()
        return int(lib.gcr_workspace_size(C.byref(pc), nq, ng, d, int(with_cameras)))

    def workspace_bytes(self) -> int:
        return int(self.lib.gcr_workspace_bytes(self.h))

    def reserve(self, nbytes: int):
        self._ok(self.lib.gcr_reserve(self.h, int(nbytes)), "gcr_reserve")

    def _need(self, p: "Params", nq: int, ng: int, d: int, with_cameras: bool = False):
        if not self.auto_reserve:
            return
        nb = self.workspace_size(p, nq, ng, d, with_cameras)
        if nb > self.workspace_bytes():
            self.reserve(nb)

    def close(self):
        if getattr(self, "h", None):
            self.lib.gcr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ok(self, st: int, what: str):
        if st != L.GCR_OK:
            msg = self.lib.gcr_last_error(self.h).decode()
            raise GcrError(f"{what}: {L.STATUS_NAMES.get(st, st)}: {msg}")

    # -- statistics
    def stats(self) -> dict:
        s = L.GcrStats()
        self._ok(self.lib.gcr_get_stats(self.h, C.byref(s)), "gcr_get_stats")
        return dict(knn_rows=s.knn_rows, knn_candidates=s.knn_candidates,
                    knn_fallback_rows=s.knn_fallback_rows, splits=s.splits,
                    knn_exhaustive_rows=s.knn_exhaustive_rows, tile_rows=s.tile_rows)

    def set_timing(self, on: bool):
        self._ok(self.lib.gcr_set_timing(self.h, int(on)), "gcr_set_timing")

    def timing(self) -> dict:
        """{class: (total ms, launches)} since the last call (synchronises)."""
        t = L.GcrTiming()
        self._ok(self.lib.gcr_get_timing(self.h, C.byref(t)), "gcr_get_timing")
        return {L.TIMER_NAMES[i]: (t.ms[i], t.launches[i]) for i in range(L.NUM_TIMERS)}

    def reset_stats(self):
        self._ok(self.lib.gcr_reset_stats(self.h), "gcr_reset_stats")

    # -- operations
    def normalize_rows(self, X: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        _check(X, torch.float32, "X", self.device)
        Y = torch.empty_like(X) if out is None else out
        self._ok(self.lib.gcr_normalize_rows(self.h, _ptr(X), _ptr(Y), X.shape[0], X.shape[1], _stream()),
                 "gcr_normalize_rows")
        return Y

    def knn(self, X: torch.Tensor, p: Params, cam: Optional[torch.Tensor] = None, cross: bool = False):
        _check(X, torch.float32, "X", self.device)
        n, d = X.shape
        idx = torch.empty((n, p.k), dtype=torch.int32, device=self.device)
        dist = torch.empty((n, p.k), dtype=torch.float32, device=self.device)
        cidx = cdist = None
        if cross:
            if cam is None:
                raise ValueError("cross list needs camera labels")
            ck = p.k if p.cross_k < 0 else p.cross_k
            cidx = torch.empty((n, ck), dtype=torch.int32, device=self.device)
            cdist = torch.empty((n, ck), dtype=torch.float32, device=self.device)
        if cam is not None:
            _check(cam, torch.int32, "cam", self.device)
        self._need(p, 0, n, d, cross)
        pc = p.c()
        self._ok(self.lib.gcr_knn(self.h, _ptr(X), n, d, _ptr(cam), C.byref(pc), _ptr(idx), _ptr(dist),
                                  _ptr(cidx), _ptr(cdist), _stream()), "gcr_knn")
        return (idx, dist, cidx, cdist) if cross else (idx, dist)

    def build_graph(self, X: torch.Tensor, p: Params, cam: Optional[torch.Tensor] = None) -> Graph:
        _check(X, torch.float32, "X", self.device)
        n, d = X.shape
        has_cross = cam is not None and p.alpha < 1.0
        if cam is not None:
            _check(cam, torch.int32, "cam", self.device)
        g = Graph(n, p.k, p.cross_k, has_cross, self.device)
        self._need(p, 0, n, d, has_cross)
        pc = p.c()
        self._ok(self.lib.gcr_build_graph(self.h, _ptr(X), n, d, _ptr(cam), C.byref(pc), C.byref(g.g),
                                          _stream()), "gcr_build_graph")
        return g

    def propagate(self, g: Graph, X: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        _check(X, torch.float32, "X", self.device)
        Y = torch.empty_like(X) if out is None else out
        self._need(Params(k=0), 0, X.shape[0], X.shape[1])
        self._ok(self.lib.gcr_propagate(self.h, C.byref(g.g), _ptr(X), _ptr(Y), X.shape[0], X.shape[1],
                                        _stream()), "gcr_propagate")
        return Y

    def propagate_noalloc(self, g: Graph, X: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """gcr_propagate_noalloc: one round with the library's fixed per-GPU
        scratch (no workspace, no allocation); `out` must be preallocated."""
        _check(X, torch.float32, "X", self.device)
        _check(out, torch.float32, "out", self.device)
        self._ok(self.lib.gcr_propagate_noalloc(self.h, C.byref(g.g), _ptr(X), _ptr(out), X.shape[0], X.shape[1],
                                                _stream()), "gcr_propagate_noalloc")
        return out

    def final_distances(self, X: torch.Tensor, nq: int, p: Params, dense: bool = True, topk: bool = False):
        _check(X, torch.float32, "X", self.device)
        n, d = X.shape
        ng = n - nq
        D = torch.empty((nq, ng), dtype=torch.float32, device=self.device) if dense else None
        ti = torch.empty((nq, p.topk_out), dtype=torch.int32, device=self.device) if topk else None
        td = torch.empty((nq, p.topk_out), dtype=torch.float32, device=self.device) if topk else None
        self._need(p, nq, ng, d)
        pc = p.c()
        self._ok(self.lib.gcr_final_distances(self.h, _ptr(X), nq, ng, d, C.byref(pc), _ptr(D), _ptr(ti),
                                              _ptr(td), _stream()), "gcr_final_distances")
        return D, ti, td

    def rerank(self, X: torch.Tensor, nq: int, p: Params, cam: Optional[torch.Tensor] = None,
               dense: bool = True, topk: bool = False, keep_features: bool = False,
               out: Optional[dict] = None, last_graph: Optional["Graph"] = None):
        """Whole re-ranking; returns dict(dist, topk_idx, topk_dist, X).
        last_graph: a Graph (from new_graph) that receives the graph of the
        last round."""
        _check(X, torch.float32, "X", self.device)
        if cam is not None:
            _check(cam, torch.int32, "cam", self.device)
        n, d = X.shape
        ng = n - nq
        o = out if out is not None else {}
        if dense and o.get("dist") is None:
            o["dist"] = torch.empty((nq, ng), dtype=torch.float32, device=self.device)
        if topk and o.get("topk_idx") is None:
            o["topk_idx"] = torch.empty((nq, p.topk_out), dtype=torch.int32, device=self.device)
            o["topk_dist"] = torch.empty((nq, p.topk_out), dtype=torch.float32, device=self.device)
        if keep_features and o.get("X") is None:
            o["X"] = torch.empty_like(X)
        self._need(p, nq, ng, d, cam is not None)
        pc = p.c()
        self._ok(self.lib.gcr_rerank(self.h, _ptr(X), nq, ng, d, _ptr(cam), C.byref(pc),
                                     _ptr(o.get("dist") if dense else None),
                                     _ptr(o.get("topk_idx") if topk else None),
                                     _ptr(o.get("topk_dist") if topk else None),
                                     _ptr(o.get("X") if keep_features else None),
                                     C.byref(last_graph.g) if last_graph is not None else None, _stream()),
                 "gcr_rerank")
        return o

    def new_graph(self, n: int, p: Params, has_cross: bool = False) -> "Graph":
        """An empty graph bound for n nodes with p.k (and p.cross_k)."""
        return Graph(n, p.k, p.cross_k, has_cross, self.device)

    def dsfp(self, X: torch.Tensor, idx: Optional[torch.Tensor], p: Params,
             out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """DSFP (Alg. 1) of X (used as given) over the neighbour lists idx
        (int32 [n, k], or None with k = 0), with p.gamma and p.rounds."""
        _check(X, torch.float32, "X", self.device)
        n, d = X.shape
        k = 0
        if idx is not None:
            _check(idx, torch.int32, "idx", self.device)
            k = idx.shape[1]
        Y = out if out is not None else torch.empty_like(X)
        self._need(Params(k=0), 0, n, d)
        self._ok(self.lib.gcr_dsfp(self.h, _ptr(X), _ptr(idx), n, d, k, p.gamma, p.rounds, _ptr(Y), _stream()),
                 "gcr_dsfp")
        return Y

    def rerank_local(self, X: torch.Tensor, nq: int, p: Params, dense: bool = True, topk: bool = False,
                     keep_features: bool = False, out: Optional[dict] = None):
        """GCR_Local re-ranking (kNN once, DSFP, final distances); returns
        dict(dist, topk_idx, topk_dist, X)."""
        _check(X, torch.float32, "X", self.device)
        n, d = X.shape
        ng = n - nq
        o = out if out is not None else {}
        if dense and o.get("dist") is None:
            o["dist"] = torch.empty((nq, ng), dtype=torch.float32, device=self.device)
        if topk and o.get("topk_idx") is None:
            o["topk_idx"] = torch.empty((nq, p.topk_out), dtype=torch.int32, device=self.device)
            o["topk_dist"] = torch.empty((nq, p.topk_out), dtype=torch.float32, device=self.device)
        if keep_features and o.get("X") is None:
            o["X"] = torch.empty_like(X)
        self._need(p, nq, ng, d)
        pc = p.c()
        self._ok(self.lib.gcr_rerank_local(self.h, _ptr(X), nq, ng, d, C.byref(pc),
                                           _ptr(o.get("dist") if dense else None),
                                           _ptr(o.get("topk_idx") if topk else None),
                                           _ptr(o.get("topk_dist") if topk else None),
                                           _ptr(o.get("X") if keep_features else None), _stream()),
                 "gcr_rerank_local")
        return o

    def profile_vectors(self, frames: torch.Tensor, offsets: torch.Tensor, groups: Optional[torch.Tensor] = None,
                        mode: str = "pvg", lam: float = 10.0) -> torch.Tensor:
        """Eq. (16) ("pvg") or Eq. (10) ("mean") profiles, L2-normalised.
        offsets / groups: int32 tensors (device copies are made as needed)."""
        _check(frames, torch.float32, "frames", self.device)
        offs_h = offsets.detach().to("cpu", torch.int32).contiguous()
        offs_d = offs_h.to(self.device)
        nt = offs_h.numel() - 1
        grp_h = grp_d = None
        if groups is not None:
            grp_h = groups.detach().to("cpu", torch.int32).contiguous()
            grp_d = grp_h.to(self.device)
        W = torch.empty((nt, frames.shape[1]), dtype=torch.float32, device=self.device)
        m = {"pvg": 0, "mean": 1}[mode]
        if self.auto_reserve:
            nb = int(self.lib.gcr_profile_workspace_size(nt, frames.shape[0], frames.shape[1], m))
            if nb > self.workspace_bytes():
                self.reserve(nb)
        self._ok(self.lib.gcr_profile_vectors(self.h, _ptr(frames), _ptr(offs_d), _ptr(grp_d), _ptr(offs_h),
                                              _ptr(grp_h), nt, frames.shape[1], m, lam, _ptr(W), _stream()),
                 "gcr_profile_vectors")
        return W

    def gcrv(self, frames, offsets, nq: int, p: Params, groups=None, cam=None, mode: str = "pvg",
             dense: bool = True, topk: bool = False):
        """Alg. 2: profile vectors of all tracklets (queries first), then
        re-ranking on them."""
        W = self.profile_vectors(frames, offsets, groups, mode, p.lam)
        out = self.rerank(W, nq, p, cam, dense=dense, topk=topk, keep_features=True)
        out["W"] = W
        return out


class Server:
    """Resident gallery + request loop (gcr_server_*).

    gallery: CUDA tensor [G, d], float32, or bfloat16 / int16 / uint16 BF16
    bit patterns.  p.rebuild_each_round must be False (the gallery graph is
    fixed).  submit() takes a host float32 array [b, d] and returns a ticket;
    wait() returns (indices int32 [b, K], distances float32 [b, K]).
    """

    def __init__(self, ctx: Context, gallery: Optional[torch.Tensor], p: Optional[Params], lanes: int = 2,
                 max_batch: int = 512, max_recomputed: int = 65536, gallery_capacity: int = 0,
                 max_requests: int = 16, mem_budget: int = 0, _load_path: Optional[str] = None):
        self.ctx = ctx
        self.lib = ctx.lib
        cfg = L.GcrServerConfig(lanes, max_batch, max_requests, max_recomputed, gallery_capacity, 0, mem_budget)
        if _load_path is not None:
            h = C.c_void_p()
            st = self.lib.gcr_server_load(ctx.h, _load_path.encode(), C.byref(cfg), C.byref(h))
            if st != L.GCR_OK:
                raise GcrError(f"gcr_server_load failed ({L.STATUS_NAMES.get(st, st)}): "
                               f"{self.lib.gcr_last_error(ctx.h).decode()}")
            self.h = h
            self._b = {}
            self._read_shape(_load_path)
            return
        if gallery.device != ctx.device or not gallery.is_contiguous():
            raise ValueError("gallery must be a contiguous tensor on the context's device")
        if gallery.dtype == torch.float32:
            dtype = 0
        elif gallery.dtype in (torch.bfloat16, torch.int16, torch.uint16):
            dtype = 1
        else:
            raise TypeError("gallery must be float32 or BF16")
        ng, d = gallery.shape
        self.d, self.K = d, p.topk_out
        h = C.c_void_p()
        pc = p.c()
        st = self.lib.gcr_server_create(ctx.h, _ptr(gallery), dtype, ng, d, C.byref(pc), C.byref(cfg), C.byref(h))
        if st != L.GCR_OK:
            raise GcrError(f"gcr_server_create failed ({L.STATUS_NAMES.get(st, st)}): "
                           f"{self.lib.gcr_last_error(ctx.h).decode()}")
        self.h = h
        self._b = {}

    def _err(self) -> str:
        return self.lib.gcr_server_last_error(self.h).decode()

    def submit(self, q) -> int:
        import numpy as np

        q = np.ascontiguousarray(q, dtype=np.float32)
        if q.ndim != 2 or q.shape[1] != self.d:
            raise ValueError(f"queries must be [b, {self.d}]")
        t = C.c_uint64()
        st = self.lib.gcr_server_submit(self.h, q.ctypes.data, q.shape[0], C.byref(t))
        if st != L.GCR_OK:
            raise GcrError(f"gcr_server_submit failed ({L.STATUS_NAMES.get(st, st)}): {self._err()}")
        self._b[t.value] = q.shape[0]
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        """(indices, distances), or None on timeout."""
        import numpy as np

        b = self._b[ticket]
        idx = np.empty((b, self.K), dtype=np.int32)
        dist = np.empty((b, self.K), dtype=np.float32)
        st = self.lib.gcr_server_wait(self.h, ticket, idx.ctypes.data, dist.ctypes.data, timeout_ms)
        if st == L.GCR_ERR_TIMEOUT:
            return None
        del self._b[ticket]
        if st != L.GCR_OK:
            raise GcrError(f"request {ticket} failed ({L.STATUS_NAMES.get(st, st)}): {self._err()}")
        return idx, dist

    def query(self, q):
        return self.wait(self.submit(q))

    @classmethod
    def load(cls, ctx: Context, path: str, lanes: int = 2, max_batch: int = 512, max_recomputed: int = 65536,
             gallery_capacity: int = 0, max_requests: int = 16, mem_budget: int = 0) -> "Server":
        """A server started from a state written by save()."""
        return cls(ctx, None, None, lanes, max_batch, max_recomputed, gallery_capacity, max_requests, mem_budget,
                   _load_path=path)

    def _read_shape(self, path: str):
        import struct

        with open(path, "rb") as f:
            head = f.read(8 + 16 + 16 + C.sizeof(L.GcrParams))
        _, d, _, _ = struct.unpack_from("<4i", head, 8)
        pr = L.GcrParams.from_buffer_copy(head[8 + 16 + 16:])
        self.d, self.K = d, pr.topk_out

    def insert(self, rows):
        """Append host float32 rows [m, d]; returns their ids (int32 [m])."""
        import numpy as np

        rows = np.ascontiguousarray(rows, dtype=np.float32)
        if rows.ndim != 2 or rows.shape[1] != self.d:
            raise ValueError(f"rows must be [m, {self.d}]")
        ids = np.empty(rows.shape[0], dtype=np.int32)
        st = self.lib.gcr_server_insert(self.h, rows.ctypes.data, rows.shape[0], ids.ctypes.data)
        if st != L.GCR_OK:
            raise GcrError(f"gcr_server_insert failed ({L.STATUS_NAMES.get(st, st)}): {self._err()}")
        return ids

    def remove(self, ids):
        import numpy as np

        ids = np.ascontiguousarray(ids, dtype=np.int32).ravel()
        st = self.lib.gcr_server_remove(self.h, ids.ctypes.data, ids.shape[0])
        if st != L.GCR_OK:
            raise GcrError(f"gcr_server_remove failed ({L.STATUS_NAMES.get(st, st)}): {self._err()}")

    def ids(self):
        """Live gallery ids in row order (increasing)."""
        import numpy as np

        n = C.c_int64()
        self.lib.gcr_server_gallery_ids(self.h, None, 0, C.byref(n))
        out = np.empty(n.value, dtype=np.int32)
        st = self.lib.gcr_server_gallery_ids(self.h, out.ctypes.data, n.value, C.byref(n))
        if st != L.GCR_OK:
            raise GcrError(f"gcr_server_gallery_ids failed: {self._err()}")
        return out

    def save(self, path: str):
        st = self.lib.gcr_server_save(self.h, path.encode())
        if st != L.GCR_OK:
            raise GcrError(f"gcr_server_save failed ({L.STATUS_NAMES.get(st, st)}): {self._err()}")

    def stats(self) -> dict:
        s = L.GcrServerStats()
        self.lib.gcr_server_get_stats(self.h, C.byref(s))
        return {f: getattr(s, f) for f, _ in L.GcrServerStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.gcr_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
