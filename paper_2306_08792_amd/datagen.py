"""Seeded synthetic inputs shaped like the paper's retrieval workloads.

The paper evaluates on person re-identification sets (Market-1501-like image
features with camera labels, MARS-like tracklets) and on image retrieval
(Section IV). None of those datasets ships here, so every input is drawn from
Gaussian identity clusters with the same shapes: the number of queries and
gallery items, the feature width, identities per split, camera labels and
tracklet lengths.

This module only draws numbers. It holds none of the re-ranking arithmetic,
and both the GPU path and the test oracle take its arrays as given.

Common rules for every generator:
  * ``rng = numpy.random.default_rng(seed)``; draws happen in the order listed
    in each function's docstring;
  * values are built in float64, each row is L2-normalised in float64, then
    cast to float32 with round-to-nearest-even;
  * queries come first in the stacked feature matrix.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = [
    "Workload",
    "plain_gcr_small",
    "cross_camera_reid",
    "video_tracklets",
    "large_retrieval",
    "clustered",
    "random_unit",
    "serving_gallery",
    "serving_trace",
    "WORKLOADS",
]


@dataclasses.dataclass
class Workload:
    """One synthetic retrieval problem.

    X: float32 [nq + ng, d], queries first, unit rows (canonical input).
    ids: int64 [nq + ng] identity label of every row (for mAP).
    cams: int32 [nq + ng] camera label or None.
    params: re-ranking hyper-parameters the workload is defined with.
    frames/offsets/groups: tracklet frames for the video workload (X is then
    None until profile vectors are made).
    """

    name: str
    nq: int
    ng: int
    d: int
    X: Optional[np.ndarray]
    ids: np.ndarray
    cams: Optional[np.ndarray]
    params: dict
    frames: Optional[np.ndarray] = None
    offsets: Optional[np.ndarray] = None
    groups: Optional[np.ndarray] = None


def _unit_rows_f32(x64: np.ndarray) -> np.ndarray:
    nrm = np.sqrt(np.einsum("ij,ij->i", x64, x64))
    nrm = np.maximum(nrm, 1e-300)
    return (x64 / nrm[:, None]).astype(np.float32)


def random_unit(n: int, d: int, seed: int = 0) -> np.ndarray:
    """n i.i.d. Gaussian directions in R^d as float32 unit rows."""
    rng = np.random.default_rng(seed)
    return _unit_rows_f32(rng.standard_normal((n, d)))


def clustered(n_centres: int, per_centre: int, d: int, sigma: float,
              seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """Small clustered set: centres ~ N(0, I), then per-sample noise.

    Draws: centres (n_centres, d); noise (n_centres * per_centre, d).
    Sample s belongs to centre s // per_centre.  Returns (X f32, ids).
    """
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((n_centres, d))
    n = n_centres * per_centre
    noise = rng.standard_normal((n, d))
    ids = np.arange(n) // per_centre
    return _unit_rows_f32(centres[ids] + sigma * noise), ids.astype(np.int64)


def plain_gcr_small(seed: int = 0) -> Workload:
    """Plain GCR, 500 queries + 1,500 gallery, d = 256 (image re-ID shape).

    Draws: centres (100, 256) ~ N(0, I); noise (2000, 256) ~ N(0, I).
    Sample s = 20 c + r has x = centre_c + 0.5 noise_s; r < 5 is a query.
    Parameters: k = 20, gamma = 0.1, L = 2 rounds, alpha = 1.
    """
    rng = np.random.default_rng(seed)
    d = 256
    centres = rng.standard_normal((100, d))
    noise = rng.standard_normal((2000, d))
    s = np.arange(2000)
    c, r = s // 20, s % 20
    x = centres[c] + 0.5 * noise
    q = r < 5
    order = np.concatenate([s[q], s[~q]])
    X = _unit_rows_f32(x[order])
    return Workload("plain_gcr_500q_1500g_d256", 500, 1500, d, X,
                    c[order].astype(np.int64), None,
                    dict(k=20, gamma=0.1, rounds=2, alpha=1.0))


def cross_camera_reid(seed: int = 0, nq: int = 3368, ng: int = 15913,
                      d: int = 2048, n_ids: int = 751, n_cams: int = 6) -> Workload:
    """Cross-camera re-ID, Market-1501-shaped (3,368 q + 15,913 g, d = 2048).

    Draws, in order: centres (n_ids, d) ~ N(0, I); camera bias 0.3 N(0, I)
    (n_cams, d); query cameras (nq) and gallery cameras (ng) uniform over
    n_cams; noise (nq + ng, d).  Identity = index mod n_ids within each
    split; x = centre + bias_cam + 0.5 noise.
    Parameters: k = 20 for both neighbour lists, gamma = 0.2, L = 3; the
    within-camera x0.5 / cross-camera x1.0 weighting is read as the blend of
    the global and cross-camera graphs with alpha = 0.5.
    """
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((n_ids, d))
    bias = 0.3 * rng.standard_normal((n_cams, d))
    qcam = rng.integers(0, n_cams, size=nq)
    gcam = rng.integers(0, n_cams, size=ng)
    n = nq + ng
    ids = np.concatenate([np.arange(nq) % n_ids, np.arange(ng) % n_ids])
    cams = np.concatenate([qcam, gcam]).astype(np.int32)
    X = np.empty((n, d), dtype=np.float32)
    step = 4096
    for a in range(0, n, step):
        b = min(n, a + step)
        noise = rng.standard_normal((b - a, d))
        X[a:b] = _unit_rows_f32(centres[ids[a:b]] + bias[cams[a:b]] + 0.5 * noise)
    return Workload(f"cross_camera_{nq}q_{ng}g_d{d}", nq, ng, d, X,
                    ids.astype(np.int64), cams,
                    dict(k=20, gamma=0.2, rounds=3, alpha=0.5))


def video_tracklets(seed: int = 0, nq: int = 1980, ng: int = 6000, d: int = 2048,
                    n_ids: int = 625, min_len: int = 4, max_len: int = 32,
                    noise_sigma: float = 0.4) -> Workload:
    """Video re-ID, MARS-shaped: 1,980 query + 6,000 gallery tracklets.

    Draws: centres (n_ids, d); tracklet lengths m_t ~ U{min_len..max_len}
    for all nq + ng tracklets (queries first); frame noise (n_frames, d).
    Tracklet t has identity t mod n_ids within its split; every frame is
    centre + 0.4 noise, normalised.  One camera group.
    Parameters: PVG lambda = 10; k = 15, gamma = 0.2, L = 2, alpha = 1.
    """
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((n_ids, d))
    nt = nq + ng
    lens = rng.integers(min_len, max_len + 1, size=nt)
    offsets = np.zeros(nt + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    nf = int(offsets[-1])
    tid = np.concatenate([np.arange(nq) % n_ids, np.arange(ng) % n_ids])
    frame_id = np.repeat(tid, lens)
    frames = np.empty((nf, d), dtype=np.float32)
    step = 8192
    for a in range(0, nf, step):
        b = min(nf, a + step)
        noise = rng.standard_normal((b - a, d))
        frames[a:b] = _unit_rows_f32(centres[frame_id[a:b]] + noise_sigma * noise)
    return Workload(f"video_{nq}q_{ng}g_d{d}", nq, ng, d, None,
                    tid.astype(np.int64), None,
                    dict(k=15, gamma=0.2, rounds=2, alpha=1.0, lam=10.0),
                    frames=frames, offsets=offsets.astype(np.int32),
                    groups=np.zeros(nt, dtype=np.int32))


def large_retrieval(seed: int = 0, nq: int = 20000, ng: int = 200000, d: int = 512,
                    n_ids: int = 5000, sigma: float = 0.6) -> Workload:
    """Large retrieval corpus: 20,000 queries + 200,000 gallery, d = 512.

    Draws: centres (n_ids, d); noise (nq + ng, d).  Identity = index mod
    n_ids within each split; x = centre + 0.6 noise.
    Parameters: k = 20, gamma = 0.2, L = 2, top-100 output.
    """
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((n_ids, d))
    n = nq + ng
    ids = np.concatenate([np.arange(nq) % n_ids, np.arange(ng) % n_ids])
    X = np.empty((n, d), dtype=np.float32)
    step = 16384
    for a in range(0, n, step):
        b = min(n, a + step)
        X[a:b] = _unit_rows_f32(centres[ids[a:b]] + sigma * rng.standard_normal((b - a, d)))
    return Workload(f"large_retrieval_{nq}q_{ng}g_d{d}", nq, ng, d, X,
                    ids.astype(np.int64), None,
                    dict(k=20, gamma=0.2, rounds=2, alpha=1.0, topk_out=100))


def serving_gallery(seed: int = 0, ng: int = 500000, d: int = 512,
                    n_ids: int = 10000, sigma: float = 0.6) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Resident gallery for serving: 500,000 x 512 stored as bfloat16.

    Draws: centres (n_ids, d); noise (ng, d).  Identity = g mod n_ids.
    The rows are normalised in float64, rounded to float32, then to
    bfloat16 with round-to-nearest-even; those bfloat16 values (returned as
    uint16 bit patterns and as their exact float32 values) are canonical.
    Returns (bits uint16 [ng, d], values float32 [ng, d], centres float64).
    """
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((n_ids, d))
    ids = np.arange(ng) % n_ids
    bits = np.empty((ng, d), dtype=np.uint16)
    step = 16384
    for a in range(0, ng, step):
        b = min(ng, a + step)
        f = _unit_rows_f32(centres[ids[a:b]] + sigma * rng.standard_normal((b - a, d)))
        u = f.view(np.uint32).astype(np.uint64)
        # round-to-nearest-even on the top 16 bits (inputs are finite)
        u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
        bits[a:b] = u.astype(np.uint16)
    vals = (bits.astype(np.uint32) << 16).view(np.float32)
    return bits, vals, centres


def serving_trace(centres: np.ndarray, n_requests: int, target_qps: float,
                  seed: int = 1, sigma: float = 0.6, max_b: int = 512):
    """Poisson request trace for the serving loop.

    Draws, per request in order: u ~ U[0, 1) giving the batch size
    b = min(max_b, floor(exp(u ln(max_b + 1)))) (log-uniform, 1..512);
    an exponential inter-arrival gap at rate target_qps / E[b]; b centre
    indices; noise (b, d).  Each query is centre + 0.6 noise, normalised.
    Returns a list of (arrival_seconds, float32 [b, d], centre ids).
    """
    rng = np.random.default_rng(seed)
    # E[b] of the log-uniform draw, by exact summation over the support
    us = np.linspace(0.0, 1.0, 200001)[:-1]
    eb = float(np.minimum(max_b, np.floor(np.exp(us * np.log(max_b + 1)))).mean())
    rate = target_qps / eb
    t = 0.0
    out = []
    n_c, d = centres.shape
    for _ in range(n_requests):
        u = rng.random()
        b = int(min(max_b, np.floor(np.exp(u * np.log(max_b + 1)))))
        b = max(b, 1)
        t += rng.exponential(1.0 / rate)
        cid = rng.integers(0, n_c, size=b)
        q = _unit_rows_f32(centres[cid] + sigma * rng.standard_normal((b, d)))
        out.append((t, q, cid))
    return out


WORKLOADS = {
    "plain_gcr_small": plain_gcr_small,
    "cross_camera_reid": cross_camera_reid,
    "video_tracklets": video_tracklets,
    "large_retrieval": large_retrieval,
}
