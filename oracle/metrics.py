"""Retrieval metrics for the test oracle (test infrastructure only).

Mean average precision over all gallery items of the query's identity, the
plain protocol the result tables report (Tables I-IV headers give Rank-1 and
mAP without further detail)."""
from __future__ import annotations

import numpy as np


def mean_average_precision(dq: np.ndarray, qids: np.ndarray, gids: np.ndarray) -> float:
    """mAP of the per-query gallery ranking by ascending distance (ties by
    gallery index)."""
    aps = []
    for t in range(dq.shape[0]):
        order = np.argsort(dq[t], kind="stable")
        rel = (gids[order] == qids[t]).astype(np.float64)
        nrel = rel.sum()
        if nrel == 0:
            continue
        hits = np.cumsum(rel)
        prec = hits / np.arange(1, len(rel) + 1)
        aps.append(float((prec * rel).sum() / nrel))
    return float(np.mean(aps)) if aps else 0.0

