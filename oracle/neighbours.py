"""Conditioning sets: the nearest preceding neighbours.

Section 2.1 (text after eq. (4)) and Section 2.2 (after eq. (6)): N_i holds
min(m, i-1) components; for a stationary process observed at locations, the
most correlated components are the nearest locations. Only components that
precede i in the ordering are eligible (the telescoping product, eq. (5)).

Reading for ties (a regular grid has many): candidates are ranked by the key
(d^2, plan index) ascending, d^2 = dx*dx + dy*dy without fused multiply-add, and
the list is returned in that order.
"""
from __future__ import annotations

import numpy as np


def knn_preceding(s: np.ndarray, m: int, queries=None) -> list:
    """For plan-ordered locations s (D x 2), return nbrs[i] (plan indices) for
    every i, or for the plan positions in `queries` (in that order)."""
    D = s.shape[0]
    out = []
    for i in (range(D) if queries is None else [int(q) for q in queries]):
        k = min(m, i)
        if k == 0:
            out.append(np.zeros(0, dtype=np.int64))
            continue
        dx = s[:i, 0] - s[i, 0]
        dy = s[:i, 1] - s[i, 1]
        d2 = dx * dx + dy * dy
        idx = np.arange(i)
        order = np.lexsort((idx, d2))          # primary d2, secondary index
        out.append(order[:k].astype(np.int64))
    return out
