"""Orderings of the locations before neighbour selection.

The paper orders the components before choosing nearest preceding neighbours
and reports the ordering cost as insignificant (Section 3.2); it names no rule.
Readings used:

* COORD: stable lexicographic sort by (x, then y, then original index).
* MAXMIN: the first point is the one nearest the centre of the bounding box
  (ties: lowest index); every next point is the unselected point whose distance
  to the nearest selected point is largest (ties: lowest index). Distances are
  compared through d^2 = dx*dx + dy*dy evaluated without fused multiply-add.
* GIVEN: a caller permutation, validated.

Returns perm with perm[i] = the user index placed at plan position i.
"""
from __future__ import annotations

import numpy as np

ORDER_GIVEN, ORDER_COORD, ORDER_MAXMIN = 0, 1, 2


def d2_to(locs: np.ndarray, px: float, py: float) -> np.ndarray:
    dx = locs[:, 0] - px
    dy = locs[:, 1] - py
    return dx * dx + dy * dy


def coord_order(locs: np.ndarray) -> np.ndarray:
    D = locs.shape[0]
    return np.lexsort((np.arange(D), locs[:, 1], locs[:, 0])).astype(np.int64)


def maxmin_order(locs: np.ndarray, n_first: int | None = None) -> np.ndarray:
    """O(D^2) maxmin ordering, written as its definition. n_first: return only
    the first n_first plan positions (the same picks, the loop stops early)."""
    D = locs.shape[0]
    if D == 0:
        return np.zeros(0, dtype=np.int64)
    n_out = D if n_first is None else max(1, min(D, int(n_first)))
    cx = (locs[:, 0].min() + locs[:, 0].max()) / 2.0
    cy = (locs[:, 1].min() + locs[:, 1].max()) / 2.0
    first = int(np.argmin(d2_to(locs, cx, cy)))        # argmin: first (lowest) index on ties
    perm = np.empty(n_out, dtype=np.int64)
    perm[0] = first
    mind2 = d2_to(locs, locs[first, 0], locs[first, 1])
    mind2[first] = -np.inf
    for t in range(1, n_out):
        j = int(np.argmax(mind2))                      # argmax: lowest index on ties
        perm[t] = j
        mind2 = np.minimum(mind2, d2_to(locs, locs[j, 0], locs[j, 1]))
        mind2[perm[:t + 1]] = -np.inf
    return perm


def given_order(perm: np.ndarray, D: int) -> np.ndarray:
    perm = np.asarray(perm, dtype=np.int64)
    if perm.shape != (D,) or not np.array_equal(np.sort(perm), np.arange(D)):
        raise ValueError("given ordering is not a permutation of 0..D-1")
    return perm


def order(locs: np.ndarray, rule: int, perm: np.ndarray | None = None) -> np.ndarray:
    if rule == ORDER_COORD:
        return coord_order(locs)
    if rule == ORDER_MAXMIN:
        return maxmin_order(locs)
    if rule == ORDER_GIVEN:
        return given_order(perm, locs.shape[0])
    raise ValueError(f"unknown ordering {rule}")
