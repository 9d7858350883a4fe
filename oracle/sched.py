"""Load-balance metric and list scheduling -- TEST ONLY.

Load balance follows the paper's definition (Section 4.1): useful time over
total time, sum_i t_i / (n * max_i t_i), for n workers with busy times t_i.
A dynamic work queue hands the next item to whichever worker frees first;
`list_schedule` simulates that for given item costs and queue order, which is
what ordering the queue by predicted cost (largest first) tries to improve.
"""
from __future__ import annotations

import heapq

import numpy as np


def load_balance(times):
    t = np.asarray(times, dtype=np.float64)
    return float(t.sum() / (t.size * t.max()))


def list_schedule(costs, n_workers):
    """Busy time per worker when items are taken in the given order."""
    heap = [(0.0, w) for w in range(n_workers)]
    busy = np.zeros(n_workers)
    for c in costs:
        t, w = heapq.heappop(heap)
        busy[w] += c
        heapq.heappush(heap, (t + c, w))
    return busy


def lpt_order(pred):
    """Indices by descending prediction; ties keep ascending index."""
    pred = np.asarray(pred)
    return np.lexsort((np.arange(pred.size), -pred))


def class_order(pred, family):
    """Largest cost class first, ascending index within a class.

    pred is a predicted log-cost per item and family its element family. An
    item's class is round((pred - med) / ln 2) in double precision, med the
    lower median of pred over the items of its family, round(x) =
    floor(x + 0.5): items within a factor of two of each other's predicted
    cost mostly share a class, and a class keeps the given (type-sorted)
    order.
    """
    p = np.asarray(pred).astype(np.float64)
    family = np.asarray(family)
    cls = np.zeros(p.size)
    for t in np.unique(family):
        sel = family == t
        med = np.sort(p[sel])[(int(sel.sum()) - 1) // 2]
        cls[sel] = np.floor((p[sel] - med) / np.log(2.0) + 0.5)
    return np.lexsort((np.arange(p.size), -cls))
