"""Accuracy of the reported k-majority candidates (Section 4's metrics).

For a stream of n items with true frequencies f:

* relative error of a reported item x: |f(x) - f^(x)| / f(x), with f^ the
  estimated count the library reports; the average relative error (ARE) is
  its mean over the reported items (the paper averages over "all of the
  measured frequencies"; the measured frequencies are those of the items the
  algorithm reports);
* precision: reported items that are true k-majority items (f * k > n) over
  all reported items;
* recall: true k-majority items that are reported over all true k-majority
  items, the latter found by exact counting.

Exact counting sorts the stream and counts runs: on the device with
PyTorch's sort-based unique for device tensors, with NumPy for host arrays.
This module measures results; nothing on the hot path uses it.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class ExactCounts:
    """Distinct item ids in increasing order (as uint32) and their counts."""
    ids: np.ndarray
    counts: np.ndarray
    n: int

    def frequency(self, items: np.ndarray) -> np.ndarray:
        """True frequency of each item (0 for items not in the stream)."""
        items = np.asarray(items, dtype=np.uint32)
        if len(self.ids) == 0:
            return np.zeros(len(items), dtype=np.uint64)
        pos = np.minimum(np.searchsorted(self.ids, items), len(self.ids) - 1)
        return np.where(self.ids[pos] == items, self.counts[pos], 0).astype(np.uint64)

    def majority(self, k: int) -> np.ndarray:
        """The true k-majority items: f * k > n."""
        sel = self.counts.astype(np.uint64) * np.uint64(k) > np.uint64(self.n)
        return self.ids[sel]


def exact_counts_host(items: np.ndarray) -> ExactCounts:
    a = np.asarray(items, dtype=np.uint32)
    ids, counts = np.unique(a, return_counts=True)
    return ExactCounts(ids.astype(np.uint32), counts.astype(np.uint64), len(a))


def exact_counts_device(d_items) -> ExactCounts:
    """Exact counts of a device tensor of 32-bit items (int32 view of uint32
    ids); the sort runs on the device, the distinct ids come to the host."""
    import torch
    t = d_items.view(torch.int32) if d_items.dtype != torch.int32 else d_items
    # widen to int64 so that the uint32 order is the numeric order
    vals, counts = torch.unique(t.to(torch.int64) & 0xFFFFFFFF, sorted=True, return_counts=True)
    ids = vals.cpu().numpy().astype(np.uint32)
    cnt = counts.cpu().numpy().astype(np.uint64)
    return ExactCounts(ids, cnt, int(t.numel()))


def metrics(reported: np.ndarray, exact: ExactCounts, k: int) -> dict:
    """ARE over the reported items, precision and recall against the exact
    k-majority set.  `reported`: entries with fields item and count."""
    items = np.asarray(reported["item"], dtype=np.uint32)
    est = np.asarray(reported["count"], dtype=np.uint64)
    f = exact.frequency(items)
    if len(items) and np.any(f == 0):
        raise ValueError("a reported item does not occur in the stream")
    rel = np.abs(est.astype(np.float64) - f.astype(np.float64)) / np.maximum(f, 1).astype(np.float64)
    true_set = exact.majority(k)
    hit = np.isin(items, true_set)
    n_rep, n_true, n_hit = int(len(items)), int(len(true_set)), int(hit.sum())
    return {
        "k": int(k),
        "reported": n_rep,
        "true_majority": n_true,
        "are": float(rel.mean()) if n_rep else 0.0,
        "max_rel_error": float(rel.max()) if n_rep else 0.0,
        "precision": n_hit / n_rep if n_rep else 1.0,
        "recall": (float(np.isin(true_set, items).sum()) / n_true) if n_true else 1.0,
    }
