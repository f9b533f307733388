"""Canonical upper-triangular 3x3 block pattern and stencil -> slot map.

Follows the paper's global Hessian compression (appendix "Global Hessian
Compression"): collect the (row, col) coordinates of every block a stencil
contributes, keep the upper triangle, sort lexicographically and remove
duplicates; each stencil then looks up where its blocks live ("PositionInData").
Placement indices are 0-based with -1 for "no contribution" (the paper's
1-based indices with 0 as the pad, appendix "Index Computation").

Rule, fixed so that two independent builders agree bit for bit:

* a stencil with k used vertices enumerates local pairs (a, b), a = 0..k-1,
  b = a..k-1 (10 / 6 / 3 pairs for k = 4 / 3 / 2), padded to w (w + 1) / 2
  entries for stencils given w entries wide (10 for w = 4; the row lists of
  stencils touching affine bodies are up to 8 wide, 36 pairs);
* a pair whose two vertices are both free has key (min(v_a, v_b), max(v_a, v_b));
  otherwise its slot is -1;
* the static part also holds (v, v) for every free vertex;
* row_ptr (n_free + 1) and col_idx (nnzb) are int32; slot[s][pair] is the index
  of the key in the sorted unique list.
"""
from __future__ import annotations

import numpy as np


def local_pairs(k):
    return [(a, b) for a in range(k) for b in range(a, k)]


def used_vertices(idx):
    """Number of used (non -1) leading entries of each stencil row."""
    return (np.asarray(idx) >= 0).sum(axis=1)


def stencil_pairs(idx):
    """(n_s, w (w + 1) / 2, 2) local vertex positions (a, b) of every pair slot,
    -1 padded (w = the width of idx)."""
    idx = np.asarray(idx)
    w = idx.shape[1] if idx.ndim == 2 else 4
    k = used_vertices(idx) if idx.size else np.zeros(0, np.int64)
    out = -np.ones((idx.shape[0], w * (w + 1) // 2, 2), np.int64)
    for kk in range(1, w + 1):
        rows = np.flatnonzero(k == kk)
        pr = np.array(local_pairs(kk))
        out[rows[:, None], np.arange(len(pr))[None, :]] = pr[None, :, :]
    return out


def build(n_free, idx_list, add_diagonal):
    """Pattern of one part.  idx_list: list of (n_s, w) int arrays (free ids
    < n_free, fixed ids >= n_free, -1 unused).  Returns row_ptr, col_idx and a
    list of (n_s, w (w + 1) / 2) int32 slot arrays, one per input array."""
    rows_all, cols_all, per = [], [], []
    for idx in idx_list:
        idx = np.asarray(idx, dtype=np.int64)
        pairs = stencil_pairs(idx)
        a, b = pairs[..., 0], pairs[..., 1]
        valid = a >= 0
        va = np.where(valid, np.take_along_axis(idx, np.maximum(a, 0), 1), -1)
        vb = np.where(valid, np.take_along_axis(idx, np.maximum(b, 0), 1), -1)
        ok = valid & (va >= 0) & (va < n_free) & (vb >= 0) & (vb < n_free)
        r = np.minimum(va, vb)
        c = np.maximum(va, vb)
        per.append((r, c, ok))
        rows_all.append(r[ok])
        cols_all.append(c[ok])
    if add_diagonal:
        rows_all.append(np.arange(n_free))
        cols_all.append(np.arange(n_free))
    keys = np.concatenate([r * n_free + c for r, c in zip(rows_all, cols_all)]) if rows_all else np.zeros(0, np.int64)
    uniq = np.unique(keys)
    rows = uniq // max(n_free, 1)
    cols = uniq % max(n_free, 1)
    row_ptr = np.zeros(n_free + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n_free), out=row_ptr[1:])
    slots = []
    for r, c, ok in per:
        s = np.searchsorted(uniq, r * n_free + c)
        slots.append(np.where(ok, s, -1).astype(np.int32))
    return row_ptr.astype(np.int32), cols.astype(np.int32), slots
