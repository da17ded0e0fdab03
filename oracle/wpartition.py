"""Oracle for the w-plane partition (FP64, CPU).  Test infrastructure only;
see the package header.

Algorithm 2 (and Algorithm 1 with signed w) opens with three steps: sort the
visibility records by increasing absolute w-term, divide the sorted records
into M w-planes of equal size, and take each plane's w-term as the average
(or the median) of its records (section 3: the kernel of a plane is computed
once for that representative w).

Readings where the paper is silent:

P1  "Equally-sized" planes for n records: plane m holds the sorted positions
    [floor(m n / M), floor((m + 1) n / M)); sizes differ by at most one.
    n >= M >= 1 (an empty plane has no w-term).
P2  Records with equal keys keep their input order (a stable sort).
P3  The statistic is taken over the sort key: |w| for Algorithm 2 (a record
    with w < 0 uses the conjugate kernel, section 4.1), w for Algorithm 1.
    The mean is the correctly rounded sum divided by the count; the median of
    an even count is the mean of the two middle values.
P4  -0.0 and +0.0 are equal keys; NaN sorts after every number (stable among
    NaNs).  These follow IEEE comparison, as NumPy's sort does.

Parity: pinned in tests/test_oracle_pins.py by a brute-force sort on tiny
inputs (a separate key function), a hand-derived example, plane-size and
ordering invariants, and exact statistics of constant planes.
"""
from __future__ import annotations

import math

import numpy as np


def sort_key(w, absolute: bool = True) -> np.ndarray:
    """The value records are sorted by (P3)."""
    w = np.asarray(w, dtype=np.float64)
    return np.abs(w) if absolute else w.copy()


def plane_bounds(n: int, n_planes: int) -> np.ndarray:
    """Start of each plane in sorted order, [M + 1] (P1)."""
    if not (n >= n_planes >= 1):
        raise ValueError("need n >= n_planes >= 1")
    return (np.arange(n_planes + 1, dtype=np.int64) * n) // n_planes


def partition(w, n_planes: int, absolute: bool = True, stat: str = "mean"):
    """(order [n] record indices in sorted order, plane_start [M + 1],
    w_plane [M]) for Algorithm 2 (absolute=True) or Algorithm 1."""
    key = sort_key(w, absolute)
    n = key.shape[0]
    start = plane_bounds(n, n_planes)
    order = np.argsort(key, kind="stable")  # P2, P4
    vals = key[order]
    w_plane = np.empty(n_planes, dtype=np.float64)
    for m in range(n_planes):
        seg = vals[start[m]:start[m + 1]]
        c = seg.shape[0]
        if stat == "mean":
            w_plane[m] = math.fsum(seg) / c if np.all(np.isfinite(seg)) else np.sum(seg) / c
        elif stat == "median":
            if c % 2:
                w_plane[m] = seg[c // 2]
            else:
                w_plane[m] = (seg[c // 2 - 1] + seg[c // 2]) / 2.0
        else:
            raise ValueError(stat)
    return order.astype(np.int64), start, w_plane
