"""Oracle for gridding with the generated kernels (FP64, CPU).  Test
infrastructure only; see the package header.

Algorithm 2 ends each w-plane's iteration by gridding the plane's visibility
records with its oversampled kernel cache.  This module writes that step
out so the fused consumer (kernels evaluated from the radial lines while
gridding, never stored) can be checked against it.

Readings:

G1  The uv grid has N x N cells of du = 1 / FOV; cell (ix, iy) holds
    uv = ((ix - N/2) du, (iy - N/2) du); rows are v, columns u.
G2  A record at uv position x = u / du + N/2 (cells) uses the nearest
    oversampled sub-kernel: i = floor(x), f = floor((x - i) os + 1/2), and
    f = os moves to (i + 1, 0).  Sub-kernel f holds samples at offsets
    (a - h) - f / os (reading R7), so cell i + a - h receives sample a.
    Decided in FP64.
G3  Cells outside the grid are skipped (the rest of the footprint is kept).
G4  A record with w < 0 uses the conjugate of the kernel computed for |w|
    (section 4.1).
G5  A record's kernel is the one of the plane the partition assigned it to
    (Algorithm 2), with that plane's support.

Parity: pinned in tests/test_oracle_gridding.py by a gather formulation
(each cell sums over the records that reach it, evaluated independently),
the Hermitian symmetry of a record paired with its (-u, -v, -w, conj V)
twin, exact placement of a single record at a cell centre, and linearity.
"""
from __future__ import annotations

import math

import numpy as np


def position(u: float, du: float, n_grid: int, oversampling: int):
    """(cell i, sub-kernel f) of a coordinate (G2)."""
    x = u / du + n_grid / 2
    i = math.floor(x)
    f = math.floor((x - i) * oversampling + 0.5)
    if f == oversampling:
        i, f = i + 1, 0
    return i, f


def grid(u, v, w, vis, order, plane_start, caches, supports, oversampling: int,
         n_grid: int, du: float) -> np.ndarray:
    """Scatter every record's kernel footprint onto the N x N grid."""
    g = np.zeros((n_grid, n_grid), dtype=np.complex128)
    order = np.asarray(order)
    for m in range(len(plane_start) - 1):
        s = int(supports[m])
        h = (s - 1) // 2
        cache = caches[m]
        for k in order[plane_start[m]:plane_start[m + 1]]:
            iu, fu = position(float(u[k]), du, n_grid, oversampling)
            iv, fv = position(float(v[k]), du, n_grid, oversampling)
            sub = cache[fv, fu]
            if w[k] < 0:
                sub = np.conj(sub)
            y0, x0 = iv - h, iu - h
            ys, xs = max(0, y0), max(0, x0)
            ye, xe = min(n_grid, y0 + s), min(n_grid, x0 + s)
            if ys >= ye or xs >= xe:
                continue
            g[ys:ye, xs:xe] += complex(vis[k]) * sub[ys - y0:ye - y0, xs - x0:xe - x0]
    return g


def grid_cell(iy: int, ix: int, u, v, w, vis, plane_of, caches, supports, oversampling: int,
              n_grid: int, du: float) -> complex:
    """One grid cell as a gather over all records (vectorised), used for
    sampled checks at full size: sum of V_k K_{m(k)} at the cell's offset."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    xu = u / du + n_grid / 2
    xv = v / du + n_grid / 2
    iu = np.floor(xu).astype(np.int64)
    iv = np.floor(xv).astype(np.int64)
    fu = np.floor((xu - iu) * oversampling + 0.5).astype(np.int64)
    fv = np.floor((xv - iv) * oversampling + 0.5).astype(np.int64)
    iu = np.where(fu == oversampling, iu + 1, iu)
    fu = np.where(fu == oversampling, 0, fu)
    iv = np.where(fv == oversampling, iv + 1, iv)
    fv = np.where(fv == oversampling, 0, fv)
    h = (np.asarray(supports)[plane_of] - 1) // 2
    a = ix - iu + h
    b = iy - iv + h
    s = 2 * h + 1
    hit = np.nonzero((a >= 0) & (a < s) & (b >= 0) & (b < s))[0]
    acc = 0.0 + 0.0j
    for k in hit:
        val = caches[plane_of[k]][fv[k], fu[k], b[k], a[k]]
        if w[k] < 0:
            val = np.conj(val)
        acc += complex(vis[k]) * val
    return acc
