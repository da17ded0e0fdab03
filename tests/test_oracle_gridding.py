"""Pins of the gridding oracle (CPU): a gather formulation, Hermitian
symmetry of mirrored record pairs, exact placement, linearity."""
import numpy as np
import pytest

import workloads as W
from oracle import gridding as G
from oracle import hankel as H
from oracle import wpartition as P


def _setup(gw, supports=None, seed=0):
    order, start, wp = P.partition(gw.w, gw.n_planes)
    rng = np.random.default_rng(seed)
    if supports is None:
        supports = 2 * rng.integers(1, (gw.max_support - 1) // 2 + 1, gw.n_planes) + 1
    caches, _ = H.generate(gw.image_size, gw.cellsize, gw.n_radial, gw.oversampling, gw.taper,
                           wp, supports)
    plane_of = np.empty(len(gw.w), dtype=np.int64)
    for m in range(gw.n_planes):
        plane_of[order[start[m]:start[m + 1]]] = m
    du = 1.0 / (gw.image_size * gw.cellsize)
    return order, start, caches, np.asarray(supports), plane_of, du


def test_scatter_equals_gather():
    gw = W.grid_small(0, n_rec=300)
    order, start, caches, sup, plane_of, du = _setup(gw)
    g = G.grid(gw.u, gw.v, gw.w, gw.vis, order, start, caches, sup, gw.oversampling,
               gw.grid_size, du)
    ref = np.zeros_like(g)
    for iy in range(gw.grid_size):
        for ix in range(gw.grid_size):
            ref[iy, ix] = G.grid_cell(iy, ix, gw.u, gw.v, gw.w, gw.vis, plane_of, caches, sup,
                                      gw.oversampling, gw.grid_size, du)
    assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_mirrored_pairs_give_a_hermitian_grid():
    gw = W.grid_small(1, n_rec=200)
    u = np.concatenate([gw.u, -gw.u])
    v = np.concatenate([gw.v, -gw.v])
    w = np.concatenate([gw.w, -gw.w])
    vis = np.concatenate([gw.vis, np.conj(gw.vis)])
    # 4 planes over 400 records: every plane boundary is even, so no +-w pair
    # (adjacent after the stable |w| sort) is split between two planes
    gw2 = W.GridWorkload("pairs", gw.image_size, gw.cellsize, gw.grid_size, gw.n_radial,
                         gw.oversampling, 4, gw.max_support, gw.taper, u, v, w, vis)
    order, start, caches, sup, _, du = _setup(gw2)
    g = G.grid(u, v, w, vis, order, start, caches, sup, gw.oversampling, gw.grid_size, du)
    n = gw.grid_size
    # cell ix <-> n - ix (row and column 0 have no mirror inside the grid)
    inner = g[1:, 1:]
    mirror = np.conj(g[1:, 1:][::-1, ::-1])
    assert np.max(np.abs(inner - mirror)) <= 1e-12 * np.max(np.abs(g))
    assert n % 2 == 0


def test_single_record_at_a_cell_centre():
    gw = W.grid_small(2, n_rec=1)
    n, os_ = gw.grid_size, gw.oversampling
    du = 1.0 / (gw.image_size * gw.cellsize)
    s = 11
    h = 5
    caches, _ = H.generate(gw.image_size, gw.cellsize, gw.n_radial, os_, gw.taper, [300.0], [s])
    for (ix, iy) in ((40, 50), (2, 93)):  # inside; clipped at the edges
        u = np.array([(ix - n / 2) * du])
        v = np.array([(iy - n / 2) * du])
        g = G.grid(u, v, np.array([300.0]), np.array([1.0 + 0j]), [0], [0, 1], caches, [s], os_,
                   n, du)
        ref = np.zeros((n, n), dtype=np.complex128)
        for b in range(s):
            for a in range(s):
                y, x = iy + b - h, ix + a - h
                if 0 <= y < n and 0 <= x < n:
                    ref[y, x] = caches[0][0, 0, b, a]
        assert np.array_equal(g, ref)
        # w < 0 uses the conjugate kernel
        g2 = G.grid(u, v, np.array([-300.0]), np.array([1.0 + 0j]), [0], [0, 1], caches, [s],
                    os_, n, du)
        assert np.array_equal(g2, np.conj(ref))


def test_position_rounding():
    du, n, os_ = 1.0, 16, 4
    assert G.position(0.0, du, n, os_) == (8, 0)
    assert G.position(0.25, du, n, os_) == (8, 1)
    assert G.position(0.99, du, n, os_) == (9, 0)       # f rounds up to os -> next cell
    i, f = G.position(-0.1, du, n, os_)
    assert (i, f) == (8, 0)                              # 7.9 -> cell 7, f = 4 -> (8, 0)


def test_linearity():
    gw = W.grid_small(3, n_rec=150)
    order, start, caches, sup, _, du = _setup(gw)
    rng = np.random.default_rng(7)
    v2 = (rng.normal(size=gw.vis.size) + 1j * rng.normal(size=gw.vis.size))
    g1 = G.grid(gw.u, gw.v, gw.w, gw.vis, order, start, caches, sup, gw.oversampling,
                gw.grid_size, du)
    g2 = G.grid(gw.u, gw.v, gw.w, v2, order, start, caches, sup, gw.oversampling,
                gw.grid_size, du)
    g3 = G.grid(gw.u, gw.v, gw.w, gw.vis.astype(np.complex128) + 2 * v2, order, start, caches,
                sup, gw.oversampling, gw.grid_size, du)
    assert np.max(np.abs(g3 - (g1 + 2 * g2))) <= 1e-12 * np.max(np.abs(g3))
