"""Gridding with the kernels on the GPU: the fused consumer (kernel values
from the spline intervals, no cache) and the cache reader, against the
gridding oracle.  FP32 atomic sums: the gate per cell is
    |G - G_ref| <= g_K * E + 1e-6 * A,
E = sum over the cell's records of |V| max|K_plane| (the kernel's normwise
error g_K: 1e-5 FP32, 1e-6 split-BF16, relative to the plane's peak) and
A = sum of |V K| (FP32 rounding of products and sums, with room for the
number of terms)."""
import numpy as np
import pytest

import workloads as W
from oracle import gridding as G
from oracle import hankel as H
from oracle import wpartition as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _bounds(gw, order, start, caches, sup, du, n):
    mags = [np.abs(c) for c in caches]
    peaks = [np.ones_like(c.real) * np.max(np.abs(c)) for c in caches]
    a = G.grid(gw.u, gw.v, gw.w, np.abs(gw.vis), order, start, mags, sup, gw.oversampling, n, du)
    e = G.grid(gw.u, gw.v, gw.w, np.abs(gw.vis), order, start, peaks, sup, gw.oversampling, n, du)
    return np.abs(a), np.abs(e)


def _check(got, ref, a, e, gk, what):
    err = np.abs(got - ref)
    tol = gk * e + 1e-6 * a + 1e-30
    worst = float(np.max(err / tol))
    print(f"  {what}: max |dG| {err.max():.3e} (max |G| {np.abs(ref).max():.3e}), "
          f"worst err / tol {worst:.3f}", flush=True)
    assert worst <= 1.0


@pytest.mark.parametrize("seed", [0, 1])
def test_small_full_grid(seed):
    from paper_1904_08463_amd import Plan, wpartition
    gw = W.grid_small(seed)
    n = gw.grid_size
    du = 1.0 / (gw.image_size * gw.cellsize)
    print(f"case grid_small{seed}: {gw.u.size} records, {gw.n_planes} planes, grid {n}", flush=True)
    rng = np.random.default_rng(seed)
    sup = 2 * rng.integers(1, (gw.max_support - 1) // 2 + 1, gw.n_planes) + 1
    order_d, start_d, wp_d = wpartition(_dev(gw.w), gw.n_planes)
    order, start, wp = P.partition(gw.w, gw.n_planes)
    assert np.array_equal(order_d.cpu().numpy(), order)
    caches, _ = H.generate(gw.image_size, gw.cellsize, gw.n_radial, gw.oversampling, gw.taper,
                           wp, sup)
    ref = G.grid(gw.u, gw.v, gw.w, gw.vis, order, start, caches, sup, gw.oversampling, n, du)
    a, e = _bounds(gw, order, start, caches, sup, du, n)
    plan = Plan(gw.image_size, gw.cellsize, gw.n_radial, gw.oversampling, sup, gw.max_support)
    taper = _dev(gw.taper)
    sup_d = plan.prepare_lines(taper, wp_d)
    assert np.array_equal(sup_d.cpu().numpy(), sup)
    args = (_dev(gw.u), _dev(gw.v), _dev(gw.w), _dev(gw.vis), order_d, start_d, sup_d)
    g = torch.zeros((n, n), dtype=torch.complex64, device="cuda")
    plan.grid(*args, g)
    _check(g.cpu().numpy(), ref, a, e, 1e-5, "fused")
    cache = plan.generate(taper, wp_d)
    offs = _dev(plan.offsets)
    g2 = torch.zeros((n, n), dtype=torch.complex64, device="cuda")
    plan.grid(*args, g2, cache=cache, cache_offsets=offs)
    _check(g2.cpu().numpy(), ref, a, e, 1e-5, "from cache")
    plan.close()


def test_paper_setting_record_subset():
    """IM-S geometry, 128 |w|-planes of the 505440 records, os 8, support up
    to 255 with 1% truncation, split-BF16 kernels; 3000 records gridded."""
    from paper_1904_08463_amd import Plan, wpartition
    gw = W.grid_paper()
    n = gw.grid_size
    du = 1.0 / (gw.image_size * gw.cellsize)
    order_d, start_d, wp_d = wpartition(_dev(gw.w), gw.n_planes)
    order, start, wp = P.partition(gw.w, gw.n_planes)
    assert np.array_equal(order_d.cpu().numpy(), order)
    rng = np.random.default_rng(11)
    keep = np.zeros(gw.u.size, dtype=bool)
    keep[rng.choice(gw.u.size, 3000, replace=False)] = True
    plane_of = np.empty(gw.u.size, dtype=np.int64)
    for m in range(gw.n_planes):
        plane_of[order[start[m]:start[m + 1]]] = m
    sub_order = order[keep[order]]
    sub_start = np.searchsorted(plane_of[sub_order], np.arange(gw.n_planes + 1))
    caches, sup, _ = H.generate_truncated(gw.image_size, gw.cellsize, gw.n_radial, gw.oversampling,
                                          gw.taper, wp, gw.max_support, frac=gw.frac)
    print(f"case paper setting: supports {sup.min()}..{sup.max()}", flush=True)
    ref = G.grid(gw.u, gw.v, gw.w, gw.vis, sub_order, sub_start, caches, sup, gw.oversampling,
                 n, du)
    a, e = _bounds(gw, sub_order, sub_start, caches, sup, du, n)
    plan = Plan(gw.image_size, gw.cellsize, gw.n_radial, gw.oversampling,
                [gw.max_support] * gw.n_planes, gw.max_support, precision="bf16x6")
    taper = _dev(gw.taper)
    plan.prepare_lines(taper, wp_d, frac=0.0)
    g = torch.zeros((n, n), dtype=torch.complex64, device="cuda")
    plan.grid(_dev(gw.u), _dev(gw.v), _dev(gw.w), _dev(gw.vis),
              _dev(sub_order.astype(np.int32)), _dev(sub_start.astype(np.int64)),
              _dev(sup.astype(np.int32)), g)
    _check(g.cpu().numpy(), ref, a, e, 1e-6, "fused, 3000 records")
    plan.close()


def test_paper_setting_fused_equals_cache():
    """All 505440 records: the fused consumer against gridding from the cache
    wkern_generate_truncated writes (same kernel values; only the order of
    the FP32 atomic sums differs)."""
    from paper_1904_08463_amd import Plan, wpartition
    gw = W.grid_paper()
    n = gw.grid_size
    order_d, start_d, wp_d = wpartition(_dev(gw.w), gw.n_planes)
    plan = Plan(gw.image_size, gw.cellsize, gw.n_radial, gw.oversampling,
                [gw.max_support] * gw.n_planes, gw.max_support, precision="bf16x6")
    taper = _dev(gw.taper)
    cache, sup_c, offs = plan.generate_truncated(taper, wp_d, gw.frac)
    sup_f = plan.prepare_lines(taper, wp_d, frac=gw.frac)
    assert torch.equal(sup_c, sup_f)
    args = (_dev(gw.u), _dev(gw.v), _dev(gw.w), _dev(gw.vis), order_d, start_d, sup_f)
    g1 = torch.zeros((n, n), dtype=torch.complex64, device="cuda")
    plan.grid(*args, g1)
    g2 = torch.zeros((n, n), dtype=torch.complex64, device="cuda")
    plan.grid(*args, g2, cache=cache, cache_offsets=offs)
    d = (g1 - g2).abs().max().item()
    m = g2.abs().max().item()
    print(f"  fused vs cache: max |dG| {d:.3e}, max |G| {m:.3e}", flush=True)
    assert d <= 1e-5 * m
    plan.close()


def test_grid_rejects_bad_arguments():
    from paper_1904_08463_amd import Plan
    from paper_1904_08463_amd.wkern import WkernError
    wl = W.plain()
    plan = Plan.from_workload(wl)
    z = lambda dt, k=4: torch.zeros(k, dtype=dt, device="cuda")  # noqa: E731
    args = (z(torch.float64), z(torch.float64), z(torch.float64), z(torch.complex64),
            z(torch.int32), z(torch.int64, 9), z(torch.int32, 8))
    with pytest.raises(WkernError):
        plan.grid(*args, torch.zeros((63, 63), dtype=torch.complex64, device="cuda"))
    with pytest.raises(WkernError):
        plan.prepare_lines(_dev(wl.taper), _dev(wl.w), frac=1.0)
    plan.close()


def test_grid_empty_and_outside_records():
    """No records: nothing happens.  Records whose footprint lies wholly or
    partly off the grid: only the cells inside are touched (G3)."""
    from paper_1904_08463_amd import Plan, wpartition
    gw = W.grid_small(4, n_rec=40, n_planes=2)
    n = gw.grid_size
    du = 1.0 / (gw.image_size * gw.cellsize)
    # push half the records near or beyond the grid edge
    u = gw.u.copy()
    u[::2] = (0.5 * n + np.linspace(-3, 8, u[::2].size)) * du
    gw.u = u
    sup = np.array([15, 9])
    order_d, start_d, wp_d = wpartition(_dev(gw.w), 2)
    order, start, wp = P.partition(gw.w, 2)
    caches, _ = H.generate(gw.image_size, gw.cellsize, gw.n_radial, gw.oversampling, gw.taper,
                           wp, sup)
    ref = G.grid(gw.u, gw.v, gw.w, gw.vis, order, start, caches, sup, gw.oversampling, n, du)
    a, e = _bounds(gw, order, start, caches, sup, du, n)
    plan = Plan(gw.image_size, gw.cellsize, gw.n_radial, gw.oversampling, sup, gw.max_support)
    sup_d = plan.prepare_lines(_dev(gw.taper), wp_d)
    g = torch.zeros((n, n), dtype=torch.complex64, device="cuda")
    empty = torch.empty(0, dtype=torch.float64, device="cuda")
    plan.grid(empty, empty, empty, torch.empty(0, dtype=torch.complex64, device="cuda"),
              torch.empty(0, dtype=torch.int32, device="cuda"),
              torch.zeros(3, dtype=torch.int64, device="cuda"), sup_d, g)
    assert g.abs().max().item() == 0.0
    plan.grid(_dev(gw.u), _dev(gw.v), _dev(gw.w), _dev(gw.vis), order_d, start_d, sup_d, g)
    _check(g.cpu().numpy(), ref, a, e, 1e-5, "edge records")
    plan.close()
