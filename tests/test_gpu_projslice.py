"""Projection-slice engine (section 4.3.1, Algorithm 2) on the GPU against
the oracle's projection-slice chain.  The engine is FP64 up to the radial
line: lines are held to 1e-12 (relative to the line's peak), caches to 1e-6
(the FP32 spline coefficients and complex64 output of the shared
resample)."""
import numpy as np
import pytest

import workloads as W
from oracle import fft2d as F
from oracle import projslice as PS

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

LINE_GATE = 1e-12
CACHE_GATE = 1e-6


def _plan(wl, engine_ws, precision="fp32"):
    from paper_1904_08463_amd import Plan
    plan = Plan.from_workload(wl, precision=precision)
    plan.set_engine("projection_slice", engine_ws)
    return plan


def _ref(wl, planes, engine_ws):
    fov = wl.image_size * wl.cellsize
    tfn = F.taper_from_samples(wl.taper, 0.5 * fov)
    fixed = wl.max_support if engine_ws == "max_support" else None
    return PS.generate(tfn, wl.w[planes], wl.support[planes], wl.oversampling, fov,
                       wl.radial_refine, wl.interp, fixed)


def _check(wl, engine_ws, planes=None, precision="fp32"):
    planes = list(range(wl.n_planes)) if planes is None else list(planes)
    print(f"case {wl.name} projection-slice {engine_ws} planes={len(planes)}", flush=True)
    plan = _plan(wl, engine_ws, precision)
    taper = torch.from_numpy(wl.taper).cuda()
    w = torch.from_numpy(wl.w).cuda()
    out = plan.generate(taper, w).cpu().numpy()
    lines = plan.generate_radial(taper, w).cpu().numpy()
    loff = np.concatenate([[0], np.cumsum(plan.nrho)])
    caches, ref_lines = _ref(wl, planes, engine_ws)
    worst_line = worst_cache = 0.0
    for j, p in enumerate(planes):
        got_l = lines[loff[p]:loff[p + 1]]
        e = np.max(np.abs(got_l - ref_lines[j])) / np.max(np.abs(ref_lines[j]))
        worst_line = max(worst_line, e)
        got = out[plan.offsets[p]:plan.offsets[p + 1]].reshape(caches[j].shape)
        e = np.max(np.abs(got - caches[j])) / np.max(np.abs(caches[j]))
        worst_cache = max(worst_cache, e)
    print(f"  worst line {worst_line:.2e}, worst cache {worst_cache:.2e}", flush=True)
    assert worst_line <= LINE_GATE
    assert worst_cache <= CACHE_GATE
    return plan, out


@pytest.mark.parametrize("engine_ws", ["per_plane", "max_support"])
@pytest.mark.parametrize("interp", ["cubic", "linear"])
def test_plain(engine_ws, interp):
    _check(W.plain(interp=interp), engine_ws)[0].close()


@pytest.mark.parametrize("seed", range(4))
def test_random_ragged(seed):
    for q in (1, 2):
        wl = W.random_small(seed, os_=3 if seed % 2 else 4, radial_refine=q,
                            interp="linear" if seed == 3 else "cubic")
        _check(wl, "per_plane")[0].close()


@pytest.mark.parametrize("engine_ws", ["per_plane", "max_support"])
def test_paper_sampled(engine_ws):
    _check(W.paper(), engine_ws, planes=[0, 31, 100, 200, 255])[0].close()


def test_batch_sampled_split_plan():
    """The full batch through the projection-slice engine on a split-BF16 plan
    (the engine ignores the plan's contraction precision)."""
    wl = W.batch()
    order = np.argsort(wl.support, kind="stable")
    planes = sorted(set(order[[0, 5000, 12000, 16383]].tolist()) | {int(np.argmax(wl.mirror))})
    _check(wl, "per_plane", planes=planes, precision="bf16x6")[0].close()


def test_mirrored_planes_exact_conjugates():
    base = W.plain()
    wl = W.plain(extra_w=[-v for v in base.w[::-1]])
    wl.mirror = W.mirror_table(wl.w, wl.support)
    plan, out = _check(wl, "per_plane")
    for p in range(wl.n_planes):
        q = wl.mirror[p]
        if q >= 0:
            assert np.array_equal(out[plan.offsets[p]:plan.offsets[p + 1]],
                                  np.conj(out[plan.offsets[q]:plan.offsets[q + 1]]))
    plan.close()


def test_engine_switch_and_gradient():
    """Back to the matrix engine gives the bits of a fresh matrix plan; the
    adjoint refuses the projection-slice engine."""
    from paper_1904_08463_amd import Plan
    from paper_1904_08463_amd.wkern import WkernError
    wl = W.plain()
    taper = torch.from_numpy(wl.taper).cuda()
    w = torch.from_numpy(wl.w).cuda()
    fresh = Plan.from_workload(wl)
    ref = fresh.generate(taper, w).cpu().numpy()
    fresh.close()
    plan = _plan(wl, "per_plane")
    ps_out = plan.generate(taper, w).cpu().numpy()
    assert not np.array_equal(ps_out, ref)
    g = torch.zeros(int(plan.offsets[-1]), dtype=torch.complex64, device="cuda")
    with pytest.raises(WkernError):
        plan.grad(taper, w, g)
    plan.set_engine("matrix")
    assert np.array_equal(plan.generate(taper, w).cpu().numpy(), ref)
    plan.close()


def test_truncated_with_projection_slice():
    from oracle import hankel as H
    wl = W.paper()
    plan = _plan(wl, "per_plane")
    taper = torch.from_numpy(wl.taper).cuda()
    w = torch.from_numpy(wl.w).cuda()
    out, sup, offs = plan.generate_truncated(taper, w, 0.01)
    out, sup, offs = out.cpu().numpy(), sup.cpu().numpy(), offs.cpu().numpy()
    planes = [0, 128, 255]
    caches, lines = _ref(wl, planes, "per_plane")
    for j, p in enumerate(planes):
        h = H.truncated_half_support(lines[j], 0.01, wl.oversampling, 1, (wl.support[p] - 1) // 2)
        assert sup[p] == 2 * h + 1
        ref = H.resample(lines[j], 2 * h + 1, wl.oversampling)
        got = out[offs[p]:offs[p + 1]].reshape(ref.shape)
        assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) <= CACHE_GATE
    plan.close()
