"""The 2D-FFT comparison path (standard algorithm, Algorithm 1) through the C
ABI against the oracle's FP64 2D twin on the same workspace: per plane
max |K_gpu - K_ref| / max |K_ref| <= 1e-6, zeros outside the support."""
import numpy as np
import pytest

import workloads as W
from oracle import fft2d as F
from oracle import hankel as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GATE = 1e-6


def _run(wl, workspace, planes=None):
    from paper_1904_08463_amd import FFT2DPlan
    print(f"case {wl.name} workspace={workspace} P={wl.n_planes}", flush=True)
    plan = FFT2DPlan.from_workload(wl, workspace=workspace)
    taper = torch.from_numpy(wl.taper).cuda()
    w = torch.from_numpy(wl.w).cuda()
    flat = plan.generate(taper, w).cpu().numpy()
    plan.close()
    fov = wl.image_size * wl.cellsize
    tfn = F.taper_from_samples(wl.taper, 0.5 * fov)
    planes = range(wl.n_planes) if planes is None else planes
    worst = 0.0
    offs = H.offsets(wl.support, wl.oversampling)
    for p in planes:
        s = int(wl.support[p])
        n_ws = F.next_pow2(wl.max_support if workspace == "max_support" else s)
        ref = F.generate(tfn, [wl.w[p]], [s], wl.oversampling, n_ws, fov)[0]
        got = flat[offs[p]:offs[p + 1]].reshape(ref.shape)
        _, mask, _ = H.sample_positions(s, wl.oversampling, 1)
        assert np.all(got[~mask] == 0)
        e = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        worst = max(worst, e)
        assert e <= GATE, (p, s, e)
    print(f"{wl.name}/{workspace}: worst error {worst:.3e}", flush=True)


@pytest.mark.parametrize("workspace", ["max_support", "per_plane"])
def test_plain(workspace):
    _run(W.plain(), workspace)


@pytest.mark.parametrize("workspace", ["max_support", "per_plane"])
def test_random_ragged(workspace):
    _run(W.random_small(4, n_planes=17, n_radial=333, os_=3, max_support=29), workspace)


def test_paper_sampled():
    _run(W.paper(), "max_support", planes=[0, 90, 255])


def test_mirrored_planes():
    base = W.plain()
    wl = W.plain(extra_w=[-v for v in base.w])
    wl.mirror = W.mirror_table(wl.w, wl.support)
    _run(wl, "per_plane")
