"""Truncation step of Algorithm 2 (section 3.1) on the GPU against the oracle:
per plane the support is chosen from the radial line (last node at or above
frac x the maximum amplitude), the layout is packed at device-computed
offsets, and the cache is sampled from the spline through the full line.
Supports are compared exactly; where the oracle's deciding node sits within
1e-6 (relative) of the threshold a one-step difference is allowed and
reported (both sides decide in FP64 but on values that differ by the
contraction's rounding).  Caches: per-plane error <= the precision's gate."""
import numpy as np
import pytest

import workloads as W
from oracle import hankel as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GATE = {"fp32": 1e-5, "bf16x6": 1e-6}


def _near_tie(line, frac, s_gpu, s_ref, qos):
    amp = np.abs(line)
    thr = frac * amp.max()
    # nodes whose decision differs between the two supports
    lo = (min(s_gpu, s_ref) - 1) // 2 * qos
    hi = (max(s_gpu, s_ref) - 1) // 2 * qos
    cand = amp[max(0, lo - qos):hi + 1]
    return np.min(np.abs(cand - thr)) <= 1e-6 * amp.max()


@pytest.mark.parametrize("precision", ["fp32", "bf16x6"])
@pytest.mark.parametrize("frac", [0.01, 0.001])
def test_truncated_paper_workload(precision, frac):
    from paper_1904_08463_amd import Plan
    base = W.paper()
    s_max = base.max_support
    sup_plan = np.full(base.n_planes, s_max, dtype=np.int32)
    print(f"case paper truncated frac={frac} precision={precision}", flush=True)
    plan = Plan(base.image_size, base.cellsize, base.n_radial, base.oversampling, sup_plan, s_max,
                precision=precision)
    taper = torch.from_numpy(base.taper).cuda()
    w = torch.from_numpy(base.w).cuda()
    out, sup, offs = plan.generate_truncated(taper, w, frac)
    out, sup, offs = out.cpu().numpy(), sup.cpu().numpy(), offs.cpu().numpy()
    assert offs[0] == 0 and np.array_equal(np.diff(offs), base.oversampling ** 2 * sup.astype(np.int64) ** 2)
    # oracle supports for every plane (lines only), caches for a sample
    geo = H.geometry(base.image_size, base.cellsize, base.n_radial, base.oversampling)
    lines = H.radial_kernels(geo, base.taper, base.w, sup_plan)
    qos = base.oversampling
    ties = 0
    for p, line in enumerate(lines):
        s_ref = 2 * H.truncated_half_support(line, frac, base.oversampling, 1, (s_max - 1) // 2) + 1
        if sup[p] != s_ref:
            assert abs(int(sup[p]) - s_ref) == 2 and _near_tie(line, frac, sup[p], s_ref, qos), p
            ties += 1
    print(f"supports {sup.min()}..{sup.max()}, {ties} threshold ties", flush=True)
    assert ties <= 2
    planes = [0, 60, 128, 200, 255]
    caches, sup_ref, _ = H.generate_truncated(base.image_size, base.cellsize, base.n_radial,
                                              base.oversampling, base.taper, base.w, s_max,
                                              frac=frac, planes=planes)
    for j, p in enumerate(planes):
        if sup[p] != sup_ref[j]:
            continue
        got = out[offs[p]:offs[p + 1]].reshape(caches[j].shape)
        e = float(np.max(np.abs(got - caches[j])) / np.max(np.abs(caches[j])))
        assert e <= GATE[precision], (p, e)
    plan.close()


def test_truncated_with_mirrors_and_small_cap():
    """Mirrored planes take their source's support; planned supports act as
    per-plane caps."""
    from paper_1904_08463_amd import Plan
    base = W.plain()
    wl = W.plain(extra_w=[-v for v in base.w])
    mir = W.mirror_table(wl.w, wl.support)
    sup_plan = np.array([31, 21, 31, 15, 31, 31, 9, 31] * 2, dtype=np.int32)
    plan = Plan(wl.image_size, wl.cellsize, wl.n_radial, wl.oversampling, sup_plan, 31, mirror=mir)
    taper = torch.from_numpy(wl.taper).cuda()
    w = torch.from_numpy(wl.w).cuda()
    out, sup, offs = plan.generate_truncated(taper, w, 0.01)
    out, sup, offs = out.cpu().numpy(), sup.cpu().numpy(), offs.cpu().numpy()
    assert np.all(sup <= sup_plan)
    for p in range(wl.n_planes):
        caches, s_ref, _ = H.generate_truncated(wl.image_size, wl.cellsize, wl.n_radial,
                                                wl.oversampling, wl.taper, wl.w, int(sup_plan[p]),
                                                frac=0.01, planes=[p])
        assert sup[p] == s_ref[0], (p, sup[p], s_ref[0])
        got = out[offs[p]:offs[p + 1]].reshape(caches[0].shape)
        e = float(np.max(np.abs(got - caches[0])) / np.max(np.abs(caches[0])))
        assert e <= 1e-5, (p, e)
        if mir[p] >= 0:
            q = mir[p]
            assert sup[p] == sup[q]
            assert np.array_equal(got, np.conj(out[offs[q]:offs[q + 1]].reshape(got.shape)))
    plan.close()


def test_truncated_rejects_bad_arguments():
    from paper_1904_08463_amd import Plan
    from paper_1904_08463_amd.wkern import WkernError
    wl = W.plain()
    plan = Plan.from_workload(wl)
    taper = torch.from_numpy(wl.taper).cuda()
    w = torch.from_numpy(wl.w).cuda()
    for frac in (0.0, 1.0, -0.5, float("nan")):
        with pytest.raises(WkernError):
            plan.generate_truncated(taper, w, frac)
    small = torch.empty(int(plan.offsets[-1]) - 1, dtype=torch.complex64, device="cuda")
    with pytest.raises(WkernError):
        plan.generate_truncated(taper, w, 0.01, out=small)
    plan.close()


def test_truncated_layout_many_planes():
    """30000 planes: the layout kernel then holds 58 KB of plane widths in
    LDS (above the default 64 KiB with its scan arrays).  The first 1000
    planes must get the supports a 1000-plane plan gives them, and the
    offsets must be the prefix sums of os^2 S^2 of the returned supports."""
    from paper_1904_08463_amd import Plan
    base = W.plain()
    n_big, n_small, os_, s_max = 30000, 1000, 2, 15
    rng = np.random.default_rng(5)
    w = np.ascontiguousarray(rng.uniform(0.0, 1000.0, n_big))
    taper = torch.from_numpy(base.taper).cuda()
    print(f"case truncated layout planes={n_big}", flush=True)
    res = {}
    for n in (n_big, n_small):
        plan = Plan(base.image_size, base.cellsize, base.n_radial, os_, np.full(n, s_max), s_max,
                    precision="fp32")
        _, sup, offs = plan.generate_truncated(taper, torch.from_numpy(w[:n]).cuda(), 0.01)
        res[n] = (sup.cpu().numpy(), offs.cpu().numpy())
        plan.close()
    sup_b, offs_b = res[n_big]
    assert np.array_equal(sup_b[:n_small], res[n_small][0])
    assert np.all((sup_b % 2 == 1) & (sup_b >= 1) & (sup_b <= s_max))
    expect = np.concatenate([[0], np.cumsum(os_ * os_ * sup_b.astype(np.int64) ** 2)])
    assert np.array_equal(offs_b, expect)


@pytest.mark.parametrize("precision", ["fp32", "bf16x6"])
@pytest.mark.parametrize("sig,os_,q", [(0.0035, 3, 1), (0.004, 8, 2), (0.007, 8, 1)])
def test_truncated_support_between_cells(precision, sig, os_, q):
    """Gaussian tapers whose 1% node k* is not a multiple of q os (the
    closed-form cases of the oracle's truncation pins): the device must round
    the half-width up, h = ceil(k* / (q os)), exactly as the oracle does;
    w = 0 and small |w| (still monotone, same k*) and a clamped plane."""
    import math
    from paper_1904_08463_amd import Plan
    base = W.plain(n_radial=2048)
    tau = np.ascontiguousarray(W.sample_taper(W.gaussian_taper(sig), 2048, base.r_max).astype(np.float32))
    w = np.array([0.0, 1.0, -1.0, 2.0], dtype=np.float64)
    sup_plan = np.array([63, 63, 63, 9], dtype=np.int32)  # the last plane is clamped
    print(f"case truncation between cells sig={sig} os={os_} q={q} {precision}", flush=True)
    plan = Plan(base.image_size, base.cellsize, 2048, os_, sup_plan, 63, radial_refine=q,
                precision=precision)
    out, sup, offs = plan.generate_truncated(torch.from_numpy(tau).cuda(),
                                             torch.from_numpy(w).cuda(), 0.01)
    out, sup, offs = out.cpu().numpy(), sup.cpu().numpy(), offs.cpu().numpy()
    geo = H.geometry(base.image_size, base.cellsize, 2048, os_, q)
    k_star = math.floor(math.sqrt(math.log(100.0) / (2 * math.pi ** 2 * sig ** 2)) / geo.drho)
    assert k_star % (q * os_) != 0
    h_expect = -(-k_star // (q * os_))
    for p in range(len(w)):
        caches, s_ref, _ = H.generate_truncated(base.image_size, base.cellsize, 2048, os_, tau, w,
                                                int(sup_plan[p]), radial_refine=q, planes=[p])
        assert sup[p] == s_ref[0], (p, sup[p], s_ref[0])
        if p < 3:
            assert sup[p] == 2 * h_expect + 1, (p, sup[p], h_expect)
        else:
            assert sup[p] == 9
        got = out[offs[p]:offs[p + 1]].reshape(caches[0].shape)
        e = float(np.max(np.abs(got - caches[0])) / np.max(np.abs(caches[0])))
        assert e <= GATE[precision], (p, e)
    plan.close()
