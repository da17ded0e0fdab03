"""w-plane partition on the GPU against the oracle (Algorithms 1 and 2,
sort / equal-size planes / mean or median).  Index work (order, plane
starts) and medians are compared bit for bit; means to 1e-13 relative
(|w|) or 1e-12 of the plane's largest |w| (signed w): the device sums in a
fixed order, the oracle rounds the exact sum once."""
import numpy as np
import pytest

import workloads as W
from oracle import hankel as H
from oracle import wpartition as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _run(w, m, absolute, stat):
    from paper_1904_08463_amd import wpartition
    order, start, wp = wpartition(torch.from_numpy(w).cuda(), m, absolute=absolute, stat=stat)
    return order.cpu().numpy(), start.cpu().numpy(), wp.cpu().numpy()


def _check(w, m, absolute, stat):
    order, start, wp = _run(w, m, absolute, stat)
    o_ref, s_ref, wp_ref = P.partition(w, m, absolute=absolute, stat=stat)
    assert np.array_equal(order, o_ref)
    assert np.array_equal(start, s_ref)
    key = P.sort_key(w, absolute)[o_ref]
    if stat == "median":
        assert np.array_equal(wp, wp_ref, equal_nan=True)
    else:
        for k in range(m):
            seg = key[s_ref[k]:s_ref[k + 1]]
            if not np.all(np.isfinite(seg)):
                assert (np.isnan(wp[k]) and np.isnan(wp_ref[k])) or wp[k] == wp_ref[k]
                continue
            scale = np.max(np.abs(seg)) if not absolute else abs(wp_ref[k])
            tol = (1e-13 if absolute else 1e-12) * max(scale, np.finfo(float).tiny)
            assert abs(wp[k] - wp_ref[k]) <= tol, (k, wp[k], wp_ref[k])
    return order, start, wp


@pytest.mark.parametrize("absolute", [True, False])
@pytest.mark.parametrize("stat", ["mean", "median"])
def test_paper_shaped_records(absolute, stat):
    w = W.vla_c_74mhz_w()
    print(f"case vla 505440 records, 128 planes, absolute={absolute}, {stat}", flush=True)
    _check(w, 128, absolute, stat)


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("absolute", [True, False])
def test_ragged_ties_and_special_values(seed, absolute):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 3000))
    w = rng.choice([-3.0, -1.0, -0.0, 0.0, 1.0, 2.5, 3.0, np.inf, -np.inf, np.nan], n)
    w = np.where(rng.random(n) < 0.6, w, rng.normal(0, 100, n))
    m = int(rng.choice([1, n, max(1, n // 7), min(n, 3)]))
    print(f"case ragged seed={seed} n={n} m={m} absolute={absolute}", flush=True)
    for stat in ("mean", "median"):
        _check(w, m, absolute, stat)


def test_multichannel_records_and_determinism():
    w = W.multichannel_w(W.vla_c_74mhz_w(), 33)  # 16.7 M records
    print(f"case multichannel n={w.size}", flush=True)
    order, start, wp = _check(w, 256, True, "mean")
    order2, start2, wp2 = _run(w, 256, True, "mean")
    assert np.array_equal(order, order2) and np.array_equal(wp.view(np.int64), wp2.view(np.int64))


def test_rejects_bad_arguments():
    from paper_1904_08463_amd import wpartition, wpartition_workspace
    from paper_1904_08463_amd.wkern import WkernError
    w = torch.zeros(10, dtype=torch.float64, device="cuda")
    with pytest.raises(WkernError):
        wpartition(w, 11)
    with pytest.raises(WkernError):
        wpartition(w, 0)
    small = torch.empty(wpartition_workspace(10) - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(WkernError):
        wpartition(w, 2, workspace=small)


def test_partition_feeds_generation():
    """Plane w-terms stay on the device and go straight into generate."""
    from paper_1904_08463_amd import Plan, wpartition
    w = W.vla_c_74mhz_w()
    _, _, wp_dev = wpartition(torch.from_numpy(w).cuda(), 16, absolute=True, stat="mean")
    _, _, wp_ref = P.partition(w, 16)
    wl = W.plain()
    plan = Plan(wl.image_size, wl.cellsize, wl.n_radial, wl.oversampling, [31] * 16, 31)
    out = plan.generate(torch.from_numpy(wl.taper).cuda(), wp_dev)
    got = out.cpu().numpy()
    caches, _ = H.generate(wl.image_size, wl.cellsize, wl.n_radial, wl.oversampling, wl.taper,
                           wp_ref, [31] * 16)
    for p in range(16):
        ref = caches[p].reshape(-1)
        seg = got[int(plan.offsets[p]):int(plan.offsets[p + 1])]
        assert np.max(np.abs(seg - ref)) / np.max(np.abs(ref)) <= 1e-5
    plan.close()
