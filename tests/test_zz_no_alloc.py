"""wkern_wpartition_noalloc (the partition with the library's static device
scratch instead of a caller workspace) against wkern_wpartition with a
workspace, through the C ABI: record order, plane starts and plane w-terms
bit for bit, on two calls in a row (the second with fewer records, so the
scratch holds the first call's contents), and no device memory taken by a
call."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _free():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return torch.cuda.mem_get_info()[0]


def _reference(wd, m, absolute, stat):
    from paper_1904_08463_amd import wpartition
    return wpartition(wd, m, absolute=absolute, stat=stat)


def test_noalloc_matches_workspace_path():
    from paper_1904_08463_amd import wpartition_noalloc
    rng = np.random.default_rng(77)
    big = W.vla_c_74mhz_w()                                  # 505440 records
    small = rng.choice(np.array([-3.0, -0.0, 0.0, 1.5, 2.25, 7.0, np.nan, np.inf]), 100003)
    small[::7] = rng.normal(0.0, 500.0, small[::7].size)     # ties, signed zeros, NaN, inf
    cases = [(big, 128, True, "mean"), (small, 37, False, "median")]
    for i, (w, m, absolute, stat) in enumerate(cases):
        print(f"case noalloc call {i}: n={w.size} M={m} absolute={absolute} stat={stat}", flush=True)
        wd = torch.from_numpy(np.ascontiguousarray(w)).cuda()
        order = torch.empty(w.size, dtype=torch.int32, device="cuda")
        start = torch.empty(m + 1, dtype=torch.int64, device="cuda")
        wp = torch.empty(m, dtype=torch.float64, device="cuda")
        before = _free()
        wpartition_noalloc(wd, m, absolute=absolute, stat=stat, order=order, plane_start=start,
                           w_plane=wp)
        if i > 0:
            assert _free() == before  # the call allocated nothing
        o_ref, s_ref, w_ref = _reference(wd, m, absolute, stat)
        assert torch.equal(order, o_ref)
        assert torch.equal(start, s_ref)
        a, b = wp.cpu().numpy(), w_ref.cpu().numpy()
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_noalloc_rejects_too_many_records():
    from paper_1904_08463_amd import wpartition_noalloc
    from paper_1904_08463_amd.wkern import NOALLOC_MAX_RECORDS, WkernError
    wd = torch.zeros(NOALLOC_MAX_RECORDS + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(WkernError) as ei:
        wpartition_noalloc(wd, 4)
    assert ei.value.status == 1 and "static scratch" in str(ei.value)
    # the largest accepted size works
    w = np.random.default_rng(3).normal(0.0, 1e3, NOALLOC_MAX_RECORDS)
    wd = torch.from_numpy(w).cuda()
    o, s, wp = wpartition_noalloc(wd, 256)
    o_ref, s_ref, w_ref = _reference(wd, 256, True, "mean")
    assert torch.equal(o, o_ref) and torch.equal(s, s_ref) and torch.equal(wp, w_ref)
