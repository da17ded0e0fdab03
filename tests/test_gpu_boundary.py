"""Boundary behaviour of the C ABI on the GPU: the device status word
(WKERN_ERR_NONFINITE through wkern_sync_status), host-side fault injection
(WKERN_FAULT: allocation, launch and capture failures release what they
allocated and leave the plan usable), the persistent tuning cache
(WKERN_TUNE_CACHE), and guard regions around the output buffer (no write
outside a plane's block)."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import hankel as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NONFINITE, OOM, DEVICE = 6, 2, 3


@pytest.fixture
def env():
    """Set environment variables for one test and restore them afterwards."""
    saved = {}

    def set_(name, value):
        if name not in saved:
            saved[name] = os.environ.get(name)
        if value is None:
            os.environ.pop(name, None)
        else:
            os.environ[name] = value
    yield set_
    for name, value in saved.items():
        if value is None:
            os.environ.pop(name, None)
        else:
            os.environ[name] = value


def _inputs(wl):
    return (torch.from_numpy(np.ascontiguousarray(wl.taper)).cuda(),
            torch.from_numpy(np.ascontiguousarray(wl.w)).cuda())


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _check_against_oracle(plan, flat, wl, gate):
    caches, _ = H.generate_workload(wl)
    for p in range(wl.n_planes):
        got = flat[plan.offsets[p]:plan.offsets[p + 1]].reshape(caches[p].shape)
        assert _rel(got, caches[p]) <= gate, p


# ---------------------------------------------------------------------------
# device status word
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("graph", [True, False])
def test_nonfinite_w_flags_its_plane(graph):
    from paper_1904_08463_amd import Plan
    from paper_1904_08463_amd.wkern import WkernError
    wl = W.plain()
    plan = Plan.from_workload(wl, precision="bf16x6")
    plan.set_graph(graph)
    taper, w = _inputs(wl)
    plan.generate(taper, w)
    plan.sync_status()  # clean inputs: no flag
    for bad in (float("nan"), float("inf"), -float("inf")):
        wb = w.clone()
        wb[5] = bad
        wb[3] = bad
        plan.generate(taper, wb)
        with pytest.raises(WkernError) as ei:
            plan.sync_status()
        assert ei.value.status == NONFINITE
        assert "plane 3" in str(ei.value), str(ei.value)
        plan.sync_status()  # the read cleared the word
    # the plan still generates correct kernels afterwards
    flat = plan.generate(taper, w).cpu().numpy()
    plan.sync_status()
    _check_against_oracle(plan, flat, wl, 1e-6)
    plan.close()


def test_nonfinite_taper_flags_every_path():
    """A NaN taper sample reaches every plane's line: flagged through the
    plain, truncated and radial-line calls; the first plane is 0."""
    from paper_1904_08463_amd import Plan
    from paper_1904_08463_amd.wkern import WkernError
    wl = W.plain()
    plan = Plan.from_workload(wl)
    taper, w = _inputs(wl)
    tb = taper.clone()
    tb[17] = float("nan")
    calls = (lambda: plan.generate(tb, w), lambda: plan.generate_truncated(tb, w, 0.01),
             lambda: plan.prepare_lines(tb, w))
    for call in calls:
        call()
        with pytest.raises(WkernError) as ei:
            plan.sync_status()
        assert ei.value.status == NONFINITE and "plane 0" in str(ei.value)
    plan.generate(taper, w)
    plan.sync_status()
    plan.close()


# ---------------------------------------------------------------------------
# fault injection
# ---------------------------------------------------------------------------
def _free_bytes():
    """Free device memory with torch's cached blocks returned to the device
    (the library allocates with hipMalloc, outside torch's allocator)."""
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("nth", [1, 4, 9])
def test_injected_allocation_failure_leaks_nothing(env, nth):
    from paper_1904_08463_amd import Plan
    from paper_1904_08463_amd.wkern import WkernError
    wl = W.paper(n_planes=64, n_radial=1024)
    # one full plan first, so that runtime state created on first use (code
    # objects, streams) is not counted
    Plan.from_workload(wl, precision="bf16x6").close()
    before = _free_bytes()
    env("WKERN_FAULT", f"alloc:{nth}")
    with pytest.raises(WkernError) as ei:
        Plan.from_workload(wl, precision="bf16x6")
    assert ei.value.status == OOM and "injected" in str(ei.value)
    env("WKERN_FAULT", None)
    assert _free_bytes() == before
    # a plan made afterwards is whole
    plan = Plan.from_workload(wl, precision="bf16x6")
    taper, w = _inputs(wl)
    flat = plan.generate(taper, w).cpu().numpy()
    caches, _ = H.generate_workload(wl, planes=[0, 31, 63])
    for j, p in enumerate([0, 31, 63]):
        got = flat[plan.offsets[p]:plan.offsets[p + 1]].reshape(caches[j].shape)
        assert _rel(got, caches[j]) <= 1e-6
    plan.close()
    del taper, w
    assert _free_bytes() == before


def test_injected_allocation_failure_in_first_gradient(env):
    """The adjoint allocates its scratch on its first call: a failure there
    releases the part already allocated, and the next call succeeds."""
    from paper_1904_08463_amd import Plan
    from paper_1904_08463_amd.wkern import WkernError
    wl = W.plain()
    plan = Plan.from_workload(wl)
    taper, w = _inputs(wl)
    g = torch.ones(int(plan.offsets[-1]), dtype=torch.complex64, device="cuda")
    before = _free_bytes()
    env("WKERN_FAULT", "alloc:3")
    with pytest.raises(WkernError) as ei:
        plan.grad(taper, w, g)
    assert ei.value.status == OOM
    env("WKERN_FAULT", None)
    assert _free_bytes() == before
    gt1, gw1 = plan.grad(taper, w, g)
    gt2, gw2 = plan.grad(taper, w, g)
    assert torch.equal(gt1, gt2) and torch.equal(gw1, gw2)
    assert torch.isfinite(gt1).all() and torch.isfinite(gw1).all()
    plan.close()


@pytest.mark.parametrize("site", ["launch:1", "launch:2", "launch:3", "capture"])
@pytest.mark.parametrize("graph", [True, False])
def test_injected_launch_or_capture_failure(env, site, graph):
    from paper_1904_08463_amd import Plan
    from paper_1904_08463_amd.wkern import WkernError
    if site == "capture" and not graph:
        pytest.skip("no capture without the graph")
    wl = W.plain()
    plan = Plan.from_workload(wl, precision="bf16x6")
    plan.set_graph(graph)
    taper, w = _inputs(wl)
    out = torch.zeros(int(plan.offsets[-1]), dtype=torch.complex64, device="cuda")
    env("WKERN_FAULT", site)
    with pytest.raises(WkernError) as ei:
        plan.generate(taper, w, out=out)
    assert ei.value.status == DEVICE and "injected" in str(ei.value)
    env("WKERN_FAULT", None)
    torch.cuda.synchronize()
    # the same pointers again: generated whole
    plan.generate(taper, w, out=out)
    _check_against_oracle(plan, out.cpu().numpy(), wl, 1e-6)
    plan.close()


# ---------------------------------------------------------------------------
# tuning cache
# ---------------------------------------------------------------------------
def test_tuning_cache_round_trip(env, tmp_path):
    from paper_1904_08463_amd import Plan
    wl = W.paper(n_planes=96, n_radial=2048)
    path = tmp_path / "tune.txt"
    env("WKERN_TUNE_CACHE", str(path))
    a = Plan.from_workload(wl, precision="bf16x6")
    ia = a.info()
    a.close()
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and "|prec1|" in lines[0] and "|abi3|" in lines[0]
    assert "|rev" in lines[0]
    # a second plan of the same geometry takes the stored result unchanged
    b = Plan.from_workload(wl, precision="bf16x6")
    assert b.info() == ia
    b.close()
    assert len(path.read_text().splitlines()) == 1
    # an edited entry is obeyed (the choice is read, not re-timed)
    key, _, rest = lines[0].split(" ", 2)
    other = "ringf64x256" if ia["variant"] != "ringf64x256" else "ringf128x128"
    path.write_text(f"{key} {Plan.VARIANTS.index(other)} {rest}\n")
    c = Plan.from_workload(wl, precision="bf16x6")
    assert c.info()["variant"] == other
    taper, w = _inputs(wl)
    flat = c.generate(taper, w).cpu().numpy()
    caches, _ = H.generate_workload(wl, planes=[0, 95])
    for j, p in enumerate([0, 95]):
        got = flat[c.offsets[p]:c.offsets[p + 1]].reshape(caches[j].shape)
        assert _rel(got, caches[j]) <= 1e-6
    c.close()
    # another precision is another key
    d = Plan.from_workload(wl, precision="fp32")
    d.close()
    assert len(path.read_text().splitlines()) == 2
    # an entry made with another kernel revision is not reused: the plan
    # times its candidates again and appends its own entry
    rev = key.split("|rev")[1].split("|")[0]
    stale = key.replace(f"|rev{rev}|", f"|rev{int(rev) - 1}|")
    path.write_text(f"{stale} {Plan.VARIANTS.index(other)} {rest}\n")
    e = Plan.from_workload(wl, precision="bf16x6")
    assert e.info()["variant"] != other
    e.close()
    kept = path.read_text().splitlines()
    assert len(kept) == 2 and kept[0].startswith(stale + " ") and kept[1].startswith(key + " ")


# ---------------------------------------------------------------------------
# output guard regions
# ---------------------------------------------------------------------------
def _mirrored_plain():
    base = W.plain()
    wl = W.plain(extra_w=[-v for v in base.w[::2]])
    wl.mirror = W.mirror_table(wl.w, wl.support)
    assert np.sum(wl.mirror >= 0) == 4
    return wl


@pytest.mark.parametrize("truncated", [False, True])
@pytest.mark.parametrize("make", [lambda: W.random_small(11, n_planes=23, n_radial=333, os_=3,
                                                         max_support=25), _mirrored_plain],
                         ids=["ragged_os3", "mirrored"])
def test_output_guard_regions_untouched(truncated, make):
    """The cache is generated into the middle of a larger buffer filled with
    a sentinel: the elements before and after it keep their bits (ragged
    supports at os 3; mirrored planes)."""
    from paper_1904_08463_amd import Plan
    wl = make()
    plan = Plan.from_workload(wl, precision="bf16x6")
    taper, w = _inputs(wl)
    total = int(plan.offsets[-1])
    guard = 4099
    buf = torch.empty(total + 2 * guard, dtype=torch.complex64, device="cuda")
    sentinel = complex(np.float32(1.25e-3), np.float32(-7.5e2))
    buf.fill_(sentinel)
    view = buf[guard:guard + total]
    if truncated:
        plan.generate_truncated(taper, w, 0.01, out=view)
    else:
        plan.generate(taper, w, out=view)
    host = buf.cpu().numpy()
    assert np.all(host[:guard] == np.complex64(sentinel))
    assert np.all(host[guard + total:] == np.complex64(sentinel))
    if not truncated:
        _check_against_oracle(plan, host[guard:guard + total], wl, 1e-6)
    plan.close()


def test_store_ceiling_diagnostic():
    """wkern_store_ceiling writes zeros over the buffer in both store
    structures and rejects misaligned or partial sizes."""
    import ctypes
    from paper_1904_08463_amd import load_library, store_ceiling
    buf = torch.full((3 * 65536 * 2 + 48,), 7.0, dtype=torch.float32, device="cuda")
    for pattern in ("one_store_per_lane", "unit_walk"):
        buf.fill_(7.0)
        store_ceiling(buf, pattern)
        assert torch.count_nonzero(buf).item() == 0
    lib = load_library()
    p = ctypes.c_void_p(buf.data_ptr())
    assert lib.wkern_store_ceiling(p, 24, 0, None) == 1          # not a multiple of 16
    assert lib.wkern_store_ceiling(ctypes.c_void_p(buf.data_ptr() + 4), 16, 0, None) == 1
    assert lib.wkern_store_ceiling(p, 16, 2, None) == 1          # unknown pattern
    assert lib.wkern_store_ceiling(None, 16, 0, None) == 1
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# debug canaries around the plan's own allocations
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision,variant", [("bf16x6", "ringw64x256"), ("bf16x6", "ringr64x256"),
                                               ("bf16x6", "ringh64x256"), ("bf16x6", "wave32x64"),
                                               ("fp32", None)])
def test_canaries_hold_on_every_path(env, precision, variant):
    """WKERN_CANARY=1: every allocation of the plan carries guard bands.
    After the plain (graph and eager), truncated, radial-line, gradient,
    gridding and projection-slice calls on ragged supports at os 3, none
    changed, and the caches still match the oracle; a byte changed by the
    host hook is reported with the buffer named, and the band is refilled."""
    from paper_1904_08463_amd import Plan, wpartition
    from paper_1904_08463_amd.wkern import WkernError
    wl = W.random_small(11, n_planes=23, n_radial=333, os_=3, max_support=25)
    env("WKERN_CANARY", "1")
    print(f"case canaries {precision} {variant}", flush=True)
    plan = Plan.from_workload(wl, precision=precision)
    env("WKERN_CANARY", None)
    if variant is not None:
        plan.set_variant(variant)
    taper, w = _inputs(wl)
    for graph in (True, False):
        plan.set_graph(graph)
        flat = plan.generate(taper, w).cpu().numpy()
        plan.sync_status()
        _check_against_oracle(plan, flat, wl, 1e-6 if precision == "bf16x6" else 1e-5)
    plan.generate_truncated(taper, w, 0.01)
    plan.generate_radial(taper, w)
    plan.sync_status()
    g = torch.ones(int(plan.offsets[-1]), dtype=torch.complex64, device="cuda")
    plan.grad(taper, w, g)
    plan.sync_status()
    # gridding: records spread over the planes' w range, fused and from the cache
    rng = np.random.default_rng(5)
    n, n_rec = 256, 4000
    du = 1.0 / (wl.image_size * wl.cellsize)
    rec_w = rng.uniform(wl.w.min(), wl.w.max(), n_rec)
    uv = rng.uniform(-0.4 * n * du, 0.4 * n * du, (2, n_rec))
    vis = (rng.standard_normal(n_rec) + 1j * rng.standard_normal(n_rec)).astype(np.complex64)
    order_d, start_d, wp_d = wpartition(torch.from_numpy(rec_w).cuda(), wl.n_planes)
    sup_d = plan.prepare_lines(taper, wp_d)
    args = tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (uv[0], uv[1], rec_w, vis))
    plan.grid(*args, order_d, start_d, sup_d, torch.zeros((n, n), dtype=torch.complex64, device="cuda"))
    cache = plan.generate(taper, wp_d)
    plan.grid(*args, order_d, start_d, sup_d, torch.zeros((n, n), dtype=torch.complex64, device="cuda"),
              cache=cache, cache_offsets=torch.from_numpy(plan.offsets).cuda())
    plan.sync_status()
    plan.set_engine("projection_slice", "per_plane")
    plan.generate(taper, w)
    plan.sync_status()
    plan.set_engine("matrix")
    # the detection path, through a byte the host changes in a guard band
    env("WKERN_FAULT", "canary")
    with pytest.raises(WkernError) as ei:
        plan.sync_status()
    env("WKERN_FAULT", None)
    assert ei.value.status == DEVICE and "canary overwritten after" in str(ei.value), str(ei.value)
    plan.sync_status()  # refilled
    plan.close()  # checks the bands once more


def test_canary_reported_at_destroy(env):
    """With canaries on, destroying the plan checks the bands: a byte the host
    hook changes is reported by wkern_destroy, and the plan is released all
    the same (a second close is a no-op)."""
    from paper_1904_08463_amd import Plan
    from paper_1904_08463_amd.wkern import WkernError
    wl = W.plain()
    env("WKERN_CANARY", "1")
    plan = Plan.from_workload(wl)
    env("WKERN_CANARY", None)
    taper, w = _inputs(wl)
    plan.generate(taper, w)
    env("WKERN_FAULT", "canary")
    with pytest.raises(WkernError) as ei:
        plan.close()
    env("WKERN_FAULT", None)
    assert ei.value.status == DEVICE and "canary" in str(ei.value)
    plan.close()
