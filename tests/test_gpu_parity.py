"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Error metric per plane: e = max |K_gpu - K_ref| / max |K_ref| over the plane's
radial line or its whole kernel cache.  Gates: FP32 contraction <= 1e-5,
split-BF16 contraction <= 1e-6 (both are the accuracy targets of the two
arithmetic paths); layout, zeros outside the circular support and the
conjugate symmetry in w are checked exactly.
"""
import numpy as np
import pytest

import workloads as W
from oracle import hankel as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GATE = {"fp32": 1e-5, "bf16x6": 1e-6}


def _plan(wl, precision=None, interp=None):
    from paper_1904_08463_amd import Plan
    return Plan.from_workload(wl, precision=precision, interp=interp)


def _inputs(wl):
    taper = torch.from_numpy(np.ascontiguousarray(wl.taper)).cuda()
    w = torch.from_numpy(np.ascontiguousarray(wl.w)).cuda()
    return taper, w


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _check_cache(plan, flat_cpu, wl, planes, ref_caches, gate, tag):
    worst = 0.0
    for j, p in enumerate(planes):
        o0, o1 = int(plan.offsets[p]), int(plan.offsets[p + 1])
        got = flat_cpu[o0:o1].reshape(ref_caches[j].shape)
        ref = ref_caches[j]
        # exactly zero outside the circular support
        _, mask, _ = H.sample_positions(int(wl.support[p]), wl.oversampling, wl.radial_refine)
        assert np.all(got[~mask] == 0), f"{tag}: plane {p} nonzero outside support"
        e = _rel(got, ref)
        worst = max(worst, e)
        assert e <= gate, f"{tag}: plane {p} (w={wl.w[p]:.3f}, S={wl.support[p]}) error {e:.3e} > {gate}"
    print(f"{tag}: worst cache error {worst:.3e} over {len(planes)} planes", flush=True)
    return worst


def _check_lines(plan, lines_cpu, wl, planes, ref_lines, gate, tag):
    offs = np.concatenate([[0], np.cumsum(plan.nrho)])
    worst = 0.0
    for j, p in enumerate(planes):
        got = lines_cpu[offs[p]:offs[p + 1]]
        e = _rel(got, ref_lines[j])
        worst = max(worst, e)
        assert e <= gate, f"{tag}: plane {p} radial error {e:.3e} > {gate}"
    print(f"{tag}: worst radial error {worst:.3e}", flush=True)
    return worst


def _run_full(wl, precision, interp=None, planes=None):
    interp = interp or wl.interp
    print(f"case {wl.name} precision={precision} interp={interp} P={wl.n_planes} Nr={wl.n_radial}",
          flush=True)
    plan = _plan(wl, precision, interp)
    taper, w = _inputs(wl)
    lines = plan.generate_radial(taper, w).cpu().numpy()
    flat = plan.generate(taper, w).cpu().numpy()
    torch.cuda.synchronize()
    planes = list(range(wl.n_planes)) if planes is None else list(planes)
    caches, ref_lines = H.generate_workload(wl, planes=planes, interp=interp)
    _check_lines(plan, lines, wl, planes, ref_lines, GATE[precision], f"{wl.name}/{precision}")
    worst = _check_cache(plan, flat, wl, planes, caches, GATE[precision], f"{wl.name}/{precision}")
    plan.close()
    return worst


@pytest.mark.parametrize("precision", ["fp32", "bf16x6"])
def test_plain_workload(precision):
    _run_full(W.plain(), precision)


def test_precision_workload_bf16x6():
    """Plain workload through the split-BF16 contraction, FP64 phase: <= 1e-6."""
    _run_full(W.precision(), "bf16x6")


@pytest.mark.parametrize("precision", ["fp32", "bf16x6"])
def test_linear_interpolation(precision):
    _run_full(W.plain(), precision, interp="linear")


@pytest.mark.parametrize("q", [2, 4])
def test_radial_refinement(q):
    _run_full(W.plain(radial_refine=q), "bf16x6")


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
@pytest.mark.parametrize("precision", ["fp32", "bf16x6"])
def test_random_ragged(seed, precision):
    """Ragged radial lengths, Nr not a multiple of the tile sizes, odd and even
    oversampling, supports down to 1."""
    os_ = [1, 3, 4, 7][seed - 1]
    wl = W.random_small(seed, n_planes=37, n_radial=[96, 333, 64, 1000][seed - 1], os_=os_,
                        max_support=[21, 15, 33, 9][seed - 1])
    _run_full(wl, precision)


def test_single_plane_support_one():
    wl = W.random_small(9, n_planes=1, n_radial=50, os_=2, max_support=1)
    _run_full(wl, "fp32")


@pytest.mark.parametrize("precision", ["fp32", "bf16x6"])
def test_conjugate_symmetry_and_determinism(precision):
    """K(-w) = conj K(w) (section 4.1), and two generations of the same plan
    agree bit for bit.  The FP32 matrix-core sums are sign-symmetric, so the
    FP32 path is conjugate bit for bit; the BF16 matrix-core sums are not, so
    the split path is held to its accuracy gate."""
    wl = W.plain(extra_w=[-v for v in W.plain().w])
    plan = _plan(wl, precision)
    taper, w = _inputs(wl)
    a = plan.generate(taper, w).cpu().numpy()
    b = plan.generate(taper, w).cpu().numpy()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    for p in range(8):
        pos = a[plan.offsets[p]:plan.offsets[p + 1]]
        neg = a[plan.offsets[p + 8]:plan.offsets[p + 9]]
        if precision == "fp32":
            assert np.array_equal(neg, np.conj(pos))
        else:
            e = _rel(neg, np.conj(pos))
            print(f"plane {p}: |K(-w) - conj K(w)| / max = {e:.3e}", flush=True)
            assert e <= GATE[precision]
    plan.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16x6"])
def test_paper_workload_sampled_planes(precision):
    """2048^2 at 3.5 arcsec, 256 planes, Nr 4096, os 8, S 7..127: oracle on a
    spread of planes covering the support range."""
    wl = W.paper()
    planes = sorted(set([0, 1, 2, 40, 85, 128, 170, 200, 230, 254, 255]))
    _run_full(wl, precision, planes=planes)


def _batch_planes(wl, n=24):
    # stratified: every channel's extreme, several supports, both signs
    order = np.argsort(wl.support, kind="stable")
    pick = set(order[np.linspace(0, len(order) - 1, n).astype(int)].tolist())
    pick |= {0, 511, 512, 1023, 15 * 1024, 15 * 1024 + 1023}
    return sorted(pick)


@pytest.mark.parametrize("precision", ["bf16x6", "fp32"])
def test_batch_workload_full_size(precision):
    """16 channels x 1024 w-planes, Nr 8192, os 8, S 7..255, all 16384 kernels in
    one generate call (the benchmark's launch); oracle on a stratified subset."""
    wl = W.batch(precision=precision)
    planes = _batch_planes(wl)
    print(f"case batch precision={precision} planes={planes}", flush=True)
    plan = _plan(wl, precision)
    taper, w = _inputs(wl)
    flat = plan.generate(taper, w)
    torch.cuda.synchronize()
    got = {}
    for p in planes:
        got[p] = flat[int(plan.offsets[p]):int(plan.offsets[p + 1])].cpu().numpy()
    del flat
    caches, _ = H.generate_workload(wl, planes=planes)
    worst = 0.0
    for j, p in enumerate(planes):
        ref = caches[j]
        e = _rel(got[p].reshape(ref.shape), ref)
        worst = max(worst, e)
        assert e <= GATE[precision], f"plane {p} S={wl.support[p]} w={wl.w[p]:.1f}: {e:.3e}"
    print(f"batch/{precision}: worst error {worst:.3e} over {len(planes)} planes", flush=True)
    plan.close()


VARIANTS = ("wave32x64", "wave32x128", "lds128x128", "lds64x256", "ring128x128", "ring64x256",
            "ring32x512", "ringf128x128", "ringf64x256", "ringf64x256w8", "ringh64x256",
            "ringr64x256", "ringw64x256")
SPLIT_ONLY = ("ring128x128", "ring64x256", "ring32x512", "ringh64x256", "ringr64x256",
              "ringw64x256")


@pytest.mark.parametrize("precision", ["fp32", "bf16x6"])
@pytest.mark.parametrize("variant", VARIANTS)
def test_every_contraction_variant(variant, precision):
    """Every candidate the autotuner may pick, on ragged random planes (one K-chunk
    of 32 stages, and one of 16: Nr 96 pads to 256) and on sampled planes of
    the paper workload."""
    if precision == "fp32" and variant in SPLIT_ONLY:
        pytest.skip("split-BF16 only variant")
    for wl, planes in ((W.random_small(5, n_planes=45, n_radial=300, os_=5, max_support=41), None),
                       (W.random_small(7, n_planes=9, n_radial=96, os_=3, max_support=21), None),
                       (W.paper(), [0, 3, 100, 255])):
        print(f"case {wl.name} variant={variant} precision={precision}", flush=True)
        plan = _plan(wl, precision)
        plan.set_variant(variant)
        taper, w = _inputs(wl)
        lines = plan.generate_radial(taper, w).cpu().numpy()
        flat = plan.generate(taper, w).cpu().numpy()
        pl = list(range(wl.n_planes)) if planes is None else planes
        caches, ref_lines = H.generate_workload(wl, planes=pl)
        _check_lines(plan, lines, wl, pl, ref_lines, GATE[precision], f"{wl.name}/{variant}")
        _check_cache(plan, flat, wl, pl, caches, GATE[precision], f"{wl.name}/{variant}")
        plan.close()


def test_running_sum_variants_agree():
    """ringh64x256 keeps an FP64 running sum of every sub-chunk's sums,
    ringr64x256 an FP32 two-sum pair, and ringw64x256 an FP64 running sum of
    the 00 product with the small products left in FP32 over the K-chunk.
    Their radial lines agree to 1e-8 of each plane's peak, far inside the 1e-6
    gate (the emulated differences of the three sums are below 1e-9).  Their
    caches, where a line difference can move the FP32 spline coefficients by
    an ulp, agree within the split path's gate."""
    wl = W.paper()
    plan = _plan(wl, "bf16x6")
    taper, w = _inputs(wl)
    got = {}
    lines = {}
    for v in ("ringh64x256", "ringr64x256", "ringw64x256"):
        plan.set_variant(v)
        got[v] = plan.generate(taper, w).cpu().numpy()
        lines[v] = plan.generate_radial(taper, w).cpu().numpy()
    loffs = np.concatenate([[0], np.cumsum(plan.nrho)])
    for v in ("ringr64x256", "ringw64x256"):
        worst_l = worst_c = 0.0
        for p in range(wl.n_planes):
            a = lines[v][loffs[p]:loffs[p + 1]]
            b = lines["ringh64x256"][loffs[p]:loffs[p + 1]]
            worst_l = max(worst_l, float(np.max(np.abs(a - b)) / np.max(np.abs(b))))
            o0, o1 = int(plan.offsets[p]), int(plan.offsets[p + 1])
            a = got[v][o0:o1]
            b = got["ringh64x256"][o0:o1]
            worst_c = max(worst_c, float(np.max(np.abs(a - b)) / np.max(np.abs(b))))
        print(f"{v} vs ringh64x256: worst line difference {worst_l:.3e}, cache {worst_c:.3e}",
              flush=True)
        assert worst_l <= 1e-8
        assert worst_c <= GATE["bf16x6"]
    plan.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16x6"])
def test_pipeline_chunks_bitwise(precision):
    """Splitting the batch into pipeline chunks (the resample of one chunk
    overlapping the other stages of the next) changes no bit of the output."""
    wl = W.paper()
    plan = _plan(wl, precision)
    taper, w = _inputs(wl)
    plan.set_chunks(1)
    ref = plan.generate(taper, w).cpu().numpy()
    for chunks in (2, 5, 16):
        plan.set_chunks(chunks)
        assert plan.info()["chunks"] == chunks
        got = plan.generate(taper, w).cpu().numpy()
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), chunks
    plan.close()


@pytest.mark.parametrize("chunks", [1, 3])
def test_graph_replays_match_eager(chunks):
    """The captured graph, replayed several times with the program's own eager
    work (clearing the output) and synchronisations in between, reproduces the
    eager launches bit for bit on every replay; a new output pointer
    re-captures."""
    wl = W.paper()
    plan = _plan(wl, "bf16x6")
    plan.set_chunks(chunks)
    taper, w = _inputs(wl)
    plan.set_graph(False)
    ref = plan.generate(taper, w).cpu().numpy()
    plan.set_graph(True)
    out = torch.empty(int(plan.offsets[-1]), dtype=torch.complex64, device="cuda")
    for rep in range(4):
        out.zero_()
        torch.cuda.synchronize()
        plan.generate(taper, w, out)
        got = out.cpu().numpy()
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), rep
    out2 = torch.full_like(out, 7.0)
    plan.generate(taper, w, out2)
    assert np.array_equal(out2.cpu().numpy().view(np.uint64), ref.view(np.uint64))
    plan.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16x6"])
def test_mirrored_planes(precision):
    """Absolute w-term (section 4.1): planes declared as the -w mirror of
    another are written as its exact conjugate, and every plane still matches
    the oracle (which computes each plane on its own)."""
    base = W.plain()
    wl = W.plain(extra_w=[-v for v in base.w[::-1]])
    wl.mirror = W.mirror_table(wl.w, wl.support)
    assert (wl.mirror >= 0).sum() == 8
    _run_full(wl, precision)
    plan = _plan(wl, precision)
    taper, w = _inputs(wl)
    a = plan.generate(taper, w).cpu().numpy()
    lines = plan.generate_radial(taper, w).cpu().numpy()
    offs = np.concatenate([[0], np.cumsum(plan.nrho)])
    for p in range(wl.n_planes):
        q = wl.mirror[p]
        if q < 0:
            continue
        assert np.array_equal(a[plan.offsets[p]:plan.offsets[p + 1]],
                              np.conj(a[plan.offsets[q]:plan.offsets[q + 1]]))
        assert np.array_equal(lines[offs[p]:offs[p + 1]], np.conj(lines[offs[q]:offs[q + 1]]))
    plan.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16x6"])
def test_longest_radial_line(precision):
    """The largest radial line the plan accepts (2048 nodes: spline LDS of
    96 KB, resample LDS of 64 KB): S = 255 at os 8 with q = 2 gives 2036
    nodes; a short plane rides along in the same batch."""
    wl = W.paper(n_planes=2)
    wl.w = np.array([19000.0, 300.0])
    wl.support = np.array([255, 9], dtype=np.int32)
    wl.max_support = 255
    wl.radial_refine = 2
    _run_full(wl, precision)


@pytest.mark.parametrize("q,os_,smax", [(1, 8, 255), (2, 3, 151), (1, 2, 301), (1, 1, 301), (1, 5, 201)])
def test_full_cache_bitwise_equals_per_sample_evaluation(q, os_, smax):
    """The full-cache resample decodes each wave's first sample once and
    writes two samples per 16-byte store; the truncated path decodes every
    sample on its own and evaluates it with the shared per-sample routine.
    Both take the same FP32 steps, so at a threshold far below every node
    (supports stay full) the two caches agree bit for bit: S >= 128,
    64 <= S < 128 and S < 64, q = 1 and 2, os = 1 (no sub-kernel split),
    odd os (8-byte stores where a plane starts at an odd element; os = 5 by
    magic-number division), mirrored planes."""
    from paper_1904_08463_amd import Plan
    base = W.random_small(61, n_planes=2, n_radial=384, os_=os_, max_support=smax,
                          radial_refine=q)
    sup = [s for s in (smax, 201, 129, 127, 101, 65, 63, 33, 7, 3, 1) if s <= smax]
    rng = np.random.default_rng(7)
    w = rng.uniform(-1200.0, 1200.0, len(sup))
    # three planes repeated with -w: written as conjugates of their sources
    w2 = np.concatenate([w, -w[:3]])
    sup2 = np.array(sup + sup[:3], dtype=np.int32)
    mir = W.mirror_table(w2, sup2)
    assert (mir >= 0).sum() == 3
    plan = Plan(base.image_size, base.cellsize, base.n_radial, os_, sup2, smax,
                radial_refine=q, precision="bf16x6", mirror=mir)
    taper = torch.from_numpy(base.taper).cuda()
    wd = torch.from_numpy(w2).cuda()
    full = plan.generate(taper, wd)
    tr, sup_t, offs_t = plan.generate_truncated(taper, wd, frac=1e-30)
    torch.cuda.synchronize()
    print(f"q={q} os={os_}: supports {sup2.tolist()}", flush=True)
    assert np.array_equal(sup_t.cpu().numpy(), sup2)
    assert np.array_equal(offs_t.cpu().numpy(), plan.offsets)
    assert torch.equal(full.view(torch.int32), tr.view(torch.int32))
    plan.close()
