#!/usr/bin/env python3
"""Throughput of batched w-kernel generation on one MI355X.

Workload: 16 channels (1.0-1.5 GHz) x 1024 w-planes with 1/|w| density on
+-[40, 40000] lambda, 2048^2 image at 3.5 arcsec, prolate-spheroidal taper
(m = 6, alpha = 1) on Nr = 8192 radial nodes, supports 7..255 px, oversampling
8: 16384 kernel caches (30.6 GB of complex64) per step, all in one generate
call.  A step is one whole generate call (screen, Hankel contraction, spline,
resample) with the inputs already resident in device memory.

The headline value is the split-BF16 path; the FP32 path is timed on the
same inputs and reported beside it.  One JSON line is printed.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"bf16x6": 2500.0, "fp32": 157.3}  # dense BF16 / FP32 matrix peaks
# HBM bytes per k_resample launch from two counter runs (FETCH_SIZE, WRITE_SIZE),
# valid only for the kernel sources they were taken with
COUNTERS = os.path.join(ROOT, "profiles", "k_resample_batch_counters.txt")
RESAMPLE_SOURCES = ("paper_1904_08463_amd/csrc/wkern_resample.hip",
                    "paper_1904_08463_amd/csrc/wkern_radial.h",
                    "paper_1904_08463_amd/csrc/wkern_tables.h")


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the single-thread oracle and host 2D-FFT timings")
    ap.add_argument("--cpu-stride", type=int, default=4,
                    help="oracle sample: every n-th plane by w of each (channel, support) group")
    ap.add_argument("--skip-fp32", action="store_true")
    ap.add_argument("--skip-fft", action="store_true")
    ap.add_argument("--fft-steps", type=int, default=2)
    ap.add_argument("--skip-projslice", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="counter pass: one warm and one measured generate of the split path, "
                         "then a 2 GiB device copy as the reference for the byte counters")
    return ap.parse_args()


def _time_path(plan, taper, w, out, steps, warmup):
    """Wall time of `steps` generate calls (captured-graph replays), then a
    separate pass with per-stage HIP events (kernels launched one by one on
    the same stream) for the stage split."""
    import torch
    for _ in range(warmup):
        plan.generate(taper, w, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.generate(taper, w, out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.set_profiling(True)
    for _ in range(steps):
        plan.generate(taper, w, out)
    stages, calls = plan.stage_times()
    plan.set_profiling(False)
    return wall, {k: v / max(calls, 1) for k, v in stages.items()}


def resample_source_digest() -> str:
    h = hashlib.sha256()
    for f in RESAMPLE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _measured_traffic():
    """HBM bytes per k_resample launch (FETCH + WRITE, each scaled by what
    the counter reads for a copy of known size), or None when the summary is
    missing or the resample sources changed after the counters were taken."""
    try:
        with open(COUNTERS) as fh:
            text = fh.read()
    except OSError:
        return None
    kv = dict(re.findall(r"^(source_sha256|traffic_bytes_per_launch):\s*(\S+)", text, re.M))
    if kv.get("source_sha256") != resample_source_digest() or "traffic_bytes_per_launch" not in kv:
        return None
    return float(kv["traffic_bytes_per_launch"])


def _contraction_roofline(plan, wl, stages, precision):
    """MFMA roofline of the Hankel contraction: algorithmic 4 Nr Nrho FLOP per
    computed plane (mirrored planes are not contracted); the split path
    executes six BF16 products per algorithmic one."""
    nrho = plan.nrho.astype(np.float64)
    computed = np.ones(wl.n_planes, dtype=bool) if plan.mirror is None else plan.mirror < 0
    flop = 4.0 * wl.n_radial * float(nrho[computed].sum())
    executed = flop * (6.0 if precision == "bf16x6" else 1.0)
    ms = stages["contraction"]
    achieved = executed / (ms * 1e-3) / 1e12
    peak = MFMA_PEAK_TFLOPS[precision]
    res = {"bound": "mfma", "kernel": "k_contract_*", "achieved": achieved, "peak": peak,
           "unit": "TFLOP/s", "frac": achieved / peak, "algorithmic_flop": flop,
           "executed_flop": executed, "ms": ms}
    if precision == "bf16x6":
        # the split contraction's utilisation target and how far it is from it
        res["target_frac"] = 0.60
        res["ms_at_target"] = executed / (0.60 * peak * 1e12) * 1e3
    return res


def _fft_paths(wl, taper, w, out, steps):
    """The standard algorithm (zero-padded 2D FFT per plane) on the same GPU:
    the paper's fixed workspace (power of two >= max support) and a per-plane
    workspace (power of two >= S_p)."""
    import torch
    from oracle import fft2d as F
    from paper_1904_08463_amd import FFT2DPlan
    res = {}
    fov = wl.image_size * wl.cellsize
    tfn = F.taper_from_samples(wl.taper, 0.5 * fov)
    order = np.argsort(wl.support, kind="stable")
    check = sorted(set(order[[0, 9000]].tolist()))
    for mode in ("max_support", "per_plane"):
        plan = FFT2DPlan.from_workload(wl, workspace=mode)
        plan.generate(taper, w, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.generate(taper, w, out)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        worst = 0.0
        for p in check:
            s = int(wl.support[p])
            n_ws = F.next_pow2(wl.max_support if mode == "max_support" else s)
            ref = F.generate(tfn, [wl.w[p]], [s], wl.oversampling, n_ws, fov)[0].reshape(-1)
            got = out[int(plan.offsets[p]):int(plan.offsets[p + 1])].cpu().numpy()
            worst = max(worst, float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
        plan.close()
        res[f"fft2d_{mode}"] = {"kernels_per_s": wl.n_planes / wall, "ms_per_step": 1000.0 * wall,
                                "steps": steps, "max_rel_err_sampled_vs_2d_twin": worst}
    return res


def _projslice_paths(wl, taper, w, out, steps):
    """The projection-slice engine (section 4.3.1) on the same batch: per-plane
    and fixed workspaces.  Errors on sampled planes against the oracle's
    projection-slice chain (parity) and against the matrix-form oracle (the
    difference between the two discretisations)."""
    from oracle import fft2d as F
    from oracle import hankel as H
    from oracle import projslice as PS
    from paper_1904_08463_amd import Plan
    fov = wl.image_size * wl.cellsize
    tfn = F.taper_from_samples(wl.taper, 0.5 * fov)
    order = np.argsort(wl.support, kind="stable")
    check = sorted(set(order[[0, 8000, 16000]].tolist()))
    ref_h, _ = H.generate_workload(wl, planes=check)
    res = {}
    for mode in ("per_plane", "max_support"):
        plan = Plan.from_workload(wl, precision="bf16x6")
        plan.set_engine("projection_slice", mode)
        wall, stages = _time_path(plan, taper, w, out, steps, 1)
        fixed = wl.max_support if mode == "max_support" else None
        ref_ps, _ = PS.generate(tfn, wl.w[check], wl.support[check], wl.oversampling, fov,
                                wl.radial_refine, wl.interp, fixed)
        e_ps = e_h = 0.0
        for j, p in enumerate(check):
            got = out[int(plan.offsets[p]):int(plan.offsets[p + 1])].cpu().numpy()
            a, b = ref_ps[j].reshape(-1), ref_h[j].reshape(-1)
            e_ps = max(e_ps, float(np.max(np.abs(got - a)) / np.max(np.abs(a))))
            e_h = max(e_h, float(np.max(np.abs(got - b)) / np.max(np.abs(b))))
        res[f"projection_slice_{mode}"] = {
            "kernels_per_s": wl.n_planes / (wall / steps), "ms_per_step": 1000.0 * wall / steps,
            "stage_ms": stages, "max_rel_err_sampled_vs_projslice_oracle": e_ps,
            "max_rel_diff_sampled_vs_matrix_form_oracle": e_h}
        plan.close()
    return res


def _gridding_paths(steps):
    """The paper's imaging setting on the synthetic records (IM-S 2048^2 at 60
    arcsec, 128 |w|-planes of 505440 records at 74 MHz, os 8, supports up to
    255 with 1% truncation, split-BF16): partition, kernels and gridding,
    once with the fused consumer (no kernel cache) and once through a
    written cache."""
    import torch
    import workloads as W
    from paper_1904_08463_amd import Plan, wpartition, wpartition_workspace
    gw = W.grid_paper()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    u, v, w, vis, taper = dev(gw.u), dev(gw.v), dev(gw.w), dev(gw.vis), dev(gw.taper)
    n = gw.grid_size
    plan = Plan(gw.image_size, gw.cellsize, gw.n_radial, gw.oversampling,
                [gw.max_support] * gw.n_planes, gw.max_support, precision="bf16x6")
    ws = torch.empty(wpartition_workspace(gw.u.size), dtype=torch.uint8, device="cuda")
    grid = torch.zeros((n, n), dtype=torch.complex64, device="cuda")
    sup = torch.empty(gw.n_planes, dtype=torch.int32, device="cuda")
    cache = torch.empty(int(plan.offsets[-1]), dtype=torch.complex64, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def fused():
        order, start, wp = wpartition(w, gw.n_planes, workspace=ws)
        ev[0].record()
        plan.prepare_lines(taper, wp, frac=gw.frac, support_out=sup)
        ev[1].record()
        grid.zero_()
        ev[2].record()
        plan.grid(u, v, w, vis, order, start, sup, grid)
        ev[3].record()

    def cached():
        order, start, wp = wpartition(w, gw.n_planes, workspace=ws)
        ev[0].record()
        _, s2, offs = plan.generate_truncated(taper, wp, gw.frac, out=cache)
        ev[1].record()
        grid.zero_()
        ev[2].record()
        plan.grid(u, v, w, vis, order, start, s2, grid, cache=cache, cache_offsets=offs)
        ev[3].record()

    res = {}
    for name, fn in (("fused", fused), ("through_cache", cached)):
        fn()
        torch.cuda.synchronize()
        kern = grd = 0.0
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
            torch.cuda.synchronize()
            kern += ev[0].elapsed_time(ev[1])
            grd += ev[2].elapsed_time(ev[3])
        wall = (time.perf_counter() - t0) / steps
        res[name] = {"records_per_s": gw.u.size / wall, "ms_per_step": 1000.0 * wall,
                     "kernels_ms": kern / steps, "gridding_ms": grd / steps,
                     "n_records": int(gw.u.size), "n_planes": gw.n_planes, "grid": n}
    sup_h = sup.cpu().numpy()
    res["supports"] = [int(sup_h.min()), int(np.median(sup_h)), int(sup_h.max())]
    res["cache_bytes_avoided"] = int(8 * gw.oversampling ** 2 * np.sum(sup_h.astype(np.int64) ** 2))
    plan.close()
    return res


def _gradient_path(steps):
    """Differentiation workload (256 planes of 2048 free taper samples, S 127,
    os 4): one forward generate and one adjoint (dL/dtaper, dL/dw from a
    dL/dcache of the cache's size), split-BF16 forward, FP64 adjoint."""
    import torch
    import workloads as W
    from paper_1904_08463_amd import Plan
    wl = W.grad()
    plan = Plan.from_workload(wl, precision="bf16x6")
    taper = torch.from_numpy(wl.taper).cuda()
    w = torch.from_numpy(wl.w).cuda()
    out = plan.generate(taper, w)
    g_out = torch.randn(out.shape, dtype=torch.complex64, device="cuda")
    g_tau = torch.empty(wl.n_radial, dtype=torch.float32, device="cuda")
    g_w = torch.empty(wl.n_planes, dtype=torch.float64, device="cuda")
    plan.grad(taper, w, g_out, g_tau, g_w)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd = bwd = 0.0
    for _ in range(steps):
        e[0].record()
        plan.generate(taper, w, out)
        e[1].record()
        plan.grad(taper, w, g_out, g_tau, g_w)
        e[2].record()
        torch.cuda.synchronize()
        fwd += e[0].elapsed_time(e[1])
        bwd += e[1].elapsed_time(e[2])
    nbytes = out.numel() * 8
    plan.close()
    return {"forward_ms": fwd / steps, "adjoint_ms": bwd / steps, "cache_bytes": int(nbytes),
            "adjoint_read_GBs": nbytes / (bwd / steps * 1e-3) / 1e9, "n_planes": wl.n_planes,
            "n_radial": wl.n_radial}


def _wpartition_paths(steps):
    """w-plane partition (sort by |w|, equal-size planes, mean |w|): the
    paper-shaped record set (505440 records, 128 planes) and the same records
    over 33 channels (16.7 M records, 256 planes)."""
    import torch
    import workloads as W
    from paper_1904_08463_amd import wpartition, wpartition_workspace
    base = W.vla_c_74mhz_w()
    res = {}
    for name, w, m in (("records_505440_planes_128", base, 128),
                       ("records_16679520_planes_256", W.multichannel_w(base, 33), 256)):
        wd = torch.from_numpy(w).cuda()
        ws = torch.empty(wpartition_workspace(w.size), dtype=torch.uint8, device="cuda")
        for _ in range(2):
            wpartition(wd, m, workspace=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            wpartition(wd, m, workspace=ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        res[name] = {"records_per_s": w.size / dt, "ms": 1000.0 * dt, "n_records": int(w.size),
                     "n_planes": m, "steps": steps}
    return res


def _guarded(fn, *args, name=None):
    """Run an auxiliary measurement; a failure is reported in its entry (as
    {name: {"error": ...}} for the ones that return several paths) instead of
    taking the headline line down with it."""
    try:
        return fn(*args)
    except Exception as exc:  # reported, not hidden
        err = {"error": f"{type(exc).__name__}: {exc}"}
        print(f"bench: {fn.__name__} failed: {err['error']}", file=sys.stderr, flush=True)
        return {name: err} if name else err


def _truncated_path(plan, taper, w, out, steps):
    """The same plan with the 1% truncation step (section 3.1): supports,
    offsets and the packed cache come back in device memory; the call is
    timed whole (lines, truncation decision, layout, resample)."""
    import torch
    _, sup, offs = plan.generate_truncated(taper, w, 0.01, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.generate_truncated(taper, w, 0.01, out=out)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    written = int(offs[-1].item()) * 8
    sup = sup.cpu().numpy()
    return {"kernels_per_s": plan.n_planes / wall, "ms_per_step": 1000.0 * wall,
            "bytes_written": written, "written_GBs": written / wall / 1e9,
            "support_min_median_max": [int(sup.min()), int(np.median(sup)), int(sup.max())]}


def _profile_pass(wl):
    """Kernels for a hardware-counter run: two generate calls of the split path
    and a plain 2 GiB device-to-device copy of known size."""
    import torch
    from paper_1904_08463_amd import Plan
    taper = torch.from_numpy(wl.taper).cuda()
    w = torch.from_numpy(wl.w).cuda()
    plan = Plan.from_workload(wl, precision="bf16x6")
    out = torch.empty(int(plan.offsets[-1]), dtype=torch.complex64, device="cuda")
    for _ in range(2):
        plan.generate(taper, w, out)
    torch.cuda.synchronize()
    plan.close()
    del out
    src = torch.ones(1 << 28, dtype=torch.float64, device="cuda")  # 2 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"profile_pass": "done", "output_bytes": int(plan.offsets[-1]) * 8,
                      "copy_bytes": 2 * (1 << 30)}), flush=True)


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        return 1


def stratified_planes(wl, stride, per_channel=1024):
    """Every stride-th plane (by w) of each (channel, support) group, and at
    least one plane of every group: covers every support and channel of the
    batch (channel-major, per_channel planes a channel)."""
    chan = np.arange(wl.n_planes) // per_channel
    picked = []
    for c in np.unique(chan):
        for s in np.unique(wl.support[chan == c]):
            g = np.nonzero((chan == c) & (wl.support == s))[0]
            g = g[np.argsort(wl.w[g], kind="stable")]
            sel = g[stride // 2::stride] if len(g) > stride else g[len(g) // 2:len(g) // 2 + 1]
            picked.extend(sel.tolist())
    return np.array(sorted(picked), dtype=np.int64)


LOG_BINS = (-16.0, 0.0, 3200)  # log10 of element-wise relative error, 0.005-decade bins


def _accuracy(wl, outs, offsets, planes, gates, max_elems=150_000_000):
    """Device caches `outs` (name -> flat complex64 tensor) against the FP64
    oracle on `planes`, streamed in chunks of at most max_elems elements.
    Per plane e_max = max|dK| / max|K_ref| and e_mean = mean|dK| / max|K_ref|;
    the 99.9th percentile of |dK| / |K_ref| over elements with |K_ref| >= 1%
    of their plane's peak (from a 0.005-decade histogram).  Also returns the
    oracle's own time (the comparison is not counted)."""
    import torch
    from oracle import hankel as H
    lo, hi, nb = LOG_BINS
    st = {n: {"emax": [], "emean": [], "hist": torch.zeros(nb, dtype=torch.float64, device="cuda"),
              "above": 0, "n_elem": 0} for n in outs}
    sizes = (offsets[planes + 1] - offsets[planes]).astype(np.int64)
    chunks, cur, acc = [], [], 0
    for p, n in zip(planes, sizes):
        if cur and acc + n > max_elems:
            chunks.append(cur)
            cur, acc = [], 0
        cur.append(int(p))
        acc += int(n)
    if cur:
        chunks.append(cur)
    t_oracle = 0.0
    for chunk in chunks:
        t0 = time.perf_counter()
        caches, _ = H.generate_workload(wl, planes=chunk)
        t_oracle += time.perf_counter() - t0
        ref = torch.from_numpy(np.concatenate([c.reshape(-1) for c in caches])).cuda()
        del caches
        sizes_c = [int(offsets[p + 1] - offsets[p]) for p in chunk]
        bounds = np.concatenate([[0], np.cumsum(sizes_c)])
        nel = torch.tensor(sizes_c, dtype=torch.float64, device="cuda")
        rabs = ref.abs()
        # per-plane reductions over contiguous slices (no atomics)
        peak = torch.stack([rabs[bounds[i]:bounds[i + 1]].max() for i in range(len(chunk))])
        big = rabs >= 0.01 * torch.repeat_interleave(peak, torch.tensor(sizes_c, device="cuda"))
        for name, out in outs.items():
            got = torch.cat([out[int(offsets[p]):int(offsets[p + 1])] for p in chunk])
            d = (got.to(torch.complex128) - ref).abs()
            dmax = torch.stack([d[bounds[i]:bounds[i + 1]].max() for i in range(len(chunk))])
            dsum = torch.stack([d[bounds[i]:bounds[i + 1]].sum() for i in range(len(chunk))])
            st[name]["emax"].append((dmax / peak).cpu().numpy())
            st[name]["emean"].append((dsum / nel / peak).cpu().numpy())
            rel = torch.log10((d[big] / rabs[big]).clamp(min=10.0 ** lo))
            st[name]["hist"] += torch.histc(rel, bins=nb, min=lo, max=hi).double()
            st[name]["above"] += int((rel > hi).sum())
            st[name]["n_elem"] += int(big.sum())
            del got, d
        del ref, rabs, big
    res = {}
    for name, v in st.items():
        emax, emean = np.concatenate(v["emax"]), np.concatenate(v["emean"])
        cdf = torch.cumsum(v["hist"], 0).cpu().numpy()
        k = int(np.searchsorted(cdf, 0.999 * v["n_elem"]))
        p999 = 10.0 ** (lo + (hi - lo) * (k + 1) / nb) if v["above"] == 0 else float("inf")
        worst = int(planes[int(np.argmax(emax))])
        res[name] = {"planes_checked": int(len(planes)), "e_max": float(emax.max()),
                     "e_max_plane": worst, "e_mean_max": float(emean.max()),
                     "e_mean_avg": float(emean.mean()),
                     "elementwise_rel_p99_9": p999,
                     "elements_above_1pct_of_peak": v["n_elem"],
                     "gate": gates[name], "accuracy_ok": bool(emax.max() <= gates[name])}
    return res, t_oracle, len(chunks)


def _oracle_single_thread(wl, planes):
    """The same oracle chain with BLAS held to one thread (NumPy's own loops
    are single-threaded), on a smaller stratified sample."""
    from threadpoolctl import threadpool_limits
    from oracle import hankel as H
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        H.generate_workload(wl, planes=planes)
        return time.perf_counter() - t0


def _cpu_fft_generator(wl, planes, workers, fixed):
    """The standard algorithm (Algorithm 1) on the host, as the paper's WP-FFT
    method runs there: screen on the power-of-two workspace (fixed: at or
    above the maximum support, as the paper's imager; else per plane),
    zero padding by os, a 2D FFT with scipy.fft over `workers` threads,
    extraction of the os^2 sub-kernels.  Returns seconds."""
    import scipy.fft
    from oracle import fft2d as F
    fov = wl.image_size * wl.cellsize
    tfn = F.taper_from_samples(wl.taper, 0.5 * fov)
    t0 = time.perf_counter()
    for p in planes:
        s = int(wl.support[p])
        n_ws = F.next_pow2(wl.max_support if fixed else s)
        scr = F.workspace_screen(tfn, float(wl.w[p]), n_ws, fov)
        big_n = wl.oversampling * n_ws
        big = np.zeros((big_n, big_n), dtype=np.complex128)
        o = big_n // 2 - n_ws // 2
        big[o:o + n_ws, o:o + n_ws] = scr
        spec = np.fft.fftshift(scipy.fft.fft2(np.fft.ifftshift(big), workers=workers))
        spec *= (fov / n_ws) ** 2
        F.extract_cache(spec, s, wl.oversampling)
    return time.perf_counter() - t0


def parallel_efficiency(t_single, t_multi, cores):
    """eta = speed-up / cores, the speed-up being the single-threaded time
    over the multi-threaded one (section 6.8, the equation beside Table 2;
    a fraction here, the paper prints percent)."""
    return (t_single / t_multi) / cores


def _cpu_baselines(wl, small):
    """Host-side comparison methods with single-thread and all-thread timings
    and the parallel efficiency eta = (t_1 / t_N) / N (section 6.8, Table 2).
    `small`: the plane sample."""
    cores = len(os.sched_getaffinity(0))
    res = {"host_cores": cores, "sample_planes": int(len(small)),
           "sample": "every 24th plane of the accuracy sample (sorted by plane index)"}
    t1 = _oracle_single_thread(wl, small)
    from oracle import hankel as H
    t0 = time.perf_counter()
    H.generate_workload(wl, planes=small)
    ta = time.perf_counter() - t0
    res["oracle"] = {"kernels_per_s_1_thread": len(small) / t1,
                     "kernels_per_s_all_threads": len(small) / ta,
                     "blas_threads_all": int(_blas_threads()),
                     "eta": parallel_efficiency(t1, ta, cores)}
    fft_planes = small[::4]
    for fixed in (False, True):
        tag = "fft2d_fixed_workspace" if fixed else "fft2d_per_plane_workspace"
        ta = _cpu_fft_generator(wl, fft_planes, cores, fixed)
        t1f = _cpu_fft_generator(wl, fft_planes, 1, fixed)
        res[tag] = {"planes": int(len(fft_planes)), "kernels_per_s_all_threads": len(fft_planes) / ta,
                    "kernels_per_s_1_thread": len(fft_planes) / t1f,
                    "eta": parallel_efficiency(t1f, ta, cores)}
    return res


def _store_ceilings(out, reps=5):
    """HBM store rate of the two plain-store structures over the whole
    kernel-cache buffer (wkern_store_ceiling): one 16-byte store per lane and
    the resample's 256 KB unit walk (units dealt to the XCDs in runs of 64).  GB/s from the best of `reps` event-timed
    launches on the launching stream."""
    import torch
    from paper_1904_08463_amd import store_ceiling
    nbytes = out.numel() * out.element_size()
    res = {}
    for name in ("one_store_per_lane", "unit_walk"):
        store_ceiling(out, name)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            store_ceiling(out, name)
            b.record()
            b.synchronize()
            best = min(best, a.elapsed_time(b))
        res[name] = {"ms": best, "GB/s": nbytes / (best * 1e-3) / 1e9}
    return res


def _machine():
    info = {"host_cores": len(os.sched_getaffinity(0))}
    try:
        with open("/proc/cpuinfo") as fh:
            info["cpu_model"] = next((ln.split(":", 1)[1].strip() for ln in fh
                                      if ln.startswith("model name")), None)
    except OSError:
        info["cpu_model"] = None
    try:
        with open("/opt/rocm/.info/version") as fh:
            info["rocm"] = fh.read().strip()
    except OSError:
        info["rocm"] = None
    try:
        import torch
        info["torch"] = torch.__version__
        info["hip_runtime"] = torch.version.hip
        info["gpu"] = torch.cuda.get_device_properties(0).gcnArchName
    except Exception:  # pragma: no cover
        pass
    # the kernel driver's version, where the box exposes it
    try:
        with open("/sys/module/amdgpu/version") as fh:
            info["amdgpu_driver"] = fh.read().strip() or None
    except OSError:
        info["amdgpu_driver"] = None
    import subprocess
    try:
        info["git_sha"] = subprocess.run(["git", "rev-parse", "HEAD"], cwd=ROOT, capture_output=True,
                                         text=True, timeout=10).stdout.strip() or None
    except Exception:
        info["git_sha"] = None
    h = hashlib.sha256()
    for sub in ("include", os.path.join("paper_1904_08463_amd", "csrc")):
        d = os.path.join(ROOT, sub)
        for f in sorted(os.listdir(d)):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    info["source_sha256"] = h.hexdigest()
    return info


def _precision_config():
    """The small Gaussian workload in split-BF16 at q = 1, 2, 4 (with w = 0, a
    lone negative w and one mirrored plane): per-plane e_max / e_mean against
    the FP64 oracle, and the agreement of the device caches with the oracle's
    zero-padded 2D DFT of the same screen inside the disc (section 4.4)."""
    import torch
    import workloads as W
    from oracle import fft2d as F
    from oracle import hankel as H
    from paper_1904_08463_amd import Plan
    res = {}
    for q in (1, 2, 4):
        base = W.plain()
        wl = W.plain(radial_refine=q, extra_w=[0.0, -300.0, -base.w[-1]], precision="bf16x6")
        wl.mirror = W.mirror_table(wl.w, wl.support)
        plan = Plan.from_workload(wl)
        flat = plan.generate(torch.from_numpy(wl.taper).cuda(),
                             torch.from_numpy(wl.w).cuda()).cpu().numpy()
        caches, _ = H.generate_workload(wl)
        twins = F.generate(wl.taper_fn, wl.w, wl.support, wl.oversampling, 128,
                           wl.image_size * wl.cellsize)
        emax, emean, e2d = [], [], []
        for p in range(wl.n_planes):
            got = flat[plan.offsets[p]:plan.offsets[p + 1]].reshape(caches[p].shape)
            pk = np.max(np.abs(caches[p]))
            d = np.abs(got - caches[p])
            emax.append(float(d.max() / pk))
            emean.append(float(d.mean() / pk))
            e2d.append(float(np.max(np.abs(got - twins[p])) / np.max(np.abs(twins[p]))))
        plan.close()
        res[f"q{q}"] = {"w": [float(x) for x in wl.w], "e_max": emax, "e_mean": emean,
                        "hankel_vs_2d_in_disc": e2d}
    return res


def main():
    args = _parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; "
                          "multi-GPU sharding of planes is a design note, not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import workloads as W
    from paper_1904_08463_amd import Plan

    torch.cuda.set_device(0)
    wl = W.batch()
    if args.profile:
        _profile_pass(wl)
        return
    taper = torch.from_numpy(wl.taper).cuda()
    w = torch.from_numpy(wl.w).cuda()

    plan = Plan.from_workload(wl, precision="bf16x6")
    total = int(plan.offsets[-1])
    out = torch.empty(total, dtype=torch.complex64, device="cuda")
    out_bytes = total * 8
    wall, stages = _time_path(plan, taper, w, out, args.steps, args.warmup)
    ms = 1000.0 * wall / args.steps
    value = wl.n_planes / (wall / args.steps)

    res_ms = stages["resample"]
    achieved = out_bytes / (res_ms * 1e-3) / 1e9
    info = plan.info()
    paths = {"bf16x6": {"kernels_per_s": value, "ms_per_step": ms,
                        "stage_ms": stages,
                        "pipeline_chunks": info["chunks"], "contraction_variant": info["variant"],
                        "autotune_ms": info["variant_ms"],
                        "contraction_roofline": _contraction_roofline(plan, wl, stages, "bf16x6")}}
    offsets = plan.offsets.copy()
    # the truncated path writes into its own buffer: `out` keeps the headline
    # cache for the accuracy check below
    out_t = torch.empty_like(out)
    paths["bf16x6_truncated_1pct"] = _guarded(_truncated_path, plan, taper, w, out_t, args.steps)
    plan.close()
    # every plane computed on its own (no use of K(-w) = conj K(w), section 4.1)
    plan_all = Plan.from_workload(wl, precision="bf16x6", use_mirror=False)
    wall1, stages1 = _time_path(plan_all, taper, w, out_t, args.steps, 1)
    paths["bf16x6_all_planes_computed"] = {"kernels_per_s": wl.n_planes / (wall1 / args.steps),
                                           "ms_per_step": 1000.0 * wall1 / args.steps,
                                           "stage_ms": stages1}
    plan_all.close()

    outs = {"bf16x6": out}
    if not args.skip_fp32:
        plan32 = Plan.from_workload(wl, precision="fp32")
        wall32, stages32 = _time_path(plan32, taper, w, out_t, args.steps, args.warmup)
        outs["fp32"] = out_t
        info32 = plan32.info()
        paths["fp32"] = {"kernels_per_s": wl.n_planes / (wall32 / args.steps),
                         "ms_per_step": 1000.0 * wall32 / args.steps, "stage_ms": stages32,
                         "pipeline_chunks": info32["chunks"],
                         "contraction_variant": info32["variant"],
                         "autotune_ms": info32["variant_ms"],
                         "contraction_roofline": _contraction_roofline(plan32, wl, stages32, "fp32")}
        plan32.close()

    # accuracy of the timed caches against the FP64 oracle on a stratified
    # sample covering every (channel, support) group; the oracle's time is the
    # CPU baseline
    planes = stratified_planes(wl, args.cpu_stride)
    acc, t_oracle, n_chunks = _accuracy(wl, outs, offsets, planes,
                                        {"bf16x6": 1e-6, "fp32": 1e-5})
    for name, a in acc.items():
        paths[name]["accuracy"] = a
    del out_t
    outs.clear()
    torch.cuda.empty_cache()
    ceilings = _guarded(_store_ceilings, out)

    if not args.skip_fft:
        paths.update(_guarded(_fft_paths, wl, taper, w, out, args.fft_steps, name="fft2d"))
    if not args.skip_projslice:
        paths.update(_guarded(_projslice_paths, wl, taper, w, out, args.steps,
                              name="projection_slice"))
    paths["wpartition"] = _guarded(_wpartition_paths, args.steps)
    paths["gridding_paper_setting"] = _guarded(_gridding_paths, args.steps)
    paths["gradient"] = _guarded(_gradient_path, args.steps)
    paths["precision_config"] = _guarded(_precision_config)
    ok = acc["bf16x6"]["accuracy_ok"]

    # the split path's speed-up over the FP32 Hankel path and over 2D-FFT
    # generation, same GPU, same run (time ratios, > 1 means the split path
    # is faster)
    def ratio(other, key="ms_per_step"):
        v = paths.get(other, {}).get(key)
        return v / ms if v else None
    speedups = {"vs_fp32_hankel_step": ratio("fp32"),
                "vs_2d_fft_per_plane_workspace": ratio("fft2d_per_plane"),
                "vs_2d_fft_fixed_workspace": ratio("fft2d_max_support")}
    c16 = stages.get("contraction")
    c32 = paths.get("fp32", {}).get("stage_ms", {}).get("contraction")
    speedups["vs_fp32_hankel_contraction"] = c32 / c16 if c16 and c32 else None
    # the running sum that carries the 128-node FP32 sub-chunk sums
    combine = {"ringr64x256": "fp32 two-sum running sum",
               "ringw64x256": "fp64 running sum of the 00 product"}.get(info["variant"],
                                                                      "fp64 running sum")

    line = {
        "metric": "w-kernels/sec at <=1e-6 rel err (split-BF16 Hankel; FP32 Hankel beside it)",
        # the metric counts kernels only when the timed cache meets its gate
        "value": value if ok else None,
        "value_unchecked": value,
        "accuracy_ok": ok,
        "unit": "kernels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"bf16x6 (fp32 accumulate, {combine})",
        "data": "synthetic",
        "config": {"workload": "batch: 16 ch x 1024 w-planes, Nr 8192, os 8, S 7..255, "
                               "2048^2 @ 3.5 arcsec, PSWF taper; 16384 kernels per step, "
                               "the -w half as conjugates (section 4.1)",
                   "n_kernels": wl.n_planes, "output_bytes": out_bytes},
        "roofline": {"bound": "hbm", "kernel": "k_resample", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": _measured_traffic(), "ms": res_ms,
                     "algorithmic_bytes": out_bytes,
                     # the same 30.6 GB written with plain stores on this device
                     "peak_measured": ceilings.get("one_store_per_lane", {}).get("GB/s"),
                     "store_ceilings": ceilings},
        "speedups": speedups,
        "paths": paths,
        "machine": _machine(),
    }
    line["cpu_baseline"] = {
        "value": len(planes) / t_oracle, "unit": "kernels/s", "cores": int(_blas_threads()),
        "kind": "oracle",
        "sample": f"{len(planes)} of {wl.n_planes} planes (every {args.cpu_stride}th by w of each "
                  f"(channel, support) group: all 16 channels, S {int(wl.support[planes].min())}.."
                  f"{int(wl.support[planes].max())}), FP64 NumPy/SciPy in {n_chunks} chunks, "
                  f"{t_oracle:.1f} s; BLAS threads {_blas_threads()}, host cores "
                  f"{len(os.sched_getaffinity(0))}; the same planes check the timed caches"}
    if not args.no_cpu_baseline:
        line["cpu_baselines"] = _guarded(_cpu_baselines, wl, planes[::24])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
