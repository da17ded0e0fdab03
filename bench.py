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
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=4,
                    help="oracle sample: every n-th plane in support order")
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
    return {"bound": "mfma", "kernel": "k_contract_*", "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": achieved / peak, "algorithmic_flop": flop,
            "executed_flop": executed, "ms": ms}


def _sampled_error(plan, out, wl, planes):
    from oracle import hankel as H
    caches, _ = H.generate_workload(wl, planes=planes)
    worst = 0.0
    for j, p in enumerate(planes):
        got = out[int(plan.offsets[p]):int(plan.offsets[p + 1])].cpu().numpy()
        ref = caches[j].reshape(-1)
        worst = max(worst, float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
    return worst


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


def _cpu_baseline(wl, stride):
    """The FP64 oracle, as it stands, on a stratified sample of the planes."""
    from oracle import hankel as H
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = 1
    order = np.argsort(wl.support, kind="stable")
    planes = order[stride // 2::stride]
    t0 = time.perf_counter()
    H.generate_workload(wl, planes=planes)
    dt = time.perf_counter() - t0
    return {
        "value": len(planes) / dt,
        "unit": "kernels/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"{len(planes)} of {wl.n_planes} planes (every {stride}th in support order, "
                  f"S {int(wl.support[planes].min())}..{int(wl.support[planes].max())}), "
                  f"FP64 NumPy/SciPy, {dt:.1f} s; BLAS threads {threads}, "
                  f"host cores {len(os.sched_getaffinity(0))}",
    }


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
    order = np.argsort(wl.support, kind="stable")
    check_planes = sorted(set(order[[0, 4000, 8000, 12000, 15000, 16000]].tolist()))
    err_bf16 = _sampled_error(plan, out, wl, check_planes)

    res_ms = stages["resample"]
    achieved = out_bytes / (res_ms * 1e-3) / 1e9
    info = plan.info()
    paths = {"bf16x6": {"kernels_per_s": value, "ms_per_step": ms,
                        "stage_ms": stages, "max_rel_err_sampled": err_bf16,
                        "pipeline_chunks": info["chunks"], "contraction_variant": info["variant"],
                        "autotune_ms": info["variant_ms"],
                        "contraction_roofline": _contraction_roofline(plan, wl, stages, "bf16x6")}}
    paths["bf16x6_truncated_1pct"] = _guarded(_truncated_path, plan, taper, w, out, args.steps)
    plan.close()
    # every plane computed on its own (no use of K(-w) = conj K(w), section 4.1)
    plan_all = Plan.from_workload(wl, precision="bf16x6", use_mirror=False)
    wall1, stages1 = _time_path(plan_all, taper, w, out, args.steps, 1)
    paths["bf16x6_all_planes_computed"] = {"kernels_per_s": wl.n_planes / (wall1 / args.steps),
                                           "ms_per_step": 1000.0 * wall1 / args.steps,
                                           "stage_ms": stages1}
    plan_all.close()

    if not args.skip_fp32:
        plan32 = Plan.from_workload(wl, precision="fp32")
        wall32, stages32 = _time_path(plan32, taper, w, out, args.steps, args.warmup)
        err32 = _sampled_error(plan32, out, wl, check_planes)
        info32 = plan32.info()
        paths["fp32"] = {"kernels_per_s": wl.n_planes / (wall32 / args.steps),
                         "ms_per_step": 1000.0 * wall32 / args.steps, "stage_ms": stages32,
                         "max_rel_err_sampled": err32, "pipeline_chunks": info32["chunks"],
                         "contraction_variant": info32["variant"],
                         "autotune_ms": info32["variant_ms"],
                         "contraction_roofline": _contraction_roofline(plan32, wl, stages32, "fp32")}
        plan32.close()

    if not args.skip_fft:
        paths.update(_guarded(_fft_paths, wl, taper, w, out, args.fft_steps, name="fft2d"))
    if not args.skip_projslice:
        paths.update(_guarded(_projslice_paths, wl, taper, w, out, args.steps,
                              name="projection_slice"))
    paths["wpartition"] = _guarded(_wpartition_paths, args.steps)
    paths["gridding_paper_setting"] = _guarded(_gridding_paths, args.steps)
    paths["gradient"] = _guarded(_gradient_path, args.steps)

    line = {
        "metric": "w-kernels/sec at <=1e-6 rel err (split-BF16 Hankel; FP32 Hankel beside it)",
        "value": value,
        "unit": "kernels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x6 (fp32 accumulate, fp64 combine)",
        "data": "synthetic",
        "config": {"workload": "batch: 16 ch x 1024 w-planes, Nr 8192, os 8, S 7..255, "
                               "2048^2 @ 3.5 arcsec, PSWF taper; 16384 kernels per step, "
                               "the -w half as conjugates (section 4.1)",
                   "n_kernels": wl.n_planes, "output_bytes": out_bytes},
        "roofline": {"bound": "hbm", "kernel": "k_resample", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": _measured_traffic(), "ms": res_ms,
                     "algorithmic_bytes": out_bytes},
        "paths": paths,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = _guarded(_cpu_baseline, wl, args.cpu_stride)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
