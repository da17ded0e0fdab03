"""The Python binding refuses tensors the library would address out of
bounds or in host memory (it raises ValueError before any library call), on
a small plan."""
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_plan_methods_validate_tensors():
    from paper_1904_08463_amd import Plan
    wl = W.plain()
    plan = Plan.from_workload(wl, precision="fp32")
    taper = torch.from_numpy(wl.taper).cuda()
    w = torch.from_numpy(wl.w).cuda()
    total = int(plan.offsets[-1])
    with pytest.raises(ValueError):
        plan.generate(taper.cpu(), w)
    with pytest.raises(ValueError):
        plan.generate(taper, w[:-1])
    with pytest.raises(ValueError):
        plan.generate(taper, w, out=torch.empty(total - 1, dtype=torch.complex64, device="cuda"))
    with pytest.raises(ValueError):
        plan.generate_radial(taper, w, out=torch.empty(int(plan.nrho.sum()), dtype=torch.complex64,
                                                       device="cuda"))
    with pytest.raises(ValueError):
        plan.generate_truncated(taper, w, 0.01, out=torch.empty(total, dtype=torch.complex64))
    with pytest.raises(ValueError):
        plan.grad(taper, w, torch.zeros(total, dtype=torch.complex64))
    with pytest.raises(ValueError):
        plan.grad(taper, w, torch.zeros(total, dtype=torch.complex64, device="cuda"),
                  grad_w=torch.empty(plan.n_planes - 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        plan.prepare_lines(taper, w, support_out=torch.empty(plan.n_planes, dtype=torch.int64,
                                                             device="cuda"))
    d = lambda dt, k: torch.zeros(k, dtype=dt, device="cuda")  # noqa: E731
    P = plan.n_planes
    good = [d(torch.float64, 5), d(torch.float64, 5), d(torch.float64, 5), d(torch.complex64, 5),
            d(torch.int32, 5), d(torch.int64, P + 1), d(torch.int32, P)]
    grid = torch.zeros((64, 64), dtype=torch.complex64, device="cuda")
    for i, bad in enumerate((d(torch.float64, 4), d(torch.float64, 4), d(torch.float64, 4),
                             d(torch.complex64, 4), d(torch.int64, 5), d(torch.int64, P),
                             d(torch.int32, P + 1))):
        args = list(good)
        if i > 0:
            args[i] = bad
        else:
            args[1] = d(torch.float64, 6)  # u sets the record count; v disagrees
        with pytest.raises(ValueError):
            plan.grid(*args, grid)
    with pytest.raises(ValueError):
        plan.grid(*good, grid, cache=d(torch.complex64, total))  # offsets missing
    with pytest.raises(ValueError):
        plan.grid(*good, grid, cache=d(torch.complex64, total), cache_offsets=d(torch.int32, P + 1))
    plan.close()


def test_fft2d_and_partition_validate_tensors():
    from paper_1904_08463_amd import wpartition
    from paper_1904_08463_amd.wkern import FFT2DPlan
    wl = W.plain()
    fp = FFT2DPlan.from_workload(wl)
    with pytest.raises(ValueError):
        fp.generate(torch.from_numpy(wl.taper), torch.from_numpy(wl.w).cuda())
    with pytest.raises(ValueError):
        fp.generate(torch.from_numpy(wl.taper).cuda(), torch.from_numpy(wl.w).cuda(),
                    out=torch.empty(3, dtype=torch.complex64, device="cuda"))
    fp.close()
    w = torch.zeros(10, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        wpartition(w, 2, workspace=torch.empty(1 << 16, dtype=torch.uint8))
