"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/wkern.h declares, validates arguments, and its layout
agrees with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import hankel as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

lib_mod = pytest.importorskip("paper_1904_08463_amd.wkern")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lib_mod.LIB_PATH):
        pytest.skip("libwkern.so not built")
    return lib_mod.load_library()


def test_header_symbols_exported(lib):
    with open(os.path.join(ROOT, "include", "wkern.h")) as f:
        hdr = f.read()
    declared = set(re.findall(r"^\S[^\n(]*?\b(wkern_[a-z_0-9]+)\s*\(", hdr, flags=re.M))
    assert declared == set(lib_mod.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_abi_version(lib):
    assert lib.wkern_abi_version() == lib_mod.ABI_VERSION


@pytest.mark.parametrize("wl", [W.plain(), W.paper(), W.random_small(3, os_=5)], ids=lambda w: w.name)
def test_layout_matches_oracle(lib, wl):
    offs, nrho = lib_mod.layout_desc(image_size=wl.image_size, cellsize=wl.cellsize,
                                     n_radial=wl.n_radial, oversampling=wl.oversampling,
                                     support=wl.support, max_support=wl.max_support,
                                     radial_refine=wl.radial_refine)
    assert np.array_equal(offs, H.offsets(wl.support, wl.oversampling))
    assert np.array_equal(nrho, H.n_rho(wl.support, wl.oversampling, wl.radial_refine))


def test_layout_batch_size(lib):
    wl = W.batch()
    offs, _ = lib_mod.layout_desc(image_size=wl.image_size, cellsize=wl.cellsize,
                                  n_radial=wl.n_radial, oversampling=wl.oversampling,
                                  support=wl.support, max_support=wl.max_support)
    # 16384 kernels of 7..255 px at os 8: 30.6 GB of complex64
    assert abs(offs[-1] * 8 / 1e9 - 30.6) < 0.1


BAD = [
    ("image_size", 0), ("cellsize", 0.0), ("cellsize", float("nan")), ("cellsize", 0.02),
    ("n_radial", 0), ("oversampling", 0), ("oversampling", 65), ("radial_refine", 0),
    ("max_support", 4), ("precision", 7), ("interp", 3),
    # an empty batch, and sizes past the documented limits
    ("n_planes", 0), ("n_radial", (1 << 20) + 1), ("radial_refine", 17), ("image_size", -5),
    ("max_support", 0),
]


@pytest.mark.parametrize("field,value", BAD)
def test_invalid_arguments(lib, field, value):
    d, sup = lib_mod.make_desc(image_size=128, cellsize=7.8125e-4, n_radial=64, oversampling=4,
                               support=[7, 9], max_support=9)
    setattr(d, field, value)
    offs = np.zeros(3, dtype=np.int64)
    st = lib.wkern_layout_desc(ctypes.byref(d), offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               None)
    assert st == 1, (field, value, lib.wkern_last_error())
    assert lib.wkern_last_error().decode()


@pytest.mark.parametrize("support", [[8], [11], [0], [-3]])
def test_invalid_supports(lib, support):
    with pytest.raises(lib_mod.WkernError) as ei:
        lib_mod.layout_desc(image_size=128, cellsize=7.8125e-4, n_radial=64, oversampling=4,
                            support=support, max_support=9)
    assert ei.value.status == 1


def test_abi_mismatch(lib):
    d, sup = lib_mod.make_desc(image_size=128, cellsize=7.8125e-4, n_radial=64, oversampling=4,
                               support=[7])
    d.abi_version = 99
    offs = np.zeros(2, dtype=np.int64)
    assert lib.wkern_layout_desc(ctypes.byref(d), offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 None) == 5


def test_null_arguments(lib):
    assert lib.wkern_layout_desc(None, None, None) == 1
    assert lib.wkern_plan(None, None) == 1
    assert lib.wkern_generate(None, None, None, None, None) == 1
    assert lib.wkern_generate_truncated(None, None, None, 0.01, None, 0, None, None, None) == 1
    assert lib.wkern_generate_radial(None, None, None, None, None) == 1
    assert lib.wkern_wpartition(None, 10, 2, 1, 0, None, 0, None, None, None, None) == 1
    assert lib.wkern_prepare_lines(None, None, None, 0.0, None, None) == 1
    assert lib.wkern_grid(None, None, None, None, None, 0, None, None, None, None, None, 64,
                          None, None) == 1
    n = ctypes.c_size_t()
    assert lib.wkern_wpartition_workspace(0, ctypes.byref(n)) == 1
    assert lib.wkern_wpartition_workspace(1 << 31, ctypes.byref(n)) == 4
    assert lib.wkern_grad(None, None, None, None, None, None, None) == 1
    assert lib.wkern_destroy(None) == 0
    for s in range(6):
        assert lib.wkern_strerror(s)


def test_radial_line_limit(lib):
    # q os h + 4 beyond the spline's capacity is rejected up front
    with pytest.raises(lib_mod.WkernError):
        lib_mod.layout_desc(image_size=128, cellsize=7.8125e-4, n_radial=64, oversampling=16,
                            support=[255], max_support=255, radial_refine=2)


def test_plan_without_device_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(lib_mod.WkernError) as ei:
        lib_mod.Plan(128, 7.8125e-4, 64, 4, [7])
    assert ei.value.status == 3


@pytest.mark.parametrize("mirror", [[0, -1], [-1, 5], [-1, 0, 1], [2, -1, -1], [-2, -1]])
def test_invalid_mirror_tables(lib, mirror):
    sup = [7, 7, 9][:len(mirror)]
    with pytest.raises(lib_mod.WkernError) as ei:
        lib_mod.layout_desc(image_size=128, cellsize=7.8125e-4, n_radial=64, oversampling=4,
                            support=sup, max_support=9, mirror=mirror)
    assert ei.value.status == 1


def test_mirror_table_of_batch_workload():
    wl = W.batch()
    m = wl.mirror
    assert (m >= 0).sum() == wl.n_planes // 2
    src = m[m >= 0]
    assert np.all(m[src] == -1)
    assert np.all(wl.w[m >= 0] == -wl.w[src])
    assert np.all(wl.support[m >= 0] == wl.support[src])


def test_binding_rejects_host_and_mis_sized_tensors():
    """The binding refuses, before any library call, a tensor the library
    would address on the device: host memory, wrong dtype, wrong size,
    non-contiguous."""
    torch = pytest.importorskip("torch")
    req = lib_mod._require
    with pytest.raises(ValueError):
        req(torch.zeros(4, dtype=torch.float32), torch.float32, "t", numel=4)
    with pytest.raises(ValueError):
        req(np.zeros(4, dtype=np.float32), torch.float32, "t")
    meta = torch.empty(8, dtype=torch.float64, device="meta")
    with pytest.raises(ValueError):
        req(meta, torch.float64, "t")
