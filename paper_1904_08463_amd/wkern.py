"""Python binding of the wkern C ABI (include/wkern.h).

Argument marshalling only: every step of kernel generation runs in the HIP
library ``libwkern.so``.  PyTorch provides device memory and streams.  If the
library has not been built, every entry point raises ``WkernError``; there is
no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwkern.so")

ABI_VERSION = 3
PRECISION = {"fp32": 0, "bf16x6": 1}
INTERP = {"linear": 0, "cubic": 1}
STATUS = {
    0: "WKERN_OK",
    1: "WKERN_ERR_INVALID_ARG",
    2: "WKERN_ERR_OUT_OF_MEMORY",
    3: "WKERN_ERR_DEVICE",
    4: "WKERN_ERR_UNSUPPORTED",
    5: "WKERN_ERR_ABI_MISMATCH",
    6: "WKERN_ERR_NONFINITE",
}

# every symbol include/wkern.h declares
EXPORTS = (
    "wkern_abi_version", "wkern_layout_desc", "wkern_plan", "wkern_layout",
    "wkern_generate", "wkern_generate_truncated", "wkern_generate_radial", "wkern_grad", "wkern_set_profiling",
    "wkern_stage_times", "wkern_plan_info", "wkern_set_variant",
    "wkern_set_chunks", "wkern_set_graph", "wkern_set_engine", "wkern_sync_status", "wkern_destroy",
    "wkern_strerror", "wkern_last_error",
    "wkern_fft2d_plan", "wkern_fft2d_generate", "wkern_fft2d_destroy",
    "wkern_wpartition_workspace", "wkern_wpartition", "wkern_wpartition_noalloc",
    "wkern_store_ceiling",
    "wkern_prepare_lines", "wkern_grid",
)


class WkernError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        self.name = STATUS.get(status, f"status {status}")
        super().__init__(f"{self.name}: {detail}")


class WkernDesc(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("image_size", ctypes.c_int32),
        ("cellsize", ctypes.c_double),
        ("n_radial", ctypes.c_int32),
        ("oversampling", ctypes.c_int32),
        ("radial_refine", ctypes.c_int32),
        ("n_planes", ctypes.c_int32),
        ("support", ctypes.POINTER(ctypes.c_int32)),
        ("max_support", ctypes.c_int32),
        ("precision", ctypes.c_int),
        ("interp", ctypes.c_int),
        ("device", ctypes.c_int32),
        ("mirror", ctypes.POINTER(ctypes.c_int32)),
    ]


_lib = None


def load_library() -> ctypes.CDLL:
    """Load the in-tree libwkern.so (raises WkernError if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise WkernError(3, f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32p, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
    desc_p = ctypes.POINTER(WkernDesc)
    lib.wkern_abi_version.restype = ctypes.c_int32
    lib.wkern_abi_version.argtypes = []
    lib.wkern_layout_desc.restype = ctypes.c_int
    lib.wkern_layout_desc.argtypes = [desc_p, i64p, i32p]
    lib.wkern_plan.restype = ctypes.c_int
    lib.wkern_plan.argtypes = [desc_p, ctypes.POINTER(vp)]
    lib.wkern_layout.restype = ctypes.c_int
    lib.wkern_layout.argtypes = [vp, i64p, i32p]
    lib.wkern_generate.restype = ctypes.c_int
    lib.wkern_generate.argtypes = [vp, vp, vp, vp, vp]
    lib.wkern_generate_truncated.restype = ctypes.c_int
    lib.wkern_generate_truncated.argtypes = [vp, vp, vp, ctypes.c_double, vp, ctypes.c_int64, vp,
                                             vp, vp]
    lib.wkern_generate_radial.restype = ctypes.c_int
    lib.wkern_generate_radial.argtypes = [vp, vp, vp, vp, vp]
    lib.wkern_grad.restype = ctypes.c_int
    lib.wkern_grad.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.wkern_set_profiling.restype = ctypes.c_int
    lib.wkern_set_profiling.argtypes = [vp, ctypes.c_int32]
    lib.wkern_stage_times.restype = ctypes.c_int
    lib.wkern_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32p]
    lib.wkern_plan_info.restype = ctypes.c_int
    lib.wkern_plan_info.argtypes = [vp, i32p, i32p, ctypes.POINTER(ctypes.c_float), i32p]
    lib.wkern_set_variant.restype = ctypes.c_int
    lib.wkern_set_variant.argtypes = [vp, ctypes.c_int32]
    lib.wkern_set_graph.restype = ctypes.c_int
    lib.wkern_set_graph.argtypes = [vp, ctypes.c_int32]
    lib.wkern_set_engine.restype = ctypes.c_int
    lib.wkern_set_engine.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    lib.wkern_set_chunks.restype = ctypes.c_int
    lib.wkern_set_chunks.argtypes = [vp, ctypes.c_int32]
    lib.wkern_sync_status.restype = ctypes.c_int
    lib.wkern_sync_status.argtypes = [vp, vp]
    lib.wkern_destroy.restype = ctypes.c_int
    lib.wkern_destroy.argtypes = [vp]
    lib.wkern_strerror.restype = ctypes.c_char_p
    lib.wkern_strerror.argtypes = [ctypes.c_int]
    lib.wkern_last_error.restype = ctypes.c_char_p
    lib.wkern_last_error.argtypes = []
    lib.wkern_fft2d_plan.restype = ctypes.c_int
    lib.wkern_fft2d_plan.argtypes = [desc_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(vp)]
    lib.wkern_fft2d_generate.restype = ctypes.c_int
    lib.wkern_fft2d_generate.argtypes = [vp, vp, vp, vp, vp]
    lib.wkern_fft2d_destroy.restype = ctypes.c_int
    lib.wkern_fft2d_destroy.argtypes = [vp]
    lib.wkern_prepare_lines.restype = ctypes.c_int
    lib.wkern_prepare_lines.argtypes = [vp, vp, vp, ctypes.c_double, vp, vp]
    lib.wkern_grid.restype = ctypes.c_int
    lib.wkern_grid.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int64, vp, vp, vp, vp, vp,
                               ctypes.c_int32, vp, vp]
    lib.wkern_wpartition_workspace.restype = ctypes.c_int
    lib.wkern_wpartition_workspace.argtypes = [ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
    lib.wkern_wpartition.restype = ctypes.c_int
    lib.wkern_wpartition.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, vp, ctypes.c_size_t, vp, vp, vp, vp]
    lib.wkern_store_ceiling.restype = ctypes.c_int
    lib.wkern_store_ceiling.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, vp]
    lib.wkern_wpartition_noalloc.restype = ctypes.c_int
    lib.wkern_wpartition_noalloc.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, vp, vp, vp, vp]
    if lib.wkern_abi_version() != ABI_VERSION:
        raise WkernError(5, f"library ABI {lib.wkern_abi_version()}, binding {ABI_VERSION}")
    _lib = lib
    return lib


def _check(status: int) -> None:
    if status != 0:
        raise WkernError(status, load_library().wkern_last_error().decode())


def make_desc(image_size: int, cellsize: float, n_radial: int, oversampling: int,
              support: Sequence[int], max_support: Optional[int] = None, radial_refine: int = 1,
              precision: str = "fp32", interp: str = "cubic", device: int = 0, mirror=None):
    """Build a WkernDesc; returns (desc, arrays it points to, to be kept alive)."""
    sup = np.ascontiguousarray(np.asarray(support, dtype=np.int32))
    mir = None if mirror is None else np.ascontiguousarray(np.asarray(mirror, dtype=np.int32))
    if max_support is None:
        max_support = int(sup.max()) if sup.size else 1
    d = WkernDesc()
    d.abi_version = ABI_VERSION
    d.image_size = int(image_size)
    d.cellsize = float(cellsize)
    d.n_radial = int(n_radial)
    d.oversampling = int(oversampling)
    d.radial_refine = int(radial_refine)
    d.n_planes = int(sup.shape[0])
    d.support = sup.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.max_support = int(max_support)
    d.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    d.interp = INTERP[interp] if isinstance(interp, str) else int(interp)
    d.device = int(device)
    if mir is not None:
        d.mirror = mir.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    return d, (sup, mir)


def layout_desc(**kw):
    """Host-only layout (no device): returns (offsets int64 [P+1], nrho int32 [P])."""
    lib = load_library()
    d, sup = make_desc(**kw)
    offs = np.zeros(d.n_planes + 1, dtype=np.int64)
    nrho = np.zeros(d.n_planes, dtype=np.int32)
    _check(lib.wkern_layout_desc(ctypes.byref(d),
                                 offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 nrho.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    del sup
    return offs, nrho


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _require(t, dtype, name, numel=None, device=None):
    """Raise ValueError unless t is a contiguous device tensor of dtype (with
    numel values, on the given device index): the library reads and writes
    these pointers on the device without knowing their extent."""
    import torch
    ok = (isinstance(t, torch.Tensor) and t.dtype == dtype and t.is_cuda and t.is_contiguous()
          and (numel is None or t.numel() == numel)
          and (device is None or t.device.index == device))
    if not ok:
        size = f" of {numel} values" if numel is not None else ""
        where = f" on cuda:{device}" if device is not None else ""
        raise ValueError(f"{name} must be a contiguous {dtype} device tensor{size}{where}")


class Plan:
    """A wkern plan (geometry, HT matrix, schedule, scratch) on one device."""

    def __init__(self, image_size: int, cellsize: float, n_radial: int, oversampling: int,
                 support: Sequence[int], max_support: Optional[int] = None,
                 radial_refine: int = 1, precision: str = "fp32", interp: str = "cubic",
                 device: int = 0, mirror=None):
        lib = load_library()
        d, (sup, mir) = make_desc(image_size, cellsize, n_radial, oversampling, support,
                                  max_support, radial_refine, precision, interp, device, mirror)
        h = ctypes.c_void_p()
        _check(lib.wkern_plan(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.device = int(device)
        self.n_planes = int(d.n_planes)
        self.n_radial = int(n_radial)
        self.support = sup.copy()
        self.mirror = None if mir is None else mir.copy()
        self.oversampling = int(oversampling)
        offs = np.zeros(self.n_planes + 1, dtype=np.int64)
        nrho = np.zeros(self.n_planes, dtype=np.int32)
        _check(lib.wkern_layout(h, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                nrho.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        self.offsets = offs
        self.nrho = nrho

    @classmethod
    def from_workload(cls, wl, precision: Optional[str] = None, interp: Optional[str] = None,
                      device: int = 0, use_mirror: bool = True) -> "Plan":
        return cls(wl.image_size, wl.cellsize, wl.n_radial, wl.oversampling, wl.support,
                   wl.max_support, wl.radial_refine, precision or wl.precision,
                   interp or wl.interp, device, wl.mirror if use_mirror else None)

    # ------------------------------------------------------------------
    def _check_inputs(self, taper, w):
        import torch
        _require(taper, torch.float32, "taper", numel=self.n_radial, device=self.device)
        _require(w, torch.float64, "w", numel=self.n_planes, device=self.device)

    def generate(self, taper, w, out=None, stream=None):
        """Kernel cache as a flat complex64 tensor [offsets[P]] (asynchronous)."""
        import torch
        self._check_inputs(taper, w)
        total = int(self.offsets[-1])
        if out is None:
            out = torch.empty(total, dtype=torch.complex64, device=taper.device)
        _require(out, torch.complex64, "out", numel=total, device=self.device)
        _check(load_library().wkern_generate(self._h, _ptr(taper), _ptr(w), _ptr(out),
                                             _stream_handle(stream)))
        return out

    def generate_truncated(self, taper, w, frac=0.01, out=None, stream=None):
        """Truncated generation: (flat complex64 cache of the untruncated size,
        int32 supports [P], int64 offsets [P + 1]) on the device."""
        import torch
        self._check_inputs(taper, w)
        total = int(self.offsets[-1])
        if out is None:
            out = torch.empty(total, dtype=torch.complex64, device=taper.device)
        # the library checks the capacity it is given against the cache size
        _require(out, torch.complex64, "out", device=self.device)
        sup = torch.empty(self.n_planes, dtype=torch.int32, device=taper.device)
        offs = torch.empty(self.n_planes + 1, dtype=torch.int64, device=taper.device)
        _check(load_library().wkern_generate_truncated(
            self._h, _ptr(taper), _ptr(w), ctypes.c_double(frac), _ptr(out),
            ctypes.c_int64(out.numel()), _ptr(sup), _ptr(offs), _stream_handle(stream)))
        return out, sup, offs

    def generate_radial(self, taper, w, out=None, stream=None):
        """Radial lines as a flat complex128 tensor [sum nrho] (asynchronous)."""
        import torch
        self._check_inputs(taper, w)
        total = int(self.nrho.sum())
        if out is None:
            out = torch.empty(total, dtype=torch.complex128, device=taper.device)
        _require(out, torch.complex128, "out", numel=total, device=self.device)
        _check(load_library().wkern_generate_radial(self._h, _ptr(taper), _ptr(w), _ptr(out),
                                                    _stream_handle(stream)))
        return out

    def grad(self, taper, w, grad_out, grad_taper=None, grad_w=None, stream=None):
        """dL/dtau [Nr] float32 and dL/dw [P] float64 from dL/dcache (asynchronous)."""
        import torch
        self._check_inputs(taper, w)
        total = int(self.offsets[-1])
        grad_out = grad_out.contiguous()
        _require(grad_out, torch.complex64, "grad_out", numel=total, device=self.device)
        if grad_taper is None:
            grad_taper = torch.empty(self.n_radial, dtype=torch.float32, device=taper.device)
        if grad_w is None:
            grad_w = torch.empty(self.n_planes, dtype=torch.float64, device=taper.device)
        _require(grad_taper, torch.float32, "grad_taper", numel=self.n_radial, device=self.device)
        _require(grad_w, torch.float64, "grad_w", numel=self.n_planes, device=self.device)
        _check(load_library().wkern_grad(self._h, _ptr(taper), _ptr(w), _ptr(grad_out),
                                         _ptr(grad_taper), _ptr(grad_w), _stream_handle(stream)))
        return grad_taper, grad_w

    def set_profiling(self, enable: bool):
        _check(load_library().wkern_set_profiling(self._h, 1 if enable else 0))

    STAGES = ("screen", "contraction", "spline", "resample")

    def stage_times(self):
        """(dict stage -> summed ms, number of profiled calls); waits for the events."""
        ms = (ctypes.c_double * 4)()
        calls = ctypes.c_int32()
        _check(load_library().wkern_stage_times(self._h, ms, ctypes.byref(calls)))
        return dict(zip(self.STAGES, list(ms))), calls.value

    VARIANTS = ("wave32x64", "wave32x128", "lds128x128", "lds64x256", "ring128x128",
                "ring64x256", "ring32x512", "ringf128x128", "ringf64x256", "ringf64x256w8",
                "ringh64x256", "ringr64x256", "ringw64x256")

    def info(self):
        """Autotuner choice, candidate timings (ms) and pipeline chunk count."""
        lib = load_library()
        v, n, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        ms = (ctypes.c_float * 16)()
        _check(lib.wkern_plan_info(self._h, ctypes.byref(v), ctypes.byref(n), ms, ctypes.byref(c)))
        return {"variant": self.VARIANTS[v.value],
                "variant_ms": {self.VARIANTS[i]: float(ms[i]) for i in range(n.value)},
                "chunks": c.value}

    def set_variant(self, variant):
        v = self.VARIANTS.index(variant) if isinstance(variant, str) else int(variant)
        _check(load_library().wkern_set_variant(self._h, v))

    def set_graph(self, enable: bool):
        _check(load_library().wkern_set_graph(self._h, 1 if enable else 0))

    def prepare_lines(self, taper, w, frac=0.0, support_out=None, stream=None):
        """Lines and spline coefficients kept in the plan for a fused grid();
        returns the device int32 supports (truncated when frac > 0)."""
        import torch
        self._check_inputs(taper, w)
        if support_out is None:
            support_out = torch.empty(self.n_planes, dtype=torch.int32, device=taper.device)
        _require(support_out, torch.int32, "support_out", numel=self.n_planes, device=self.device)
        _check(load_library().wkern_prepare_lines(self._h, _ptr(taper), _ptr(w), ctypes.c_double(frac),
                                                  _ptr(support_out), _stream_handle(stream)))
        return support_out

    def grid(self, u, v, w, vis, order, plane_start, support, grid, cache=None,
             cache_offsets=None, stream=None):
        """Add every record's kernel footprint onto grid (complex64 [N, N]):
        fused from the prepared lines (cache None) or from a kernel cache."""
        import torch
        n = u.numel() if isinstance(u, torch.Tensor) else -1
        P, dev = self.n_planes, self.device
        for t, dt, name, cnt in ((u, torch.float64, "u", n), (v, torch.float64, "v", n),
                                 (w, torch.float64, "w", n), (vis, torch.complex64, "vis", n),
                                 (order, torch.int32, "order", None),
                                 (plane_start, torch.int64, "plane_start", P + 1),
                                 (support, torch.int32, "support", P)):
            _require(t, dt, name, numel=cnt, device=dev)
        _require(grid, torch.complex64, "grid", device=dev)
        if grid.dim() != 2 or grid.shape[0] != grid.shape[1]:
            raise ValueError("grid must be square")
        if (cache is None) != (cache_offsets is None):
            raise ValueError("cache and cache_offsets go together")
        if cache is not None:
            _require(cache, torch.complex64, "cache", device=dev)
            _require(cache_offsets, torch.int64, "cache_offsets", numel=P + 1, device=dev)
        _check(load_library().wkern_grid(
            self._h, _ptr(u), _ptr(v), _ptr(w), _ptr(vis), u.numel(), _ptr(order),
            _ptr(plane_start), _ptr(support), None if cache is None else _ptr(cache),
            None if cache_offsets is None else _ptr(cache_offsets), grid.shape[0], _ptr(grid),
            _stream_handle(stream)))
        return grid

    ENGINES = {"matrix": 0, "projection_slice": 1}
    PS_WORKSPACE = {"max_support": 0, "per_plane": 1}

    def set_engine(self, engine: str = "matrix", workspace: str = "per_plane"):
        """Radial-line engine: "matrix" (HT matrix on the matrix cores) or
        "projection_slice" (section 4.3.1, FP64), with the projection-slice
        workspace per plane or fixed at the maximum support."""
        _check(load_library().wkern_set_engine(self._h, self.ENGINES[engine],
                                               self.PS_WORKSPACE[workspace]))

    def sync_status(self, stream=None):
        """Wait for the stream, then raise WkernError (WKERN_ERR_NONFINITE) if a
        generating call since the last check produced a non-finite radial-line
        value; clears the device status word."""
        _check(load_library().wkern_sync_status(self._h, _stream_handle(stream)))

    def set_chunks(self, chunks: int):
        _check(load_library().wkern_set_chunks(self._h, int(chunks)))

    def plane_views(self, flat):
        """Per-plane [os, os, S, S] views of a flat cache tensor."""
        os_ = self.oversampling
        return [flat[int(self.offsets[p]):int(self.offsets[p + 1])].view(
            os_, os_, int(self.support[p]), int(self.support[p])) for p in range(self.n_planes)]

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None  # released even when destroy reports an error
            _check(load_library().wkern_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class FFT2DPlan:
    """The standard algorithm (2D FFT of the zero-padded workspace) on the GPU,
    for comparison with Plan; same output layout."""

    WORKSPACE = {"max_support": 0, "per_plane": 1}

    def __init__(self, image_size: int, cellsize: float, n_radial: int, oversampling: int,
                 support: Sequence[int], max_support: Optional[int] = None,
                 workspace: str = "max_support", workspace_bytes: int = 0, device: int = 0,
                 mirror=None):
        lib = load_library()
        d, (sup, mir) = make_desc(image_size, cellsize, n_radial, oversampling, support,
                                  max_support, 1, "fp32", "cubic", device, mirror)
        h = ctypes.c_void_p()
        _check(lib.wkern_fft2d_plan(ctypes.byref(d), self.WORKSPACE[workspace],
                                    int(workspace_bytes), ctypes.byref(h)))
        self._h = h
        self.device = int(device)
        self.n_planes = int(d.n_planes)
        self.n_radial = int(n_radial)
        self.offsets, _ = layout_desc(image_size=image_size, cellsize=cellsize, n_radial=n_radial,
                                      oversampling=oversampling, support=sup,
                                      max_support=d.max_support)

    @classmethod
    def from_workload(cls, wl, workspace: str = "max_support", device: int = 0,
                      use_mirror: bool = True):
        return cls(wl.image_size, wl.cellsize, wl.n_radial, wl.oversampling, wl.support,
                   wl.max_support, workspace, 0, device, wl.mirror if use_mirror else None)

    def generate(self, taper, w, out=None, stream=None):
        import torch
        total = int(self.offsets[-1])
        _require(taper, torch.float32, "taper", numel=self.n_radial, device=self.device)
        _require(w, torch.float64, "w", numel=self.n_planes, device=self.device)
        if out is None:
            out = torch.empty(total, dtype=torch.complex64, device=taper.device)
        _require(out, torch.complex64, "out", numel=total, device=self.device)
        _check(load_library().wkern_fft2d_generate(self._h, _ptr(taper), _ptr(w), _ptr(out),
                                                   _stream_handle(stream)))
        return out

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            _check(load_library().wkern_fft2d_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


WSTAT = {"mean": 0, "median": 1}


def wpartition_workspace(n_records: int, device: int = 0) -> int:
    """Device workspace bytes wpartition needs for n_records records."""
    import torch
    lib = load_library()
    n = ctypes.c_size_t()
    with torch.cuda.device(device):
        _check(lib.wkern_wpartition_workspace(int(n_records), ctypes.byref(n)))
    return int(n.value)


def wpartition(w, n_planes: int, absolute: bool = True, stat: str = "mean", workspace=None,
               stream=None):
    """w-plane partition of visibility records (asynchronous): returns device
    tensors (order int32 [n], plane_start int64 [M + 1], w_plane float64 [M]).
    w: device float64 [n]."""
    import torch
    if w.dtype != torch.float64 or not w.is_cuda or w.dim() != 1:
        raise ValueError("w must be a 1-D float64 device tensor")
    w = w.contiguous()
    n = w.numel()
    dev = w.device
    if workspace is None:
        workspace = torch.empty(wpartition_workspace(n, dev.index or 0), dtype=torch.uint8,
                                device=dev)
    _require(workspace, torch.uint8, "workspace", device=dev.index)
    order = torch.empty(n, dtype=torch.int32, device=dev)
    start = torch.empty(n_planes + 1, dtype=torch.int64, device=dev)
    w_plane = torch.empty(n_planes, dtype=torch.float64, device=dev)
    _check(load_library().wkern_wpartition(
        _ptr(w), n, int(n_planes), 1 if absolute else 0, WSTAT[stat], _ptr(workspace),
        workspace.numel(), _ptr(order), _ptr(start), _ptr(w_plane), _stream_handle(stream)))
    return order, start, w_plane


NOALLOC_MAX_RECORDS = 1 << 20


def wpartition_noalloc(w, n_planes: int, absolute: bool = True, stat: str = "mean", order=None,
                       plane_start=None, w_plane=None, stream=None):
    """wpartition without a workspace (the library's static device scratch;
    at most 2^20 records; calls on one device must not overlap).  Outputs
    may be passed in (order int32 [n], plane_start int64 [M + 1], w_plane
    float64 [M]); any that is None is allocated here with torch."""
    import torch
    if w.dtype != torch.float64 or not w.is_cuda or w.dim() != 1:
        raise ValueError("w must be a 1-D float64 device tensor")
    w = w.contiguous()
    n = w.numel()
    dev = w.device
    if order is None:
        order = torch.empty(n, dtype=torch.int32, device=dev)
    if plane_start is None:
        plane_start = torch.empty(n_planes + 1, dtype=torch.int64, device=dev)
    if w_plane is None:
        w_plane = torch.empty(n_planes, dtype=torch.float64, device=dev)
    _require(order, torch.int32, "order", numel=n, device=dev.index)
    _require(plane_start, torch.int64, "plane_start", numel=n_planes + 1, device=dev.index)
    _require(w_plane, torch.float64, "w_plane", numel=n_planes, device=dev.index)
    with torch.cuda.device(dev):
        _check(load_library().wkern_wpartition_noalloc(
            _ptr(w), n, int(n_planes), 1 if absolute else 0, WSTAT[stat], _ptr(order),
            _ptr(plane_start), _ptr(w_plane), _stream_handle(stream)))
    return order, plane_start, w_plane


STORE_PATTERNS = {"one_store_per_lane": 0, "unit_walk": 1}


def store_ceiling(buf, pattern: str = "one_store_per_lane", stream=None):
    """Write zeros over the device tensor buf with the given store structure
    (diagnostic: the device's store ceilings, for the resample's roofline)."""
    import torch
    if not (isinstance(buf, torch.Tensor) and buf.is_cuda and buf.is_contiguous()):
        raise ValueError("buf must be a contiguous device tensor")
    nbytes = buf.numel() * buf.element_size()
    _check(load_library().wkern_store_ceiling(_ptr(buf), nbytes - nbytes % 16,
                                              STORE_PATTERNS[pattern], _stream_handle(stream)))
