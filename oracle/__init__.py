"""FP64 CPU oracle for w-projection kernel generation (test infrastructure).

This package is test infrastructure only.  Nothing in the product path may
import, call, link or execute it: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP path; the only module both sides import is ``workloads`` (seeded
inputs, none of the method's arithmetic).

What it computes (Lucas, Skipper & Scaife 2019, "Fast W-Projection for
Wide-field Imaging"):

* ``hankel``   -- the optimised algorithm (section 4.4, Algorithm 2): screen
  tau(r) * G(r, w) with G from the w-projection kernel equation (section
  2.5), the order-0 Hankel transform (section 4.3, equation ht) as a discrete
  transform matrix times the sampled screen, radial cubic/linear spline
  (section 4.3.2) and extraction of the oversampled kernel cache.
* ``fft2d``    -- the standard algorithm (section 3, Algorithm 1): the same
  screen on a Cartesian workspace, zero padded by the oversampling factor,
  2D DFT, kernel cache extraction.  This is the twin the Hankel path is
  compared against inside the circular region (section 4.4).
* ``projslice`` -- the paper's own Hankel engine (section 4.3.1): 1D
  projection of the workspace screen, zero-padded 1D FFT, then the same
  interpolation as ``hankel``.
* ``gridding`` -- the step that consumes the kernels in Algorithm 2:
  each record's oversampled sub-kernel added onto the uv grid.
* ``wpartition`` -- the w-plane partition that opens Algorithms 1 and 2:
  sort by (absolute) w, equal-size planes, average or median w per plane.
* ``adjoint``  -- the exact gradient of a real loss of the kernel cache with
  respect to the taper samples and the w values (no paper counterpart; the
  chain rule applied to the functions above).

Parity status of each function is listed in its docstring.  Readings of the
paper where it is silent or ambiguous are listed in ``hankel``'s header.
"""
from . import hankel, fft2d, adjoint, gridding, projslice, wpartition  # noqa: F401
