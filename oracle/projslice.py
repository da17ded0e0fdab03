"""Oracle for the projection-slice Hankel engine (FP64, CPU).  Test
infrastructure only; see the package header.

Section 4.3.1 computes the order-0 Hankel transform of the radially
symmetric IConv-kernel through the projection-slice theorem: the 1D Fourier
transform of the kernel's projection onto a line is the slice of its 2D
Fourier transform along that line.  Algorithm 2 spells the steps out per
w-plane: screen on the (undersampled) workspace, 1D projection, zero padding
by the oversampling ratio, 1D FFT; the radial line then goes through the
same interpolation and cache extraction as the matrix-form transform
(oracle.hankel.resample).

Readings (in addition to R1-R10 of oracle.hankel and F1-F3 of
oracle.fft2d, which fix the workspace grid, the disc, the taper
interpolation and the transform's sign and scale):

PS1 The workspace of a plane is the power of two at or above its full width
    S_p (section 4.2, workspace undersampling), or at or above the maximum
    support for every plane (the fixed setting of sections 5 and 6.4), and
    at least 2 (a centred workspace needs an even width); it is doubled
    until the padded transform reaches the line's last node,
    q os N_ws / 2 >= nrho = q os h + 4.
PS2 Projection onto the l axis: p(l) = sum over m of s(l, m) dm; transform
    K(rho) = sum over l of p(l) exp(-j 2 pi rho l) dl, zero padded by q os so
    that the line has the matrix form's spacing du / (q os) (reading R9).
    By the discrete projection-slice theorem this line is, sample for
    sample, the v = 0 row of the zero-padded 2D transform of the same
    workspace (oracle.fft2d.padded_transform).

Parity: pinned in tests/test_oracle_pins.py against the 2D twin's v = 0 row
(an independent 2D FFT of the same screen), against the Gaussian closed
form on a smooth-edged workload, and by brute-force summation on a tiny grid.
"""
from __future__ import annotations

import math

import numpy as np

from . import fft2d as F
from . import hankel as H

TWO_PI = 2.0 * math.pi


def workspace_size(support: int, oversampling: int, radial_refine: int = 1,
                   min_width: int | None = None) -> int:
    """N_ws of a plane (PS1)."""
    n = F.next_pow2(max(support, min_width or 0, 2))
    nrho = radial_refine * oversampling * ((support - 1) // 2) + 4
    while radial_refine * oversampling * n // 2 < nrho:
        n *= 2
    return n


def projection(scr: np.ndarray, fov: float) -> np.ndarray:
    """p(l) = sum_m s(l, m) dm on the workspace (rows m, columns l) (PS2)."""
    return scr.sum(axis=0) * (fov / scr.shape[0])


def line(taper_fn, w: float, support: int, oversampling: int, fov: float,
         radial_refine: int = 1, n_ws: int | None = None) -> np.ndarray:
    """Radial line K(rho_k), k = 0 .. q os h + 3, by projection and a zero-
    padded 1D FFT (Algorithm 2)."""
    n_ws = n_ws or workspace_size(support, oversampling, radial_refine)
    pad = radial_refine * oversampling
    nrho = pad * ((support - 1) // 2) + 4
    if pad * n_ws // 2 < nrho:
        raise ValueError("workspace too small for the line")
    p = projection(F.workspace_screen(taper_fn, w, n_ws, fov), fov)
    big = np.zeros(pad * n_ws, dtype=np.complex128)
    c = pad * n_ws // 2
    big[c - n_ws // 2:c + n_ws // 2] = p
    spec = np.fft.fftshift(np.fft.fft(np.fft.ifftshift(big))) * (fov / n_ws)
    return spec[c:c + nrho].copy()


def generate(taper_fn, w, support, oversampling: int, fov: float, radial_refine: int = 1,
             interp: str = "cubic", fixed_width: int | None = None):
    """Kernel caches [os][os][S][S] of every plane through the projection-slice
    line and the matrix form's interpolation.  fixed_width: one workspace for
    all planes at or above this width (PS1), else per plane."""
    w = np.asarray(w, dtype=np.float64)
    support = np.asarray(support)
    caches, lines = [], []
    for p in range(len(w)):
        s = int(support[p])
        n_ws = workspace_size(s, oversampling, radial_refine, fixed_width)
        k = line(taper_fn, float(w[p]), s, oversampling, fov, radial_refine, n_ws)
        lines.append(k)
        caches.append(H.resample(k, s, oversampling, radial_refine, interp))
    return caches, lines


def brute_line(scr: np.ndarray, fov: float, pad: int, nrho: int) -> np.ndarray:
    """K(rho_k) = sum_{l, m} s(l, m) exp(-j 2 pi rho_k l) dl dm written out as
    a double loop; used only to pin ``line`` on tiny grids."""
    n_ws = scr.shape[0]
    dl = fov / n_ws
    out = np.zeros(nrho, dtype=np.complex128)
    for k in range(nrho):
        rho = k / (pad * fov)
        acc = 0.0 + 0.0j
        for x in range(n_ws):
            lx = (x - n_ws // 2) * dl
            ph = np.exp(-1j * TWO_PI * rho * lx)
            for y in range(n_ws):
                acc += scr[y, x] * ph
        out[k] = acc * dl * dl
    return out
