"""Oracle for the optimised w-projection kernel generator (FP64, CPU).

Test infrastructure only; see the package header.  Follows Lucas, Skipper &
Scaife (2019), section 4 and Algorithm 2, in the paper's order:

  screen (w-kernel times IAA-kernel, section 2.5 eq. wproj_G and Algorithm 2)
  -> order-0 Hankel transform (section 4.3, eq. ht) as a matrix-vector product
     with a discrete HT matrix computed once (section 4.3)
  -> spline through the radial line with precomputed coefficients (4.3.2)
  -> oversampled 2D kernels over the circular support (4.4, Algorithm 2).

Readings taken where the paper is silent or ambiguous:

R1  Screen sign: G = exp(-j 2 pi w (n - 1)) with n = sqrt(1 - r^2), i.e.
    s(r) = tau(r) exp(+j 2 pi w phi(r)) with phi = 1 - n, evaluated in the
    cancellation-free form phi = r^2 / (1 + sqrt(1 - r^2)).  J0 is even, so
    the transform direction does not matter for the Hankel route.
R2  The 1/n factor of the wide-field equation is not part of the screen
    (Algorithm 2 multiplies only the w-kernel and the IAA-kernel).
R3  Normalisation: continuous-FT units, K(rho) = 2 pi int s(r) J0(2 pi rho r)
    r dr; no peak or sum normalisation.
R4  Discrete HT matrix: midpoint nodes r_i = (i + 1/2) dr, dr = r_max / Nr,
    weights r_i dr:  M[k, i] = 2 pi J0(2 pi rho_k r_i) r_i dr.
R5  r_max = image_size * cellsize / 2 (circular image region of diameter
    equal to the image size, section 4.4 and section 6.1); du = 1 / FOV.
R6  Supports are odd full widths S, half-width h = (S - 1) / 2.
R7  Oversampled sub-kernel (fv, fu) is sampled at uv offsets
    ((a - h) - fu / os, (b - h) - fv / os) cells; layout [fv][fu][b][a].
R8  Circular support: integer test X^2 + Y^2 <= (os h)^2 with
    X = os (a - h) - fu, Y = os (b - h) - fv; zero outside.
R9  Radial uv nodes rho_k = k du / (q os), q >= 1 (q = 1 is the spacing du/os
    the 1D zero padding by os gives), k = 0 .. q os h + 3.
R10 Cubic spline: interpolating, s'(0) = 0 (radial symmetry), natural
    (s'' = 0) at the last node; linear option = piecewise linear.
R11 Truncation (section 3.1 and Algorithm 2: the 1D conv-kernel is cut
    where its amplitude falls below a fraction f, default 1%, of its
    maximum): on the radial line computed for the maximum support, k* is
    the last node with |K(rho_k)| >= f max_k |K(rho_k)|; the plane's
    half-width is h = ceil(k* / (q os)) uv cells (so the circular support
    reaches rho_{k*}), clamped to the maximum half-width.  The cache is then
    sampled from the spline through the full line.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.linalg import solve_banded
from scipy.special import j0

TWO_PI = 2.0 * math.pi


@dataclass(frozen=True)
class Geometry:
    image_size: int
    cellsize: float
    n_radial: int
    oversampling: int
    radial_refine: int
    fov: float
    r_max: float
    du: float
    dr: float
    drho: float
    r: np.ndarray      # [Nr] radial image nodes
    phi: np.ndarray    # [Nr] 1 - sqrt(1 - r^2)


def geometry(image_size: int, cellsize: float, n_radial: int, oversampling: int,
             radial_refine: int = 1) -> Geometry:
    """Image- and uv-plane sampling (readings R4, R5, R9).  Parity: pinned by the
    closed-form Hankel tests (a wrong dr, r_i or rho_k spacing fails them)."""
    fov = image_size * cellsize
    r_max = 0.5 * fov
    du = 1.0 / fov
    dr = r_max / n_radial
    r = (np.arange(n_radial, dtype=np.float64) + 0.5) * dr
    phi = r * r / (1.0 + np.sqrt(1.0 - r * r))
    drho = du / (radial_refine * oversampling)
    return Geometry(image_size, cellsize, n_radial, oversampling, radial_refine,
                    fov, r_max, du, dr, drho, r, phi)


def half_support(support) -> np.ndarray:
    return (np.asarray(support, dtype=np.int64) - 1) // 2


def n_rho(support, oversampling: int, radial_refine: int = 1) -> np.ndarray:
    """Radial uv nodes per plane: q os h + 4 (three nodes beyond the last one
    any sample of the circular support reaches, reading R9)."""
    return radial_refine * oversampling * half_support(support) + 4


def offsets(support, oversampling: int) -> np.ndarray:
    """Start of each plane's [os][os][S][S] block in the concatenated cache, in
    complex elements; planes in the caller's order."""
    sizes = oversampling * oversampling * np.asarray(support, dtype=np.int64) ** 2
    return np.concatenate([[0], np.cumsum(sizes)])


def hankel_matrix(rho: np.ndarray, geo: Geometry) -> np.ndarray:
    """Discrete order-0 HT matrix (section 4.3, eq. ht, with k = 2 pi rho and the
    2 pi of the 2D FT of a radial function), midpoint rule (R4):
        M[k, i] = 2 pi J0(2 pi rho_k r_i) r_i dr.
    Parity: pinned by the Gaussian, Fresnel-chirp, disc and Airy closed forms."""
    arg = TWO_PI * np.outer(rho, geo.r)
    return TWO_PI * j0(arg) * (geo.r * geo.dr)[None, :]


def screen(taper: np.ndarray, w: np.ndarray, geo: Geometry) -> np.ndarray:
    """Image-domain convolution kernel on the radial nodes (Algorithm 2: w-kernel
    times IAA-kernel; section 2.5 eq. wproj_G; reading R1):
        s[i, p] = tau_i exp(+j 2 pi w_p phi_i).
    Parity: pinned by the disc closed form at rho = 0 (sign of the phase) and by
    the Fresnel-chirp closed form."""
    tau = np.asarray(taper, dtype=np.float64)
    theta = TWO_PI * np.outer(geo.phi, np.asarray(w, dtype=np.float64))
    return tau[:, None] * np.exp(1j * theta)


def radial_kernels(geo: Geometry, taper, w, support) -> list:
    """Hankel transform of each plane's screen, K_p[k] = sum_i M[k, i] s[i, p]
    for k < Nrho(p) (section 4.3: the HT as the product of the HT matrix, built
    once, with the sampled screen)."""
    nr = n_rho(support, geo.oversampling, geo.radial_refine)
    rho = np.arange(int(nr.max()), dtype=np.float64) * geo.drho
    m = hankel_matrix(rho, geo)
    s = screen(taper, w, geo)
    full = m @ s
    return [full[: int(nr[p]), p].copy() for p in range(len(nr))]


# --------------------------------------------------------------------------
# Interpolation (section 4.3.2)
# --------------------------------------------------------------------------
def spline_second_derivatives(y: np.ndarray) -> np.ndarray:
    """Second derivatives m_k of the interpolating cubic spline through
    (k, y_k), k = 0..n-1, unit spacing, with s'(0) = 0 and s''(n-1) = 0 (R10).

    Rows of the tridiagonal system (one per node):
      k = 0:        2 m_0 + m_1 = 6 (y_1 - y_0)                  (s'(0) = 0)
      0 < k < n-1:  m_{k-1} + 4 m_k + m_{k+1} = 6 (y_{k-1} - 2 y_k + y_{k+1})
      k = n-1:      m_{n-1} = 0                                   (natural)
    ``y`` may be [n] or [n, batch] and complex.  Parity: pinned by scipy's
    CubicSpline with the same end conditions and by exact reproduction of
    cubics that satisfy them.
    """
    y = np.asarray(y)
    n = y.shape[0]
    if n < 2:
        raise ValueError("a spline needs at least two nodes")
    ab = np.zeros((3, n))
    rhs = np.zeros(y.shape, dtype=np.result_type(y, np.float64))
    # super-diagonal (row 0), diagonal (row 1), sub-diagonal (row 2) in banded form
    ab[1, 0] = 2.0
    ab[0, 1] = 1.0
    rhs[0] = 6.0 * (y[1] - y[0])
    for k in range(1, n - 1):
        ab[2, k - 1] = 1.0
        ab[1, k] = 4.0
        ab[0, k + 1] = 1.0
        rhs[k] = 6.0 * (y[k - 1] - 2.0 * y[k] + y[k + 1])
    ab[1, n - 1] = 1.0
    if n >= 2:
        ab[2, n - 2] = 0.0
    rhs[n - 1] = 0.0
    return solve_banded((1, 1), ab, rhs)


def spline_eval(y: np.ndarray, m: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Evaluate the cubic spline (unit node spacing) at positions t in [0, n-1]:
    on [k, k+1] with u = t - k,
      s = (1-u) y_k + u y_{k+1} + ((1-u)^3 - (1-u)) m_k / 6 + (u^3 - u) m_{k+1} / 6."""
    n = y.shape[0]
    k = np.clip(np.floor(t).astype(np.int64), 0, n - 2)
    u = t - k
    v = 1.0 - u
    return (v * y[k] + u * y[k + 1]
            + (v ** 3 - v) * m[k] / 6.0 + (u ** 3 - u) * m[k + 1] / 6.0)


def linear_eval(y: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Piecewise-linear interpolation through (k, y_k)."""
    n = y.shape[0]
    k = np.clip(np.floor(t).astype(np.int64), 0, n - 2)
    u = t - k
    return (1.0 - u) * y[k] + u * y[k + 1]


def sample_positions(support: int, oversampling: int, radial_refine: int = 1):
    """Integer offsets of the kernel cache samples (R7, R8): returns
    (d2, mask) with shape [os][os][S][S], d2 = X^2 + Y^2, and the radial
    position of each sample in units of drho, t = q sqrt(d2)."""
    h = (support - 1) // 2
    os_ = oversampling
    fv = np.arange(os_)[:, None, None, None]
    fu = np.arange(os_)[None, :, None, None]
    b = np.arange(support)[None, None, :, None]
    a = np.arange(support)[None, None, None, :]
    x = os_ * (a - h) - fu
    y = os_ * (b - h) - fv
    d2 = x * x + y * y
    mask = d2 <= (os_ * h) ** 2
    t = radial_refine * np.sqrt(d2.astype(np.float64))
    return d2, mask, t


def resample(k_line: np.ndarray, support: int, oversampling: int, radial_refine: int = 1,
             interp: str = "cubic") -> np.ndarray:
    """Interpolate the radial line onto the oversampled circular kernel cache of
    one plane (section 4.3.2 and Algorithm 2): [os][os][S][S] complex, zero
    outside the circular support."""
    _, mask, t = sample_positions(support, oversampling, radial_refine)
    out = np.zeros(mask.shape, dtype=np.complex128)
    tt = t[mask]
    if interp == "cubic":
        m = spline_second_derivatives(k_line)
        out[mask] = spline_eval(k_line, m, tt)
    elif interp == "linear":
        out[mask] = linear_eval(k_line, tt)
    else:
        raise ValueError(interp)
    return out


def generate(image_size, cellsize, n_radial, oversampling, taper, w, support,
             radial_refine: int = 1, interp: str = "cubic", planes=None):
    """Whole chain of Algorithm 2 (kernel generation part) for the selected planes
    (default: all).  Returns (caches, lines): per-plane [os][os][S][S] complex128
    caches and the radial lines K_p."""
    geo = geometry(image_size, cellsize, n_radial, oversampling, radial_refine)
    w = np.asarray(w, dtype=np.float64)
    support = np.asarray(support)
    idx = np.arange(len(w)) if planes is None else np.asarray(planes)
    lines = radial_kernels(geo, taper, w[idx], support[idx])
    caches = [resample(lines[j], int(support[p]), oversampling, radial_refine, interp)
              for j, p in enumerate(idx)]
    return caches, lines


def truncated_half_support(line: np.ndarray, frac: float, oversampling: int,
                           radial_refine: int, h_max: int) -> int:
    """Half-width after truncation at `frac` of the maximum amplitude (R11)."""
    amp = np.abs(np.asarray(line))
    above = np.nonzero(amp >= frac * amp.max())[0]
    k_star = int(above[-1])
    h = -(-k_star // (radial_refine * oversampling))  # ceil
    return min(h, h_max)


def generate_truncated(image_size, cellsize, n_radial, oversampling, taper, w, max_support,
                       frac: float = 0.01, radial_refine: int = 1, interp: str = "cubic",
                       planes=None):
    """Algorithm 2 with the truncation step: every plane's radial line is
    computed for the maximum support, its support is chosen by R11, and its
    cache is sampled from the spline through the full line.  Returns
    (caches, supports, lines)."""
    geo = geometry(image_size, cellsize, n_radial, oversampling, radial_refine)
    w = np.asarray(w, dtype=np.float64)
    idx = np.arange(len(w)) if planes is None else np.asarray(planes)
    h_max = (max_support - 1) // 2
    lines = radial_kernels(geo, taper, w[idx], np.full(len(idx), max_support))
    supports, caches = [], []
    for line in lines:
        h = truncated_half_support(line, frac, oversampling, radial_refine, h_max)
        s = 2 * h + 1
        supports.append(s)
        caches.append(resample(line, s, oversampling, radial_refine, interp))
    return caches, np.asarray(supports, dtype=np.int32), lines


def generate_workload(wl, planes=None, interp=None):
    """Convenience wrapper taking a ``workloads.Workload``."""
    return generate(wl.image_size, wl.cellsize, wl.n_radial, wl.oversampling,
                    wl.taper, wl.w, wl.support, wl.radial_refine,
                    interp or wl.interp, planes)
