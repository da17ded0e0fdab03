"""Oracle twin: standard w-projection kernel generation by 2D FFT (FP64, CPU).

Test infrastructure only; see the package header.  Follows Algorithm 1 of
Lucas, Skipper & Scaife (2019) (section 3 and 3.1): the w-kernel times the
IAA-kernel on a Cartesian image-domain workspace, zero padding by the
oversampling ratio, a 2D FFT, extraction of the oversampled kernel cache.
Workspace undersampling (section 4.2) sets the workspace to the next power of
two at or above the full kernel width.

Readings (in addition to the ones in ``oracle.hankel``):

F1  Workspace pixel l_x = (x - N_ws/2) * FOV/N_ws, x = 0..N_ws-1, and the screen
    is zero outside the open disc r < r_max; the strict inequality removes the
    unpaired row/column at -N_ws/2 so the sampled screen is even.
F2  The forward transform carries exp(-j 2 pi (u l + v m)) (section 1, eq.
    interferom_smallfov) and the area element (FOV/N_ws)^2, so that it
    approximates the continuous 2D FT; the padded transform has uv spacing
    du / os, so the sample at uv offset (X, Y) du/os is bin (X, Y) from the
    centre.
F3  A taper given only as radial samples is evaluated at Cartesian radii by
    linear interpolation in r between the midpoint nodes (held constant
    inside the first node).
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def next_pow2(n: int) -> int:
    """Smallest power of two >= n (section 4.2 and section 6.4: the workspace is
    the power of two at or above the full kernel size 2 support + 1)."""
    p = 1
    while p < n:
        p *= 2
    return p


def taper_from_samples(samples, r_max: float):
    """Callable of r built from radial samples at the midpoint nodes (F3)."""
    tau = np.asarray(samples, dtype=np.float64)
    nr = tau.shape[0]
    nodes = (np.arange(nr) + 0.5) * (r_max / nr)
    return lambda r: np.interp(np.asarray(r, dtype=np.float64), nodes, tau)


def workspace_screen(taper_fn, w: float, n_ws: int, fov: float) -> np.ndarray:
    """IConv-kernel of Algorithm 1 on an n_ws^2 workspace (rows = m, cols = l):
    tau(r) exp(+j 2 pi w (1 - sqrt(1 - r^2))) inside r < r_max, zero outside."""
    dl = fov / n_ws
    r_max = 0.5 * fov
    l = (np.arange(n_ws) - n_ws // 2) * dl
    r2 = l[None, :] ** 2 + l[:, None] ** 2
    inside = r2 < r_max * r_max
    r2c = np.where(inside, r2, 0.0)
    phi = r2c / (1.0 + np.sqrt(1.0 - r2c))
    val = taper_fn(np.sqrt(r2c)) * np.exp(1j * TWO_PI * w * phi)
    return np.where(inside, val, 0.0)


def padded_transform(scr: np.ndarray, oversampling: int, fov: float) -> np.ndarray:
    """Zero pad the centred workspace by os (Algorithm 1) and transform (F2).
    Returns the centred spectrum: index L/2 + X along each axis is uv offset
    X du / os, L = os n_ws."""
    n_ws = scr.shape[0]
    big_n = oversampling * n_ws
    big = np.zeros((big_n, big_n), dtype=np.complex128)
    o = big_n // 2 - n_ws // 2
    big[o:o + n_ws, o:o + n_ws] = scr
    dl = fov / n_ws
    spec = np.fft.fft2(np.fft.ifftshift(big)) * dl * dl
    return np.fft.fftshift(spec)


def extract_cache(spec: np.ndarray, support: int, oversampling: int) -> np.ndarray:
    """Kernel cache [os][os][S][S] from the centred spectrum, with the same
    sample offsets and circular support as the Hankel path (readings R7, R8)."""
    big_n = spec.shape[0]
    h = (support - 1) // 2
    os_ = oversampling
    fv = np.arange(os_)[:, None, None, None]
    fu = np.arange(os_)[None, :, None, None]
    b = np.arange(support)[None, None, :, None]
    a = np.arange(support)[None, None, None, :]
    x = os_ * (a - h) - fu
    y = os_ * (b - h) - fv
    x, y = np.broadcast_arrays(x, y)
    mask = x * x + y * y <= (os_ * h) ** 2
    c = big_n // 2
    if os_ * h + os_ > c:
        raise ValueError("kernel support exceeds the padded workspace")
    out = spec[c + y, c + x]
    return np.where(mask, out, 0.0)


def generate(taper_fn, w, support, oversampling: int, n_ws: int, fov: float):
    """Algorithm 1 (kernel generation part) for each plane; one workspace size for
    all planes.  Returns a list of [os][os][S][S] complex128 caches."""
    w = np.asarray(w, dtype=np.float64)
    support = np.asarray(support)
    out = []
    for p in range(len(w)):
        spec = padded_transform(workspace_screen(taper_fn, float(w[p]), n_ws, fov),
                                oversampling, fov)
        out.append(extract_cache(spec, int(support[p]), oversampling))
    return out


def direct_dft(scr: np.ndarray, oversampling: int, fov: float, xs, ys) -> np.ndarray:
    """Brute-force 2D DFT of a workspace screen at uv offsets (X, Y) du/os:
    sum over pixels of s(l, m) exp(-j 2 pi (u l + v m)) dl^2.  Used only to pin
    ``padded_transform`` on small grids."""
    n_ws = scr.shape[0]
    dl = fov / n_ws
    du = 1.0 / fov
    l = (np.arange(n_ws) - n_ws // 2) * dl
    xs = np.asarray(xs)
    ys = np.asarray(ys)
    out = np.zeros(xs.shape, dtype=np.complex128)
    for idx in np.ndindex(xs.shape):
        u = xs[idx] * du / oversampling
        v = ys[idx] * du / oversampling
        ph = np.exp(-1j * TWO_PI * (u * l[None, :] + v * l[:, None]))
        out[idx] = np.sum(scr * ph) * dl * dl
    return out
