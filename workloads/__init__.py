"""Seeded synthetic inputs for w-kernel generation.

This module is shared by the oracle, the tests and the benchmark.  It holds
only the *inputs* of the method (per-plane w values, per-plane supports, the
image-domain anti-aliasing taper sampled on the radial nodes, geometry
scalars); it performs none of the method's arithmetic (no screen, no Hankel
transform, no interpolation, no layout).

The taper is handed to the method as samples at the normalised radial
positions nu_i = (i + 1/2) / Nr of r / r_max (the midpoint nodes of the
discrete Hankel quadrature); a workload therefore fixes nu_i -> tau_i.

Workloads (their shapes follow the paper's experiments, section 5 and the
imager settings IM-S / IM-L):

* ``plain``      8 w-planes, w in [0, 1000] lambda, Gaussian taper
                 sigma = 0.02 on r <= 0.05, Nr = 128, support 31, os 4.
* ``paper``      2048^2 image at 3.5 arcsec, 256 w-planes on [0, 20000]
                 lambda, prolate-spheroidal taper (m = 6, alpha = 1),
                 Nr = 4096, support 7..127 growing with |w|, os 8.
* ``precision``  ``plain`` run through the split-BF16 contraction.
* ``batch``      16 channels (1.0-1.5 GHz) x 1024 w-planes with 1/|w|
                 density on +-[40, 40000] lambda, Nr = 8192, os 8,
                 supports 7..255: 16384 kernels in one launch.
* ``grad``       256 w-planes on [0, 1000] lambda, 2048 free taper samples
                 (seeded spheroidal + N(0, 1e-3)), support 127, os 4.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED = 1904
ARCSEC = math.pi / (180.0 * 3600.0)


@dataclass
class Workload:
    name: str
    image_size: int
    cellsize: float          # radians (direction-cosine increment)
    n_radial: int
    oversampling: int
    radial_refine: int
    w: np.ndarray            # float64 [P], wavelengths
    support: np.ndarray      # int32 [P], odd full widths
    max_support: int
    taper: np.ndarray        # float32 [Nr], samples at nu_i = (i+1/2)/Nr
    precision: str = "fp32"  # "fp32" | "bf16x6"
    interp: str = "cubic"    # "cubic" | "linear"
    taper_fn: object = field(default=None, repr=False)  # callable of r (radians) or None
    notes: str = ""
    mirror: object = field(default=None, repr=False)  # int32 [P]: -1 or the plane with -w

    @property
    def n_planes(self) -> int:
        return int(self.w.shape[0])

    @property
    def r_max(self) -> float:
        return 0.5 * self.image_size * self.cellsize


def mirror_table(w: np.ndarray, support: np.ndarray) -> np.ndarray:
    """Pairs planes whose w values are exact negatives of each other (same
    support): the later plane of a pair gets the index of the earlier one,
    every other plane -1.  w = 0 is never paired."""
    w = np.asarray(w, dtype=np.float64)
    mir = np.full(w.shape[0], -1, dtype=np.int32)
    open_ = {}  # (w, support) of an unpaired plane -> its index
    for p in range(w.shape[0]):
        if w[p] == 0.0:
            continue
        q = open_.pop((float(-w[p]), int(support[p])), None)
        if q is not None:
            mir[p] = q
        else:
            open_.setdefault((float(w[p]), int(support[p])), p)
    return mir


def nodes_nu(n_radial: int) -> np.ndarray:
    """Normalised radial sample positions nu_i = (i + 1/2)/Nr of the taper."""
    return (np.arange(n_radial, dtype=np.float64) + 0.5) / n_radial


# --------------------------------------------------------------------------
# Tapers (image-domain anti-aliasing functions, the IAA-kernel of section 3)
# --------------------------------------------------------------------------
def gaussian_taper(sigma: float):
    """Radially symmetric Gaussian AA function exp(-r^2 / (2 sigma^2))."""
    return lambda r: np.exp(-np.asarray(r, dtype=np.float64) ** 2 / (2.0 * sigma * sigma))


def _pswf_nystrom(c: float, alpha: float, n_nodes: int = 160):
    """Order-0 prolate spheroidal function psi_{alpha,0}(c, nu) on [-1, 1].

    It is the even eigenfunction with the largest eigenvalue of
        lambda psi(nu) = int_{-1}^{1} exp(i c nu eta) (1 - eta^2)^alpha psi(eta) d eta,
    discretised with Gauss-Jacobi(alpha, alpha) nodes (Nystrom).  For even
    psi the kernel reduces to cos(c nu eta).  Returns a callable of nu,
    normalised so that psi(0) = 1.
    """
    from scipy.special import roots_jacobi

    eta, wts = roots_jacobi(n_nodes, alpha, alpha)
    sw = np.sqrt(wts)
    kern = np.cos(c * np.outer(eta, eta))
    sym = sw[:, None] * kern * sw[None, :]
    vals, vecs = np.linalg.eigh(sym)
    j = int(np.argmax(vals))
    lam = vals[j]
    psi_nodes = vecs[:, j] / sw

    def psi(nu):
        nu = np.asarray(nu, dtype=np.float64)
        return (np.cos(c * np.multiply.outer(nu, eta)) @ (wts * psi_nodes)) / lam

    p0 = float(psi(np.array(0.0)))
    return lambda nu: psi(nu) / p0, lam, (eta, wts, psi_nodes)


def spheroidal_taper(r_max: float, m: int = 6, alpha: float = 1.0, n_nodes: int = 160):
    """psi_{alpha,0}(c = pi m / 2, r / r_max) / psi(0), as a callable of r."""
    fn, _, _ = _pswf_nystrom(math.pi * m / 2.0, alpha, n_nodes)
    return lambda r: fn(np.asarray(r, dtype=np.float64) / r_max)


def sample_taper(fn, n_radial: int, r_max: float) -> np.ndarray:
    return np.asarray(fn(nodes_nu(n_radial) * r_max), dtype=np.float64).astype(np.float32)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
def plain(n_radial: int = 128, precision: str = "fp32", interp: str = "cubic",
          radial_refine: int = 1, extra_w=()) -> Workload:
    """8 w-planes at bin centres of [0, 1000] lambda, Gaussian taper sigma 0.02,
    r in [0, 0.05] (N = 128, cell = 7.8125e-4), support 31, os 4."""
    n, cell = 128, 7.8125e-4
    r_max = 0.5 * n * cell
    w = 1000.0 * (np.arange(8) + 0.5) / 8.0
    if len(extra_w):
        w = np.concatenate([w, np.asarray(extra_w, dtype=np.float64)])
    fn = gaussian_taper(0.02)
    return Workload(
        name="plain", image_size=n, cellsize=cell, n_radial=n_radial, oversampling=4,
        radial_refine=radial_refine, w=w.astype(np.float64),
        support=np.full(w.shape[0], 31, dtype=np.int32), max_support=31,
        taper=sample_taper(fn, n_radial, r_max), precision=precision, interp=interp,
        taper_fn=fn,
        notes="Gaussian sigma=0.02; w bin centres of [0,1000]")


def precision(**kw) -> Workload:
    wl = plain(precision="bf16x6", **kw)
    wl.name = "precision"
    return wl


def paper(n_planes: int = 256, n_radial: int = 4096, precision: str = "fp32") -> Workload:
    """2048^2 image at 3.5 arcsec (FOV ~2 deg), 256 w-planes on [0, 20000] lambda,
    PSWF taper (m=6, alpha=1), Nr = 4096, os 8; half-support 3 + rint(60 w / 20000)."""
    n, cell = 2048, 3.5 * ARCSEC
    r_max = 0.5 * n * cell
    w = 20000.0 * (np.arange(n_planes) + 0.5) / n_planes
    h = 3 + np.rint(60.0 * np.abs(w) / 20000.0).astype(np.int64)
    fn = spheroidal_taper(r_max)
    return Workload(
        name="paper", image_size=n, cellsize=cell, n_radial=n_radial, oversampling=8,
        radial_refine=1, w=w, support=(2 * h + 1).astype(np.int32), max_support=127,
        taper=sample_taper(fn, n_radial, r_max), precision=precision, taper_fn=fn,
        notes="PSWF m=6 alpha=1; w bin centres of [0,20000]; S = 7..127")


def batch_w(n_w: int = 1024, n_chan: int = 16):
    """1/|w| density: |w|_j = 40 * 1000^((j+1/2)/(n_w/2)), mirrored to negatives;
    channel c scales w by nu_c / 1 GHz, nu_c = 1.0 + 0.5 c / (n_chan - 1) GHz.
    Plane order: channel-major, w ascending within a channel."""
    half = n_w // 2
    mag = 40.0 * 1000.0 ** ((np.arange(half) + 0.5) / half)
    wv = np.concatenate([-mag[::-1], mag])
    if n_chan > 1:
        nu = 1.0 + 0.5 * np.arange(n_chan) / (n_chan - 1)
    else:
        nu = np.ones(1)
    return (nu[:, None] * wv[None, :]).reshape(-1)


def batch(n_w: int = 1024, n_chan: int = 16, n_radial: int = 8192,
          precision: str = "bf16x6") -> Workload:
    """Config of the batching experiment: paper geometry and taper, Nr = 8192,
    os 8, half-support 3 + rint(124 |w| / max|w|) (S = 7..255)."""
    n, cell = 2048, 3.5 * ARCSEC
    r_max = 0.5 * n * cell
    w = batch_w(n_w, n_chan)
    h = 3 + np.rint(124.0 * np.abs(w) / np.max(np.abs(w))).astype(np.int64)
    fn = spheroidal_taper(r_max)
    sup = (2 * h + 1).astype(np.int32)
    return Workload(
        name="batch", image_size=n, cellsize=cell, n_radial=n_radial, oversampling=8,
        radial_refine=1, w=w, support=sup, max_support=255,
        taper=sample_taper(fn, n_radial, r_max), precision=precision, taper_fn=fn,
        notes="16 ch x 1024 w, 1/|w| density on +-[40,40000], S = 7..255",
        mirror=mirror_table(w, sup))


def grad(n_planes: int = 256, n_radial: int = 2048, noise: float = 1e-3,
         precision: str = "fp32") -> Workload:
    """Differentiation workload: r_max = 0.05 (N 128, cell 7.8125e-4), Nr = 2048
    free taper samples psi(3 pi, nu) + N(0, noise) (seed 1904), w on [0, 1000],
    support 127, os 4."""
    n, cell = 128, 7.8125e-4
    r_max = 0.5 * n * cell
    w = 1000.0 * (np.arange(n_planes) + 0.5) / n_planes
    fn = spheroidal_taper(r_max)
    rng = np.random.default_rng(SEED)
    tau = fn(nodes_nu(n_radial) * r_max) + rng.normal(0.0, noise, n_radial)
    return Workload(
        name="grad", image_size=n, cellsize=cell, n_radial=n_radial, oversampling=4,
        radial_refine=1, w=w, support=np.full(n_planes, 127, dtype=np.int32),
        max_support=127, taper=tau.astype(np.float32), precision=precision, taper_fn=None,
        notes="free taper samples (PSWF + noise), S = 127")


def fd_directions(n: int, count: int = 16, seed: int = SEED) -> np.ndarray:
    """Seeded unit directions [count, n] for directional finite differences."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(count, n))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def fd_taper_coords(n: int, count: int = 32, tail: int = 8) -> np.ndarray:
    """Taper coordinates for finite differences: count - tail spread over the
    radial nodes and the last `tail` nodes (next to r_max)."""
    spread = np.rint(np.linspace(0, n - tail - 1, count - tail)).astype(np.int64)
    return np.concatenate([spread, np.arange(n - tail, n)])


def random_small(seed: int, n_planes: int = 5, n_radial: int = 96, os_: int = 3,
                 max_support: int = 21, precision: str = "fp32", interp: str = "cubic",
                 radial_refine: int = 1) -> Workload:
    """Small randomised workload for property tests: random signed w, random odd
    supports, a random smooth taper."""
    rng = np.random.default_rng(seed)
    n, cell = 128, 7.8125e-4
    w = rng.uniform(-1500.0, 1500.0, n_planes)
    h = rng.integers(0, (max_support - 1) // 2 + 1, n_planes)
    nu = nodes_nu(n_radial)
    coef = rng.normal(0.0, 0.3, 4)
    tau = np.exp(-(nu / 0.45) ** 2) * (1.0 + coef[0] * nu + coef[1] * nu ** 2) + 0.01 * coef[2]
    return Workload(
        name=f"random{seed}", image_size=n, cellsize=cell, n_radial=n_radial,
        oversampling=os_, radial_refine=radial_refine, w=w,
        support=(2 * h + 1).astype(np.int32), max_support=max_support,
        taper=tau.astype(np.float32), precision=precision, interp=interp,
        notes="randomised property-test workload")


# --------------------------------------------------------------------------
# Visibility w coordinates: the input of the w-plane partition
# --------------------------------------------------------------------------
C_LIGHT = 299792458.0


def y_array(n_per_arm: int = 9, arm_m: float = 1900.0, az0_deg: float = 5.0,
            seed: int = SEED) -> np.ndarray:
    """East-north-up positions (m) of a Y-shaped array: three arms at azimuths
    az0, az0 + 120, az0 + 240 deg with antennas at d_k = arm (k / n)^1.7,
    k = 1..n, plus a seeded 1 m jitter."""
    rng = np.random.default_rng(seed)
    pos = []
    for arm in range(3):
        az = np.deg2rad(az0_deg + 120.0 * arm)
        for k in range(1, n_per_arm + 1):
            d = arm_m * (k / n_per_arm) ** 1.7
            pos.append([d * np.sin(az), d * np.cos(az), 0.0])
    return np.asarray(pos) + rng.normal(0.0, 1.0, (3 * n_per_arm, 3)) * [1.0, 1.0, 0.1]


def uvw_tracks(enu: np.ndarray, freq_hz: float, dec_deg: float, lat_deg: float,
               n_times: int, ha_span_h: float = 12.0):
    """(u, v, w) in wavelengths of every baseline at n_times hour angles evenly
    spread over +-ha_span/2; records time-major (all baselines of a dump, then
    the next dump), as a measurement set holds them."""
    lat, dec = np.deg2rad(lat_deg), np.deg2rad(dec_deg)
    e, n_, u_ = enu[:, 0], enu[:, 1], enu[:, 2]
    xyz = np.stack([-np.sin(lat) * n_ + np.cos(lat) * u_, e,
                    np.cos(lat) * n_ + np.sin(lat) * u_], axis=1)
    a, b = np.triu_indices(enu.shape[0], 1)
    bl = (xyz[b] - xyz[a]) * (freq_hz / C_LIGHT)
    ha = np.deg2rad(15.0 * ha_span_h * ((np.arange(n_times) + 0.5) / n_times - 0.5))
    sh, ch = np.sin(ha)[:, None], np.cos(ha)[:, None]
    X, Y, Z = bl[:, 0][None, :], bl[:, 1][None, :], bl[:, 2][None, :]
    u = sh * X + ch * Y
    v = -np.sin(dec) * ch * X + np.sin(dec) * sh * Y + np.cos(dec) * Z
    w = np.cos(dec) * ch * X - np.cos(dec) * sh * Y + np.sin(dec) * Z
    return u.reshape(-1), v.reshape(-1), w.reshape(-1)


def vla_c_74mhz_w(n_times: int = 1440) -> np.ndarray:
    """w of the partition workload shaped like the paper's simulation (section
    5): a 27-antenna Y array of C-configuration extent at 74 MHz, pointing at
    dec +47.34 deg from latitude 34.08 deg, 351 baselines x 1440 dumps over
    +-6 h = 505440 records."""
    _, _, w = uvw_tracks(y_array(), 74e6, 47.339, 34.079, n_times)
    return w


def multichannel_w(w: np.ndarray, n_chan: int, f_lo: float = 1.0, f_hi: float = 1.5) -> np.ndarray:
    """The same records over n_chan channels, w scaled by nu_c / nu_lo,
    nu_c evenly spaced on [f_lo, f_hi]; channel-major."""
    if n_chan == 1:
        return np.asarray(w, dtype=np.float64).copy()
    nu = f_lo + (f_hi - f_lo) * np.arange(n_chan) / (n_chan - 1)
    return (np.asarray(w, dtype=np.float64)[None, :] * (nu / f_lo)[:, None]).reshape(-1)


def point_source_vis(u, v, w, sources) -> np.ndarray:
    """Visibilities of point sources (amplitude, l, m):
    V = sum A exp(-j 2 pi (u l + v m + w (n - 1))), n = sqrt(1 - l^2 - m^2)
    (the measurement equation of section 1 with the w-term kept); complex64."""
    vis = np.zeros(np.shape(u), dtype=np.complex128)
    for a, l, m in sources:
        n = math.sqrt(1.0 - l * l - m * m)
        vis += a * np.exp(-2j * math.pi * (u * l + v * m + w * (n - 1.0)))
    return vis.astype(np.complex64)


def diagonal_sources(n_src: int = 5, max_deg: float = 12.0):
    """Equal 1 Jy sources on the image diagonal from the centre out to
    max_deg (the 5DIAG layout of section 5)."""
    out = []
    for k in range(n_src):
        rad = math.radians(max_deg) * k / max(n_src - 1, 1)
        out.append((1.0, rad / math.sqrt(2.0), -rad / math.sqrt(2.0)))
    return out


@dataclass
class GridWorkload:
    name: str
    image_size: int
    cellsize: float
    grid_size: int
    n_radial: int
    oversampling: int
    n_planes: int
    max_support: int
    taper: np.ndarray       # float32 [Nr]
    u: np.ndarray           # float64 [n] wavelengths
    v: np.ndarray
    w: np.ndarray
    vis: np.ndarray         # complex64 [n]
    frac: float = 0.01      # kernel truncation fraction


def grid_paper(n_times: int = 1440, n_planes: int = 128, n_radial: int = 4096) -> GridWorkload:
    """The paper's imaging setting on the synthetic records: IM-S (2048^2 at
    60 arcsec), 128 |w|-planes, os 8, maximum support 255 (half-width 127),
    1% truncation, Gaussian AA taper (sigma = r_max / 6), five 1 Jy sources on
    the diagonal out to 12 deg; 505440 records at 74 MHz."""
    n, cell = 2048, 60.0 * ARCSEC
    r_max = 0.5 * n * cell
    enu = y_array()
    u, v, w = uvw_tracks(enu, 74e6, 47.339, 34.079, n_times)
    vis = point_source_vis(u, v, w, diagonal_sources())
    fn = gaussian_taper(r_max / 6.0)
    return GridWorkload("grid_paper", n, cell, n, n_radial, 8, n_planes, 255,
                        sample_taper(fn, n_radial, r_max), u, v, w, vis)


def grid_small(seed: int = 0, n_rec: int = 600, n_planes: int = 6, grid_size: int = 96,
               os_: int = 4, max_support: int = 15) -> GridWorkload:
    """Small gridding case for full-grid parity: plain geometry (r_max 0.05),
    random records inside the grid and random complex visibilities."""
    rng = np.random.default_rng(SEED + seed)
    n, cell = 128, 7.8125e-4
    du = 1.0 / (n * cell)
    half = 0.5 * grid_size * du
    u = rng.uniform(-0.8 * half, 0.8 * half, n_rec)
    v = rng.uniform(-0.8 * half, 0.8 * half, n_rec)
    w = rng.uniform(-1000.0, 1000.0, n_rec)
    vis = (rng.normal(size=n_rec) + 1j * rng.normal(size=n_rec)).astype(np.complex64)
    fn = gaussian_taper(0.02)
    return GridWorkload(f"grid_small{seed}", n, cell, grid_size, 128, os_, n_planes, max_support,
                        sample_taper(fn, 128, 0.5 * n * cell), u, v, w, vis)


WORKLOADS = {
    "plain": plain,
    "paper": paper,
    "precision": precision,
    "batch": batch,
    "grad": grad,
}
