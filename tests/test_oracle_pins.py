"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms of the Hankel transform, special cases that reduce to textbook results,
Parseval, an independent library routine, brute force on tiny inputs, or
values the paper prints (tests/golden/).  Together they are chosen so that a
dropped factor, a wrong sign or index, or a transposed operand anywhere in the
oracle fails at least one of them.
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest
from scipy.interpolate import CubicSpline
from scipy.special import j1

import workloads as W
from oracle import adjoint as A
from oracle import projslice as PS
from oracle import fft2d as F
from oracle import hankel as H

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# Hankel matrix: closed forms (section 4.3, eq. ht)
# ---------------------------------------------------------------------------
def _chirp_gaussian_err(nr, w, sig=0.01):
    """Gaussian under a quadratic (Fresnel) chirp: s = exp(-a r^2) with
    a = 1/(2 sig^2) - j pi w has the 2D FT (pi/a) exp(-pi^2 rho^2 / a)."""
    geo = H.geometry(200, 1e-3, nr, 4)          # r_max = 0.1 = 10 sigma
    rho = np.linspace(0.0, 60.0, 121)
    a = 1.0 / (2 * sig * sig) - 1j * math.pi * w
    k = H.hankel_matrix(rho, geo) @ np.exp(-a * geo.r ** 2)
    ref = (math.pi / a) * np.exp(-math.pi ** 2 * rho ** 2 / a)
    return np.max(np.abs(k - ref)) / np.max(np.abs(ref))


@pytest.mark.parametrize("w", [0.0, 100.0, 1000.0])
def test_hankel_matrix_fresnel_gaussian_closed_form(w):
    e1024 = _chirp_gaussian_err(1024, w)
    e4096 = _chirp_gaussian_err(4096, w)
    assert e4096 < 4e-7
    # midpoint rule: second-order convergence in Nr
    assert 12.0 < e1024 / e4096 < 20.0


def test_hankel_w0_gaussian_closed_form():
    """w = 0 reduces to the transform of the taper alone: 2 pi sig^2 exp(-2 pi^2 sig^2 rho^2)."""
    sig = 0.01
    geo = H.geometry(200, 1e-3, 4096, 4)
    rho = np.linspace(0, 80, 161)
    k = H.hankel_matrix(rho, geo) @ np.exp(-geo.r ** 2 / (2 * sig * sig))
    ref = 2 * math.pi * sig * sig * np.exp(-2 * math.pi ** 2 * sig * sig * rho ** 2)
    assert np.max(np.abs(k - ref)) / ref[0] < 4e-7


@pytest.mark.parametrize("nr,tol", [(128, 1.5e-4), (8192, 3e-8)])
def test_hankel_w0_disc_is_airy(nr, tol):
    """Uniform disc of radius R: K(rho) = R J1(2 pi rho R) / rho (normalised by pi R^2)."""
    geo = H.geometry(128, 7.8125e-4, nr, 4)
    r_ = geo.r_max
    rho = np.arange(1, 400) * geo.drho
    k = H.hankel_matrix(rho, geo) @ np.ones(nr)
    ref = r_ * j1(2 * math.pi * rho * r_) / rho
    assert np.max(np.abs(k - ref)) / (math.pi * r_ * r_) < tol


@pytest.mark.parametrize("w", [100.0, 1000.0, -700.0])
def test_screen_and_hankel_disc_exact_phase_rho0(w):
    """rho = 0 with the exact phase over the disc r <= R (uniform taper):
    K(0) = 2 pi [F(1) - F(n_R)], F(n) = exp(c (n - 1)) (n / c - 1 / c^2),
    c = -j 2 pi w, n_R = sqrt(1 - R^2).  Goes through oracle.hankel.screen,
    so it pins the sign of the phase and the cancellation-free phi."""
    geo = H.geometry(128, 7.8125e-4, 8192, 4)
    c = -2j * math.pi * w

    def fn(n):
        return np.exp(c * (n - 1.0)) * (n / c - 1.0 / c ** 2)

    ref = 2 * math.pi * (fn(1.0) - fn(math.sqrt(1.0 - geo.r_max ** 2)))
    lines = H.radial_kernels(geo, np.ones(8192), np.array([w]), np.array([3]))
    got = lines[0][0]
    assert abs(got - ref) / abs(ref) < 2e-7
    # the opposite sign of the phase would give the conjugate: far off
    assert abs(np.conj(got) - ref) / abs(ref) > 1e-2


def test_hankel_parseval():
    """2 pi int |K|^2 rho d rho = 2 pi int tau^2 r dr, independent of w (|G| = 1)."""
    geo = H.geometry(200, 1e-3, 4096, 4)
    tau = np.exp(-geo.r ** 2 / (2 * 0.01 ** 2))
    drho = 0.05
    rho = np.arange(0, int(400 / drho)) * drho
    m = H.hankel_matrix(rho, geo)
    rhs = 2 * math.pi * np.sum(tau ** 2 * geo.r) * geo.dr
    for w in (0.0, 100.0, 300.0):
        k = m @ (tau * np.exp(2j * math.pi * w * geo.phi))
        lhs = 2 * math.pi * np.sum(np.abs(k) ** 2 * rho) * drho
        assert abs(lhs - rhs) / rhs < 2e-6


def test_j0_against_mpmath():
    """scipy's J0 (the oracle's) against mpmath's arbitrary-precision Bessel J0
    over the argument range of the largest workload (2 pi rho_max r_max ~ 400)."""
    from scipy.special import j0
    xs = np.concatenate([np.linspace(0, 10, 41), np.linspace(10, 420, 83), [2.404825557695773]])
    for x in xs:
        # absolute error of a few ulp of the argument's phase (x * eps grows with x)
        assert abs(j0(x) - float(mpmath.besselj(0, x))) < 1e-15 + 1e-17 * x


def test_geometry_phi_cancellation_free():
    geo = H.geometry(2048, W.ARCSEC * 3.5, 8192, 8)
    with mpmath.workdps(60):
        exact = np.array([float(1 - mpmath.sqrt(1 - mpmath.mpf(r) ** 2)) for r in geo.r[::511]])
    assert np.max(np.abs(geo.phi[::511] - exact) / exact) < 1e-15


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------
def test_conjugate_symmetry_in_w():
    """K(-w) = conj K(w) for a real taper (section 4.1)."""
    wl = W.plain(extra_w=[-62.5, -937.5])
    caches, _ = H.generate_workload(wl)
    for p_pos, p_neg in ((0, 8), (7, 9)):
        assert np.max(np.abs(caches[p_neg] - np.conj(caches[p_pos]))) <= 1e-15 * np.max(np.abs(caches[p_pos]))


def test_linearity_in_taper():
    wl = W.plain()
    geo = H.geometry(wl.image_size, wl.cellsize, wl.n_radial, wl.oversampling)
    rng = np.random.default_rng(W.SEED)
    t1 = rng.normal(size=wl.n_radial)
    t2 = rng.normal(size=wl.n_radial)
    k1 = H.radial_kernels(geo, t1, wl.w, wl.support)
    k2 = H.radial_kernels(geo, t2, wl.w, wl.support)
    k12 = H.radial_kernels(geo, 0.3 * t1 - 1.7 * t2, wl.w, wl.support)
    for a, b, c in zip(k1, k2, k12):
        assert np.max(np.abs(c - (0.3 * a - 1.7 * b))) <= 1e-13 * np.max(np.abs(c))


def test_supports_reach_only_existing_nodes():
    for s in (1, 3, 7, 31, 127, 255):
        for os_ in (1, 4, 8):
            for q in (1, 2):
                _, mask, t = H.sample_positions(s, os_, q)
                n = int(H.n_rho([s], os_, q)[0])
                h = (s - 1) // 2
                # the farthest sample sits on node q os h; three nodes lie beyond it
                assert t[mask].max() == q * os_ * h
                assert n - 1 - q * os_ * h == 3


# ---------------------------------------------------------------------------
# interpolation (section 4.3.2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 3, 5, 28, 257])
def test_spline_matches_scipy_cubicspline(n):
    rng = np.random.default_rng(n)
    y = rng.normal(size=n) + 1j * rng.normal(size=n)
    m = H.spline_second_derivatives(y)
    t = np.sort(rng.uniform(0, n - 1, 500))
    x = np.arange(n, dtype=float)
    ref = (CubicSpline(x, y.real, bc_type=((1, 0.0), (2, 0.0)))(t)
           + 1j * CubicSpline(x, y.imag, bc_type=((1, 0.0), (2, 0.0)))(t))
    got = H.spline_eval(y, m, t)
    assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(y)))
    # interpolation property at the nodes
    assert np.max(np.abs(H.spline_eval(y, m, x) - y)) < 1e-13


def test_spline_reproduces_admissible_cubic():
    """A cubic with s'(0) = 0 and s''(n-1) = 0 is reproduced exactly."""
    n = 40
    c = 0.7
    b = -3.0 * c * (n - 1)
    f = lambda t: 2.0 + b * t ** 2 + c * t ** 3  # noqa: E731
    x = np.arange(n, dtype=float)
    m = H.spline_second_derivatives(f(x))
    t = np.linspace(0, n - 1, 777)
    assert np.max(np.abs(H.spline_eval(f(x), m, t) - f(t))) < 1e-9 * np.max(np.abs(f(t)))


def test_linear_matches_numpy_interp():
    rng = np.random.default_rng(3)
    y = rng.normal(size=50)
    t = rng.uniform(0, 49, 300)
    assert np.max(np.abs(H.linear_eval(y, t) - np.interp(t, np.arange(50), y))) < 1e-14


# ---------------------------------------------------------------------------
# 2D-FFT twin (Algorithm 1)
# ---------------------------------------------------------------------------
def test_fft2d_matches_direct_dft():
    fov = 0.1
    n_ws = 16
    os_ = 2
    scr = F.workspace_screen(W.gaussian_taper(0.02), 300.0, n_ws, fov)
    spec = F.padded_transform(scr, os_, fov)
    xs, ys = np.meshgrid(np.arange(-6, 7), np.arange(-5, 6))
    ref = F.direct_dft(scr, os_, fov, xs, ys)
    c = spec.shape[0] // 2
    got = spec[c + ys, c + xs]
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))


def test_fft2d_parseval():
    fov, n_ws, os_ = 0.1, 64, 4
    scr = F.workspace_screen(W.gaussian_taper(0.02), 500.0, n_ws, fov)
    spec = F.padded_transform(scr, os_, fov)
    dl = fov / n_ws
    du = 1.0 / (os_ * n_ws * dl)
    lhs = np.sum(np.abs(spec) ** 2) * du * du
    rhs = np.sum(np.abs(scr) ** 2) * dl * dl
    assert abs(lhs - rhs) / rhs < 1e-12


def _hankel_exact_rho(geo, tau, w, support, os_):
    """Hankel sum evaluated at each sample's exact radius (no spline)."""
    d2, mask, _ = H.sample_positions(support, os_, 1)
    uniq, inv = np.unique(d2[mask], return_inverse=True)
    rho = geo.du * np.sqrt(uniq.astype(float)) / os_
    vals = H.hankel_matrix(rho, geo) @ (np.asarray(tau, float) * np.exp(2j * math.pi * w * geo.phi))
    out = np.zeros(mask.shape, complex)
    out[mask] = vals[inv]
    return out, mask


def test_hankel_vs_2d_in_circle_plain():
    """Section 4.4: the Hankel route equals the 2D FFT route inside the circular
    region.  Plain workload (Gaussian sigma 0.02 cut at r_max = 0.05): the
    remaining difference is the Cartesian staircase of the disc edge."""
    wl = W.plain()
    caches, _ = H.generate_workload(wl)
    ffts = F.generate(wl.taper_fn, wl.w, wl.support, wl.oversampling, 128, wl.image_size * wl.cellsize)
    for c_h, c_f in zip(caches, ffts):
        assert np.max(np.abs(c_h - c_f)) / np.max(np.abs(c_f)) < 1e-3


def test_hankel_vs_2d_in_circle_smooth_edge():
    """With a taper that vanishes smoothly at r_max the two routes agree to the
    quadrature error (exact-radius Hankel at Nr = 4096 vs 2D DFT)."""
    r_max = 0.05
    base = W.gaussian_taper(0.02)
    fn = lambda r: base(r) * np.clip(1 - (np.asarray(r) / r_max) ** 2, 0, None) ** 2  # noqa: E731
    geo = H.geometry(128, 7.8125e-4, 4096, 4)
    tau = fn(geo.r)
    for w in (62.5, 562.5, 937.5):
        ref, mask = _hankel_exact_rho(geo, tau, w, 31, 4)
        got = F.generate(fn, [w], [31], 4, 128, 0.1)[0]
        assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-6


def test_resample_layout_against_exact_radius():
    """The spline cache at refinement q = 4 matches the exact-radius Hankel sum:
    pins the sample offsets X, Y, the circular mask and the radial scale."""
    geo = H.geometry(128, 7.8125e-4, 128, 4, radial_refine=4)
    wl = W.plain()
    caches, _ = H.generate(128, 7.8125e-4, 128, 4, wl.taper, wl.w, wl.support, radial_refine=4)
    for p in (0, 5, 7):
        ref, _ = _hankel_exact_rho(geo, wl.taper, wl.w[p], 31, 4)
        assert np.max(np.abs(caches[p] - ref)) / np.max(np.abs(ref)) < 1e-6


# ---------------------------------------------------------------------------
# gradient (adjoint)
# ---------------------------------------------------------------------------
def _small_grad_case():
    wl = W.random_small(11, n_planes=4, n_radial=48, os_=2, max_support=15)
    wl.support[:] = np.array([15, 11, 13, 9], dtype=np.int32)
    return wl


def _loss(wl, tau, w):
    caches, _ = H.generate(wl.image_size, wl.cellsize, wl.n_radial, wl.oversampling, tau, w,
                           wl.support, wl.radial_refine, wl.interp)
    return A.energy_outside_loss(caches, wl.support, wl.oversampling, inner_half=2)


@pytest.mark.parametrize("interp", ["cubic", "linear"])
def test_adjoint_matches_central_fd(interp):
    wl = _small_grad_case()
    wl.interp = interp
    tau = wl.taper.astype(np.float64)
    w = wl.w.copy()
    loss, g = _loss(wl, tau, w)
    g_tau, g_w = A.grad(wl.image_size, wl.cellsize, wl.n_radial, wl.oversampling, tau, w,
                        wl.support, g, wl.radial_refine, interp)
    h = 1e-4
    fd_tau = np.zeros_like(tau)
    for i in range(len(tau)):
        tp, tm = tau.copy(), tau.copy()
        tp[i] += h
        tm[i] -= h
        fd_tau[i] = (_loss(wl, tp, w)[0] - _loss(wl, tm, w)[0]) / (2 * h)
    fd_w = np.zeros_like(w)
    for p in range(len(w)):
        wp, wm = w.copy(), w.copy()
        wp[p] += h
        wm[p] -= h
        fd_w[p] = (_loss(wl, tau, wp)[0] - _loss(wl, tau, wm)[0]) / (2 * h)
    assert np.max(np.abs(g_tau - fd_tau)) / np.max(np.abs(fd_tau)) < 1e-6
    assert np.max(np.abs(g_w - fd_w)) / np.max(np.abs(fd_w)) < 1e-6


@pytest.mark.parametrize("interp", ["cubic", "linear"])
def test_resample_adjoint_dot_product(interp):
    rng = np.random.default_rng(5)
    s, os_, q = 13, 3, 2
    n = int(H.n_rho([s], os_, q)[0])
    y = rng.normal(size=n) + 1j * rng.normal(size=n)
    g = rng.normal(size=(os_, os_, s, s)) + 1j * rng.normal(size=(os_, os_, s, s))
    ry = H.resample(y, s, os_, q, interp)
    lhs = np.real(np.vdot(g, ry))
    rhs = np.real(np.vdot(A.resample_adjoint(g, n, s, os_, q, interp), y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ---------------------------------------------------------------------------
# sizing statements the paper prints (tests/golden/paper_sizing.json)
# ---------------------------------------------------------------------------
def test_paper_sizing_statements():
    with open(os.path.join(GOLDEN, "paper_sizing.json")) as f:
        g = json.load(f)
    kc = g["kernel_cache_counts"]
    assert kc["oversampling"] ** 2 == kc["kernels_per_plane"]
    assert kc["oversampling"] ** 2 * kc["n_planes"] == kc["kernels_total"]
    sw = g["support_to_width"]
    assert 2 * sw["half_support"] + 1 == sw["full_width"]
    # the oracle's layout gives a full width S block per sub-kernel
    offs = H.offsets([sw["full_width"]], kc["oversampling"])
    assert offs[1] == kc["kernels_per_plane"] * sw["full_width"] ** 2
    wu = g["workspace_undersampling"]
    for hs, ws, fs in zip(wu["half_support"], wu["workspace"], wu["fft_size"]):
        assert F.next_pow2(2 * hs + 1) == ws
        assert wu["oversampling"] * ws == fs
    pf = g["padded_full_image"]
    assert pf["image_size"] * pf["oversampling"] == pf["padded"]
    assert round(pf["padded"] ** 2 * 16 / 1e9) == pf["gigabytes"]


# ---------------------------------------------------------------------------
# truncation (section 3.1, Algorithm 2)
# ---------------------------------------------------------------------------
def test_truncation_gaussian_closed_form():
    """w = 0, Gaussian taper: K = 2 pi sig^2 exp(-2 pi^2 sig^2 rho^2) falls to 1%
    of its peak at rho_1 = sqrt(ln 100 / (2 pi^2 sig^2)); the truncated
    half-width is the first whole uv cell at or beyond it."""
    sig = 0.004
    wl = W.plain(n_radial=2048)
    fn = W.gaussian_taper(sig)
    tau = W.sample_taper(fn, 2048, wl.r_max)
    geo = H.geometry(wl.image_size, wl.cellsize, 2048, 4)
    _, sup, lines = H.generate_truncated(wl.image_size, wl.cellsize, 2048, 4, tau, [0.0], 63)
    rho1 = math.sqrt(math.log(100.0) / (2 * math.pi ** 2 * sig ** 2))
    k1 = rho1 / geo.drho
    # the last node above 1% is floor(k1) (K is monotone here)
    assert int(sup[0]) == 2 * math.ceil(math.floor(k1) / 4) + 1
    assert 1 < sup[0] < 63


# (sigma, os, q): the closed-form 1% node k1 lies well inside a node interval
# (fractional part between 0.2 and 0.8) and floor(k1) is not a multiple of
# q os, so rounding the half-width up or down, or stopping at the first node
# below the threshold instead of the last one at or above it, give different
# supports.
_TRUNC_CASES = [(0.0035, 3, 1), (0.0045, 3, 2), (0.005, 4, 1), (0.004, 8, 2),
                (0.005, 8, 2), (0.007, 8, 1)]


@pytest.mark.parametrize("sig,os_,q", _TRUNC_CASES)
def test_truncation_gaussian_node_between_cells(sig, os_, q):
    """w = 0 and a Gaussian taper of width sig, far inside the disc: the
    line is K(rho) = 2 pi sig^2 exp(-2 pi^2 sig^2 rho^2) (decreasing), so the
    last node at or above 1% of the peak is k* = floor(k1), k1 = rho_1 / drho
    with rho_1 = sqrt(ln 100 / (2 pi^2 sig^2)).  The circular support must
    reach rho_{k*}: the smallest half-width h with q os h >= k*
    (section 3.1, Algorithm 2: the kernel is cut where it falls below the
    fraction of its peak, so nothing at or above it is cut)."""
    wl = W.plain(n_radial=2048)
    tau = W.sample_taper(W.gaussian_taper(sig), 2048, wl.r_max)
    geo = H.geometry(wl.image_size, wl.cellsize, 2048, os_, q)
    k1 = math.sqrt(math.log(100.0) / (2 * math.pi ** 2 * sig ** 2)) / geo.drho
    k_star = math.floor(k1)
    assert 0.2 < k1 - k_star < 0.8 and k_star % (q * os_) != 0  # the case discriminates
    _, sup, lines = H.generate_truncated(wl.image_size, wl.cellsize, 2048, os_, tau, [0.0], 63,
                                         radial_refine=q)
    # the discrete line agrees with the closed form well below the margin
    amp = np.abs(lines[0])
    assert amp[k_star] >= 0.01 * amp.max() > amp[k_star + 1]
    h = (int(sup[0]) - 1) // 2
    assert q * os_ * h >= k_star           # the support reaches rho_{k*}
    assert q * os_ * (h - 1) < k_star      # and is the smallest that does
    assert 1 < sup[0] < 63


def test_truncation_clamped_at_planned_support():
    """A kernel wider than the planned maximum: the line (computed for the
    maximum, q os h_max + 4 nodes) stays above 1% to its last node, so the
    rule asks for more than h_max and the support is clamped to S_max."""
    sig, os_, s_max = 0.0035, 4, 21          # closed-form k* = 55, line has 44 nodes
    wl = W.plain(n_radial=2048)
    tau = W.sample_taper(W.gaussian_taper(sig), 2048, wl.r_max)
    _, sup, lines = H.generate_truncated(wl.image_size, wl.cellsize, 2048, os_, tau, [0.0], s_max)
    amp = np.abs(lines[0])
    assert len(amp) == os_ * (s_max - 1) // 2 + 4 and amp[-1] >= 0.01 * amp.max()
    assert int(sup[0]) == s_max
    # with a wider plan the same kernel gets its own (narrower than 2 h + 3) support
    _, sup_w, _ = H.generate_truncated(wl.image_size, wl.cellsize, 2048, os_, tau, [0.0], 63)
    assert s_max < int(sup_w[0]) < 63


@pytest.mark.parametrize("line,frac,os_,q,h_max,h_expect", [
    # dips below 1% at node 2 and comes back above at node 4: the last node
    # at or above the threshold decides (k* = 4), h = ceil(4 / 3) = 2
    ([1.0, 0.5, 0.001, 0.002, 0.05, 0.003, 0.0, 0.0, 0.0], 0.01, 3, 1, 3, 2),
    # a node exactly at the threshold counts; amplitude of a complex value
    ([1.0, 0.2, 0.1, 0.006 + 0.008j, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0], 0.01, 2, 1, 4, 2),
    # the peak need not be at rho = 0; negative values count by magnitude
    ([0.3, -2.0, 0.9, 0.05, -0.021, 0.025, 0.019, 0.0, 0.0, 0.0, 0.0], 0.01, 2, 2, 2, 2),
    # k* = 9 at the end of a 10-node line asks for ceil(9 / 2) = 5 > h_max = 4
    ([1.0] * 10, 0.01, 2, 1, 4, 4),
    # only the peak is above: k* = 0 gives a single-pixel kernel
    ([1.0, 0.001, 0.0, 0.0, 0.0], 0.01, 4, 1, 1, 0),
])
def test_truncation_rule_hand_lines(line, frac, os_, q, h_max, h_expect):
    assert H.truncated_half_support(np.asarray(line), frac, os_, q, h_max) == h_expect


def test_truncation_monotone_and_clamped():
    wl = W.paper(n_planes=8, n_radial=1024)
    prev = None
    for frac in (0.1, 0.01, 0.001, 1e-6):
        _, sup, _ = H.generate_truncated(wl.image_size, wl.cellsize, wl.n_radial, wl.oversampling,
                                         wl.taper, wl.w, 63, frac=frac)
        assert np.all(sup <= 63) and np.all(sup % 2 == 1)
        if prev is not None:
            assert np.all(sup >= prev)
        prev = sup
    assert np.all(prev == 63)  # a tiny fraction keeps the maximum support


def test_truncated_cache_uses_full_line():
    wl = W.plain()
    caches, sup, lines = H.generate_truncated(wl.image_size, wl.cellsize, wl.n_radial,
                                              wl.oversampling, wl.taper, wl.w[:3], 31)
    for c, s, line in zip(caches, sup, lines):
        assert c.shape == (4, 4, s, s)
        assert len(line) == H.n_rho([31], 4)[0]
        np.testing.assert_array_equal(c, H.resample(line, int(s), 4))


# ---------------------------------------------------------------------------
# Projection-slice engine (section 4.3.1, Algorithm 2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("w", [0.0, 300.0, 937.5])
@pytest.mark.parametrize("os_,q", [(4, 1), (3, 1), (2, 2)])
def test_projslice_line_is_the_2d_transform_axis(w, os_, q):
    """Discrete projection-slice theorem: the padded 1D transform of the
    projection equals the v = 0 row of the padded 2D transform (oracle.fft2d)
    of the same workspace, sample for sample."""
    wl = W.plain()
    fov = wl.image_size * wl.cellsize
    n_ws = 64
    line = PS.line(wl.taper_fn, w, 31, os_, fov, q, n_ws)
    spec = F.padded_transform(F.workspace_screen(wl.taper_fn, w, n_ws, fov), q * os_, fov)
    c = spec.shape[0] // 2
    ref = spec[c, c:c + line.shape[0]]
    assert np.max(np.abs(line - ref)) / np.max(np.abs(ref)) < 1e-12


def test_projslice_brute_force_tiny():
    wl = W.plain()
    fov = wl.image_size * wl.cellsize
    scr = F.workspace_screen(wl.taper_fn, 700.0, 8, fov)
    line = PS.line(wl.taper_fn, 700.0, 5, 3, fov, 1, 8)
    ref = PS.brute_line(scr, fov, 3, line.shape[0])
    assert np.max(np.abs(line - ref)) / np.max(np.abs(ref)) < 1e-13


def test_projslice_gaussian_closed_form():
    """w = 0 and a Gaussian taper far inside the disc: the line is the
    Gaussian's transform 2 pi sig^2 exp(-2 pi^2 sig^2 rho^2)."""
    sig, fov = 0.004, 0.1
    line = PS.line(W.gaussian_taper(sig), 0.0, 31, 4, fov, 1, 256)
    rho = np.arange(line.shape[0]) / (4 * fov)
    ref = 2 * math.pi * sig * sig * np.exp(-2 * math.pi ** 2 * sig * sig * rho ** 2)
    assert np.max(np.abs(line - ref)) / ref[0] < 1e-12


def test_projslice_agrees_with_matrix_form_on_smooth_edge():
    """Both transforms approximate the same continuous HT: with a taper that
    vanishes smoothly at r_max they agree to the quadrature errors."""
    r_max, fov = 0.05, 0.1
    base = W.gaussian_taper(0.02)
    fn = lambda r: base(r) * np.clip(1 - (np.asarray(r) / r_max) ** 2, 0, None) ** 2  # noqa: E731
    geo = H.geometry(128, 7.8125e-4, 4096, 4)
    tau = fn(geo.r)
    for w in (62.5, 562.5, 937.5):
        k_h = H.radial_kernels(geo, tau, [w], [31])[0]
        k_p = PS.line(fn, w, 31, 4, fov, 1, 128)
        assert np.max(np.abs(k_h - k_p)) / np.max(np.abs(k_h)) < 2e-6


@pytest.mark.parametrize("s,os_,q,min_w,n", [(7, 8, 1, None, 8), (9, 8, 1, None, 16),
                                             (255, 8, 1, None, 256), (31, 1, 1, None, 64),
                                             (1, 1, 1, None, 8), (7, 8, 1, 255, 256),
                                             (31, 4, 2, None, 32), (1, 8, 1, None, 2)])
def test_projslice_workspace_size(s, os_, q, min_w, n):
    assert PS.workspace_size(s, os_, q, min_w) == n


# ---------------------------------------------------------------------------
# Taper input (prolate spheroidal) and a second route to the gradient
# ---------------------------------------------------------------------------
def test_pswf_alpha0_matches_scipy_pro_ang1():
    from scipy.special import pro_ang1
    c = 3 * math.pi
    fn, _, _ = W._pswf_nystrom(c, 0.0)
    x = np.linspace(-0.99, 0.99, 41)
    ref = np.array([pro_ang1(0, 0, c, xi)[0] for xi in x]) / pro_ang1(0, 0, c, 0.0)[0]
    assert np.max(np.abs(fn(x) - ref)) < 1e-13


def test_pswf_alpha1_eigen_equation_and_convergence():
    """At alpha = 1 (the taper the workloads use) no library routine exists:
    the Nystrom solution must satisfy its integral equation under an
    independent adaptive quadrature and be converged in the node count."""
    from scipy.integrate import quad
    c = 3 * math.pi
    fn, lam, _ = W._pswf_nystrom(c, 1.0, 200)
    fn160, lam160, _ = W._pswf_nystrom(c, 1.0, 160)
    x = np.linspace(0.0, 1.0, 21)
    assert np.max(np.abs(fn(x) - fn160(x))) < 1e-13 and abs(lam - lam160) < 1e-13
    for nu in (0.0, 0.3, 0.7, 0.95):
        val = quad(lambda e: math.cos(c * nu * e) * (1 - e * e) * float(fn(np.array(e))), -1, 1,
                   limit=200, epsabs=1e-14)[0]
        assert abs(val - lam * float(fn(np.array(nu)))) < 1e-12


@pytest.mark.parametrize("interp", ["cubic", "linear"])
def test_adjoint_matches_torch_autodiff(interp):
    """The hand-written adjoint against automatic differentiation of a torch
    (FP64, CPU) re-expression of the forward chain: screen, HT matrix as a
    constant, spline system written out here as a dense solve, spline
    evaluation at the cache's sample radii, window loss."""
    torch = pytest.importorskip("torch")
    image_size, cell, nr, os_, q = 128, 7.8125e-4, 64, 3, 1
    support = [15, 11, 15]
    rng = np.random.default_rng(3)
    w = np.array([80.0, 420.0, 910.0])
    tau = np.exp(-(W.nodes_nu(nr) / 0.5) ** 2) * (1 + 0.1 * rng.normal(size=nr))
    geo = H.geometry(image_size, cell, nr, os_, q)
    nrho = H.n_rho(support, os_, q)
    m_const = torch.tensor(H.hankel_matrix(np.arange(int(nrho.max())) * geo.drho, geo))
    phi = torch.tensor(geo.phi)
    t_tau = torch.tensor(tau, requires_grad=True)
    t_w = torch.tensor(w, requires_grad=True)
    loss = 0.0
    caches = []
    for p in range(len(w)):
        n = int(nrho[p])
        s = t_tau * torch.exp(1j * 2 * math.pi * t_w[p] * phi)
        k = m_const[:n].to(torch.complex128) @ s
        _, mask, t = H.sample_positions(support[p], os_, q)
        tt = torch.tensor(t[mask])
        kk = torch.clamp(torch.floor(tt).long(), 0, n - 2)
        u = (tt - kk).to(torch.complex128)
        v = 1 - u
        val = v * k[kk] + u * k[kk + 1]
        if interp == "cubic":
            # rows: 2 m0 + m1 = 6 (y1 - y0); m_{j-1} + 4 m_j + m_{j+1} = 6 (y_{j-1} - 2 y_j + y_{j+1}); m_{n-1} = 0
            tm = torch.zeros((n, n), dtype=torch.complex128)
            rhs = torch.zeros(n, dtype=torch.complex128)
            tm[0, 0], tm[0, 1] = 2, 1
            rhs = rhs.index_put((torch.tensor([0]),), 6 * (k[1] - k[0]).reshape(1))
            idx = torch.arange(1, n - 1)
            tm[idx, idx - 1], tm[idx, idx], tm[idx, idx + 1] = 1, 4, 1
            rhs = rhs.index_put((idx,), 6 * (k[idx - 1] - 2 * k[idx] + k[idx + 1]))
            tm[n - 1, n - 1] = 1
            msec = torch.linalg.solve(tm, rhs)
            val = val + (v ** 3 - v) * msec[kk] / 6 + (u ** 3 - u) * msec[kk + 1] / 6
        cache = torch.zeros(mask.shape, dtype=torch.complex128)
        cache[torch.tensor(mask)] = val
        win = torch.tensor(A.window_mask(support[p], os_, 4))
        loss = loss + (cache[win].abs() ** 2).sum()
        caches.append(cache.detach().numpy())
    loss.backward()
    ref, _ = H.generate(image_size, cell, nr, os_, tau, w, support, q, interp)
    for c_t, c_o in zip(caches, ref):
        assert np.max(np.abs(c_t - c_o)) <= 1e-12 * np.max(np.abs(c_o))
    _, g_caches = A.energy_outside_loss(caches, support, os_, 4)
    g_tau, g_w = A.grad(image_size, cell, nr, os_, tau, w, support, g_caches, q, interp)
    assert np.max(np.abs(g_tau - t_tau.grad.numpy())) <= 1e-10 * np.max(np.abs(g_tau))
    assert np.max(np.abs(g_w - t_w.grad.numpy())) <= 1e-10 * np.max(np.abs(g_w))


def test_adjoint_matches_stored_finite_differences():
    """The oracle's adjoint on the full differentiation workload (256 planes,
    2048 free taper samples, window loss) against the stored central
    differences of the oracle's forward (tests/golden/make_grad_fd.py):
    every w-coordinate (O(h^2) truncation, about 3e-6), 32 taper
    coordinates and 16 directions (the loss is quadratic in the taper, so
    these differences are exact up to rounding)."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "grad_fd.json")) as f:
        fd = json.load(f)
    wl = W.grad()
    tau = wl.taper.astype(np.float64)
    caches, _ = H.generate(wl.image_size, wl.cellsize, wl.n_radial, wl.oversampling, tau, wl.w,
                           wl.support, 1, "cubic")
    _, g = A.energy_outside_loss(caches, wl.support, wl.oversampling, fd["inner_half"])
    gt, gw = A.grad(wl.image_size, wl.cellsize, wl.n_radial, wl.oversampling, tau, wl.w,
                    wl.support, g, 1, "cubic")
    coords = np.asarray(fd["tau_coords"])
    assert np.array_equal(coords, W.fd_taper_coords(wl.n_radial))
    assert np.max(np.abs(gw - np.asarray(fd["w_fd"]))) <= 1e-5 * np.max(np.abs(gw))
    assert np.max(np.abs(gt[coords] - np.asarray(fd["tau_fd"]))) <= 1e-10 * np.max(np.abs(gt))
    d_fd = np.asarray(fd["direction_fd"])
    assert np.max(np.abs(W.fd_directions(wl.n_radial) @ gt - d_fd) / np.abs(d_fd)) <= 1e-8


# the bench's parallel-efficiency reporter against the paper's own table
# (tests/golden/paper_table2.json: section 6.8, Table 2)
def test_parallel_efficiency_reproduces_table_2():
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    with open(os.path.join(GOLDEN, "paper_table2.json")) as f:
        table = json.load(f)
    for row in table["rows"]:
        eta = bench.parallel_efficiency(row["single_s"], row["multi_s"], table["cores"])
        assert round(100 * eta) == row["efficiency_pct"], row
    # the unrounded values of the three rows
    etas = [bench.parallel_efficiency(r["single_s"], r["multi_s"], 4) for r in table["rows"]]
    assert np.allclose(etas, [0.4310, 0.6012, 0.7015], atol=5e-4)
