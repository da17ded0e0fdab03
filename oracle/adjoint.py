"""Oracle gradient of a real loss of the kernel cache (FP64, CPU).

Test infrastructure only; see the package header.  The paper has no
gradient; this is the chain rule through the functions of ``oracle.hankel``
written as explicit transposes:

  cache = R(K)      R: spline + sampling, a real-linear map (real coefficients)
  K     = M s       M: the discrete HT matrix (real)
  s_i   = tau_i exp(j theta_i),  theta_i = 2 pi w phi_i

For a real loss L and G = dL/dRe(cache) + j dL/dIm(cache) (the convention
of torch for complex tensors):
  G_K = R^T G,  G_s = M^T G_K,  u = G_s exp(-j theta),
  dL/dtau_i = sum_p Re u_{i p},   dL/dw_p = sum_i 2 pi phi_i tau_i Im u_{i p}.
Parity: pinned by central finite differences of ``oracle.hankel.generate``
and by dot-product (adjoint) identities.
"""
from __future__ import annotations

import math

import numpy as np

from . import hankel as H

TWO_PI = 2.0 * math.pi


def spline_system(n: int):
    """Dense T and D with T m = D y for the spline of ``hankel`` (same rows as
    ``hankel.spline_second_derivatives``)."""
    t = np.zeros((n, n))
    d = np.zeros((n, n))
    t[0, 0], t[0, 1] = 2.0, 1.0
    d[0, 0], d[0, 1] = -6.0, 6.0
    for k in range(1, n - 1):
        t[k, k - 1], t[k, k], t[k, k + 1] = 1.0, 4.0, 1.0
        d[k, k - 1], d[k, k], d[k, k + 1] = 6.0, -12.0, 6.0
    t[n - 1, n - 1] = 1.0
    return t, d


def resample_adjoint(g_cache: np.ndarray, n: int, support: int, oversampling: int,
                     radial_refine: int = 1, interp: str = "cubic") -> np.ndarray:
    """R^T applied to a cache-shaped complex gradient: returns the gradient of the
    radial line K_p (length n)."""
    _, mask, t = H.sample_positions(support, oversampling, radial_refine)
    g = np.asarray(g_cache)[mask]
    tt = t[mask]
    k = np.clip(np.floor(tt).astype(np.int64), 0, n - 2)
    u = tt - k
    v = 1.0 - u
    gy = np.zeros(n, dtype=np.complex128)
    np.add.at(gy, k, v * g)
    np.add.at(gy, k + 1, u * g)
    if interp == "linear":
        return gy
    gm = np.zeros(n, dtype=np.complex128)
    np.add.at(gm, k, (v ** 3 - v) / 6.0 * g)
    np.add.at(gm, k + 1, (u ** 3 - u) / 6.0 * g)
    tm, dm = spline_system(n)
    z = np.linalg.solve(tm.T, gm)
    return gy + dm.T @ z


def grad(image_size, cellsize, n_radial, oversampling, taper, w, support, g_caches,
         radial_refine: int = 1, interp: str = "cubic"):
    """Gradient of L w.r.t. the taper samples [Nr] and the w values [P], given the
    per-plane cache gradients ``g_caches`` (list of [os][os][S][S] complex)."""
    geo = H.geometry(image_size, cellsize, n_radial, oversampling, radial_refine)
    w = np.asarray(w, dtype=np.float64)
    tau = np.asarray(taper, dtype=np.float64)
    nr = H.n_rho(support, oversampling, radial_refine)
    rho = np.arange(int(nr.max())) * geo.drho
    m = H.hankel_matrix(rho, geo)
    theta = TWO_PI * np.outer(geo.phi, w)
    g_tau = np.zeros(n_radial)
    g_w = np.zeros(len(w))
    for p in range(len(w)):
        n = int(nr[p])
        gk = resample_adjoint(g_caches[p], n, int(support[p]), oversampling,
                              radial_refine, interp)
        gs = m[:n].T @ gk
        u = gs * np.exp(-1j * theta[:, p])
        g_tau += u.real
        g_w[p] = np.sum(TWO_PI * geo.phi * tau * u.imag)
    return g_tau, g_w


def window_mask(support: int, oversampling: int, inner_half: int) -> np.ndarray:
    """Samples of a [os][os][S][S] cache outside the (2 inner_half + 1)-px window:
    max(|X|, |Y|) > inner_half * os."""
    h = (support - 1) // 2
    os_ = oversampling
    fv = np.arange(os_)[:, None, None, None]
    fu = np.arange(os_)[None, :, None, None]
    b = np.arange(support)[None, None, :, None]
    a = np.arange(support)[None, None, None, :]
    x = os_ * (a - h) - fu
    y = os_ * (b - h) - fv
    return np.maximum(np.abs(x), np.abs(y)) > inner_half * os_


def energy_outside_loss(caches, support, oversampling, inner_half: int = 31):
    """L = sum_p sum |K_p|^2 over samples outside the window, and dL/dK
    (torch convention: dL/dRe + j dL/dIm = 2 K on those samples)."""
    loss = 0.0
    grads = []
    for p, c in enumerate(caches):
        msk = window_mask(int(support[p]), oversampling, inner_half)
        loss += float(np.sum(np.abs(c[msk]) ** 2))
        grads.append(np.where(msk, 2.0 * c, 0.0))
    return loss, grads
