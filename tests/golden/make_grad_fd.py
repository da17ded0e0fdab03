"""Writes tests/golden/grad_fd.json: central finite differences (h = 1e-4) of
the FP64 oracle's window loss on the differentiation workload (256 w-planes,
2048 free taper samples, S 127, os 4, loss = kernel energy outside the 63-px
window), for every w-coordinate, 32 taper coordinates (the last 8 next to
r_max) and 16 seeded unit directions in the taper.  Calls only oracle/ and
the seeded input generators; run from the repository root:
    python tests/golden/make_grad_fd.py
The loss is quadratic in the taper (the cache is linear in it), so the
taper differences carry no truncation error; the w differences carry
O(h^2) (about 2e-6 relative)."""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import adjoint as A  # noqa: E402
from oracle import hankel as H  # noqa: E402

H_STEP = 1e-4
INNER_HALF = 31


def loss(tau, w, planes=None):
    wl = W.grad()
    caches, _ = H.generate(wl.image_size, wl.cellsize, wl.n_radial, wl.oversampling, tau, w,
                           wl.support, wl.radial_refine, wl.interp, planes)
    sup = wl.support if planes is None else wl.support[np.asarray(planes)]
    return A.energy_outside_loss(caches, sup, wl.oversampling, INNER_HALF)[0]


def fd_w(p):
    wl = W.grad()
    tau = wl.taper.astype(np.float64)
    wp, wm = wl.w.copy(), wl.w.copy()
    wp[p] += H_STEP
    wm[p] -= H_STEP
    return (loss(tau, wp, [p]) - loss(tau, wm, [p])) / (2 * H_STEP)


def fd_tau(v):
    wl = W.grad()
    tau = wl.taper.astype(np.float64)
    return (loss(tau + H_STEP * v, wl.w) - loss(tau - H_STEP * v, wl.w)) / (2 * H_STEP)


def main():
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    wl = W.grad()
    n = wl.n_radial
    coords = W.fd_taper_coords(n)
    dirs = W.fd_directions(n)
    t0 = time.time()
    with ProcessPoolExecutor(max_workers=os.cpu_count()) as ex:
        gw = list(ex.map(fd_w, range(wl.n_planes)))
        unit = [np.eye(1, n, int(i))[0] for i in coords]
        gt = list(ex.map(fd_tau, unit))
        gd = list(ex.map(fd_tau, list(dirs)))
    out = {
        "_cite": "differentiation workload (no paper counterpart); central differences of the "
                 "oracle's window loss, written by tests/golden/make_grad_fd.py",
        "h": H_STEP, "inner_half": INNER_HALF, "workload": "workloads.grad()",
        "w_fd": gw, "tau_coords": [int(i) for i in coords], "tau_fd": gt,
        "directions": "workloads.fd_directions(2048, 16, 1904)", "direction_fd": gd,
        "seconds": time.time() - t0,
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "grad_fd.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote grad_fd.json in {out['seconds']:.0f} s")


if __name__ == "__main__":
    main()
