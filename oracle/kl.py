"""Karhunen-Loeve basis of a separable exponential covariance (oracle).

Covariance on the conductor rectangle: C(x, y) = exp(-|dx|/l - |dy|/l),
the product of two 1-D exponential kernels exp(-c |s - t|), c = 1/l, on
[-a, a].  Their eigenpairs are known in closed form (Ghanem and Spanos,
"Stochastic Finite Elements", Sec. 2.3):

* even modes  phi(s) = cos(w s) / sqrt(a + sin(2 w a) / (2 w)),
              with  c cos(w a) - w sin(w a) = 0,
* odd modes   phi(s) = sin(w s) / sqrt(a - sin(2 w a) / (2 w)),
              with  w cos(w a) + c sin(w a) = 0,
* eigenvalue  lam = 2 c / (w^2 + c^2).

2-D modes are products phi_i(x - xc) phi_j(y - yc) with lam_i lam_j,
ordered by eigenvalue (descending), ties broken by the smaller x-index i.
The log-conductivity of the workload is
    ln sigma_e = ln sigma0 + s * sum_k sqrt(lam_k) phi_k(c_e) xi_k
at element centroids c_e inside the conductor.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def roots_1d(a: float, c: float, n: int):
    """First n 1-D modes, ascending in w (descending eigenvalue).

    Returns a list of (w, parity) with parity 0 = even (cos), 1 = odd (sin).
    Even root k lies in [k pi, k pi + pi/2] / a, odd root k in
    [k pi + pi/2, (k+1) pi] / a; both bracket a sign change of the smooth
    (pole-free) forms of the transcendental equations.
    """
    out = []
    k = 0
    while len(out) < n:
        fe = lambda w: c * math.cos(w * a) - w * math.sin(w * a)
        lo, hi = k * math.pi / a, (k * math.pi + math.pi / 2) / a
        out.append((brentq(fe, lo, hi, xtol=1e-15, rtol=4 * np.finfo(float).eps, maxiter=500), 0))
        fo = lambda w: w * math.cos(w * a) + c * math.sin(w * a)
        lo, hi = (k * math.pi + math.pi / 2) / a, (k + 1) * math.pi / a
        out.append((brentq(fo, lo, hi, xtol=1e-15, rtol=4 * np.finfo(float).eps, maxiter=500), 1))
        k += 1
    out.sort(key=lambda t: t[0])
    return out[:n]


def eig_1d(w: float, c: float) -> float:
    return 2.0 * c / (w * w + c * c)


def phi_1d(s: np.ndarray, w: float, parity: int, a: float) -> np.ndarray:
    s = np.asarray(s, dtype=np.float64)
    if parity == 0:
        return np.cos(w * s) / math.sqrt(a + math.sin(2 * w * a) / (2 * w))
    return np.sin(w * s) / math.sqrt(a - math.sin(2 * w * a) / (2 * w))


def modes_2d(box, corr_len: float, n_modes: int, n_1d: int = 12):
    """Top n_modes 2-D modes: list of (lam, (i, w_i, par_i), (j, w_j, par_j))."""
    x0, x1, y0, y1 = box
    ax, ay = 0.5 * (x1 - x0), 0.5 * (y1 - y0)
    c = 1.0 / corr_len
    rx = roots_1d(ax, c, n_1d)
    ry = roots_1d(ay, c, n_1d)
    cand = []
    for i, (wi, pi) in enumerate(rx):
        for j, (wj, pj) in enumerate(ry):
            cand.append((eig_1d(wi, c) * eig_1d(wj, c), i, j, wi, pi, wj, pj))
    cand.sort(key=lambda t: (-t[0], t[1]))
    return [(lam, (i, wi, pi), (j, wj, pj)) for lam, i, j, wi, pi, wj, pj in cand[:n_modes]]


def table(centroids: np.ndarray, box, corr_len: float, n_modes: int) -> np.ndarray:
    """sqrt(lam_k) phi_k(c_e) for the given centroids: [n_elem, n_modes]."""
    x0, x1, y0, y1 = box
    xc, yc = 0.5 * (x0 + x1), 0.5 * (y0 + y1)
    ax, ay = 0.5 * (x1 - x0), 0.5 * (y1 - y0)
    cols = []
    for lam, (i, wi, pi), (j, wj, pj) in modes_2d(box, corr_len, n_modes):
        cols.append(math.sqrt(lam) * phi_1d(centroids[:, 0] - xc, wi, pi, ax)
                    * phi_1d(centroids[:, 1] - yc, wj, pj, ay))
    return np.stack(cols, axis=1)
