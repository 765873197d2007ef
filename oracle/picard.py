"""Implicit Euler with a nonlinear reluctivity nu(|B|) (oracle).

Eq. (1) allows a nonlinear permeability.  With B = curl(A_z e_z) =
(dA/dy, -dA/dx), |B_e|^2 = |grad a_h|^2 is constant on each P1 element.
The conductor follows nu(|B|) = k1' exp(k2' |B|^2) + k3' with per-sample
scaled coefficients; air stays linear.

Each implicit Euler step (Eq. (7)) is solved by the fixed-point (Picard)
iteration: a^(0) = a_k; for i = 0, 1, ...: nu^(i) = nu(|grad a^(i)|^2),
K^(i) = K(nu^(i)), (M/dt + K^(i)) delta = r(t_{k+1}) - K^(i) a_k,
a^(i+1) = a_k + delta; stop when ||a^(i+1) - a^(i)||_2 <= tol ||a^(i+1)||_2
(or after picard_max iterations, which is flagged).  The Joule-loss term of
the step uses the final increment.  Every iteration refactors A (banded
Cholesky).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import cho_solve_banded, cholesky_banded

from . import fem, mesh as meshmod


def b_squared(m: meshmod.Mesh, grads: np.ndarray, a: np.ndarray) -> np.ndarray:
    """|grad a_h|^2 per element, boundary nodes at zero."""
    full = np.zeros(m.n * m.n)
    inner = m.dof >= 0
    full[inner] = a[m.dof[inner]]
    g = np.einsum("ea,eak->ek", full[m.tri], grads)
    return g[:, 0] ** 2 + g[:, 1] ** 2


def solve_sample(problem, xi, steps_per_period: int, n_periods: int, a0=None, m=None,
                 kl_table=None, return_counts: bool = False, return_traj: bool = False):
    if m is None:
        m = meshmod.build(problem.n_nodes)
    mat = problem.material
    sigma, nu = fem.materials(problem, m, xi)
    cond = meshmod.conductor_mask(m, problem)
    k1, k2, k3 = fem.nonlinear_coeffs(problem, xi)
    grads = fem.basis_gradients(m)
    M = fem.assemble_mass(m, sigma)
    S = fem.load_shape(problem, m)
    n = steps_per_period * n_periods
    dt = problem.period / steps_per_period
    bw = fem.bandwidth(m)
    a = np.zeros(m.n_dof) if a0 is None else np.array(a0, dtype=np.float64)
    q = 0.0
    counts = np.zeros(n, dtype=np.int64)
    flagged = False
    traj = [a.copy()]

    def nu_of(state):
        out = nu.copy()
        out[cond] = k1 * np.exp(k2 * b_squared(m, grads, state)[cond]) + k3
        return out

    for k in range(n):
        t = (k + 1) * dt
        rhs_src = fem.source_value(problem, t) * S
        a_it = a
        it = 0
        while True:
            K = fem.assemble_stiffness(m, nu_of(a_it), grads)
            cb = cholesky_banded(fem.to_banded_lower(M / dt + K, bw), lower=True)
            d = cho_solve_banded((cb, True), rhs_src - K @ a)
            a_new = a + d
            it += 1
            done = np.linalg.norm(a_new - a_it) <= mat.picard_tol * np.linalg.norm(a_new)
            a_it = a_new
            if done:
                break
            if it >= mat.picard_max:
                flagged = True
                break
        counts[k] = it
        q += float(d @ (M @ d)) / dt
        a = a_new
        if return_traj:
            traj.append(a.copy())
    Q = q / (n * dt)
    if return_counts and return_traj:
        return Q, a, counts, flagged, traj
    if return_counts:
        return Q, a, counts, flagged
    return Q, a
