"""Implicit Euler time stepping and the Joule-loss QoI (oracle).

Section II-A, Eqs. (6)-(7): M (a_{k+1} - a_k)/dt + K a_{k+1} = r(t_{k+1}).
The oracle solves the algebraically identical increment form
    (M/dt + K) delta_k = r(t_{k+1}) - K a_k,   a_{k+1} = a_k + delta_k,
factoring A = M/dt + K once per (sample, dt) with banded Cholesky
(LAPACK dpbtrf) and solving each step with dpbtrs.

Section III-B, Eq. (26): Q = (1/T) int_0^T (da/dt)^T M (da/dt) dt.  With the
backward difference of Eq. (6) on each step the integrand is constant on
(t_k, t_{k+1}], so Q = (1/T) sum_k delta_k^T M delta_k / dt, T = n dt.
Times come from the integer step index: t_k = k dt; a(t_0) = 0 unless given.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.linalg import cho_solve_banded, cholesky_banded

from . import fem, kl, mesh as meshmod


@dataclass
class System:
    """One sample's semi-discrete system M da/dt + K a = J(t) S (Eq. (3))."""
    problem: object
    mesh: meshmod.Mesh
    sigma: np.ndarray
    nu: np.ndarray
    M: object
    K: object
    S: np.ndarray


def build_system(problem, xi, m: meshmod.Mesh = None, kl_table=None) -> System:
    if m is None:
        m = meshmod.build(problem.n_nodes)
    sigma, nu = fem.materials(problem, m, xi, kl_table)
    return System(problem, m, sigma, nu, fem.assemble_mass(m, sigma),
                  fem.assemble_stiffness(m, nu), fem.load_shape(problem, m))


class Stepper:
    """Banded-Cholesky implicit Euler for one (system, dt)."""

    def __init__(self, sysm: System, dt: float):
        self.sys = sysm
        self.dt = dt
        A = sysm.M / dt + sysm.K
        self.cb = cholesky_banded(fem.to_banded_lower(A, fem.bandwidth(sysm.mesh)), lower=True)

    def step(self, a: np.ndarray, k_global: int):
        """One step from a = a(t_k), k = k_global; returns (a_{k+1}, delta^T M delta / dt)."""
        t = (k_global + 1) * self.dt
        b = fem.source_value(self.sys.problem, t) * self.sys.S - self.sys.K @ a
        d = cho_solve_banded((self.cb, True), b)
        return a + d, float(d @ (self.sys.M @ d)) / self.dt

    def run(self, a0: np.ndarray, n_steps: int, k0: int = 0):
        """n_steps from a0 at global step index k0; returns (a_end, sum of step terms)."""
        a = np.array(a0, dtype=np.float64, copy=True)
        q = 0.0
        for k in range(n_steps):
            a, dq = self.step(a, k0 + k)
            q += dq
        return a, q


def solve_sample(problem, xi, steps_per_period: int, n_periods: int, a0=None, m=None, kl_table=None):
    """Q (Eq. (26)) and the final state of one sample on one time grid."""
    sysm = build_system(problem, xi, m, kl_table)
    n = steps_per_period * n_periods
    dt = problem.period / steps_per_period
    st = Stepper(sysm, dt)
    if a0 is None:
        a0 = np.zeros(sysm.mesh.n_dof)
    a, q = st.run(a0, n)
    return q / (n * dt), a


def kl_table_for(problem, m):
    """Centroid KL table for the conductor elements (KL material only)."""
    if problem.material.kind != fem.MAT_KL:
        return None
    cond = meshmod.conductor_mask(m, problem)
    return kl.table(m.centroid[cond], problem.conductor, problem.material.corr_len,
                    problem.material.n_modes)
