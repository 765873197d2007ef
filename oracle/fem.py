"""P1 finite elements for the 2-D eddy-current problem (oracle).

Section II-A of the paper, Eqs. (1)-(5): with A = A_z e_z and w_i = N_i e_z,
    M_ij = int sigma N_i N_j,   K_ij = int nu grad N_i . grad N_j,
    r_i(t) = int J_s(t) N_i.
Per element (exact P1 integrals):
    M_e = sigma_e |T| / 12 (1 + delta_ij),   K_e = nu_e |T| G G^T,
    r_e = J(t) |T| / 3 on source-strip elements,
with G the constant basis gradients.  Boundary rows and columns are
dropped (A = 0 Dirichlet).  Assembly uses SciPy sparse matrices; linear
solves use symmetric banded storage (lower bandwidth N - 1).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import kl, mesh as meshmod

MAT_LOGNORMAL_SCALAR, MAT_KL, MAT_NONLINEAR = 0, 1, 2


def basis_gradients(m: meshmod.Mesh) -> np.ndarray:
    """Constant gradients of the three P1 basis functions per element: [n_elem, 3, 2]."""
    v = m.xy[m.tri]
    x, y = v[..., 0], v[..., 1]
    two_a = 2.0 * m.area
    g = np.empty((len(m.tri), 3, 2))
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        g[:, a, 0] = (y[:, b] - y[:, c]) / two_a
        g[:, a, 1] = (x[:, c] - x[:, b]) / two_a
    return g


def materials(problem, m: meshmod.Mesh, xi: np.ndarray, kl_table=None):
    """Element conductivity and reluctivity for one sample xi.

    Air (everything outside the conductor, source strip included):
    sigma = 0, nu = nu_air.  Conductor, per material kind:
    * scalar lognormal: sigma = sigma0 exp(s_sigma xi_0), nu = nu_cond exp(s_nu xi_1);
    * KL field: ln sigma_e = ln sigma0 + s_kl sum_k sqrt(lam_k) phi_k(c_e) xi_k, nu = nu_cond;
    * nonlinear: sigma = sigma0; nu is set by ``picard`` from |B|, here the
      value at B = 0 (k1' + k3') is returned.
    """
    mat = problem.material
    cond = meshmod.conductor_mask(m, problem)
    sigma = np.zeros(len(m.tri))
    nu = np.full(len(m.tri), mat.nu_air)
    xi = np.asarray(xi, dtype=np.float64)
    if mat.kind == MAT_LOGNORMAL_SCALAR:
        sigma[cond] = mat.sigma0 * math.exp(mat.s_sigma * xi[0])
        nu[cond] = mat.nu_cond * math.exp(mat.s_nu * xi[1])
    elif mat.kind == MAT_KL:
        if kl_table is None:
            kl_table = kl.table(m.centroid[cond], problem.conductor, mat.corr_len, mat.n_modes)
        g = kl_table @ xi[: mat.n_modes]
        sigma[cond] = np.exp(math.log(mat.sigma0) + mat.s_kl * g)
        nu[cond] = mat.nu_cond
    elif mat.kind == MAT_NONLINEAR:
        sigma[cond] = mat.sigma0
        k1, _, k3 = nonlinear_coeffs(problem, xi)
        nu[cond] = k1 + k3
    else:
        raise ValueError("unknown material kind")
    return sigma, nu


def nonlinear_coeffs(problem, xi):
    """Per-sample scaled curve coefficients k_i' = k_i exp(s_k xi_i)."""
    mat = problem.material
    xi = np.asarray(xi, dtype=np.float64)
    return (mat.k1 * math.exp(mat.s_k * xi[0]), mat.k2 * math.exp(mat.s_k * xi[1]),
            mat.k3 * math.exp(mat.s_k * xi[2]))


def _scatter(m: meshmod.Mesh, local: np.ndarray) -> sp.csr_matrix:
    """Assemble [n_elem, 3, 3] local matrices into the interior-DoF matrix."""
    nd = m.n_dof
    g = m.dof[m.tri]                             # [n_elem, 3]
    rows = np.repeat(g[:, :, None], 3, axis=2)
    cols = np.repeat(g[:, None, :], 3, axis=1)
    keep = (rows >= 0) & (cols >= 0)
    return sp.coo_matrix((local[keep], (rows[keep], cols[keep])), shape=(nd, nd)).tocsr()


def mass_local(m: meshmod.Mesh, sigma: np.ndarray) -> np.ndarray:
    base = (np.ones((3, 3)) + np.eye(3)) / 12.0
    return (sigma * m.area)[:, None, None] * base[None]


def stiffness_local(m: meshmod.Mesh, nu: np.ndarray, grads=None) -> np.ndarray:
    if grads is None:
        grads = basis_gradients(m)
    return (nu * m.area)[:, None, None] * np.einsum("eak,ebk->eab", grads, grads)


def assemble_mass(m, sigma) -> sp.csr_matrix:
    return _scatter(m, mass_local(m, sigma))


def assemble_stiffness(m, nu, grads=None) -> sp.csr_matrix:
    return _scatter(m, stiffness_local(m, nu, grads))


def load_shape(problem, m: meshmod.Mesh) -> np.ndarray:
    """S with r(t) = J(t) S: S_i = sum over strip elements e containing i of |T_e|/3."""
    strip = meshmod.strip_mask(m, problem)
    s = np.zeros(m.n_dof)
    g = m.dof[m.tri[strip]]
    a = m.area[strip]
    for k in range(3):
        ok = g[:, k] >= 0
        np.add.at(s, g[ok, k], a[ok] / 3.0)
    return s


def source_value(problem, t: float) -> float:
    """J(t) = J0 sin(2 pi f t)."""
    return problem.J0 * math.sin(2.0 * math.pi * problem.freq * t)


def to_banded_lower(A: sp.spmatrix, bw: int) -> np.ndarray:
    """Lower symmetric banded storage ab[i - j, j] = A[i, j] (i >= j)."""
    c = sp.tril(A).tocoo()
    ab = np.zeros((bw + 1, A.shape[0]))
    d = c.row - c.col
    if np.any(d > bw):
        raise ValueError("matrix exceeds the stated bandwidth")
    ab[d, c.col] = c.data
    return ab


def bandwidth(m: meshmod.Mesh) -> int:
    return m.n - 1
