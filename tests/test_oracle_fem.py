"""Pins of the oracle's mesh, KL basis and P1 assembly (Section II-A, Eqs. (2)-(5))."""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.linalg as sl

import workloads as W
from oracle import fem, kl, mesh, timestep


def homogeneous(n, J0=1.0e6):
    mat = W.Material(kind=W.MAT_LOGNORMAL_SCALAR)
    return W.Problem(n, mat, conductor=(0.0, 1.0, 0.0, 1.0), J0=J0)


@pytest.mark.parametrize("n", [3, 5, 9, 33, 65, 129])
def test_mesh_counts(n):
    m = mesh.build(n)
    assert m.n_dof == (n - 2) ** 2
    assert len(m.tri) == 2 * (n - 1) ** 2
    assert np.allclose(m.area, 0.5 / (n - 1) ** 2, rtol=0, atol=1e-18)
    # every element's centroid is at least h/15 from the region edges (no ties)
    prob = W.Problem(n)
    x, y = m.centroid[:, 0], m.centroid[:, 1]
    for e in (0.3, 0.7, 0.1, 0.2):
        assert np.min(np.abs(x - e)) > m.h / 16
    for e in (0.3, 0.7):
        assert np.min(np.abs(y - e)) > m.h / 16


def _dense_quadrature(m, sigma, nu):
    """Independent route: basis functions from the inverse Vandermonde of each
    triangle, mass by the 3-point edge-midpoint rule (exact for quadratics),
    stiffness from the linear coefficients; full node numbering."""
    nn = m.n * m.n
    Mf = np.zeros((nn, nn))
    Kf = np.zeros((nn, nn))
    for e, t in enumerate(m.tri):
        P = m.xy[t]
        V = np.column_stack([np.ones(3), P])
        coef = np.linalg.inv(V)             # column a: N_a = c0 + c1 x + c2 y
        area = 0.5 * abs(np.linalg.det(V))
        mids = 0.5 * (P + np.roll(P, -1, axis=0))
        Nq = np.column_stack([np.ones(3), mids]) @ coef   # [q, a]
        Mloc = sigma[e] * area / 3.0 * (Nq.T @ Nq)
        G = coef[1:, :].T
        Kloc = nu[e] * area * (G @ G.T)
        Mf[np.ix_(t, t)] += Mloc
        Kf[np.ix_(t, t)] += Kloc
    inner = np.where(m.dof >= 0)[0]
    order = inner[np.argsort(m.dof[inner])]
    return Mf, Kf, order


def test_assembly_matches_quadrature_route():
    w = W.plain_fp64_33()
    p = W.Problem(9, w.problem.material)
    m = mesh.build(9)
    xi = W.level_xi(w, 0, 1)[0]
    sigma, nu = fem.materials(p, m, xi)
    rng = np.random.default_rng(1)
    sigma = sigma * (1 + 0.5 * rng.random(len(sigma)))   # fully heterogeneous elements
    nu = nu * (1 + 0.5 * rng.random(len(nu)))
    Mf, Kf, order = _dense_quadrature(m, sigma, nu)
    M = fem.assemble_mass(m, sigma).toarray()
    K = fem.assemble_stiffness(m, nu).toarray()
    assert np.allclose(M, Mf[np.ix_(order, order)], rtol=1e-14, atol=1e-14 * np.abs(Mf).max())
    assert np.allclose(K, Kf[np.ix_(order, order)], rtol=1e-14, atol=1e-14 * np.abs(Kf).max())
    # total mass over all nodes (boundary included) = sum sigma_e |T_e|
    assert math.isclose(Mf.sum(), float(np.sum(sigma * m.area)), rel_tol=1e-13)


def test_homogeneous_stiffness_is_five_point_laplacian():
    n = 9
    m = mesh.build(n)
    nu = np.full(len(m.tri), 3.0)
    K = fem.assemble_stiffness(m, nu).toarray()
    nd = n - 2
    for d in range(m.n_dof):
        i, j = d % nd, d // nd
        assert K[d, d] == pytest.approx(12.0, rel=1e-15)
        for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            ii, jj = i + di, j + dj
            if 0 <= ii < nd and 0 <= jj < nd:
                assert K[d, jj * nd + ii] == pytest.approx(-3.0, rel=1e-15)
        for di, dj in ((1, 1), (-1, -1), (1, -1), (-1, 1)):
            ii, jj = i + di, j + dj
            if 0 <= ii < nd and 0 <= jj < nd:
                assert abs(K[d, jj * nd + ii]) < 1e-15


def test_mass_row_sums_and_pattern():
    n = 9
    m = mesh.build(n)
    M = fem.assemble_mass(m, np.full(len(m.tri), 2.0)).toarray()
    nd = n - 2
    for d in range(m.n_dof):
        i, j = d % nd, d // nd
        if 0 < i < nd - 1 and 0 < j < nd - 1:
            assert M[d].sum() == pytest.approx(2.0 * m.h ** 2, rel=1e-14)
        # "/" diagonal couples (i,j) with (i+1,j+1); "\" diagonal does not
        if i + 1 < nd and j + 1 < nd:
            assert M[d, (j + 1) * nd + i + 1] > 0
        if i + 1 < nd and j > 0:
            assert M[d, (j - 1) * nd + i + 1] == 0


def test_load_shape_total():
    p = W.Problem(33)
    m = mesh.build(33)
    S = fem.load_shape(p, m)
    strip = mesh.strip_mask(m, p)
    # all three vertices of strip elements that are interior receive |T|/3
    expected = sum(m.area[e] / 3.0 for e in np.where(strip)[0] for v in m.tri[e] if m.dof[v] >= 0)
    assert S.sum() == pytest.approx(expected, rel=1e-14)
    assert S.sum() == pytest.approx(strip.sum() * m.area[0] * (1 - 0), rel=0.1)


@pytest.mark.parametrize("n", [5, 9, 17])
def test_banded_cholesky_equals_dense_solve(n):
    w = W.plain_fp64_33()
    p = W.Problem(n, w.problem.material)
    xi = W.level_xi(w, 0, 1)[0]
    s = timestep.build_system(p, xi)
    A = (s.M / 1e-4 + s.K)
    ab = fem.to_banded_lower(A, fem.bandwidth(s.mesh))
    cb = sl.cholesky_banded(ab, lower=True)
    b = np.random.default_rng(n).standard_normal(s.mesh.n_dof)
    x = sl.cho_solve_banded((cb, True), b)
    xd = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(x - xd) <= 1e-13 * np.linalg.norm(xd)


# ---------------------------------------------------------------- KL basis
def test_kl_roots_satisfy_transcendental_equations():
    a, c = 0.2, 5.0
    for w, par in kl.roots_1d(a, c, 12):
        r = c - w * math.tan(w * a) if par == 0 else w + c * math.tan(w * a)
        assert abs(r) <= 1e-12 * max(c, w)


def test_kl_1d_eigen_equation_by_quadrature():
    """int_{-a}^{a} exp(-c|s-t|) phi(t) dt = lam phi(s), checked numerically."""
    a, c = 0.2, 5.0
    for w, par in kl.roots_1d(a, c, 6):
        lam = kl.eig_1d(w, c)
        for s in (-0.17, -0.05, 0.0, 0.11, 0.19):
            f = lambda t: math.exp(-c * abs(s - t)) * float(kl.phi_1d(np.array([t]), w, par, a)[0])
            lhs = si.quad(f, -a, s, epsabs=1e-14, epsrel=1e-13)[0] + si.quad(f, s, a, epsabs=1e-14, epsrel=1e-13)[0]
            rhs = lam * float(kl.phi_1d(np.array([s]), w, par, a)[0])
            assert lhs == pytest.approx(rhs, rel=1e-9, abs=1e-12)


def test_kl_orthonormal_and_trace():
    a, c = 0.2, 5.0
    modes = kl.roots_1d(a, c, 200)
    lam = [kl.eig_1d(w, c) for w, _ in modes]
    # Mercer: sum of all eigenvalues = int C(s,s) ds = 2a; roots are spaced
    # pi/(2a) apart, so the tail beyond n modes is about 8 c a^2 / (pi^2 n)
    tail = 8 * c * a * a / (math.pi ** 2 * len(lam))
    assert sum(lam) + tail == pytest.approx(2 * a, rel=2e-5)
    assert sum(lam[:12]) < 2 * a
    x, wq = np.polynomial.legendre.leggauss(200)
    x, wq = a * x, a * wq
    P = np.stack([kl.phi_1d(x, w, par, a) for w, par in modes[:8]])
    G = (P * wq) @ P.T
    assert np.allclose(G, np.eye(8), atol=1e-12)


def test_kl_2d_order_and_eigenvalues():
    md = kl.modes_2d((0.3, 0.7, 0.3, 0.7), 0.2, 9)
    idx = [(i, j) for _, (i, _, _), (j, _, _) in md[:8]]
    assert idx == [(0, 0), (0, 1), (1, 0), (0, 2), (2, 0), (1, 1), (0, 3), (3, 0)]
    lam = [l for l, _, _ in md]
    assert all(lam[k] >= lam[k + 1] for k in range(8))
    assert lam[7] > lam[8]                 # no tie at the 8-mode cut-off
    # 2-D Mercer trace over the square = its area
    roots = kl.roots_1d(0.2, 5.0, 400)
    l1 = np.array([kl.eig_1d(w, 5.0) for w, _ in roots])
    assert np.sum(np.outer(l1, l1)) == pytest.approx(0.16, rel=5e-3)


def test_kl_field_variance_bounded():
    """sum_k lam_k phi_k(x)^2 <= C(x, x) = 1 at every centroid (truncation)."""
    p = W.Problem(33, W.Material(kind=W.MAT_KL))
    m = mesh.build(33)
    cond = mesh.conductor_mask(m, p)
    T = kl.table(m.centroid[cond], p.conductor, 0.2, 8)
    v = np.sum(T ** 2, axis=1)
    assert np.all(v <= 1.0 + 1e-12) and np.all(v > 0.2)


def test_lumped_row_sum_is_twice_consistent_diagonal():
    """Row-sum lumping of the boundary-inclusive P1 mass matrix (Eq. (4)) equals
    twice its diagonal at every interior node, for a heterogeneous sigma (KL field
    in the conductor, zero in air): the identity the library's lumped-mass option
    rests on."""
    prob = W.Problem(17, W.Material(kind=W.MAT_KL))
    xi = W.normals(0, 47, 0, range(1), 8)[0]
    s = timestep.build_system(prob, xi)
    n = prob.n_nodes
    lump = np.zeros(n * n)
    for k in range(3):
        np.add.at(lump, s.mesh.tri[:, k], s.sigma * s.mesh.area / 3.0)
    inner = s.mesh.dof >= 0
    row = np.zeros(s.mesh.n_dof)
    row[s.mesh.dof[inner]] = lump[inner]
    diag = s.M.diagonal()
    assert np.max(np.abs(row - 2.0 * diag)) <= 1e-12 * np.max(np.abs(row))
    assert np.max(row) > 0.0


def test_load_shape_column_strip_closed_form():
    """Eq. (5), r_i = int J N_i: on an 11-node mesh (h = 0.1) the strip
    [0.1, 0.2] holds exactly the cell column x in [0.1, 0.2].  A P1 hat function
    of the "/" mesh integrates to h^2 and is point-symmetric about its node, so
    half of it (h^2 / 2) lies on either side of the node's vertical line.  Hence
    S_i = h^2 / 2 for interior nodes on x = 0.1 and x = 0.2, and 0 elsewhere."""
    n = 11
    p = W.Problem(n, strip=(0.1, 0.2))
    m = mesh.build(n)
    S = fem.load_shape(p, m)
    h = 0.1
    for j in range(1, n - 1):
        for i in range(1, n - 1):
            d = m.dof[j * n + i]
            want = h * h / 2 if i in (1, 2) else 0.0
            assert S[d] == pytest.approx(want, rel=1e-13, abs=1e-18), (i, j)


def test_load_shape_by_point_quadrature():
    """Eq. (5) by a route that never forms |T|/3: each strip triangle's basis
    functions are evaluated at its three edge midpoints (barycentric coordinates
    from a 3x3 solve against the vertex coordinates), weighted by area/3 (the
    midpoint rule, exact for P1 integrands), and scattered to interior nodes."""
    n = 17
    p = W.Problem(n)
    m = mesh.build(n)
    strip = mesh.strip_mask(m, p)
    ref = np.zeros(m.n_dof)
    for e in np.where(strip)[0]:
        P = m.xy[m.tri[e]]
        V = np.vstack([np.ones(3), P.T])               # columns: (1, x, y) of each vertex
        area = 0.5 * abs(np.linalg.det(V))
        mids = 0.5 * (P + np.roll(P, -1, axis=0))
        for q in mids:
            bary = np.linalg.solve(V, np.array([1.0, q[0], q[1]]))   # N_a(q)
            for a in range(3):
                d = m.dof[m.tri[e][a]]
                if d >= 0:
                    ref[d] += area / 3.0 * bary[a]
    S = fem.load_shape(p, m)
    assert np.max(np.abs(S - ref)) <= 1e-15 * np.max(np.abs(ref))
    assert np.count_nonzero(ref) == np.count_nonzero(S)
