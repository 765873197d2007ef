"""Pins of the oracle's implicit Euler step and Joule-loss QoI
(Section II-A, Eqs. (6)-(7); Section III-B, Eq. (26))."""
import dataclasses
import math

import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp

import workloads as W
from oracle import fem, mesh, picard, timestep


def homogeneous(n, J0=0.0):
    return W.Problem(n, W.Material(kind=W.MAT_LOGNORMAL_SCALAR), conductor=(0.0, 1.0, 0.0, 1.0), J0=J0)


def test_lumped_mass_sine_mode_closed_form():
    """Homogeneous square, lumped mass, no source: the sampled sine mode decays
    by exactly (1 + lam dt)^-n with lam = nu (4 - 2cos(p pi h) - 2cos(q pi h)) / (sigma h^2)."""
    n, p_, q_ = 17, 2, 3
    prob = homogeneous(n)
    s = timestep.build_system(prob, np.zeros(2))
    # row-sum lumping of the full (boundary-inclusive) mass matrix: sum of sigma |T|/3
    lump = np.zeros(n * n)
    for k in range(3):
        np.add.at(lump, s.mesh.tri[:, k], s.sigma * s.mesh.area / 3.0)
    inner = s.mesh.dof >= 0
    diag = np.zeros(s.mesh.n_dof)
    diag[s.mesh.dof[inner]] = lump[inner]
    s = dataclasses.replace(s, M=sp.diags(diag).tocsr())
    h = 1.0 / (n - 1)
    x = np.arange(1, n - 1) * h
    v = np.outer(np.sin(q_ * math.pi * x), np.sin(p_ * math.pi * x)).ravel()   # row j, column i
    sig, nu = prob.material.sigma0, prob.material.nu_cond
    lam = nu * (4 - 2 * math.cos(p_ * math.pi * h) - 2 * math.cos(q_ * math.pi * h)) / (sig * h * h)
    dt = 1e-4
    st = timestep.Stepper(s, dt)
    a, _ = st.run(v, 25)
    ref = (1 + lam * dt) ** -25 * v
    assert np.linalg.norm(a - ref) <= 1e-12 * np.linalg.norm(ref)


def test_consistent_mass_generalised_eigenvector():
    n = 9
    prob = homogeneous(n)
    s = timestep.build_system(prob, np.zeros(2))
    lam, V = sl.eigh(s.K.toarray(), s.M.toarray())
    dt = 2e-4
    st = timestep.Stepper(s, dt)
    for k in (0, 5, 20):
        a, _ = st.run(V[:, k], 30)
        ref = (1 + lam[k] * dt) ** -30 * V[:, k]
        assert np.linalg.norm(a - ref) <= 1e-12 * np.linalg.norm(ref)


def test_forced_mode_qoi_closed_form():
    """Source g(t) M v with (K, M)-eigenvector v: scalar recurrence
    c_{k+1} = (c_k/dt + g_{k+1}) / (1/dt + lam), and Eq. (26) becomes
    Q = sum (c_{k+1} - c_k)^2 v^T M v / (T dt)."""
    n = 9
    prob = homogeneous(n, J0=1.0e3)
    s = timestep.build_system(prob, np.zeros(2))
    lam, V = sl.eigh(s.K.toarray(), s.M.toarray())
    v = V[:, 3]
    s = dataclasses.replace(s, S=s.M @ v)
    spp, nper = 40, 2
    dt = prob.period / spp
    st = timestep.Stepper(s, dt)
    a, qsum = st.run(np.zeros(s.mesh.n_dof), spp * nper)
    c, acc = 0.0, 0.0
    vMv = float(v @ (s.M @ v))
    for k in range(spp * nper):
        g = prob.J0 * math.sin(2 * math.pi * prob.freq * (k + 1) * dt)
        cn = (c / dt + g) / (1 / dt + lam[3])
        acc += (cn - c) ** 2 * vMv / dt
        c = cn
    assert np.linalg.norm(a - c * v) <= 1e-10 * np.linalg.norm(c * v)
    assert qsum == pytest.approx(acc, rel=1e-10)


def test_discrete_energy_identity():
    """sum d^T M d/dt = sum d^T r_{k+1} - (a_N^T K a_N - a_0^T K a_0)/2 - sum d^T K d / 2."""
    w = W.plain_fp64_33()
    prob = W.Problem(17, w.problem.material)
    xi = W.level_xi(w, 0, 1)[0]
    s = timestep.build_system(prob, xi)
    dt = prob.period / 32
    st = timestep.Stepper(s, dt)
    a = np.zeros(s.mesh.n_dof)
    lhs = 0.0
    rhs = 0.0
    half_kd = 0.0
    for k in range(48):
        an, dq = st.step(a, k)
        d = an - a
        lhs += dq
        r = fem.source_value(prob, (k + 1) * dt) * s.S
        rhs += float(d @ r)
        half_kd += 0.5 * float(d @ (s.K @ d))
        a = an
    rhs -= 0.5 * float(a @ (s.K @ a)) + half_kd
    assert lhs == pytest.approx(rhs, rel=1e-10)


def test_qoi_quadratic_in_source_and_positive():
    w = W.plain_fp64_33()
    xi = W.level_xi(w, 0, 2)
    p1 = W.Problem(17, w.problem.material, J0=1.0e6)
    p2 = W.Problem(17, w.problem.material, J0=2.0e6)
    for x in xi:
        q1, a1 = timestep.solve_sample(p1, x, 32, 1)
        q2, a2 = timestep.solve_sample(p2, x, 32, 1)
        assert q1 > 0
        assert q2 == pytest.approx(4 * q1, rel=1e-12)
        assert np.allclose(a2, 2 * a1, rtol=1e-12, atol=1e-14 * np.abs(a2).max())


def test_zero_conductivity_gives_zero_loss():
    w = W.plain_fp64_33()
    mat = dataclasses.replace(w.problem.material, sigma0=0.0)
    p = W.Problem(9, mat)
    s = timestep.build_system(p, np.zeros(2))
    # sigma = 0 everywhere -> M = 0, IE reduces to the static solve K a = r each step
    st = timestep.Stepper(s, 1e-3)
    a, q = st.run(np.zeros(s.mesh.n_dof), 3)
    assert q == 0.0
    ref = np.linalg.solve(s.K.toarray(), fem.source_value(p, 3e-3) * s.S)
    assert np.linalg.norm(a - ref) <= 1e-12 * np.linalg.norm(ref)


# ---------------------------------------------------------------- Picard
def test_picard_linear_limit():
    """k2 = 0: nu = k1' + k3' is constant, the fixed point is reached in one
    solve plus one confirming iteration and equals the linear solution."""
    mat = W.Material(kind=W.MAT_NONLINEAR, k2=0.0)
    prob = W.Problem(9, mat)
    xi = np.array([0.3, -1.0, 0.7])
    Q, a, counts, flagged = picard.solve_sample(prob, xi, 16, 1, return_counts=True)
    Ql, al = timestep.solve_sample(prob, xi, 16, 1)
    assert not flagged and np.all(counts == 2)
    assert Q == pytest.approx(Ql, rel=1e-13)
    assert np.linalg.norm(a - al) <= 1e-13 * np.linalg.norm(al)


def test_picard_fixed_point_satisfies_nonlinear_step():
    """Every converged step solves the nonlinear Eq. (7) with nu taken at a_{k+1}:
    M (a_{k+1} - a_k)/dt + K(nu(a_{k+1})) a_{k+1} = r(t_{k+1})."""
    mat = W.Material(kind=W.MAT_NONLINEAR, k2=1.0e3)      # strong nonlinearity for this weak field
    prob = W.Problem(9, mat)
    xi = np.array([0.1, 0.4, -0.2])
    m = mesh.build(9)
    Q, a_end, counts, flagged, traj = picard.solve_sample(prob, xi, 8, 1, return_counts=True,
                                                          return_traj=True)
    assert not flagged and counts.max() > 2
    sigma, nu = fem.materials(prob, m, xi)
    cond = mesh.conductor_mask(m, prob)
    k1, k2, k3 = fem.nonlinear_coeffs(prob, xi)
    g = fem.basis_gradients(m)
    M = fem.assemble_mass(m, sigma)
    S = fem.load_shape(prob, m)
    dt = prob.period / 8
    for k in range(8):
        a0, a1 = traj[k], traj[k + 1]
        nu_e = nu.copy()
        nu_e[cond] = k1 * np.exp(k2 * picard.b_squared(m, g, a1)[cond]) + k3
        K = fem.assemble_stiffness(m, nu_e, g)
        r = fem.source_value(prob, (k + 1) * dt) * S
        res = M @ (a1 - a0) / dt + K @ a1 - r
        assert np.linalg.norm(res) <= 1e-6 * np.linalg.norm(K @ a1)


def test_b_squared_linear_field_and_hand_elements():
    """|B_e|^2 = |grad a_h|^2 per element (Eq. (1) with B = curl(A e_z)).

    (1) a = alpha x + beta y sampled on interior nodes: on every element with no
    boundary vertex the P1 interpolant is that linear field, so |grad a|^2 =
    alpha^2 + beta^2 exactly (up to rounding).
    (2) Hand values on a 4-node mesh (h = 1/3), interior DoFs (1,1)=1, (2,1)=2,
    (1,2)=3, (2,2)=5 (boundary zero).  In cell (1,1) the lower triangle
    (1,1),(2,1),(2,2) has d/dx = (2-1)/h, d/dy = (5-2)/h, |g|^2 = 10/h^2 = 90;
    the upper one (1,1),(2,2),(1,2) has d/dx = (5-3)/h, d/dy = (3-1)/h, 8/h^2 = 72.
    In cell (0,0) the lower triangle (0,0),(1,0),(1,1) has d/dy = 1/h, 9; the upper
    one (0,0),(1,1),(0,1) has d/dx = 1/h, 9.  In cell (2,0) the lower triangle
    (2,0),(3,0),(3,1) is all boundary, 0; the upper one (2,0),(3,1),(2,1) has
    d/dx = (0-2)/h, d/dy = (2-0)/h, 8/h^2 = 72."""
    n = 9
    m = mesh.build(n)
    g = fem.basis_gradients(m)
    alpha, beta = 0.37, -1.9
    nd = n - 2
    a = np.zeros(m.n_dof)
    for j in range(1, n - 1):
        for i in range(1, n - 1):
            a[(j - 1) * nd + (i - 1)] = alpha * i * m.h + beta * j * m.h
    b2 = picard.b_squared(m, g, a)
    interior = np.all(m.dof[m.tri] >= 0, axis=1)
    assert interior.sum() > 0
    assert np.allclose(b2[interior], alpha ** 2 + beta ** 2, rtol=1e-12, atol=0)
    assert np.all(np.abs(b2[~interior] - (alpha ** 2 + beta ** 2)) > 1e-6)

    m4 = mesh.build(4)
    g4 = fem.basis_gradients(m4)
    b4 = picard.b_squared(m4, g4, np.array([1.0, 2.0, 3.0, 5.0]))

    def elem(i, j, upper):
        return 2 * (j * 3 + i) + (1 if upper else 0)

    want = {(1, 1, 0): 90.0, (1, 1, 1): 72.0, (0, 0, 0): 9.0, (0, 0, 1): 9.0,
            (2, 0, 0): 0.0, (2, 0, 1): 72.0}
    for (i, j, up), v in want.items():
        e = elem(i, j, up)
        c = m4.centroid[e]
        assert (c[0] - i / 3) * 3 == pytest.approx(2 / 3 if not up else 1 / 3)
        assert b4[e] == pytest.approx(v, rel=1e-13, abs=1e-12), (i, j, up)
