"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Tolerances: FP64 path 1e-10 relative on Q and on the final state; mixed
path (FP32 CG inside FP64 refinement) 1e-6 relative on Q.  Operator applies
are compared entry-wise at FP64 rounding level.
"""
import dataclasses
import sys

import numpy as np
import pytest

import workloads as W
from oracle import fem, mesh as omesh, mlmc as omlmc, parareal as opara, timestep as ots

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_19246_amd as mq
    mq.load()
    yield


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mqmod():
    import paper_2507_19246_amd as mq
    from paper_2507_19246_amd import _lib
    return mq, _lib


def oracle_q(problem, xi, spp, nper):
    m = omesh.build(problem.n_nodes)
    tab = ots.kl_table_for(problem, m)
    out = [ots.solve_sample(problem, x, spp, nper, m=m, kl_table=tab) for x in xi]
    return np.array([o[0] for o in out]), np.stack([o[1] for o in out])


@pytest.mark.parametrize("n,kind", [(5, 0), (9, 1), (33, 0), (33, 1), (129, 1)])
def test_operator_apply_matches_oracle(n, kind):
    mq, L = mqmod()
    say(f"apply n={n} kind={kind}")
    prob = W.Problem(n, W.Material(kind=kind))
    p = mq.Problem(prob, L.MQ_PREC_FP64)
    nxi = prob.material.n_xi
    xi = W.normals(3, 11, 0, range(3), nxi)
    rng = np.random.default_rng(n)
    x = rng.standard_normal((3, prob.n_dof))
    dt = 1e-4
    m = omesh.build(n)
    tab = ots.kl_table_for(prob, m)
    for which in (L.MQ_APPLY_A, L.MQ_APPLY_M, L.MQ_APPLY_K):
        y = mq.debug_apply(p, which, dt, xi, x).cpu().numpy()
        for s in range(3):
            sysm = ots.build_system(prob, xi[s], m, tab)
            Mat = {L.MQ_APPLY_A: sysm.M / dt + sysm.K, L.MQ_APPLY_M: sysm.M, L.MQ_APPLY_K: sysm.K}[which]
            ref = Mat @ x[s]
            scale = abs(Mat) @ np.abs(x[s]) + 1e-300
            assert np.max(np.abs(y[s] - ref) / scale.max()) < 1e-14, (which, s)
    p.close()


@pytest.mark.parametrize("pc", [1, 2])
def test_plain_fp64_33_full_parity(pc):
    """Plain MC, FP64, 33x33, 16 samples, 64 steps: Q and a_N within 1e-10."""
    mq, L = mqmod()
    w = W.plain_fp64_33()
    lv = w.levels[0]
    xi = W.level_xi(w, 0)
    say(f"plain fp64 33 full precond={pc}")
    p = mq.Problem(w.problem, L.MQ_PREC_FP64, precond=pc)
    qf, qc, fs, rc, st = mq.mlmc_level_run(p, lv.steps_per_period, 0, lv.n_periods, xi, want_state=True)
    assert rc == 0 and qc is None
    say("stats", st)
    qref, aref = oracle_q(w.problem, xi, lv.steps_per_period, lv.n_periods)
    q = qf.cpu().numpy()
    err = np.abs(q - qref) / np.abs(qref)
    say("max rel err Q", err.max())
    assert err.max() <= 1e-10
    a = fs.cpu().numpy()
    for s in range(len(xi)):
        assert np.linalg.norm(a[s] - aref[s]) <= 1e-10 * np.linalg.norm(aref[s])
    p.close()


@pytest.mark.parametrize("n,path,pc,tile", [(33, 1, 1, 0), (33, 1, 2, 0), (33, 2, 1, 0), (33, 2, 2, 0),
                                            (65, 1, 1, 0), (65, 1, 2, 0), (65, 2, 1, 0), (65, 2, 2, 0),
                                            (129, 1, 2, 1), (129, 1, 2, 2), (129, 1, 1, 2), (129, 2, 2, 0),
                                            (65, 2, 2, 2), (65, 2, 1, 2)])
def test_mixed_kl_coupled_level(n, path, pc, tile):
    """Mixed precision, KL field, coupled fine/coarse run: Q within 1e-6
    (resident/streaming path, Jacobi/multigrid preconditioner on either path,
    both resident workgroup shapes at 129 x 129)."""
    mq, L = mqmod()
    prob = W.Problem(n, W.Material(kind=W.MAT_KL))
    xi = W.normals(0, 21, 1, range(6 if n < 129 else 3), 8)
    say(f"mixed kl n={n} path={path} precond={pc} tile={tile}")
    p = mq.Problem(prob, L.MQ_PREC_MIXED, path=path, precond=pc, tile=tile)
    assert p.info.precond == pc
    if tile:
        assert p.info.tile == tile and p.info.block == (1024 if tile == 1 else 512)
        assert p.path == (L.MQ_PATH_STREAMING if path == 2 else L.MQ_PATH_RESIDENT)
    qf, qc, _, rc, st = mq.mlmc_level_run(p, 32, 16, 2, xi)
    assert rc == 0
    say("stats", st)
    rf, _ = oracle_q(prob, xi, 32, 2)
    rcq, _ = oracle_q(prob, xi, 16, 2)
    ef = np.abs(qf.cpu().numpy() - rf) / np.abs(rf)
    ec = np.abs(qc.cpu().numpy() - rcq) / np.abs(rcq)
    say("max rel err fine/coarse", ef.max(), ec.max())
    assert ef.max() <= 1e-6 and ec.max() <= 1e-6
    p.close()


@pytest.mark.parametrize("n,path,levels,sweeps", [(65, 1, 2, 4), (65, 1, 3, 0), (65, 2, 2, 6), (33, 1, 1, 8)])
def test_mg_truncated_hierarchy(n, path, levels, sweeps):
    """Multigrid with a capped coarse hierarchy and damped-Jacobi sweeps at its
    coarsest level (both paths): Q within 1e-6 of the oracle."""
    mq, L = mqmod()
    prob = W.Problem(n, W.Material(kind=W.MAT_KL))
    xi = W.normals(0, 24, 1, range(4), 8)
    say(f"truncated mg n={n} path={path} levels={levels} sweeps={sweeps}")
    p = mq.Problem(prob, L.MQ_PREC_MIXED, path=path, precond=L.MQ_PRECOND_MULTIGRID,
                   mg_levels=levels, mg_coarse_sweeps=sweeps)
    qf, _, _, rc, st = mq.mlmc_level_run(p, 32, 0, 2, xi)
    assert rc == 0
    rf, _ = oracle_q(prob, xi, 32, 2)
    err = np.max(np.abs(qf.cpu().numpy() - rf) / np.abs(rf))
    say("max rel err", err, "iters/step", st["inner_iters"] / st["sample_steps"])
    assert err <= 1e-6
    p.close()


def test_streaming_fp64_matches_oracle():
    mq, L = mqmod()
    w = W.plain_fp64_33()
    xi = W.level_xi(w, 0, 4)
    p = mq.Problem(w.problem, L.MQ_PREC_FP64, path=L.MQ_PATH_STREAMING)
    qf, _, _, rc, st = mq.mlmc_level_run(p, 64, 0, 1, xi)
    qref, _ = oracle_q(w.problem, xi, 64, 1)
    assert np.max(np.abs(qf.cpu().numpy() - qref) / qref) <= 1e-10
    p.close()


def test_deterministic_and_alone_equals_mix():
    mq, L = mqmod()
    prob = W.Problem(33, W.Material(kind=W.MAT_KL))
    xi = W.normals(0, 22, 0, range(10), 8)
    p = mq.Problem(prob, L.MQ_PREC_MIXED)
    q1 = mq.mlmc_level_run(p, 32, 16, 1, xi)[0].cpu().numpy()
    q2 = mq.mlmc_level_run(p, 32, 16, 1, xi)[0].cpu().numpy()
    assert np.array_equal(q1, q2)
    for k in (0, 7):
        qa = mq.mlmc_level_run(p, 32, 16, 1, xi[k:k + 1])[0].cpu().numpy()
        assert qa[0] == q1[k]
    p.close()


def test_mlmc_estimate_matches_oracle():
    mq, L = mqmod()
    rng = np.random.default_rng(3)
    qf = [rng.normal(10, 1, 37), rng.normal(1, 0.1, 11), rng.normal(0.1, 0.01, 5)]
    qc = [None, rng.normal(1, 0.1, 11), rng.normal(0.1, 0.01, 5)]
    e, y, v = mq.mlmc_estimate([torch.tensor(q, dtype=torch.float64, device="cuda") for q in qf],
                               [None] + [torch.tensor(q, dtype=torch.float64, device="cuda") for q in qc[1:]])
    er, yr, vr = omlmc.estimate(qf, qc)
    assert float(e) == pytest.approx(er, rel=1e-14)
    assert np.allclose(y.cpu().numpy(), yr, rtol=1e-13)
    assert np.allclose(v.cpu().numpy(), vr, rtol=1e-12)


@pytest.mark.parametrize("path", [1, 2])
def test_parareal_matches_oracle(path):
    mq, L = mqmod()
    prob = W.Problem(17, W.Material(kind=W.MAT_KL))
    xi = W.normals(0, 23, 0, range(3), 8)
    p = mq.Problem(prob, L.MQ_PREC_FP64, path=path)
    say(f"parareal path={path}")
    # fixed K = M: the serial fine solution
    q, it, fs, rc, st = mq.parareal_run(p, 1, 6, 4, 1, 6, 0.0, xi, fixed_k=6, want_state=True)
    for s in range(3):
        ref = opara.serial_fine(prob, xi[s], 1, 6, 4)
        assert float(q[s]) == pytest.approx(ref["Q"], rel=1e-10)
        a = fs[s].cpu().numpy()
        assert np.linalg.norm(a - ref["state"]) <= 1e-10 * np.linalg.norm(ref["state"])
    assert np.all(it.cpu().numpy() == 6)
    # tolerance mode: K as the oracle (within one: the stop test compares a
    # jump near tol), and Q as the oracle's Parareal stopped at the same K
    q, it, fs, rc, st = mq.parareal_run(p, 1, 8, 8, 1, 8, 1e-5, xi)
    for s in range(3):
        ref = opara.run(prob, xi[s], 1, 8, 8, 1, k_max=8, tol=1e-5)
        assert abs(int(it[s]) - ref["K"]) <= 1
        if int(it[s]) != ref["K"]:
            ref = opara.run(prob, xi[s], 1, 8, 8, 1, k_max=8, tol=1e-5, fixed_k=int(it[s]))
        assert float(q[s]) == pytest.approx(ref["Q"], rel=1e-9)
    p.close()


@pytest.mark.parametrize("path", [1, 2])
def test_parareal_fixed_k_below_m_matches_oracle(path):
    """Parareal stopped at a fixed k < M (Eq. (12)): the slices after k are not
    yet exact, so Q and the final state depend on every coarse correction
    F + (C_new - C_old) made so far.  They match the oracle's Parareal at the
    same k within 1e-10 (FP64), and differ from the serial fine run by far
    more than that, so the comparison sees the correction."""
    mq, L = mqmod()
    prob = W.Problem(17, W.Material(kind=W.MAT_KL))
    xi = W.normals(0, 24, 0, range(3), 8)
    p = mq.Problem(prob, L.MQ_PREC_FP64, path=path)
    m = omesh.build(17)
    tab = ots.kl_table_for(prob, m)
    for k in (1, 2, 3):
        say(f"parareal fixed_k={k} of M=6, path={path}")
        q, it, fs, rc, st = mq.parareal_run(p, 1, 6, 4, 1, 6, 0.0, xi, fixed_k=k, want_state=True)
        assert rc == 0 and np.all(it.cpu().numpy() == k)
        assert np.all(mq.last_flags() == 0)
        for s in range(3):
            ref = opara.run(prob, xi[s], 1, 6, 4, 1, k_max=6, tol=0.0, fixed_k=k, m=m, kl_table=tab)
            ser = opara.serial_fine(prob, xi[s], 1, 6, 4, m=m, kl_table=tab)
            assert ref["K"] == k
            assert float(q[s]) == pytest.approx(ref["Q"], rel=1e-10)
            a = fs[s].cpu().numpy()
            assert np.linalg.norm(a - ref["state"]) <= 1e-10 * np.linalg.norm(ref["state"])
            assert np.linalg.norm(ref["state"] - ser["state"]) > 1e-6 * np.linalg.norm(ser["state"])
    p.close()


def test_parareal_kmax_warning_flags_every_sample():
    """Tolerance mode with k_max = 2 and a tolerance no sample reaches: the call
    returns MQ_WARN_NOT_CONVERGED, every sample carries MQ_FLAG_PARAREAL_KMAX,
    and Q is the oracle's Parareal stopped at k = 2."""
    mq, L = mqmod()
    prob = W.Problem(17, W.Material(kind=W.MAT_KL))
    xi = W.normals(0, 25, 0, range(2), 8)
    p = mq.Problem(prob, L.MQ_PREC_FP64)
    q, it, _, rc, _ = mq.parareal_run(p, 1, 6, 4, 1, 2, 1e-14, xi)
    assert rc == L.MQ_WARN_NOT_CONVERGED
    f = mq.last_flags()
    assert len(f) == 2 and np.all(f == L.MQ_FLAG_PARAREAL_KMAX)
    for s in range(2):
        ref = opara.run(prob, xi[s], 1, 6, 4, 1, k_max=2, tol=1e-14)
        assert int(it[s]) == ref["K"] == 2
        assert float(q[s]) == pytest.approx(ref["Q"], rel=1e-10)
    p.close()


@pytest.mark.parametrize("path", [1, 2])
def test_solver_caps_flag_instances(path):
    """Tiny max_iter and max_sweeps: every step stops at the cap, the call
    returns MQ_WARN_NOT_CONVERGED, every instance carries MQ_FLAG_NOT_CONVERGED
    (fine instances, then coarse, per level) and the results stay finite."""
    mq, L = mqmod()
    prob = W.Problem(17, W.Material(kind=W.MAT_KL))
    xi = W.normals(0, 26, 0, range(3), 8)
    p = mq.Problem(prob, L.MQ_PREC_FP64, path=path, max_iter=2, max_sweeps=1)
    say(f"solver caps path={path}")
    qf, qc, _, rc, st = mq.mlmc_level_run(p, 8, 4, 1, xi)
    assert rc == L.MQ_WARN_NOT_CONVERGED
    f = mq.last_flags()
    assert len(f) == 6 and np.all(f == L.MQ_FLAG_NOT_CONVERGED)
    assert st["n_not_converged"] == 6 and st["n_failed"] == 0
    assert bool(torch.isfinite(qf).all()) and bool(torch.isfinite(qc).all())
    qfs, qcs, rcm, stm = mq.mlmc_multilevel_run(p, [(4, 0, 1), (8, 4, 1)], [xi[:2], xi])
    assert rcm == L.MQ_WARN_NOT_CONVERGED and stm["n_not_converged"] == 2 + 6
    assert len(mq.last_flags()) == 2 + 6
    p.close()


def test_picard_cap_flags_and_matches_oracle():
    """picard_max = 1: every step makes one Picard iteration (nu lagged at a_k)
    and stops at the cap.  The call returns MQ_WARN_NOT_CONVERGED, every
    instance carries MQ_FLAG_PICARD_CAP, and Q is the oracle's with the same
    cap (FP64, 1e-9)."""
    from oracle import picard as opic
    mq, L = mqmod()
    prob = W.Problem(33, W.Material(kind=W.MAT_NONLINEAR, k2=5.0e2, picard_max=1))
    xi = W.normals(0, 27, 0, range(3), 3)
    p = mq.Problem(prob, L.MQ_PREC_FP64, tol=1e-12, inner_rtol=1e-9)
    qf, _, _, rc, st = mq.mlmc_level_run(p, 16, 0, 1, xi)
    assert rc == L.MQ_WARN_NOT_CONVERGED
    f = mq.last_flags()
    assert len(f) == 3 and np.all(f & L.MQ_FLAG_PICARD_CAP) and st["n_not_converged"] == 3
    assert st["picard_iters"] == 3 * 16
    m = omesh.build(33)
    for s in range(3):
        Q, a, counts, flagged = opic.solve_sample(prob, xi[s], 16, 1, m=m, return_counts=True)
        assert flagged and np.all(counts == 1)
        assert float(qf[s]) == pytest.approx(Q, rel=1e-9)
    p.close()


@pytest.mark.parametrize("path", [1, 2])
def test_nonfinite_instance_leaves_others_correct(path):
    """A finite input whose conductivity overflows (sigma = inf) gives that
    instance a non-finite residual: it carries MQ_FLAG_FAILED and a non-finite
    Q, the call returns MQ_WARN_NOT_CONVERGED, and the other instances of the
    same launch still match the oracle within 1e-10 (FP64)."""
    mq, L = mqmod()
    prob = W.Problem(17, W.Material(kind=W.MAT_KL))
    xi = W.normals(0, 28, 0, range(4), 8)
    xi[2, 0] = 1.0e4  # exp(0.3 sqrt(lambda_1) phi_1 xi) overflows on the conductor
    p = mq.Problem(prob, L.MQ_PREC_FP64, path=path, max_iter=400)
    say(f"non-finite instance path={path}")
    qf, _, _, rc, st = mq.mlmc_level_run(p, 8, 0, 1, xi)
    assert rc == L.MQ_WARN_NOT_CONVERGED
    f = mq.last_flags()
    assert f[2] & L.MQ_FLAG_FAILED and st["n_failed"] == 1
    assert not np.isfinite(float(qf[2]))
    good = [0, 1, 3]
    assert np.all(f[good] == 0)
    qref, _ = oracle_q(prob, xi[good], 8, 1)
    assert np.max(np.abs(qf.cpu().numpy()[good] - qref) / qref) <= 1e-10
    p.close()


def test_nonfinite_xi_rejected():
    mq, L = mqmod()
    prob = W.Problem(9, W.Material(kind=W.MAT_KL))
    p = mq.Problem(prob, L.MQ_PREC_MIXED)
    xi = np.zeros((2, 8))
    xi[1, 3] = np.nan
    with pytest.raises(L.MQError) as e:
        mq.mlmc_level_run(p, 8, 0, 1, xi)
    assert e.value.code == L.MQ_ERR_NONFINITE
    p.close()


def test_empty_and_malformed_inputs_rejected():
    """Empty sample sets and malformed level or Parareal descriptions are
    rejected on the host before any launch; the handle stays usable."""
    mq, L = mqmod()
    prob = W.Problem(9, W.Material(kind=W.MAT_KL))
    p = mq.Problem(prob, L.MQ_PREC_MIXED)
    empty = np.zeros((0, p.n_xi))
    two = W.normals(0, 31, 0, range(2), p.n_xi)
    bad = [
        ("level, no samples", lambda: mq.mlmc_level_run(p, 8, 0, 1, empty)),
        ("level, zero steps", lambda: mq.mlmc_level_run(p, 0, 0, 1, two)),
        ("level, zero periods", lambda: mq.mlmc_level_run(p, 8, 4, 0, two)),
        ("parareal, no samples", lambda: mq.parareal_run(p, 1, 4, 2, 1, 4, 1e-8, empty)),
        ("parareal, no slices", lambda: mq.parareal_run(p, 1, 0, 2, 1, 4, 1e-8, two)),
        ("parareal, k_max 0", lambda: mq.parareal_run(p, 1, 4, 2, 1, 0, 1e-8, two)),
        ("parareal, negative tol", lambda: mq.parareal_run(p, 1, 4, 2, 1, 4, -1.0, two)),
        ("estimate, empty level", lambda: mq.mlmc_estimate([torch.zeros(0, dtype=torch.float64, device="cuda")], [None])),
    ]
    for name, call in bad:
        say(f"malformed input: {name}")
        with pytest.raises(L.MQError) as e:
            call()
        assert e.value.code == L.MQ_ERR_INVALID_ARG, name
    qf, _, _, rc, _ = mq.mlmc_level_run(p, 8, 0, 1, two)
    assert rc == 0 and bool(torch.isfinite(qf).all())
    p.close()


def test_initial_state_eigenmode_and_oracle():
    """mq_set_initial_state.  Homogeneous square, no source, a_0 a generalised
    eigenvector v of (K, M): implicit Euler (Eq. (7)) gives a_n = (1 + lam dt)^-n v,
    and Eq. (26) the loss from the scalar increments (v^T M v = 1).  With the KL
    material and the source on, a seeded random a_0 gives the oracle's Q (fine and
    coupled coarse) and final state, Parareal at K = M from U_0 = a_0 gives the
    serial fine run, and None restores a_0 = 0."""
    import scipy.linalg as sl
    mq, L = mqmod()
    hom = W.Problem(9, W.Material(kind=W.MAT_LOGNORMAL_SCALAR), conductor=(0.0, 1.0, 0.0, 1.0), J0=0.0)
    s = ots.build_system(hom, np.zeros(2))
    lam, V = sl.eigh(s.K.toarray(), s.M.toarray())
    p = mq.Problem(hom, L.MQ_PREC_FP64)
    spp, nper = 4, 2
    nst, dt = spp * nper, hom.period / spp
    for k in (0, 7, 30):
        say(f"initial state: eigenmode {k}, lam dt = {lam[k] * dt:.3e}")
        p.set_initial_state(V[:, k])
        qf, _, fs, rc, _ = mq.mlmc_level_run(p, spp, 0, nper, np.zeros((1, 2)), want_state=True)
        assert rc == 0
        c = (1.0 + lam[k] * dt) ** -np.arange(nst + 1.0)
        ref = c[-1] * V[:, k]
        a = fs[0].cpu().numpy()
        assert np.linalg.norm(a - ref) <= 1e-10 * np.linalg.norm(ref)
        qref = np.sum(np.diff(c) ** 2) / dt / (nst * dt)
        assert float(qf[0]) == pytest.approx(qref, rel=1e-10)
    p.close()

    prob = W.Problem(17, W.Material(kind=W.MAT_KL))
    m = omesh.build(17)
    tab = ots.kl_table_for(prob, m)
    xi = W.normals(0, 37, 0, range(3), 8)
    p = mq.Problem(prob, L.MQ_PREC_FP64)
    _, a_scale = ots.solve_sample(prob, xi[0], 16, 1, m=m, kl_table=tab)
    a0 = np.random.default_rng(11).standard_normal(p.n_dof) * np.abs(a_scale).max()
    say("initial state: random a_0, KL material, level run and Parareal")
    p.set_initial_state(a0)
    qf, qc, fs, rc, _ = mq.mlmc_level_run(p, 16, 8, 1, xi, want_state=True)
    qp, it, fsp, rcp, _ = mq.parareal_run(p, 1, 4, 4, 1, 4, 0.0, xi, fixed_k=4, want_state=True)
    assert rc == 0 and rcp == 0
    for i in range(3):
        qref, aref = ots.solve_sample(prob, xi[i], 16, 1, a0=a0, m=m, kl_table=tab)
        qcref, _ = ots.solve_sample(prob, xi[i], 8, 1, a0=a0, m=m, kl_table=tab)
        assert float(qf[i]) == pytest.approx(qref, rel=1e-10)
        assert float(qc[i]) == pytest.approx(qcref, rel=1e-10)
        assert np.linalg.norm(fs[i].cpu().numpy() - aref) <= 1e-10 * np.linalg.norm(aref)
        assert float(qp[i]) == pytest.approx(qref, rel=1e-10)
        assert np.linalg.norm(fsp[i].cpu().numpy() - aref) <= 1e-10 * np.linalg.norm(aref)
    # a rejected a_0 keeps the previous one; None restores zeros
    bad = a0.copy()
    bad[5] = np.inf
    with pytest.raises(L.MQError) as e:
        p.set_initial_state(bad)
    assert e.value.code == L.MQ_ERR_NONFINITE
    qf2, _, _, _, _ = mq.mlmc_level_run(p, 16, 0, 1, xi[:1])
    assert float(qf2[0]) == float(qf[0])
    p.set_initial_state(None)
    qf0, _, _, _, _ = mq.mlmc_level_run(p, 16, 0, 1, xi[:1])
    q0ref, _ = ots.solve_sample(prob, xi[0], 16, 1, m=m, kl_table=tab)
    assert float(qf0[0]) == pytest.approx(q0ref, rel=1e-10)
    p.close()


@pytest.mark.parametrize("n", [5, 9, 17])
def test_small_mesh_resident_multigrid_fp64(n):
    """Regression: on meshes with fewer full-grid nodes than (rows x threads) of
    the resident workgroup, the thread-private multigrid planes (iterate,
    D^{-1/2}) need their own room in the work slot; with full-grid-sized planes
    the FP64 iterate overwrote the scaling on the 9-node mesh (Q = inf).  FP64
    resident multigrid, Jacobi and streaming multigrid all give the oracle's Q
    and final state."""
    mq, L = mqmod()
    prob = W.Problem(n, W.Material(kind=W.MAT_KL))
    xi = W.normals(0, 41, 0, range(3), 8)
    qref, aref = oracle_q(prob, xi, 8, 1)
    cases = [(L.MQ_PATH_RESIDENT, L.MQ_PRECOND_MULTIGRID), (L.MQ_PATH_RESIDENT, L.MQ_PRECOND_JACOBI),
             (L.MQ_PATH_STREAMING, L.MQ_PRECOND_MULTIGRID)]
    for path, pc in cases:
        say(f"small mesh n={n} path={path} precond={pc}")
        p = mq.Problem(prob, L.MQ_PREC_FP64, path=path, precond=pc)
        assert p.info.precond == pc
        qf, _, fs, rc, st = mq.mlmc_level_run(p, 8, 0, 1, xi, want_state=True)
        assert rc == 0 and st["n_failed"] == 0
        assert np.max(np.abs(qf.cpu().numpy() - qref) / np.abs(qref)) <= 1e-10
        assert np.linalg.norm(fs.cpu().numpy() - aref) <= 1e-10 * np.linalg.norm(aref)
        p.close()


def test_host_pointer_handle_matches_device_handle():
    """mem_kind = MQ_MEM_HOST: initial state, level run, multilevel run and
    Parareal take host arrays through the C ABI and give the device handle's
    results bit for bit; the calls without a host form refuse such a handle."""
    import ctypes as C
    mq, L = mqmod()
    prob = W.Problem(17, W.Material(kind=W.MAT_KL))
    xi = np.ascontiguousarray(W.normals(0, 43, 0, range(4), 8), dtype=np.float64)
    pdv = mq.Problem(prob, L.MQ_PREC_MIXED)
    ph = mq.Problem(prob, L.MQ_PREC_MIXED, mem_kind=L.MQ_MEM_HOST)
    lib = ph.lib

    def P(a):
        return a.ctypes.data_as(C.c_void_p)

    say("host handle: initial state + level run")
    a0 = np.ascontiguousarray(np.random.default_rng(5).standard_normal(ph.n_dof) * 1e-4)
    pdv.set_initial_state(a0)
    assert lib.mq_set_initial_state(ph.h, P(a0)) == 0
    qf_d, qc_d, fs_d, rc_d, _ = mq.mlmc_level_run(pdv, 16, 8, 1, xi, want_state=True)
    qf, qc, fs = np.zeros(4), np.zeros(4), np.zeros((4, ph.n_dof))
    lv = L.LevelDesc(16, 8, 1, 0)
    st = L.RunStats()
    rc = lib.mlmc_level_run(ph.h, C.byref(lv), 4, P(xi), P(qf), P(qc), P(fs), C.byref(st))
    assert rc == rc_d == 0
    np.testing.assert_array_equal(qf, qf_d.cpu().numpy())
    np.testing.assert_array_equal(qc, qc_d.cpu().numpy())
    np.testing.assert_array_equal(fs, fs_d.cpu().numpy())
    pdv.set_initial_state(None)
    assert lib.mq_set_initial_state(ph.h, None) == 0

    say("host handle: multilevel run")
    levels = [(8, 0, 1), (16, 8, 1)]
    xs = [xi[:3].copy(), xi[1:].copy()]
    qfs_d, qcs_d, rcm_d, _ = mq.mlmc_multilevel_run(pdv, levels, xs)
    lvs = (L.LevelDesc * 2)(*[L.LevelDesc(a, b, c, 0) for a, b, c in levels])
    ns = (C.c_int32 * 2)(3, 3)
    qfh = [np.zeros(3), np.zeros(3)]
    qch = [None, np.zeros(3)]
    px = (C.c_void_p * 2)(*[x.ctypes.data for x in xs])
    pf = (C.c_void_p * 2)(*[q.ctypes.data for q in qfh])
    pc = (C.c_void_p * 2)(None, qch[1].ctypes.data)
    assert lib.mlmc_multilevel_run(ph.h, 2, lvs, ns, px, pf, pc, C.byref(st)) == rcm_d == 0
    for l in range(2):
        np.testing.assert_array_equal(qfh[l], qfs_d[l].cpu().numpy())
    np.testing.assert_array_equal(qch[1], qcs_d[1].cpu().numpy())

    say("host handle: Parareal")
    qp_d, it_d, fsp_d, rcp_d, _ = mq.parareal_run(pdv, 1, 4, 4, 1, 4, 1e-6, xi, want_state=True)
    qp, itp, fsp = np.zeros(4), np.zeros(4, dtype=np.int32), np.zeros((4, ph.n_dof))
    pd = L.PararealDesc(1, 4, 4, 1, 4, 0, 1e-6)
    rcp = lib.parareal_run(ph.h, C.byref(pd), 4, P(xi), P(qp), P(itp), P(fsp), C.byref(st))
    assert rcp == rcp_d
    np.testing.assert_array_equal(qp, qp_d.cpu().numpy())
    np.testing.assert_array_equal(itp, it_d.cpu().numpy())
    np.testing.assert_array_equal(fsp, fsp_d.cpu().numpy())

    say("host handle: calls without a host form")
    with pytest.raises(L.MQError) as e:
        mq.debug_apply(ph, 0, 1e-3, xi[:1], np.zeros((1, ph.n_dof)))
    assert e.value.code == L.MQ_ERR_INVALID_ARG
    with pytest.raises(L.MQError) as e:
        mq.mlmc_combined_run(ph, [(8, 0, 1), (16, 8, 1)], xs)
    assert e.value.code == L.MQ_ERR_INVALID_ARG
    pdv.close()
    ph.close()


def test_lumped_mass_sine_mode_closed_form():
    """Lumped-mass option on the homogeneous square, no source: the sampled sine
    mode v = sin(p pi x) sin(q pi y) is an eigenvector, so implicit Euler (Eq. (7))
    gives a_n = (1 + lam dt)^-n v with lam = nu (4 - 2 cos(p pi h) - 2 cos(q pi h)) /
    (sigma h^2), and Eq. (26) the loss sigma h^2 |v|^2 sum_k (c_{k+1} - c_k)^2 / (dt T)."""
    import math
    mq, L = mqmod()
    for n, path in ((17, L.MQ_PATH_AUTO), (33, L.MQ_PATH_STREAMING)):
        hom = W.Problem(n, W.Material(kind=W.MAT_LOGNORMAL_SCALAR), conductor=(0.0, 1.0, 0.0, 1.0), J0=0.0)
        p = mq.Problem(hom, L.MQ_PREC_FP64, path=path, mass=L.MQ_MASS_LUMPED)
        h = 1.0 / (n - 1)
        x = np.arange(1, n - 1) * h
        sig, nu = hom.material.sigma0, hom.material.nu_cond
        spp, nper = 8, 2
        nst, dt = spp * nper, hom.period / spp
        for pq in ((1, 1), (2, 3), (n - 3, 1)):
            say(f"lumped mass n={n} path={path} mode={pq}")
            v = np.outer(np.sin(pq[1] * math.pi * x), np.sin(pq[0] * math.pi * x)).ravel()  # row j, column i
            lam = nu * (4 - 2 * math.cos(pq[0] * math.pi * h) - 2 * math.cos(pq[1] * math.pi * h)) / (sig * h * h)
            p.set_initial_state(v)
            qf, _, fs, rc, _ = mq.mlmc_level_run(p, spp, 0, nper, np.zeros((1, 2)), want_state=True)
            assert rc == 0
            c = (1.0 + lam * dt) ** -np.arange(nst + 1.0)
            a = fs[0].cpu().numpy()
            assert np.linalg.norm(a - c[-1] * v) <= 1e-10 * np.linalg.norm(c[-1] * v)
            qref = sig * h * h * float(v @ v) * np.sum(np.diff(c) ** 2) / dt / (nst * dt)
            assert float(qf[0]) == pytest.approx(qref, rel=1e-10)
        p.close()


def test_single_dof_mesh():
    mq, L = mqmod()
    prob = W.Problem(3, W.Material(kind=W.MAT_LOGNORMAL_SCALAR), conductor=(0, 1, 0, 1), strip=(0, 1))
    xi = np.array([[0.1, -0.3]])
    p = mq.Problem(prob, L.MQ_PREC_FP64)
    qf, _, fs, rc, _ = mq.mlmc_level_run(p, 16, 0, 1, xi, want_state=True)
    qref, aref = oracle_q(prob, xi, 16, 1)
    assert float(qf[0]) == pytest.approx(qref[0], rel=1e-12)
    p.close()


@pytest.mark.parametrize("n,prec,k2", [(33, 0, 5.0e2), (33, 1, 5.0e2), (65, 1, 2.17)])
def test_picard_nonlinear_matches_oracle(n, prec, k2):
    """Nonlinear reluctivity nu(|B|) solved per step by Picard iteration in the
    kernel; Q and the Picard iteration totals against the oracle."""
    from oracle import picard as opic
    mq, L = mqmod()
    prob = W.Problem(n, W.Material(kind=W.MAT_NONLINEAR, k2=k2))
    xi = W.normals(0, 31, 0, range(3), 3)
    say(f"picard n={n} prec={prec} k2={k2}")
    solver = dict(tol=1e-12, inner_rtol=1e-9) if prec == 0 else dict(tol=1e-10, inner_rtol=1e-5)
    p = mq.Problem(prob, prec, **solver)
    qf, _, _, rc, st = mq.mlmc_level_run(p, 16, 0, 1, xi)
    assert rc == 0
    m = omesh.build(n)
    ref_q, ref_its = [], 0
    for x in xi:
        Q, a, counts, flagged = opic.solve_sample(prob, x, 16, 1, m=m, return_counts=True)
        assert not flagged
        ref_q.append(Q)
        ref_its += int(counts.sum())
    err = np.max(np.abs(qf.cpu().numpy() - np.array(ref_q)) / np.abs(ref_q))
    say("picard iterations gpu", st["picard_iters"], "oracle", ref_its, "max rel err", err)
    assert err <= (1e-9 if prec == 0 else 1e-6)
    assert abs(st["picard_iters"] - ref_its) <= len(xi) * 16 // 4
    p.close()


def test_adaptive_mlmc_matches_oracle():
    """Adaptive MLMC (Eq. (11), run-time level variances): the sample counts
    the device run settles on equal the oracle driver's on the same input
    pools, and the estimate agrees to the FP64 tolerance."""
    mq, L = mqmod()
    prob = W.Problem(33, W.Material(kind=W.MAT_KL))
    levels = [(16, 0, 1), (32, 16, 1), (64, 32, 1)]
    n_max = [3000, 200, 200]
    pools = [W.normals(0, 40, l, range(n_max[l]), 8) for l in range(3)]
    eps, pilot = 20.0, 16
    p = mq.Problem(prob, L.MQ_PREC_FP64)
    e, y, v, n, qf, qc, rc, st = mq.mlmc_adaptive_run(p, levels, pools, eps, n_pilot=pilot)
    assert rc == 0
    say("device: E", e, "N", n, "V", v)
    m = omesh.build(33)
    tab = ots.kl_table_for(prob, m)

    def q_of(l, k0, k1):
        spp, cs, nper = levels[l]
        xs = pools[l][k0:k1]
        f = np.array([ots.solve_sample(prob, x, spp, nper, m=m, kl_table=tab)[0] for x in xs])
        c = np.array([ots.solve_sample(prob, x, cs, nper, m=m, kl_table=tab)[0] for x in xs]) if cs else None
        return f, c

    C = [nper * (spp + cs) for spp, cs, nper in levels]
    e_o, y_o, v_o, n_o, rounds = omlmc.adaptive(q_of, C, eps, pilot, n_max)
    say("oracle: E", e_o, "N", list(n_o), "rounds", rounds)
    assert list(n) == list(n_o)
    assert abs(e - e_o) <= 1e-10 * abs(e_o)
    assert np.allclose(v, v_o, rtol=1e-8)
    assert sum(vi / ni for vi, ni in zip(v, n)) <= 0.5 * eps * eps
    p.close()


def test_multimesh_mlmc_matches_oracle():
    """Spatial + temporal levels: level l on mesh l (17, 33, 65 nodes per side),
    its coupled coarse run on mesh l - 1 with the same input; every Q against
    the oracle on the matching mesh, and the estimator against the oracle's."""
    mq, L = mqmod()
    meshes = [17, 33, 65]
    levels = [(16, 0, 1), (32, 16, 1), (64, 32, 1)]
    ns = [5, 3, 2]
    probs = [W.Problem(n, W.Material(kind=W.MAT_KL)) for n in meshes]
    hs = [mq.Problem(pb, L.MQ_PREC_MIXED) for pb in probs]
    xis = [W.normals(0, 41, l, range(ns[l]), 8) for l in range(3)]
    qf, qc, rc, st = mq.mlmc_multimesh_run(hs, levels, xis)
    assert rc == 0
    rf, rcq = [], [None]
    for l in range(3):
        f, _ = oracle_q(probs[l], xis[l], levels[l][0], levels[l][2])
        rf.append(f)
        e = np.max(np.abs(qf[l].cpu().numpy() - f) / np.abs(f))
        say("level", l, "fine err", e)
        assert e <= 1e-6
        if l > 0:
            c, _ = oracle_q(probs[l - 1], xis[l], levels[l][1], levels[l][2])
            rcq.append(c)
            ec = np.max(np.abs(qc[l].cpu().numpy() - c) / np.abs(c))
            say("level", l, "coarse err", ec)
            assert ec <= 1e-6
    e_gpu, _, _ = mq.mlmc_estimate(qf, qc)
    e_ref, _, _ = omlmc.estimate(rf, rcq)
    assert abs(float(e_gpu) - e_ref) <= 1e-6 * abs(e_ref)
    for h in hs:
        h.close()


def test_combined_run_matches_oracle():
    """MLMC with Parareal on the finest level (17 x 17, FP64, 3 levels, M = 4,
    coarse propagator = level 0's time grid): levels 0-1 and level 2's coupled
    coarse values as the oracle's level runs, level 2's fine values and K as the
    oracle's Parareal, the executed Parareal work as the oracle's propagator
    counts; level 2's coupled coarse values equal mlmc_level_run's bit for bit."""
    mq, L = mqmod()
    prob = W.Problem(17, W.Material(kind=W.MAT_KL))
    levels = [(8, 0, 1), (16, 8, 1), (32, 16, 1)]
    ns = (5, 4, 3)
    xis = [W.normals(0, 25, l, range(n), 8) for l, n in enumerate(ns)]
    p = mq.Problem(prob, L.MQ_PREC_FP64)
    say("combined 17 fp64")
    qf, qc, it, rc, st, cs = mq.mlmc_combined_run(p, levels, xis, n_slices=4, tol=1e-6)
    say("combined stats", cs)
    assert rc == 0 and cs["n_slices"] == 4 and cs["coarse_steps_per_period"] == 8
    for l in range(3):
        spp, cspp, nper = levels[l]
        rf, rcq = omlmc.level_run(prob, spp, cspp, nper, xis[l])
        if l < 2:
            assert np.max(np.abs(qf[l].cpu().numpy() - rf) / np.abs(rf)) <= 1e-10
        if l > 0:
            assert np.max(np.abs(qc[l].cpu().numpy() - rcq) / np.abs(rcq)) <= 1e-10
    _, qc_lvl, _, _, _ = mq.mlmc_level_run(p, 32, 16, 1, xis[2])
    assert np.array_equal(qc[2].cpu().numpy(), qc_lvl.cpu().numpy())
    fine_ev = coarse_ev = 0
    all_k_match = True
    for s in range(ns[2]):
        ref = opara.run(prob, xis[2][s], 1, 4, 8, 2, k_max=4, tol=1e-6)
        k = int(it[s])
        say("sample", s, "K", k, "oracle K", ref["K"])
        assert abs(k - ref["K"]) <= 1
        if k == ref["K"]:
            assert float(qf[2][s]) == pytest.approx(ref["Q"], rel=1e-9)
            fine_ev += ref["fine_evals"]
            coarse_ev += ref["coarse_evals"]
        else:
            all_k_match = False
    if all_k_match:
        assert cs["para_fine_steps"] == 8 * fine_ev and cs["para_coarse_steps"] == 2 * coarse_ev
    # M from Eq. (25): the largest power of two <= max(2, n_c,para) dividing both step counts
    qf2, _, _, rc2, _, cs2 = mq.mlmc_combined_run(p, levels, xis, tol=1e-6)
    m = cs2["n_slices"]
    assert rc2 == 0 and m >= 2 and (m & (m - 1)) == 0 and 32 % m == 0 and 8 % m == 0
    assert m <= max(2, cs2["n_c_para"]) and (2 * m > max(2, cs2["n_c_para"]) or 8 % (2 * m) != 0)
    for l in range(2):
        assert np.array_equal(qf2[l].cpu().numpy(), qf[l].cpu().numpy())
    p.close()


def test_tail_split_is_bitwise():
    """Short instances run as chains of dependent pieces (split_steps) when that
    shortens the launch: on a level mix shaped like the three-level workload and
    sized to the device's slots, every Q equals the unsplit run's bit for bit,
    and a few against the oracle."""
    mq, L = mqmod()
    prob = W.Problem(17, W.Material(kind=W.MAT_KL))
    p0 = mq.Problem(prob, L.MQ_PREC_MIXED, path=L.MQ_PATH_RESIDENT, split_steps=-1)
    p1 = mq.Problem(prob, L.MQ_PREC_MIXED, path=L.MQ_PATH_RESIDENT, split_steps=16)
    probe = W.normals(0, 26, 0, range(4096), 8)
    _, _, _, rc, st = mq.mlmc_level_run(p0, 2, 0, 1, probe)
    G = st["grid"]
    ns = (2 * G, max(2, G // 2), max(2, G // 8))
    levels = [(16, 0, 4), (32, 16, 4), (64, 32, 4)]
    xis = [W.normals(0, 27, l, range(n), 8) for l, n in enumerate(ns)]
    say("tail split: slots", G, "samples", ns)
    qf0, qc0, rc0, st0 = mq.mlmc_multilevel_run(p0, levels, xis)
    qf1, qc1, rc1, st1 = mq.mlmc_multilevel_run(p1, levels, xis)
    say("unsplit", st0["kernel_ms"], "ms; split", st1["kernel_ms"], "ms, entries", st1["n_pieces"])
    assert rc0 == 0 and rc1 == 0
    assert st0["n_pieces"] == 0 and st1["n_pieces"] > st1["n_instances"]
    assert st1["n_instances"] == st0["n_instances"] and st1["sample_steps"] == st0["sample_steps"]
    assert st1["inner_iters"] == st0["inner_iters"] and st1["n_failed"] == 0
    for l in range(3):
        assert np.array_equal(qf0[l].cpu().numpy(), qf1[l].cpu().numpy()), l
        if l > 0:
            assert np.array_equal(qc0[l].cpu().numpy(), qc1[l].cpu().numpy()), l
    rf, _ = oracle_q(prob, xis[0][:3], 16, 4)
    assert np.max(np.abs(qf1[0][:3].cpu().numpy() - rf) / np.abs(rf)) <= 1e-6
    p0.close()
    p1.close()

