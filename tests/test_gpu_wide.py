"""The wide path (one instance at a time over the whole device, inner
iterations replayed from a captured graph) against the FP64 oracle.

Same bar as the other paths: FP64 1e-10 relative on Q and on the final
state, mixed precision 1e-6 relative on Q.  The full-size cases use the
stored oracle values of `tests/golden/full_size_oracle.json`.
"""
import json
import os
import sys
import time

import numpy as np
import pytest

import workloads as W
from oracle import mesh as omesh, timestep as ots

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size_oracle.json")


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


def oracle_q(problem, xi, spp, nper):
    m = omesh.build(problem.n_nodes)
    tab = ots.kl_table_for(problem, m)
    out = [ots.solve_sample(problem, x, spp, nper, m=m, kl_table=tab) for x in xi]
    return np.array([o[0] for o in out]), np.stack([o[1] for o in out])


@pytest.mark.parametrize("n,ns", [(33, 4), (65, 4), (129, 2)])
def test_wide_mixed_coupled_level(n, ns):
    """Mixed precision, KL field, coupled fine/coarse instances."""
    import paper_2507_19246_amd as mq
    from paper_2507_19246_amd import _lib as L
    prob = W.Problem(n, W.Material(kind=W.MAT_KL))
    xi = W.normals(0, 31, 1, range(ns), 8)
    say(f"wide mixed n={n} samples={ns}")
    p = mq.Problem(prob, L.MQ_PREC_MIXED, path=L.MQ_PATH_WIDE)
    assert p.path == L.MQ_PATH_WIDE and p.info.precond == L.MQ_PRECOND_MULTIGRID
    qf, qc, _, rc, st = mq.mlmc_level_run(p, 32, 16, 2, xi)
    assert rc == 0
    say("stats", st)
    assert st["path"] == L.MQ_PATH_WIDE and st["n_instances"] == 2 * ns
    rf, _ = oracle_q(prob, xi, 32, 2)
    rcq, _ = oracle_q(prob, xi, 16, 2)
    ef = np.abs(qf.cpu().numpy() - rf) / np.abs(rf)
    ec = np.abs(qc.cpu().numpy() - rcq) / np.abs(rcq)
    say("max rel err fine/coarse", ef.max(), ec.max())
    assert ef.max() <= 1e-6 and ec.max() <= 1e-6
    p.close()


def test_wide_fp64_state_matches_oracle():
    """FP64 on the wide path: Q and the final state within 1e-10."""
    import paper_2507_19246_amd as mq
    from paper_2507_19246_amd import _lib as L
    w = W.plain_fp64_33()
    xi = W.level_xi(w, 0, 3)
    say("wide fp64 33")
    p = mq.Problem(w.problem, L.MQ_PREC_FP64, path=L.MQ_PATH_WIDE)
    qf, _, a, rc, st = mq.mlmc_level_run(p, 64, 0, 1, xi, want_state=True)
    assert rc == 0
    qref, aref = oracle_q(w.problem, xi, 64, 1)
    eq = np.max(np.abs(qf.cpu().numpy() - qref) / qref)
    ea = np.max(np.abs(a.cpu().numpy() - aref)) / np.max(np.abs(aref))
    say("err q", eq, "err a", ea)
    assert eq <= 1e-10 and ea <= 1e-10
    p.close()


def test_wide_equals_streaming_257():
    """257 x 257: the wide and streaming paths agree, and the serial fine
    run of the Parareal workload's stored sample matches the oracle."""
    import paper_2507_19246_amd as mq
    from paper_2507_19246_amd import _lib as L
    with open(GOLDEN) as f:
        g = json.load(f)["parareal_257"][0]
    w = W.parareal_257()
    pr = w.parareal
    xi = W.level_xi(w, 0, first=g["sample"], n=1)
    spp = pr.n_slices * pr.fine_steps_per_slice // pr.n_periods
    say("wide 257 spp", spp, "periods", pr.n_periods)
    pw = mq.Problem(w.problem, L.MQ_PREC_MIXED, path=L.MQ_PATH_WIDE)
    t0 = time.perf_counter()
    qw, _, _, rc, st = mq.mlmc_level_run(pw, spp, 0, pr.n_periods, xi)
    tw = time.perf_counter() - t0
    assert rc == 0
    pw.close()
    ps = mq.Problem(w.problem, L.MQ_PREC_MIXED, path=L.MQ_PATH_STREAMING)
    t0 = time.perf_counter()
    qs, _, _, rc2, _ = mq.mlmc_level_run(ps, spp, 0, pr.n_periods, xi)
    ts = time.perf_counter() - t0
    assert rc2 == 0
    ps.close()
    ew = abs(float(qw[0]) - g["q_serial"]) / g["q_serial"]
    es = abs(float(qs[0]) - g["q_serial"]) / g["q_serial"]
    say(f"wide {tw:.3f} s err {ew:.2e}; streaming {ts:.3f} s err {es:.2e}; iters/step",
        st["inner_iters"] / st["sample_steps"])
    assert ew <= 1e-6 and es <= 1e-6


def test_wide_513_request():
    """The stored 513 x 513 request of the serving stream, run on the wide
    path: Q against the oracle's value."""
    import paper_2507_19246_amd as mq
    from paper_2507_19246_amd import _lib as L
    with open(GOLDEN) as f:
        g = json.load(f)["serving"][0]
    r = W.serving_stream(4096)[g["index"]]
    assert r.n_nodes == 513
    prob = W.Problem(513, W.Material(kind=W.MAT_KL))
    say("wide 513", r.steps_per_period, r.n_periods)
    p = mq.Problem(prob, L.MQ_PREC_MIXED, path=L.MQ_PATH_WIDE)
    t0 = time.perf_counter()
    q, _, _, rc, st = mq.mlmc_level_run(p, r.steps_per_period, 0, r.n_periods, np.asarray(r.xi)[None, :])
    dt = time.perf_counter() - t0
    assert rc == 0
    e = abs(float(q[0]) - g["q"]) / g["q"]
    say(f"wide 513: {dt:.3f} s, err {e:.2e}, iters/step {st['inner_iters'] / st['sample_steps']:.1f}")
    assert e <= 1e-6
    p.close()


def test_wide_rejects_what_it_does_not_run():
    import paper_2507_19246_amd as mq
    from paper_2507_19246_amd import _lib as L
    prob = W.Problem(33, W.Material(kind=W.MAT_KL))
    p = mq.Problem(prob, L.MQ_PREC_MIXED, path=L.MQ_PATH_WIDE)
    xi = W.normals(0, 32, 0, range(2), 8)
    with pytest.raises(Exception):
        mq.parareal_run(p, 1, 4, 8, 1, 4, 1e-8, xi)
    p.close()
    with pytest.raises(Exception):
        mq.Problem(W.Problem(33, W.Material(kind=W.MAT_NONLINEAR)), L.MQ_PREC_MIXED, path=L.MQ_PATH_WIDE)
    with pytest.raises(Exception):
        mq.Problem(W.Problem(34, W.Material(kind=W.MAT_KL)), L.MQ_PREC_MIXED, path=L.MQ_PATH_WIDE,
                   precond=L.MQ_PRECOND_MULTIGRID)


@pytest.mark.parametrize("n,pc", [(33, 1), (34, 0)])
def test_wide_jacobi_fp64_matches_oracle(n, pc):
    """The wide path with Jacobi-preconditioned CG (the plain one-sample-per-launch
    FP64 form; chosen automatically where the mesh has no multigrid hierarchy):
    Q and the final state within 1e-10 of the oracle."""
    import paper_2507_19246_amd as mq
    from paper_2507_19246_amd import _lib as L
    prob = W.Problem(n, W.Material(kind=W.MAT_KL))
    xi = W.normals(0, 36, 0, range(2), 8)
    say(f"wide jacobi fp64 n={n}")
    p = mq.Problem(prob, L.MQ_PREC_FP64, path=L.MQ_PATH_WIDE, precond=pc)
    assert p.path == L.MQ_PATH_WIDE and p.info.precond == L.MQ_PRECOND_JACOBI
    qf, qc, a, rc, st = mq.mlmc_level_run(p, 16, 8, 1, xi, want_state=True)
    assert rc == 0 and st["path"] == L.MQ_PATH_WIDE and st["n_instances"] == 4
    qref, aref = oracle_q(prob, xi, 16, 1)
    qcref, _ = oracle_q(prob, xi, 8, 1)
    eq = max(np.max(np.abs(qf.cpu().numpy() - qref) / qref), np.max(np.abs(qc.cpu().numpy() - qcref) / qcref))
    ea = np.linalg.norm(a.cpu().numpy() - aref) / np.linalg.norm(aref)
    say("err q", eq, "err a", ea, "iters/step", st["inner_iters"] / st["sample_steps"])
    assert eq <= 1e-10 and ea <= 1e-10
    assert np.all(mq.last_flags() == 0)
    p.close()
