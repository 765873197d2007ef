"""Continuous-batching server (mq_server_*) through the C ABI.

Each request's Q must be bitwise identical whether it runs alone or inside a
mix of other meshes and time grids, must equal mlmc_level_run of the same
input at level 0 bitwise (launch splitting resumes exactly), and must match
the FP64 oracle within the mixed-precision QoI tolerance (1e-6 relative).
Requests use the serving mix generator (Poisson arrivals, mixed meshes and
steps per period) at reduced mesh sizes.
"""
import sys
import time

import numpy as np
import pytest

import workloads as W
from oracle import mesh as omesh, timestep as ots

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BUDGET = 8 << 30


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


def kl_problem(n):
    return W.Problem(n, W.Material(kind=W.MAT_KL))


def drain(srv, n_expected, timeout_s=90.0):
    """Poll until n_expected results arrived (bounded wait)."""
    out = {}
    t0 = time.monotonic()
    while len(out) < n_expected:
        for r in srv.poll(256):
            out[r.ticket] = r
        if time.monotonic() - t0 > timeout_s:
            raise AssertionError(f"server produced {len(out)} of {n_expected} results in {timeout_s} s")
        time.sleep(0.002)
    assert srv.pending() == 0
    return out


def level_q(mq, L, n, spp, nper, xis):
    p = mq.Problem(kl_problem(n), L.MQ_PREC_MIXED)
    qf, _, _, rc, _ = mq.mlmc_level_run(p, spp, 0, nper, np.asarray(xis))
    assert rc == 0
    q = qf.cpu().numpy()
    p.close()
    return q


def test_server_alone_equals_mix_and_level_run():
    mq, L = mqmod()
    reqs = W.serving_stream(12, rate_hz=400.0, meshes=(33, 65), weights=(0.5, 0.5), steps=(8, 20, 32))
    probe = reqs[7]
    say("serving probe", probe.n_nodes, probe.steps_per_period)
    # alone; chunk 16 splits 2 x 20 steps into 16 + 16 + 8
    srv = mq.Server(kl_problem(probe.n_nodes), L.MQ_PREC_MIXED, BUDGET, chunk_steps=16)
    t = srv.submit(probe.n_nodes, probe.steps_per_period, probe.n_periods, probe.xi, user_id=99)
    res = drain(srv, 1)
    srv.close()
    alone = res[t]
    assert alone.status == 0 and alone.user_id == 99
    assert alone.t_submit_ns <= alone.t_start_ns <= alone.t_done_ns
    # in a mix: arrivals paced by the generator while earlier requests run
    srv = mq.Server(kl_problem(33), L.MQ_PREC_MIXED, BUDGET, chunk_steps=16)
    t0 = time.monotonic()
    tickets = []
    for r in reqs:
        while time.monotonic() - t0 < r.arrival_s:
            time.sleep(0.0005)
        tickets.append(srv.submit(r.n_nodes, r.steps_per_period, r.n_periods, r.xi, user_id=r.rid))
    res = drain(srv, len(reqs))
    srv.close()
    mixed = res[tickets[7]]
    say("alone", alone.q, "mix", mixed.q)
    assert mixed.q == alone.q
    assert mixed.inner_iters == alone.inner_iters
    # every request equals mlmc_level_run of its input at level 0, bit for bit
    groups = {}
    for i, r in enumerate(reqs):
        groups.setdefault((r.n_nodes, r.steps_per_period), []).append(i)
    for (n, spp), idx in groups.items():
        q = level_q(mq, L, n, spp, reqs[0].n_periods, [reqs[i].xi for i in idx])
        for k, i in enumerate(idx):
            got = res[tickets[i]]
            assert got.status == 0
            assert got.q == q[k], (n, spp, i, got.q, q[k])
    # and the probe against the FP64 oracle
    prob = kl_problem(probe.n_nodes)
    m = omesh.build(probe.n_nodes)
    ref = ots.solve_sample(prob, np.array(probe.xi), probe.steps_per_period, probe.n_periods, m=m,
                           kl_table=ots.kl_table_for(prob, m))[0]
    err = abs(alone.q - ref) / abs(ref)
    say("serving probe vs oracle", err)
    assert err <= 1e-6


def test_server_budget_and_validation():
    mq, L = mqmod()
    xi = tuple(W.normals(0, 4, 0, [0], 8)[0])
    # a budget below one mesh class's memory: the request completes with MQ_ERR_BUSY
    srv = mq.Server(kl_problem(33), L.MQ_PREC_MIXED, 1 << 16)
    t = srv.submit(33, 8, 1, xi)
    res = drain(srv, 1)
    assert res[t].status == L.MQ_ERR_BUSY
    # invalid requests are refused at submission
    with pytest.raises(L.MQError):
        srv.submit(2, 8, 1, xi)
    with pytest.raises(L.MQError):
        srv.submit(33, 8, 1, xi[:3])
    with pytest.raises(L.MQError):
        srv.submit(33, 8, 1, (float("nan"),) + xi[1:])
    srv.close()


def test_server_max_inflight_one_serialises():
    """max_inflight = 1: requests run one at a time and still give the
    mixed-run results."""
    mq, L = mqmod()
    reqs = W.serving_stream(4, meshes=(17, 33), weights=(0.5, 0.5), steps=(8, 12))
    srv = mq.Server(kl_problem(17), L.MQ_PREC_MIXED, BUDGET, max_inflight=1, chunk_steps=5)
    tickets = [srv.submit(r.n_nodes, r.steps_per_period, r.n_periods, r.xi) for r in reqs]
    res = drain(srv, len(reqs))
    srv.close()
    spans = sorted((res[t].t_start_ns, res[t].t_done_ns) for t in tickets)
    for a, b in zip(spans, spans[1:]):
        assert a[1] <= b[0]
    for r, t in zip(reqs, tickets):
        q = level_q(mq, L, r.n_nodes, r.steps_per_period, r.n_periods, [r.xi])
        assert res[t].status == 0 and res[t].q == q[0]


def test_server_wide_lane():
    """Large requests on the wide lane: with wide_min_nodes = 65 and a queue
    of one, a burst of 65 x 65 requests runs partly on the wide lane and the
    rest batched; every result equals mlmc_level_run of its input on the path
    that ran it, bit for bit, and the oracle within 1e-6.  33 x 33 requests in
    the same burst are batched as usual."""
    mq, L = mqmod()
    reqs = W.serving_stream(10, rate_hz=1e6, meshes=(33, 65), weights=(0.3, 0.7), steps=(16, 24))
    srv = mq.Server(kl_problem(33), L.MQ_PREC_MIXED, BUDGET, chunk_steps=16, wide_min_nodes=65, wide_queue=1)
    tickets = [srv.submit(r.n_nodes, r.steps_per_period, r.n_periods, r.xi, user_id=r.rid) for r in reqs]
    res = drain(srv, len(reqs))
    srv.close()
    for i, r in enumerate(reqs):
        got = res[tickets[i]]
        say("request", i, r.n_nodes, r.steps_per_period, "status", got.status, got.message.decode(errors="replace"))
    n_wide = 0
    for i, r in enumerate(reqs):
        got = res[tickets[i]]
        assert got.status == 0 and got.user_id == r.rid
        qb = level_q(mq, L, r.n_nodes, r.steps_per_period, r.n_periods, [r.xi])[0]
        if r.n_nodes == 65:
            pw = mq.Problem(kl_problem(65), L.MQ_PREC_MIXED, path=L.MQ_PATH_WIDE)
            qw = float(mq.mlmc_level_run(pw, r.steps_per_period, 0, r.n_periods, np.asarray([r.xi]))[0][0])
            pw.close()
            assert got.q in (qw, qb), (i, got.q, qw, qb)
            n_wide += got.q == qw and qw != qb
        else:
            assert got.q == qb
        prob = kl_problem(r.n_nodes)
        m = omesh.build(r.n_nodes)
        ref = ots.solve_sample(prob, np.array(r.xi), r.steps_per_period, r.n_periods, m=m,
                               kl_table=ots.kl_table_for(prob, m))[0]
        assert abs(got.q - ref) / abs(ref) <= 1e-6
    say("65 x 65 requests on the wide lane:", n_wide, "of", sum(r.n_nodes == 65 for r in reqs))
    assert n_wide >= 1
