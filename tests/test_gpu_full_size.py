"""Parity at the benchmark workloads' full sizes, on sampled outputs.

The expected values come from `tests/golden/full_size_oracle.json`, written by
`tests/golden/make_full_size.py` (FP64 oracle only).  The GPU side runs each
workload in the configuration its bench line uses (tuned knobs, same kernels
and launch shapes); the mixed-precision tolerance on Q is 1e-6 relative.
"""
import json
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size_oracle.json")
TOL = 1e-6


@pytest.fixture(scope="module")
def golden():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with open(GOLDEN) as f:
        return json.load(f)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return abs(a - b) / abs(b)


def test_full_size_mlmc3_129(golden):
    """All levels of the 129x129 MLMC workload in one launch; sampled Q (fine
    and coupled coarse) against the oracle."""
    import paper_2507_19246_amd as mq
    from paper_2507_19246_amd import _lib as L, autotune
    w = W.mlmc3_mixed_129()
    levels = [(lv.steps_per_period, lv.coarse_steps_per_period, lv.n_periods) for lv in w.levels]
    xis = [W.level_xi(w, l) for l in range(len(w.levels))]
    prob, knobs = autotune.tuned_problem(w.problem, L.MQ_PREC_MIXED)
    say("full-size C1", knobs)
    qf, qc, rc, st = mq.mlmc_multilevel_run(prob, levels, xis)
    assert rc == 0
    for g in golden["mlmc3_129"]:
        l, s = g["level"], g["sample"]
        e = rel(float(qf[l][s]), g["q_fine"])
        say("level", l, "sample", s, "fine err", e)
        assert e <= TOL
        if g["q_coarse"] is not None:
            assert rel(float(qc[l][s]), g["q_coarse"]) <= TOL
    prob.close()


def test_full_size_parareal_257(golden):
    """Parareal on the 257x257 workload (32 slices, 1 coarse step per slice,
    k_max 8, tol 1e-8) for one sample: Q and K against the oracle's Parareal,
    and the serial fine run against the oracle's."""
    import paper_2507_19246_amd as mq
    from paper_2507_19246_amd import _lib as L, autotune
    w = W.parareal_257()
    pr = w.parareal
    g = golden["parareal_257"][0]
    xi = W.level_xi(w, 0, first=g["sample"], n=1)
    prob, knobs = autotune.tuned_problem(w.problem, L.MQ_PREC_MIXED)
    say("full-size C2", knobs, "oracle K", g["k"])
    q, it, _, rc, st = mq.parareal_run(prob, pr.n_periods, pr.n_slices, pr.fine_steps_per_slice,
                                       pr.coarse_steps_per_slice, pr.k_max, pr.tol, xi)
    k = int(it[0])
    e = rel(float(q[0]), g["q_parareal"])
    say("parareal K", k, "err vs oracle parareal", e)
    assert abs(k - g["k"]) <= 1
    assert e <= TOL
    spp = pr.n_slices * pr.fine_steps_per_slice // pr.n_periods
    qs, _, _, rc2, _ = mq.mlmc_level_run(prob, spp, 0, pr.n_periods, xi)
    assert rc2 == 0
    assert rel(float(qs[0]), g["q_serial"]) <= TOL
    prob.close()


def test_full_size_nonlinear_129(golden):
    """Level 0 of the nonlinear MLMC workload (Picard per step), sampled Q."""
    import paper_2507_19246_amd as mq
    from paper_2507_19246_amd import _lib as L, autotune
    w = W.nonlinear_mlmc4_129()
    lv = w.levels[0]
    xi = W.level_xi(w, 0, n=2)
    prob, knobs = autotune.tuned_problem(w.problem, L.MQ_PREC_MIXED)
    q, _, _, rc, st = mq.mlmc_level_run(prob, lv.steps_per_period, 0, lv.n_periods, xi)
    assert rc == 0
    for g in golden["nonlinear_129"]:
        assert not g["flagged"]
        e = rel(float(q[g["sample"]]), g["q"])
        say("nonlinear sample", g["sample"], "err", e)
        assert e <= TOL
    ref_its = sum(g["picard_iters"] for g in golden["nonlinear_129"])
    assert abs(st["picard_iters"] - ref_its) <= lv.steps_per_period * lv.n_periods // 2
    prob.close()


def test_full_size_nonlinear_129_finest_level(golden):
    """The finest level of the nonlinear MLMC workload (512 fine and 256 coupled
    coarse Picard steps): Q of both runs of its first sample against the oracle."""
    import paper_2507_19246_amd as mq
    from paper_2507_19246_amd import _lib as L, autotune
    w = W.nonlinear_mlmc4_129()
    level = len(w.levels) - 1
    lv = w.levels[level]
    xi = W.level_xi(w, level, n=1)
    prob, knobs = autotune.tuned_problem(w.problem, L.MQ_PREC_MIXED)
    qf, qc, _, rc, st = mq.mlmc_level_run(prob, lv.steps_per_period, lv.coarse_steps_per_period, lv.n_periods, xi)
    assert rc == 0
    g = golden["nonlinear_129_top"][0]
    assert g["level"] == level and g["sample"] == 0 and not g["flagged"]
    ef, ec = rel(float(qf[0]), g["q_fine"]), rel(float(qc[0]), g["q_coarse"])
    say("nonlinear finest level: err fine", ef, "coarse", ec, "picard", st["picard_iters"])
    assert ef <= TOL and ec <= TOL
    ref_its = g["picard_iters_fine"] + g["picard_iters_coarse"]
    assert abs(st["picard_iters"] - ref_its) <= (lv.steps_per_period + lv.coarse_steps_per_period) * lv.n_periods // 2
    prob.close()


def test_full_size_serving_513(golden):
    """A 513x513 request of the serving stream through the server."""
    import time
    import paper_2507_19246_amd as mq
    from paper_2507_19246_amd import _lib as L
    g = golden["serving"][0]
    r = W.serving_stream(4096)[g["index"]]
    assert r.n_nodes == g["n_nodes"] == 513
    srv = mq.Server(W.Problem(65, W.Material(kind=W.MAT_KL)), L.MQ_PREC_MIXED, 32 << 30)
    t = srv.submit(r.n_nodes, r.steps_per_period, r.n_periods, r.xi)
    res, t0 = None, time.monotonic()
    while res is None:
        out = srv.poll(4)
        if out:
            res = out[0]
        assert time.monotonic() - t0 < 100, "513x513 request did not finish in 100 s"
        time.sleep(0.01)
    srv.close()
    assert res.ticket == t and res.status == 0
    e = rel(res.q, g["q"])
    say("513x513 request", r.steps_per_period, "steps/period: err", e,
        "latency ms", (res.t_done_ns - res.t_submit_ns) / 1e6)
    assert e <= TOL


def test_full_size_513_streaming_batch(golden):
    """The stored 513x513 request run four times in one batched launch of the
    streaming kernel (the coarse levels from level 3 on in LDS): every copy
    equal, and equal to the oracle's value."""
    import paper_2507_19246_amd as mq
    from paper_2507_19246_amd import _lib as L, autotune
    g = golden["serving"][0]
    r = W.serving_stream(4096)[g["index"]]
    prob = W.Problem(513, W.Material(kind=W.MAT_KL))
    p, knobs = autotune.tuned_problem(prob, L.MQ_PREC_MIXED, path=L.MQ_PATH_STREAMING)
    assert p.path == L.MQ_PATH_STREAMING
    xi = np.repeat(np.asarray(r.xi, dtype=np.float64)[None, :], 4, axis=0)
    q, _, _, rc, st = mq.mlmc_level_run(p, r.steps_per_period, 0, r.n_periods, xi)
    assert rc == 0 and st["path"] == L.MQ_PATH_STREAMING and st["n_instances"] == 4
    qs = q.cpu().numpy()
    e = rel(float(qs[0]), g["q"])
    say("513x513 streaming batch: err", e, "iters/step", st["inner_iters"] / st["sample_steps"])
    assert np.all(qs == qs[0])
    assert e <= TOL
    p.close()


def test_tuned_knobs_are_found():
    """The committed autotuner cache has this device's entries for the bench
    workloads, so every bench line runs its tuned configuration."""
    import paper_2507_19246_amd  # noqa: F401
    from paper_2507_19246_amd import _lib as L, autotune
    say("device id", autotune.device_id())
    for w in (W.mlmc3_mixed_129(), W.parareal_257(), W.nonlinear_mlmc4_129()):
        assert autotune.lookup(w.problem, L.MQ_PREC_MIXED) is not None, w.name
