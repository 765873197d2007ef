"""The library's cost model (mq_cost_model, host arithmetic) against the
oracle's, which the paper's worked example and Table II pin
(tests/test_oracle_parareal_mlmc.py).  No GPU needed."""
import json
import os

import pytest

from oracle import costmodel as cm

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def mq():
    import torch  # noqa: F401  (load the HIP runtime that torch ships first)
    from paper_2507_19246_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmq.so not built")
    import paper_2507_19246_amd as mq
    return mq


CASES = [
    # C_l, N_l, K, M, n_cores
    (cm.exp_cost(1.0, 10.0, 2), [1000, 100, 10], 2, 16, 256),
    (cm.exp_cost(1.0, 2.0, 2), [512, 128, 32], 3, 4, 256),
    (cm.exp_cost(3.0, 4.0, 3), [900, 200, 40, 6], 5, 32, 1024),
    ([256.0, 512.0, 1024.0], [512, 128, 32], 4, 4, 256),
    ([0.7, 5.0, 41.0, 300.0, 2000.0], [4000, 700, 90, 12, 2], 7, 64, 512),
]


@pytest.mark.parametrize("C,N,K,M,nc", CASES)
def test_cost_model_matches_oracle(mq, C, N, K, M, nc):
    out = mq.cost_model(C, N, K, M, nc)
    L = len(C) - 1
    tp, ep = cm.tau_para(K, M, C[L], C[L - 2]), cm.effort_para(K, M, C[L], C[L - 2])
    assert out["tau_para"] == pytest.approx(tp, rel=1e-14)
    assert out["effort_para"] == pytest.approx(ep, rel=1e-14)
    tr, er = cm.ref_cost(C, N)
    tc, ec = cm.comb_cost(C, N, tp, ep)
    assert out["tau_ref"] == pytest.approx(tr, rel=1e-14) and out["effort_ref"] == pytest.approx(er, rel=1e-14)
    assert out["tau_comb"] == pytest.approx(tc, rel=1e-14) and out["effort_comb"] == pytest.approx(ec, rel=1e-14)
    assert out["speedup"] == pytest.approx(tr / tc, rel=1e-14)
    assert out["s_inf"] == pytest.approx(cm.s_inf_ratio(C), rel=1e-14)
    assert out["eps_inf"] == pytest.approx(cm.effort_ratio(C, N, K, M), rel=1e-13)
    r = C[L] / C[L - 1]
    assert out["kappa"] == cm.kappa(r, M)
    assert out["batches"] == cm.batches(C, N, nc)
    assert out["n_c_para"] == cm.cores_per_parareal_sample(C, N, nc)
    if C[0] == 1.0 and out["n_c_para"] >= 1:
        # the printed finite-core form (r^L, r^{L-2}) holds for C_l = r^l
        assert out["s_nc"] == pytest.approx(cm.speedup_finite(C, N, nc, K, r), rel=1e-13)


def test_cost_model_paper_numbers(mq):
    """The worked example of Eq. (21) (r = 10, L = 2) and Table II's derived counts."""
    g = json.load(open(os.path.join(GOLD, "paper_costmodel.json")))
    num, den = g["s_inf_exact_fraction"]
    out = mq.cost_model(cm.exp_cost(1.0, g["r"], g["L"]), [1, 1, 1], 1, 4, 1)
    assert out["s_inf"] == pytest.approx(num / den, rel=1e-14)
    t2 = json.load(open(os.path.join(GOLD, "paper_table2.json")))
    C = [lv["runtime_s"] for lv in t2["levels"]]
    N = [lv["n_samples"] for lv in t2["levels"]]
    out = mq.cost_model(C, N, 1, 16, t2["n_cores"])
    assert out["n_c_para"] == t2["printed"]["cores_per_parareal_sample"]
    assert out["batches"] == [58, 1, 1]


@pytest.mark.parametrize("n,kappa", [(1, 0), (2, 0), (4, 0), (8, 0), (16, 1), (32, 2), (64, 3), (1000, 9)])
def test_cost_model_kappa_r10(mq, n, kappa):
    assert mq.cost_model(cm.exp_cost(1.0, 10.0, 2), [1, 1, 1], 1, n, 1)["kappa"] == kappa


def test_cost_model_rejects_bad_input(mq):
    from paper_2507_19246_amd import _lib
    with pytest.raises(_lib.MQError):
        mq.cost_model([1.0, 2.0], [1, 1], 1, 2, 1)       # needs level L-2
    with pytest.raises(_lib.MQError):
        mq.cost_model([1.0, 2.0, 4.0], [1, 1, 1], 5, 4, 1)  # K > M
    with pytest.raises(_lib.MQError):
        mq.cost_model([1.0, 0.0, 4.0], [1, 1, 1], 1, 4, 1)
