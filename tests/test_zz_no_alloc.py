"""The allocation-free level run (mlmc_level_run_noalloc) through the C ABI
against mlmc_level_run on the same inputs: bitwise equal Q (fine and coupled
coarse), final states and per-instance flags, on two calls in a row with the
second smaller (fewer samples, then a smaller mesh on another handle, so the
shared workspace holds the larger call's leftovers); a run beyond the fixed
workspace is refused before any launch and leaves the handle usable."""
import ctypes as C
import sys

import numpy as np
import pytest

import workloads as W

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


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def noalloc_run(p, spp, cspp, nper, xi, want_state=True):
    from paper_2507_19246_amd import _lib as L
    n = xi.shape[0]
    xd = torch.tensor(xi, dtype=torch.float64, device="cuda")
    qf = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    qc = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda") if cspp else None
    fs = torch.full((n, p.n_dof), float("nan"), dtype=torch.float64, device="cuda") if want_state else None
    lv = L.LevelDesc(spp, cspp, nper, 0)
    st = L.RunStats()
    torch.cuda.synchronize()
    rc = p.lib.mlmc_level_run_noalloc(p.h, C.byref(lv), n, _ptr(xd), _ptr(qf), _ptr(qc), _ptr(fs), C.byref(st))
    return rc, qf, qc, fs, st


def check_equal(p, spp, cspp, nper, xi):
    import paper_2507_19246_amd as mq
    rc, qf, qc, fs, st = noalloc_run(p, spp, cspp, nper, xi)
    assert rc == 0, p.lib.mq_last_error()
    flags = mq.last_flags()
    rf, rcq, rfs, rrc, rst = mq.mlmc_level_run(p, spp, cspp, nper, xi, want_state=True)
    assert rrc == 0
    assert np.array_equal(qf.cpu().numpy(), rf.cpu().numpy())
    if cspp:
        assert np.array_equal(qc.cpu().numpy(), rcq.cpu().numpy())
    assert np.array_equal(fs.cpu().numpy(), rfs.cpu().numpy())
    assert np.array_equal(flags, mq.last_flags())
    assert st.sample_steps == rst["sample_steps"] and st.n_instances == rst["n_instances"]
    say(f"  noalloc grid {st.grid} vs {rst['grid']}, {st.kernel_ms:.1f} ms vs {rst['kernel_ms']:.1f} ms")


def test_noalloc_level_run_equals_level_run():
    import paper_2507_19246_amd as mq
    from paper_2507_19246_amd import _lib as L
    big = W.Problem(65, W.Material(kind=W.MAT_KL))
    p1 = mq.Problem(big, L.MQ_PREC_MIXED)
    say("noalloc: 65x65 mixed, 24 samples, coupled level")
    check_equal(p1, 32, 16, 1, W.normals(0, 51, 0, range(24), 8))
    say("noalloc: 65x65 mixed, 7 samples (second call, smaller)")
    check_equal(p1, 16, 8, 1, W.normals(0, 52, 0, range(7), 8))
    small = W.Problem(33, W.Material(kind=W.MAT_LOGNORMAL_SCALAR))
    p2 = mq.Problem(small, L.MQ_PREC_FP64)
    say("noalloc: 33x33 FP64, 5 samples, level 0 (other handle, smaller mesh)")
    check_equal(p2, 16, 0, 1, W.normals(0, 53, 0, range(5), 2))
    # beyond the fixed workspace: refused before any launch, handle still usable
    say("noalloc: oversized run refused")
    n_big = 200000
    xi = torch.zeros((1, 8), dtype=torch.float64, device="cuda")
    q = torch.zeros(1, dtype=torch.float64, device="cuda")
    lv = L.LevelDesc(16, 0, 1, 0)
    rc = p1.lib.mlmc_level_run_noalloc(p1.h, C.byref(lv), n_big, _ptr(xi), _ptr(q), None, None, None)
    assert rc == L.MQ_ERR_INVALID_ARG
    assert b"workspace" in p1.lib.mq_last_error()
    check_equal(p1, 16, 0, 1, W.normals(0, 54, 0, range(3), 8))
    p1.close()
    p2.close()
