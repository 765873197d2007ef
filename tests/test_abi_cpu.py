"""Host-side checks of the C ABI: the library loads, exports every function
that include/mq.h declares, its ctypes structs match the C layout, and calls
without a GPU fail cleanly with the documented status codes."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "mq.h")


def header_functions():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (load the HIP runtime that torch ships first)
    from paper_2507_19246_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmq.so not built")
    return _lib.load()


def test_header_declares_the_boundary():
    fns = header_functions()
    for name in ["fem_setup", "mlmc_level_run", "parareal_run", "mlmc_estimate", "mlmc_adaptive_run", "mq_debug_apply",
                 "mlmc_combined_run", "mq_cost_model", "mq_set_initial_state",
                 "mq_server_create", "mq_submit", "mq_poll", "mq_server_destroy", "mq_last_error"]:
        assert name in fns


def test_every_declared_symbol_is_exported(lib):
    from paper_2507_19246_amd import _lib
    fns = header_functions()
    for name in fns:
        assert hasattr(lib, name), name
    assert set(fns) == set(_lib.SIGNATURES), set(fns) ^ set(_lib.SIGNATURES)


def test_struct_layout_matches_c(tmp_path):
    from paper_2507_19246_amd import _lib
    structs = {"mq_problem_desc": _lib.ProblemDesc, "mq_problem_info": _lib.ProblemInfo,
               "mq_run_stats": _lib.RunStats, "mq_level_desc": _lib.LevelDesc,
               "mq_parareal_desc": _lib.PararealDesc, "mq_server_desc": _lib.ServerDesc,
               "mq_request": _lib.Request, "mq_result": _lib.Result, "mq_adaptive_desc": _lib.AdaptiveDesc,
               "mq_combined_desc": _lib.CombinedDesc, "mq_combined_stats": _lib.CombinedStats,
               "mq_cost_in": _lib.CostIn, "mq_cost_out": _lib.CostOut}
    src = tmp_path / "sz.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HDR}"', 'int main(void){']
    for cname in structs:
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
    lines.append('printf("off_tol %zu\\n", offsetof(mq_problem_desc, tol));')
    lines.append('printf("off_kernel_ms %zu\\n", offsetof(mq_run_stats, kernel_ms));')
    lines.append('printf("off_t_done %zu\\n", offsetof(mq_result, t_done_ns));')
    lines.append('printf("off_mg_sweeps %zu\\n", offsetof(mq_problem_desc, mg_coarse_sweeps));')
    lines.append('printf("off_busy %zu\\n", offsetof(mq_run_stats, busy_ms));')
    lines.append('printf("off_wide_queue %zu\\n", offsetof(mq_server_desc, wide_queue));')
    lines.append('printf("off_s_nc %zu\\n", offsetof(mq_cost_out, s_nc));')
    lines.append('printf("off_level_slots %zu\\n", offsetof(mq_combined_stats, level_slots));')
    lines.append('printf("off_mem_kind %zu\\n", offsetof(mq_problem_desc, mem_kind));')
    lines.append('printf("off_mass %zu\\n", offsetof(mq_problem_desc, mass));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-o", str(exe), str(src)])
    out = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, cls in structs.items():
        assert int(out[cname]) == C.sizeof(cls), cname
    assert int(out["off_tol"]) == _lib.ProblemDesc.tol.offset
    assert int(out["off_kernel_ms"]) == _lib.RunStats.kernel_ms.offset
    assert int(out["off_t_done"]) == _lib.Result.t_done_ns.offset
    assert int(out["off_mg_sweeps"]) == _lib.ProblemDesc.mg_coarse_sweeps.offset
    assert int(out["off_busy"]) == _lib.RunStats.busy_ms.offset
    assert int(out["off_wide_queue"]) == _lib.ServerDesc.wide_queue.offset
    assert int(out["off_s_nc"]) == _lib.CostOut.s_nc.offset
    assert int(out["off_level_slots"]) == _lib.CombinedStats.level_slots.offset
    assert int(out["off_mem_kind"]) == _lib.ProblemDesc.mem_kind.offset
    assert int(out["off_mass"]) == _lib.ProblemDesc.mass.offset


def test_no_device_and_invalid_arguments(lib):
    import torch
    from paper_2507_19246_amd import _lib
    import workloads as W
    from paper_2507_19246_amd.api import default_desc
    d = default_desc(W.plain_fp64_33().problem, _lib.MQ_PREC_FP64)
    h = C.c_void_p()
    bad = _lib.ProblemDesc.from_buffer_copy(d)
    bad.n_nodes = 2
    assert lib.fem_setup(C.byref(bad), None, C.byref(h)) == _lib.MQ_ERR_INVALID_ARG
    assert b"n_nodes" in lib.mq_last_error()
    bad = _lib.ProblemDesc.from_buffer_copy(d)
    bad.tol = 0.0
    assert lib.fem_setup(C.byref(bad), None, C.byref(h)) == _lib.MQ_ERR_INVALID_ARG
    if not torch.cuda.is_available():
        assert lib.fem_setup(C.byref(d), None, C.byref(h)) == _lib.MQ_ERR_NO_DEVICE
        assert not h.value
    # estimator argument validation happens before any device work
    ns = (C.c_int32 * 2)(3, 0)
    null = (C.c_void_p * 2)()
    assert lib.mlmc_estimate(2, ns, null, null, None, None) == _lib.MQ_ERR_INVALID_ARG
    assert lib.mq_problem_destroy(None) == _lib.MQ_OK


def test_autotune_candidates_and_cache_key():
    """Host logic of the autotuner: candidate sets per mesh and precision."""
    import workloads as W
    from paper_2507_19246_amd import _lib, autotune
    c129 = autotune.candidates(W.Problem(129, W.Material(kind=W.MAT_KL)), _lib.MQ_PREC_MIXED)
    assert {c["tile"] for c in c129} == {1, 2}
    assert {c["precond"] for c in c129} == {_lib.MQ_PRECOND_JACOBI, _lib.MQ_PRECOND_MULTIGRID}
    assert all(c["mg_omega"] == 0.0 for c in c129 if c["precond"] == _lib.MQ_PRECOND_JACOBI)
    # 100 x 100 nodes: no multigrid (98 interior nodes is not 2^k - 1), both tiles
    c100 = autotune.candidates(W.Problem(100, W.Material(kind=W.MAT_KL)), _lib.MQ_PREC_FP64)
    assert {c["precond"] for c in c100} == {_lib.MQ_PRECOND_JACOBI}
    assert {c["inner_rtol"] for c in c100} == {1e-10}
    c33 = autotune.candidates(W.Problem(33, W.Material(kind=W.MAT_KL)), _lib.MQ_PREC_MIXED)
    assert {c["tile"] for c in c33} == {1}
    c257 = autotune.candidates(W.Problem(257, W.Material(kind=W.MAT_KL)), _lib.MQ_PREC_MIXED)
    assert {c["tile"] for c in c257} == {1, 2}
    assert {c["precond"] for c in c257} == {_lib.MQ_PRECOND_MULTIGRID}
    k = autotune.cache_key("dev", W.Problem(33, W.Material(kind=W.MAT_KL)), _lib.MQ_PREC_MIXED)
    assert k == "dev|n33|mat1|prec1"
