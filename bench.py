#!/usr/bin/env python3
"""Throughput / latency benchmark of the batched MLMC hot path on one MI355X.

Default workload (--workload mlmc3): MLMC with 3 time levels on the
129x129-node eddy-current model (KL-8 lognormal conductivity, 64/128/256
steps per period over 4 periods, 512/128/32 samples, coupled level
differences), FP32 CG inside FP64 iterative refinement.  One benchmark step =
one full MLMC estimate: device assembly of every sample, all implicit-Euler
runs of all levels in one persistent launch, the Joule-loss QoIs and the
estimator of Eq. (9).  Inputs (xi) are resident in device memory before the
timed region.

Printed: one JSON line with sample-steps/s (whole job), p50/p99 per-sample
latency, QoI error against the FP64 oracle and against the plain FP64 GPU
path (one sample per launch, Jacobi-preconditioned CG), the roofline of the
dominant kernel and the oracle timed on the host cores.

Other workloads, one JSON line each in the same shape:
  --workload parareal   Parareal on the finest level (257x257, 64 samples,
                        32 slices of 32 fine steps, 1 coarse step per slice,
                        K <= 8, tol 1e-8); value = useful (serial-equivalent)
                        sample-steps/s, beside the batched serial fine run.
  --workload nonlinear  MLMC with 4 levels and the nonlinear reluctivity
                        (Picard per step), 129x129, 1024/256/64/16 samples.
  --workload adaptive   adaptive MLMC (Eq. (11)) on the 129x129 model to
                        --target-rmse, level variances estimated at run time.
  --workload serving    Poisson stream of sample-solve requests (mixed meshes
                        65..513, 64..1024 steps per period, 2 periods) into the
                        continuous-batching server; the first --requests of
                        the stream at --rate requests/s.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3     # MI355X published FP32 vector peak
HBM_PEAK_GBS = 8000.0               # MI355X HBM3E
CG_FLOPS_PER_DOF_ITER = 26          # 7-point scaled stencil (14) + CG vector updates and dots (12)
# one multigrid-preconditioned CG iteration on the fine level: the CG stencil
# and vector work (26), the V(1,1) cycle's residual and post-smoothing stencils
# (2 x 14), smoothing/residual updates (6), restriction and prolongation (8),
# plus the coarse levels (1/4 + 1/16 + ... of that work)
MG_FLOPS_PER_DOF_ITER = 26 + (28 + 6 + 8) * 4.0 / 3.0
CG_BYTES_PER_DOF_ITER_FP32 = 72     # modelled streaming traffic of one FP32 CG iteration
# algorithmic HBM bytes of the mixed-precision path per DoF (the method's own
# traffic with every vector streamed once per pass): one FP32 CG iteration
# (stencil 7 x 4 + vectors 16, fused updates 28), one FP64 refinement residual
# (M and K coefficients, state and increment), one time step's outer work
# (K a_k, M d, state and increment updates)
ALG_BYTES_CG_ITER_FP32 = 72
ALG_BYTES_FP64_RESIDUAL = 120
ALG_BYTES_STEP = 150
# MI355X LDS: 128 B per clock per compute unit (the CDNA3 figure, kept as the
# conservative bound for CDNA4), 256 compute units at 2.4 GHz
LDS_PEAK_GBS = 128 * 256 * 2.4
# the paper's own results (one 180-core CPU machine, Julia + GetDP, no GPU):
# context for the numbers of this line, not a target
PAPER_CONTEXT = {
    "speedup_of_mlmc_from_parareal": "12-45% (1.12x FE model, 1.45x circuit model)",
    "extra_effort_core_seconds": "15-18% (1.18x FE model, 1.15x circuit model)",
    "single_sample_parareal_speedup": "2.69 (FE model, 16 cores per sample), 2.93 (circuit model)",
    "hardware": "one machine with 180 CPU cores; Julia (DifferentialEquations.jl, MultilevelEstimators.jl, "
                "Distributed.jl) with GetDP/Gmsh; no GPU; precision not stated",
    "source": "Sec. III (results), Sec. IV (conclusions), Table II",
}


def _kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    h.update(open(os.path.join(ROOT, "paper_2507_19246_amd", "csrc", "kernels.hip"), "rb").read())
    return h.hexdigest()[:16]


def profile_value(name: str, key: str):
    """A figure from a committed profile summary (`key: value` lines), or None when
    the kernel source changed since it was taken."""
    return measured_traffic(name, key)


def measured_traffic(name: str, key: str = "traffic_bytes_per_launch"):
    """HBM bytes per launch (or per run: key) from the committed counter summary,
    or None when the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("traffic_"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("traffic_source_sha256") != _kernel_source_hash():
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def _oracle_task(args):
    """One oracle solve (runs in a worker process with one BLAS thread)."""
    problem, xi, spp, nper = args
    from oracle import timestep
    t = time.perf_counter()
    q, _ = timestep.solve_sample(problem, xi, spp, nper)
    return q, spp * nper, time.perf_counter() - t


def host_buffer_rate(w, levels, xis_np, knobs, L, qfs_dev, qcs_dev):
    """One multilevel run of the same workload through a host-pointer handle
    (mem_kind = MQ_MEM_HOST): xi goes in and Q comes out over PCIe inside the
    timed call.  Results must equal the device-resident run's bit for bit."""
    import ctypes as C
    import numpy as np
    from paper_2507_19246_amd import autotune
    ph, _ = autotune.tuned_problem(w.problem, L.MQ_PREC_MIXED, **dict(knobs, mem_kind=L.MQ_MEM_HOST))
    nl = len(levels)
    lvs = (L.LevelDesc * nl)(*[L.LevelDesc(a, b, c, 0) for a, b, c in levels])
    xs = [np.ascontiguousarray(x, dtype=np.float64) for x in xis_np]
    ns = (C.c_int32 * nl)(*[x.shape[0] for x in xs])
    qf = [np.zeros(x.shape[0]) for x in xs]
    qc = [np.zeros(x.shape[0]) if levels[l][1] > 0 else None for l, x in enumerate(xs)]
    px = (C.c_void_p * nl)(*[x.ctypes.data for x in xs])
    pf = (C.c_void_p * nl)(*[q.ctypes.data for q in qf])
    pc = (C.c_void_p * nl)(*[(q.ctypes.data if q is not None else None) for q in qc])
    st = L.RunStats()
    t0 = time.perf_counter()
    rc = ph.lib.mlmc_multilevel_run(ph.h, nl, lvs, ns, px, pf, pc, C.byref(st))
    wall = time.perf_counter() - t0
    ph.close()
    if rc < 0:
        return {"error": rc}
    same = all(np.array_equal(qf[l], qfs_dev[l].cpu().numpy()) for l in range(nl)) and all(
        qc[l] is None or np.array_equal(qc[l], qcs_dev[l].cpu().numpy()) for l in range(nl))
    in_b = sum(x.nbytes for x in xs)
    out_b = sum(q.nbytes for q in qf) + sum(q.nbytes for q in qc if q is not None)
    return {"value": st.sample_steps / wall, "unit": "sample-steps/s", "steps": 1,
            "bytes_in": in_b, "bytes_out": out_b, "equal_to_device_run": bool(same),
            "note": "multilevel run through a host-pointer handle (xi in, Q out over PCIe, blocking); "
                    "the estimator is not part of it"}


def cpu_baseline(w, xis, n_per_level=(12, 4, 2)):
    """Time the FP64 oracle on a bounded sample of the same workload."""
    import multiprocessing as mp
    tasks, keys = [], []
    for l, lv in enumerate(w.levels):
        for s in range(min(n_per_level[l], lv.n_samples)):
            tasks.append((w.problem, xis[l][s], lv.steps_per_period, lv.n_periods))
            keys.append((l, s, "f"))
            if lv.coarse_steps_per_period:
                tasks.append((w.problem, xis[l][s], lv.coarse_steps_per_period, lv.n_periods))
                keys.append((l, s, "c"))
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16, len(tasks)))
    env_threads = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env_threads:
        os.environ[k] = "1"
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_task, tasks)
    wall = time.perf_counter() - t0
    for k, v in env_threads.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v
    steps = sum(r[1] for r in res)
    cpu_s = sum(r[2] for r in res)
    sample = {f"level{l}": n for l, n in enumerate(n_per_level)}
    return {
        "value": steps / wall, "unit": "sample-steps/s", "cores": cores, "kind": "oracle",
        "sample": (f"{steps} sample-steps: first {list(n_per_level)} samples of levels 0/1/2 of the "
                   f"same workload (coupled runs included), {cpu_s:.1f} core-s, banded-Cholesky FP64"),
    }, {keys[i]: res[i][0] for i in range(len(res))}


def _cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _oracle_pool(tasks, fn):
    """Run oracle tasks in a spawn pool with one BLAS thread per worker."""
    import multiprocessing as mp
    cores = max(1, min(_cores(), 16, len(tasks)))
    env_threads = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env_threads:
        os.environ[k] = "1"
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(fn, tasks)
    wall = time.perf_counter() - t0
    for k, v in env_threads.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v
    return res, wall, cores


def _picard_task(args):
    problem, xi, spp, nper = args
    from oracle import picard
    t = time.perf_counter()
    q, _ = picard.solve_sample(problem, xi, spp, nper)
    return q, spp * nper, time.perf_counter() - t


def _contract(metric_unit, value, elapsed, args, config, dtype="f32+f64"):
    return {
        "metric": "sample-steps/s + p50/p99 sample latency vs plain FP64, QoI rel err <= 1e-6",
        "value": value, "unit": metric_unit, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config,
    }


def _hbm_roofline(kernel, bytes_per_launch, avg_launch_s, traffic=None, model=""):
    gbs = bytes_per_launch / avg_launch_s / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": traffic, "kernel": kernel, "avg_launch_ms": 1e3 * avg_launch_s,
            "algorithmic_bytes_per_launch": bytes_per_launch, "model": model}


def bench_parareal(args, mq, L, W, np, torch):
    """Parareal on the finest level (257x257, 64 samples); value = useful sample-steps/s."""
    w = W.parareal_257()
    pr = w.parareal
    if args.coarse_steps > 0:
        import dataclasses
        pr = dataclasses.replace(pr, coarse_steps_per_slice=args.coarse_steps)
    xi_np = W.level_xi(w, 0)
    xi = torch.tensor(xi_np, dtype=torch.float64, device="cuda")
    from paper_2507_19246_amd import autotune
    prob, knobs = autotune.tuned_problem(w.problem, L.MQ_PREC_MIXED)
    nd = prob.n_dof
    n_f = pr.n_slices * pr.fine_steps_per_slice
    useful = xi.shape[0] * n_f

    def step():
        return mq.parareal_run(prob, pr.n_periods, pr.n_slices, pr.fine_steps_per_slice,
                               pr.coarse_steps_per_slice, pr.k_max, pr.tol, xi)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        q, it, _, rc, st = step()
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # the same samples as one batched serial fine run (no Parareal)
    spp = n_f // pr.n_periods
    qp = q.cpu().numpy()
    if args.no_serial:
        qsr, sts, serial_s = qp, None, None
    else:
        torch.cuda.synchronize()
        ts = time.perf_counter()
        qs, _, _, _, sts = mq.mlmc_level_run(prob, spp, 0, pr.n_periods, xi)
        torch.cuda.synchronize()
        serial_s = time.perf_counter() - ts
        qsr = qs.cpu().numpy()
    iters = it.cpu().numpy()
    executed = stats[-1]["sample_steps"]
    avg_kern_s = sum(s["kernel_ms"] for s in stats) / len(stats) / 1e3
    inner = stats[-1]["inner_iters"]
    resid = stats[-1]["sweeps"] + executed  # FP64 residual passes: one per sweep plus the converged check
    bytes_launches = nd * (ALG_BYTES_CG_ITER_FP32 * inner + ALG_BYTES_FP64_RESIDUAL * resid + ALG_BYTES_STEP * executed)
    res = _contract("sample-steps/s", useful * args.steps / elapsed, elapsed, args, {
        "workload": w.name, "mesh": "257x257", "n_dof": nd, "samples": int(xi.shape[0]),
        "fine_steps": n_f, "slices": pr.n_slices, "coarse_steps_per_slice": pr.coarse_steps_per_slice,
        "k_max": pr.k_max, "tol": pr.tol, "path": "resident" if stats[-1]["path"] == 1 else "streaming",
        "launch_block": stats[-1]["block"], "knobs": dict(knobs, precond=prob.info.precond)})
    res.update({
        "useful_sample_steps": useful, "executed_sample_steps": executed,
        "extra_effort": executed / useful,
        "parareal_iterations": {"min": int(iters.min()), "max": int(iters.max()), "mean": float(iters.mean())},
        "status": rc, "latency_ms": 1e3 * elapsed / args.steps,
        "serial_fine_batched": None if sts is None else {
            "value": useful / serial_s, "unit": "sample-steps/s", "wall_ms": 1e3 * serial_s,
            "cg_iters_per_sample_step": sts["inner_iters"] / sts["sample_steps"]},
        "q_max_rel_diff_parareal_vs_serial": None if sts is None else float(np.max(np.abs(qp - qsr) / np.abs(qsr))),
        "cg_iters_per_executed_step": inner / executed,
        "roofline": _hbm_roofline("k_ie_stream<float,%d,multigrid>" % stats[-1]["block"], bytes_launches, avg_kern_s,
                                  # (the committed counters are of the 1-step coarse propagator run)
                                  measured_traffic("ie_stream_parareal_257_hbm_counters.md", "traffic_bytes_per_run")
                                  if pr.coarse_steps_per_slice == 1 else None,
                                  f"{ALG_BYTES_CG_ITER_FP32} B per DoF and CG iteration + "
                                  f"{ALG_BYTES_FP64_RESIDUAL} B per DoF and FP64 residual + "
                                  f"{ALG_BYTES_STEP} B per DoF and executed step; units of the launch: "
                                  f"{inner} CG iterations, {resid} residuals, {executed} steps over {nd} DoF"),
    })
    if not args.no_cpu_baseline and sts is not None:
        tasks = [(w.problem, xi_np[s], spp, pr.n_periods) for s in range(2)]
        out, wall, cores = _oracle_pool(tasks, _oracle_task)
        errs = [abs(qsr[s] - out[s][0]) / abs(out[s][0]) for s in range(len(tasks))]
        res["cpu_baseline"] = {"value": sum(o[1] for o in out) / wall, "unit": "sample-steps/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"serial fine runs ({n_f} steps) of the first {len(tasks)} samples, "
                                         "banded-Cholesky FP64"}
        res["qoi_max_rel_err_serial_vs_fp64_oracle"] = max(errs)
        res["qoi_max_rel_err_parareal_vs_fp64_oracle"] = max(
            abs(qp[s] - out[s][0]) / abs(out[s][0]) for s in range(len(tasks)))
    prob.close()
    return res


def bench_nonlinear(args, mq, L, W, np, torch):
    """MLMC with 4 levels and the nonlinear reluctivity (Picard), 129x129."""
    w = W.nonlinear_mlmc4_129()
    levels = [(lv.steps_per_period, lv.coarse_steps_per_period, lv.n_periods) for lv in w.levels]
    xis_np = [W.level_xi(w, l) for l in range(len(w.levels))]
    xis = [torch.tensor(x, dtype=torch.float64, device="cuda") for x in xis_np]
    from paper_2507_19246_amd import autotune
    prob, knobs = autotune.tuned_problem(w.problem, L.MQ_PREC_MIXED)
    nd = prob.n_dof

    def step():
        qfs, qcs, rc, st = mq.mlmc_multilevel_run(prob, levels, xis)
        e, y, v = mq.mlmc_estimate(qfs, qcs)
        return qfs, qcs, e, rc, st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        qfs, qcs, e, rc, st = step()
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sample_steps = sum(s["sample_steps"] for s in stats)
    avg_kern_s = sum(s["kernel_ms"] for s in stats) / len(stats) / 1e3
    units = nd * stats[-1]["inner_iters"]
    flops_unit = MG_FLOPS_PER_DOF_ITER if prob.info.precond == L.MQ_PRECOND_MULTIGRID else CG_FLOPS_PER_DOF_ITER
    tf = flops_unit * units / avg_kern_s / 1e12
    res = _contract("sample-steps/s", sample_steps / elapsed, elapsed, args, {
        "workload": w.name, "mesh": "129x129", "n_dof": nd,
        "levels_steps_per_period": [lv.steps_per_period for lv in w.levels], "n_periods": w.levels[0].n_periods,
        "samples_per_level": [lv.n_samples for lv in w.levels], "sample_steps_per_step": stats[-1]["sample_steps"],
        "picard_tol": w.problem.material.picard_tol, "launch": [stats[-1]["grid"], stats[-1]["block"]],
        "knobs": dict(knobs, tile=prob.info.tile, precond=prob.info.precond)})
    res.update({
        "p50_latency_ms": st["lat_p50_ms"], "p99_latency_ms": st["lat_p99_ms"], "status": rc,
        "mlmc_estimate": float(e),
        "picard_iters_per_sample_step": stats[-1]["picard_iters"] / stats[-1]["sample_steps"],
        "cg_iters_per_sample_step": stats[-1]["inner_iters"] / stats[-1]["sample_steps"],
        "roofline": {"bound": "alu", "achieved": tf, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tf / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": measured_traffic("ie_resident_nonlinear_mlmc4_129_hbm_counters.md"),
                     "kernel": "k_ie_resident<float,128,16,8,64,%s,nonlinear>" % (
                         "multigrid" if prob.info.precond == L.MQ_PRECOND_MULTIGRID else "jacobi"),
                     "avg_launch_ms": 1e3 * avg_kern_s, "flops_per_dof_iter": flops_unit},
    })
    if not args.no_cpu_baseline:
        lv = w.levels[0]
        tasks = [(w.problem, xis_np[0][s], lv.steps_per_period, lv.n_periods) for s in range(4)]
        out, wall, cores = _oracle_pool(tasks, _picard_task)
        q0 = qfs[0].cpu().numpy()
        res["cpu_baseline"] = {"value": sum(o[1] for o in out) / wall, "unit": "sample-steps/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"first {len(tasks)} samples of level 0 ({lv.steps_per_period * lv.n_periods}"
                                         " steps each, Picard with a banded-Cholesky refactorisation per iteration)"}
        res["qoi_max_rel_err_vs_fp64_oracle"] = max(abs(q0[s] - out[s][0]) / abs(out[s][0]) for s in range(len(tasks)))
    prob.close()
    return res


def bench_adaptive(args, mq, L, W, np, torch):
    """Adaptive MLMC (Eq. (11)) on the 129x129 three-level model: pilot samples,
    then rounds of one launch each until the sample counts meet the target RMSE."""
    from paper_2507_19246_amd import autotune
    w = W.mlmc3_mixed_129()
    levels = [(lv.steps_per_period, lv.coarse_steps_per_period, lv.n_periods) for lv in w.levels]
    n_max = [8192, 2048, 1024]
    pools = [torch.tensor(W.level_xi(w, l, n=n_max[l]), dtype=torch.float64, device="cuda") for l in range(3)]
    prob, knobs = autotune.tuned_problem(w.problem, L.MQ_PREC_MIXED)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e, y, v, n, _, _, rc, st = mq.mlmc_adaptive_run(prob, levels, pools, args.target_rmse, n_pilot=32)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    args.steps, args.warmup = 1, 0
    res = _contract("sample-steps/s", st["sample_steps"] / elapsed, elapsed, args, {
        "workload": "adaptive-mlmc3-mixed-129x129-kl8", "mesh": "129x129",
        "levels_steps_per_period": [lv.steps_per_period for lv in w.levels], "n_periods": w.levels[0].n_periods,
        "target_rmse": args.target_rmse, "var_fraction": 0.5, "n_pilot": 32, "n_max": n_max,
        "knobs": dict(knobs, precond=prob.info.precond)})
    res.update({"status": rc, "mlmc_estimate": e, "samples_per_level": n, "level_means": y,
                "level_variances": v, "estimator_std": float(np.sqrt(sum(vi / ni for vi, ni in zip(v, n)))),
                "sample_steps": st["sample_steps"], "kernel_ms": st["kernel_ms"], "roofline": None,
                "cpu_baseline": None})
    prob.close()
    return res


def bench_combined(args, mq, L, W, np, torch):
    """MLMC with Parareal on the finest level (Section II-D) on the three-level
    129x129 model: the plain MLMC estimate as reference, then the combined run
    (levels 0-1 batched, level 2 by Parareal with the level-0 time grid as coarse
    propagator, at once); measured times and effort against Eqs. (15)-(25) with
    C_l = one sample of level l alone."""
    from paper_2507_19246_amd import autotune
    w = W.mlmc3_mixed_129()
    levels = [(lv.steps_per_period, lv.coarse_steps_per_period, lv.n_periods) for lv in w.levels]
    xis = [torch.tensor(W.level_xi(w, l), dtype=torch.float64, device="cuda") for l in range(3)]
    prob, knobs = autotune.tuned_problem(w.problem, L.MQ_PREC_MIXED)
    Lf = len(levels) - 1
    useful = sum(x.shape[0] * lv[2] * (lv[0] + lv[1]) for x, lv in zip(xis, levels))

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    # warm-up of both paths (the combined run sets up its second handle here)
    mq.mlmc_multilevel_run(prob, levels, xis)
    mq.mlmc_combined_run(prob, levels, xis, tol=args.para_tol)
    (ref, t_ref) = timed(lambda: mq.mlmc_multilevel_run(prob, levels, xis))
    (comb, t_comb) = timed(lambda: mq.mlmc_combined_run(prob, levels, xis, tol=args.para_tol))
    qf, qc, it, rc, st, cs = comb
    e_ref = float(mq.mlmc_estimate(ref[0], ref[1])[0])
    e_comb = float(mq.mlmc_estimate(qf, qc)[0])
    # C_l: one sample of level l alone (fine run), and the level-L serial fine runs batched
    C_ms = []
    for l, (spp, _, nper) in enumerate(levels):
        _, t = timed(lambda: mq.mlmc_level_run(prob, spp, 0, nper, xis[l][:1]))
        C_ms.append(1e3 * t)
    _, t_serial_L = timed(lambda: mq.mlmc_level_run(prob, levels[Lf][0], 0, levels[Lf][2], xis[Lf]))
    M, kmax = cs["n_slices"], cs["max_k"]
    N = [x.shape[0] for x in xis]
    model = mq.cost_model(C_ms, N, kmax, M, cs["n_cores"])
    steps = [lv[0] * lv[2] for lv in levels]
    model_steps = mq.cost_model(steps, N, kmax, M, cs["n_cores"])
    Kv = it.cpu().numpy()
    pred_effort = sum(mq.cost_model(steps, N, int(k), M, cs["n_cores"])["effort_para"] for k in Kv)
    args.steps, args.warmup = 1, 1
    res = _contract("sample-steps/s", useful / t_comb, t_comb, args, {
        "workload": "combined-mlmc3-mixed-129x129-kl8-512/128/32-parareal-level2",
        "mesh": "129x129", "levels_steps_per_period": [lv[0] for lv in levels], "n_periods": levels[0][2],
        "n_slices": M, "coarse_propagator_steps_per_period": cs["coarse_steps_per_period"],
        "parareal_tol": args.para_tol, "knobs": dict(knobs, precond=prob.info.precond)})
    res.update({
        "status": rc, "reference_mlmc_sample_steps_per_s": useful / t_ref,
        "measured": {"t_ref_ms": 1e3 * t_ref, "t_comb_ms": 1e3 * t_comb, "speedup": t_ref / t_comb,
                     "ms_levels": cs["ms_levels"], "ms_parareal": cs["ms_parareal"],
                     "level_L_serial_fine_ms": 1e3 * t_serial_L,
                     "level_L_parareal_speedup": 1e3 * t_serial_L / cs["ms_parareal"],
                     "K_mean": cs["mean_k"], "K_max": kmax, "n_c_para_eq25": cs["n_c_para"],
                     "n_cores_slots": cs["n_cores"], "level_slots": cs["level_slots"],
                     "parareal_effort_steps_per_sample": (cs["para_fine_steps"] + cs["para_coarse_steps"]) / N[Lf],
                     "estimate": e_comb, "estimate_reference": e_ref,
                     "estimate_rel_diff": abs(e_comb - e_ref) / abs(e_ref)},
        "predicted": {"C_ms_one_sample": C_ms, "tau_para_ms_eq15": model["tau_para"],
                      "level_L_parareal_speedup": C_ms[Lf] / model["tau_para"],
                      "speedup_unlimited_eq17_18": model["speedup"], "s_inf_eq21": model["s_inf"],
                      "kappa_eq22": model_steps["kappa"], "eps_inf_eq23": model["eps_inf"],
                      "batches_eq24": model["batches"], "speedup_n_cores": model["s_nc"],
                      "parareal_effort_steps_per_sample_eq16": pred_effort / N[Lf]},
        "sample_steps_executed": st["sample_steps"], "roofline": None, "cpu_baseline": None})
    prob.close()
    return res


def _serve(mq, L, W, np, torch, reqs, limit_s, label, wide_min_nodes=0, wide_load_limit=0):
    """Submit `reqs` at their arrival times into a fresh server; wait for all results."""
    base = W.Problem(65, W.Material(kind=W.MAT_KL))
    srv = mq.Server(base, L.MQ_PREC_MIXED, hbm_budget_bytes=96 << 30, max_inflight=4096, n_streams=2,
                    wide_min_nodes=wide_min_nodes, wide_load_limit=wide_load_limit)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_report = t0
    done = {}
    i = 0
    while len(done) < len(reqs):
        now = time.perf_counter() - t0
        while i < len(reqs) and reqs[i].arrival_s <= now:
            r = reqs[i]
            srv.submit(r.n_nodes, r.steps_per_period, r.n_periods, r.xi, user_id=i)
            i += 1
        for r in srv.poll(1024):
            done[r.ticket] = r
        if time.perf_counter() - t_report > 10.0:
            t_report = time.perf_counter()
            print(f"serving ({label}): {i} submitted, {len(done)} done, {t_report - t0:.0f} s",
                  file=sys.stderr, flush=True)
        if time.perf_counter() - t0 > limit_s:
            srv.close()
            raise RuntimeError(f"serving run exceeded {limit_s} s ({len(done)} of {len(reqs)} done)")
        time.sleep(0.0005)
    elapsed = time.perf_counter() - t0
    srv.close()
    lat = np.array([(r.t_done_ns - r.t_submit_ns) / 1e6 for r in done.values()])
    steps = sum(reqs[r.user_id].steps_per_period * reqs[r.user_id].n_periods for r in done.values())
    # algorithmic bytes of the work done (same per-DoF figures as the batched lines)
    alg = {}
    for r in done.values():
        q = reqs[r.user_id]
        nd = (q.n_nodes - 2) ** 2
        st_ = q.steps_per_period * q.n_periods
        b = nd * (ALG_BYTES_CG_ITER_FP32 * r.inner_iters + ALG_BYTES_FP64_RESIDUAL * (r.sweeps + st_)
                  + ALG_BYTES_STEP * st_)
        a = alg.setdefault(q.n_nodes, {"bytes": 0.0, "steps": 0, "cg_iters": 0, "wide": 0})
        a["bytes"] += b
        a["steps"] += st_
        a["cg_iters"] += r.inner_iters
        a["wide"] += int(r.path == L.MQ_PATH_WIDE)
    by_mesh = {}
    for r in done.values():
        by_mesh.setdefault(reqs[r.user_id].n_nodes, []).append((r.t_done_ns - r.t_submit_ns) / 1e6)
    return {
        "sample_steps_per_s": steps / elapsed, "requests_per_s": len(done) / elapsed, "wall_s": elapsed,
        "p50_latency_ms": float(np.percentile(lat, 50)), "p99_latency_ms": float(np.percentile(lat, 99)),
        "failed": sum(1 for r in done.values() if r.status < 0),
        "latency_ms_by_mesh": {str(k): {"n": len(v), "p50": float(np.percentile(v, 50)),
                                        "p99": float(np.percentile(v, 99))} for k, v in sorted(by_mesh.items())},
        "algorithmic": alg,
    }


def bench_serving(args, mq, L, W, np, torch):
    """Poisson request stream into the continuous-batching server: the offered
    rate (saturating), then a stable load at 0.7 x the measured capacity."""
    reqs = W.serving_stream(args.requests, rate_hz=args.rate)
    sat = _serve(mq, L, W, np, torch, reqs, args.serving_limit_s, "offered rate", args.wide_min_nodes,
                 args.wide_load_limit)
    args.steps, args.warmup = 1, 0
    res = _contract("sample-steps/s", sat["sample_steps_per_s"], sat["wall_s"], args, {
        "workload": f"serving-kl8-mixed-{len(reqs)}req-{args.rate:g}rps",
        "meshes": list(W.SERVING_MESHES), "mesh_weights": list(W.SERVING_MESH_WEIGHTS),
        "steps_per_period": list(W.SERVING_STEPS), "n_periods": 2, "requests": len(reqs),
        "rate_req_per_s": args.rate, "lanes_per_mesh": 2, "chunk_steps": 32,
        "wide_min_nodes": 513 if args.wide_min_nodes == 0 else args.wide_min_nodes,
        "wide_load_limit": args.wide_load_limit or "half the compute units",
        "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "0")) or None})
    res.update({k: sat[k] for k in ("p50_latency_ms", "p99_latency_ms", "requests_per_s", "failed",
                                    "latency_ms_by_mesh")})
    if args.stable_requests > 0:
        rate = 0.7 * sat["requests_per_s"]
        st = _serve(mq, L, W, np, torch, W.serving_stream(args.stable_requests, rate_hz=rate),
                    args.serving_limit_s, "stable load", args.wide_min_nodes, args.wide_load_limit)
        st["rate_req_per_s"] = rate
        st["requests"] = args.stable_requests
        st.pop("algorithmic", None)
        res["stable_load"] = st
    alg = sat["algorithmic"]
    tot = sum(a["bytes"] for a in alg.values())
    gbs = tot / sat["wall_s"] / 1e9
    res["roofline"] = {
        "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
        "traffic": None, "kernel": "k_ie_resident (65, 129), k_ie_stream (257, 513 batched), k_w_* (513 wide lane)",
        "scope": "whole job: algorithmic bytes of all served requests over the run's wall time (launches of "
                 "several lanes overlap, so per-launch durations do not add up to it)",
        "bytes_per_dof": {"fp32_cg_iteration": ALG_BYTES_CG_ITER_FP32, "fp64_residual": ALG_BYTES_FP64_RESIDUAL,
                          "time_step": ALG_BYTES_STEP},
        "by_mesh": {str(k): {"algorithmic_bytes": a["bytes"], "sample_steps": a["steps"],
                             "cg_iters_per_step": a["cg_iters"] / max(1, a["steps"]), "wide_lane_requests": a["wide"],
                             "share_of_bytes": a["bytes"] / tot} for k, a in sorted(alg.items())}}
    res["cpu_baseline"] = None if args.no_cpu_baseline else serving_cpu_baseline(reqs)
    return res


def _serving_oracle_task(args):
    n_nodes, xi, spp = args
    import workloads as W
    from oracle import timestep
    prob = W.Problem(n_nodes, W.Material(kind=W.MAT_KL))
    t = time.perf_counter()
    timestep.solve_sample(prob, xi, spp, 1)
    return n_nodes, spp, time.perf_counter() - t


def serving_cpu_baseline(reqs, per_mesh=((65, 4), (129, 2), (257, 1), (513, 1)), spp=64):
    """Oracle on a bounded sample of the stream: per mesh size, its first requests
    run for one period at 64 steps per period (one factorisation, 64 solves); the
    per-core rate of each mesh size is applied to every request of the stream."""
    import numpy as np
    tasks = []
    for n_nodes, k in per_mesh:
        mine = [r for r in reqs if r.n_nodes == n_nodes][:k]
        tasks += [(n_nodes, np.asarray(r.xi), spp) for r in mine]
    out, wall, cores = _oracle_pool(tasks, _serving_oracle_task)
    per_core = {}
    for n_nodes, s_, t in out:
        a = per_core.setdefault(n_nodes, [0, 0.0])
        a[0] += s_
        a[1] += t
    rate = {n: a[0] / a[1] for n, a in per_core.items()}
    steps = sum(r.steps_per_period * r.n_periods for r in reqs)
    core_s = sum(r.steps_per_period * r.n_periods / rate[r.n_nodes] for r in reqs)
    return {"value": cores * steps / core_s, "unit": "sample-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"per mesh size the first {dict(per_mesh)} requests of the stream, one period at {spp} steps "
                      f"per period each ({sum(a[1] for a in per_core.values()):.1f} core-s, banded-Cholesky FP64); "
                      "the measured per-core rate of each mesh size applied to all requests (factorisation "
                      "amortised over 64 steps: an upper bound on the oracle's time for longer requests), spread "
                      "over the cores",
            "per_core_sample_steps_per_s": {str(n): r_ for n, r_ in sorted(rate.items())},
            "extrapolated_stream_core_s": core_s}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-baseline", action="store_true")
    ap.add_argument("--fp64-samples", type=int, default=4,
                    help="samples of the plain FP64 one-sample-per-call baseline")
    ap.add_argument("--no-host-buffers", action="store_true",
                    help="skip the PCIe-inclusive run through a host-pointer handle")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (HBM counter calibration)")
    ap.add_argument("--workload", default="mlmc3",
                    choices=["mlmc3", "parareal", "nonlinear", "serving", "adaptive", "combined"])
    ap.add_argument("--para-tol", type=float, default=1e-8, help="combined: Parareal jump tolerance")
    ap.add_argument("--target-rmse", type=float, default=50.0, help="adaptive: target RMSE of the estimate (W/m)")
    ap.add_argument("--requests", type=int, default=4096, help="serving: requests taken from the stream")
    ap.add_argument("--rate", type=float, default=200.0, help="serving: arrival rate (requests/s)")
    ap.add_argument("--wide-min-nodes", type=int, default=0,
                    help="serving: smallest mesh of the wide lane (0: the library default 513; -1: no wide lane)")
    ap.add_argument("--wide-load-limit", type=int, default=0,
                    help="serving: batched requests above which the wide lane is not used (0: library default)")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="serving: hardware queues of the process (GPU_MAX_HW_QUEUES, at most 32; 0: leave as set)")
    ap.add_argument("--serving-limit-s", type=float, default=720.0, help="serving: wall-clock cap of the run")
    ap.add_argument("--no-serial", action="store_true", help="parareal: skip the batched serial comparison run")
    ap.add_argument("--coarse-steps", type=int, default=0,
                    help="parareal: coarse IE steps per slice (0: the workload's 1; 8 = the level L-2 grid)")
    ap.add_argument("--stable-requests", type=int, default=64,
                    help="serving: requests of the stable-load run at 0.7 x the measured capacity (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library runs on one GPU only "
              "(samples would shard across GPUs with one final all-reduce of the level sums)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "serving" and args.hw_queues > 0:
        # two lanes (streams) per mesh size plus the wide lane: streams beyond the
        # process's hardware queues share one and run one after another
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
    import numpy as np
    import torch

    import workloads as W
    import paper_2507_19246_amd as mq
    from paper_2507_19246_amd import _lib as L

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        nbytes = 1 << 30
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": nbytes, "bytes_written": nbytes, "launches": 3}}))
        return
    if args.workload != "mlmc3":
        fn = {"parareal": bench_parareal, "nonlinear": bench_nonlinear, "serving": bench_serving,
              "adaptive": bench_adaptive, "combined": bench_combined}[args.workload]
        print(json.dumps(fn(args, mq, L, W, np, torch)), flush=True)
        return
    w = W.mlmc3_mixed_129()
    levels = [(lv.steps_per_period, lv.coarse_steps_per_period, lv.n_periods) for lv in w.levels]
    xis_np = [W.level_xi(w, l) for l in range(len(w.levels))]
    xis = [torch.tensor(x, dtype=torch.float64, device="cuda") for x in xis_np]
    # launch/solver knobs measured by the autotuner for this device (committed cache), else defaults
    from paper_2507_19246_amd import autotune
    prob, knobs = autotune.tuned_problem(w.problem, L.MQ_PREC_MIXED)
    nd = prob.n_dof

    def step():
        qfs, qcs, rc, st = mq.mlmc_multilevel_run(prob, levels, xis)
        e, y, v = mq.mlmc_estimate(qfs, qcs)
        return qfs, qcs, e, y, v, rc, st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step()
        stats.append(out[-1])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    qfs, qcs, e, y, v, rc, st = out
    sample_steps = sum(s["sample_steps"] for s in stats)
    value = sample_steps / elapsed
    pcie = None if args.no_host_buffers else host_buffer_rate(w, levels, xis_np, knobs, L, qfs, qcs)
    kern_ms = [s["kernel_ms"] for s in stats]
    avg_kern_s = sum(kern_ms) / len(kern_ms) / 1e3
    per_launch = lambda k: sum(s[k] for s in stats) / len(stats)
    inner_l, sweeps_l, steps_l = per_launch("inner_iters"), per_launch("sweeps"), per_launch("sample_steps")
    units = nd * inner_l   # DoF-iterations per launch
    resid_l = sweeps_l + steps_l   # FP64 residual passes: one per sweep plus the converged check
    alg_bytes = nd * (ALG_BYTES_CG_ITER_FP32 * inner_l + ALG_BYTES_FP64_RESIDUAL * resid_l + ALG_BYTES_STEP * steps_l)
    alg_gbs = alg_bytes / avg_kern_s / 1e9
    flops_unit = MG_FLOPS_PER_DOF_ITER if prob.info.precond == L.MQ_PRECOND_MULTIGRID else CG_FLOPS_PER_DOF_ITER
    achieved_tflops = flops_unit * units / avg_kern_s / 1e12
    prof = "ie_resident_mlmc3_129_hbm_counters.md"
    traffic = measured_traffic(prof)
    lds_bytes = profile_value("ie_resident_mlmc3_129_lds_counters.md", "lds_bytes_per_launch")

    # QoI error of the mixed path against FP64 references
    q_mixed = [q.cpu().numpy() for q in qfs]
    qc_mixed = [q.cpu().numpy() if q is not None else None for q in qcs]
    result = {}
    fp64 = None
    if not args.no_fp64_baseline:
        # plain FP64 GPU path: one sample per call over the whole device, grid-wide
        # Jacobi-preconditioned FP64 CG passes driven by a host loop (wide path, S = 1)
        p64 = mq.Problem(w.problem, L.MQ_PREC_FP64, path=L.MQ_PATH_WIDE, precond=L.MQ_PRECOND_JACOBI)
        lv = w.levels[0]
        nb = args.fp64_samples
        mq.mlmc_level_run(p64, lv.steps_per_period, 0, 1, xis[0][:1])  # warm-up (graph capture, buffers)
        lat, errs, steps64 = [], [], 0
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for s in range(nb):
            t1 = time.perf_counter()
            q64, _, _, _, st64 = mq.mlmc_level_run(p64, lv.steps_per_period, 0, lv.n_periods, xis[0][s:s + 1])
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t1)
            steps64 += st64["sample_steps"]
            errs.append(abs(float(q64[0]) - q_mixed[0][s]) / abs(float(q64[0])))
        wall64 = time.perf_counter() - tb
        p64.close()
        fp64 = {"value": steps64 / wall64, "unit": "sample-steps/s",
                "p50_latency_ms": 1e3 * float(np.percentile(lat, 50)),
                "p99_latency_ms": 1e3 * float(np.percentile(lat, 99)),
                "samples": nb, "sample_steps_each": lv.steps_per_period * lv.n_periods,
                "cg_iters_per_sample_step": st64["inner_iters"] / st64["sample_steps"],
                "path": "FP64 Jacobi-PCG, one sample per call over the whole device (grid-wide passes, "
                        "host-driven loop, batches of 4 iterations replayed from a captured graph); "
                        "level-0 samples of the same workload",
                "latency_definition": "call start to return (Q in device memory)",
                "qoi_max_rel_err_mixed_vs_fp64": max(errs)}
        result["plain_fp64_gpu"] = fp64

    cpu = None
    qerr_oracle = None
    if not args.no_cpu_baseline:
        cpu, oq = cpu_baseline(w, xis_np)
        errs = []
        for (l, s, kind), q in oq.items():
            g = q_mixed[l][s] if kind == "f" else qc_mixed[l][s]
            errs.append(abs(g - q) / abs(q))
        qerr_oracle = max(errs)

    res = {
        "metric": "sample-steps/s + p50/p99 sample latency vs plain FP64, QoI rel err <= 1e-6",
        "value": value,
        "unit": "sample-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "mesh": "129x129", "n_dof": nd,
                   "levels_steps_per_period": [lv.steps_per_period for lv in w.levels],
                   "n_periods": w.levels[0].n_periods,
                   "samples_per_level": [lv.n_samples for lv in w.levels],
                   "sample_steps_per_step": stats[-1]["sample_steps"],
                   "path": "resident" if stats[-1]["path"] == 1 else "streaming",
                   "launch": [stats[-1]["grid"], stats[-1]["block"]],
                   "knobs": dict(knobs, tile=prob.info.tile, precond=prob.info.precond)},
        "p50_latency_ms": st["lat_p50_ms"],
        "p99_latency_ms": st["lat_p99_ms"],
        "latency_definition": "per sample: call start on the host to its Q (fine and coupled coarse) "
                              "readable in host memory (completion records in coherent pinned memory, "
                              "polled during the launch); last timed step",
        "qoi_max_rel_err_vs_fp64_oracle": qerr_oracle,
        "mlmc_estimate": float(e),
        "cg_iters_per_sample_step": stats[-1]["inner_iters"] / stats[-1]["sample_steps"],
        "roofline": {"bound": "hbm", "achieved": alg_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg_gbs / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": ("k_ie_resident<float,128,%d,%d,64,%s>" % (
                         16 if prob.info.tile != 2 else 32, 8 if prob.info.tile != 2 else 4,
                         "multigrid" if prob.info.precond == L.MQ_PRECOND_MULTIGRID else "jacobi")),
                     "avg_launch_ms": 1e3 * avg_kern_s,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "bytes_per_dof": {"fp32_cg_iteration": ALG_BYTES_CG_ITER_FP32,
                                       "fp64_residual": ALG_BYTES_FP64_RESIDUAL, "time_step": ALG_BYTES_STEP},
                     "units_per_launch": {"dof": nd, "cg_iterations": inner_l, "fp64_residuals": resid_l,
                                          "sample_steps": steps_l},
                     "measured_hbm_gbs": None if traffic is None else traffic / avg_kern_s / 1e9,
                     "measured_hbm_frac": None if traffic is None else traffic / avg_kern_s / 1e9 / HBM_PEAK_GBS,
                     "note": "achieved = the algorithmic bytes of the work done (as if every vector were "
                             "streamed from HBM) per launch time; this kernel keeps the CG vectors in "
                             "registers and LDS, so measured HBM traffic (counters) is lower",
                     "on_chip": None if lds_bytes is None else {
                         "bound": "lds", "achieved": lds_bytes / avg_kern_s / 1e9, "peak": LDS_PEAK_GBS,
                         "unit": "GB/s", "frac": lds_bytes / avg_kern_s / 1e9 / LDS_PEAK_GBS,
                         "lds_bytes_per_launch": lds_bytes},
                     "alu": {"achieved": achieved_tflops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS, "flops_per_dof_iter": flops_unit},
                     "precond": "multigrid" if prob.info.precond == L.MQ_PRECOND_MULTIGRID else "jacobi"},
        "paper_context": PAPER_CONTEXT,
        "cpu_baseline": cpu,
        "pcie_inclusive": pcie,
    }
    res.update(result)
    if fp64:
        res["speedup_vs_plain_fp64"] = value / fp64["value"]
        res["p99_latency_vs_plain_fp64"] = st["lat_p99_ms"] / fp64["p99_latency_ms"]
    prob.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
