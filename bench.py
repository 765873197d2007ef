#!/usr/bin/env python3
"""Throughput / latency benchmark of the batched MLMC hot path on one MI355X.

Workload: MLMC with 3 time levels on the 129x129-node eddy-current model
(KL-8 lognormal conductivity, 64/128/256 steps per period over 4 periods,
512/128/32 samples, coupled level differences), FP32 CG inside FP64
iterative refinement.  One benchmark step = one full MLMC estimate: device
assembly of every sample, all implicit-Euler runs of all levels in one
persistent launch, the Joule-loss QoIs and the estimator of Eq. (9).
Inputs (xi) are resident in device memory before the timed region.

Printed: one JSON line with sample-steps/s (whole job), p50/p99 per-sample
latency, QoI error against the FP64 oracle and against the plain FP64 GPU
path (one sample per launch), the roofline of the dominant kernel and the
oracle timed on the host cores.
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


def _kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    h.update(open(os.path.join(ROOT, "paper_2507_19246_amd", "csrc", "kernels.hip"), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(name: str):
    """HBM bytes per launch from the committed counter summary, or None when the
    kernel source changed since the counters were taken."""
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
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _oracle_task(args):
    """One oracle solve (runs in a worker process with one BLAS thread)."""
    problem, xi, spp, nper = args
    from oracle import timestep
    t = time.perf_counter()
    q, _ = timestep.solve_sample(problem, xi, spp, nper)
    return q, spp * nper, time.perf_counter() - t


def cpu_baseline(w, xis, n_per_level=(4, 1, 1)):
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(samples would shard across GPUs with one final all-reduce of the level sums)",
              file=sys.stderr)
        sys.exit(2)

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
    w = W.mlmc3_mixed_129()
    levels = [(lv.steps_per_period, lv.coarse_steps_per_period, lv.n_periods) for lv in w.levels]
    xis_np = [W.level_xi(w, l) for l in range(len(w.levels))]
    xis = [torch.tensor(x, dtype=torch.float64, device="cuda") for x in xis_np]
    prob = mq.Problem(w.problem, L.MQ_PREC_MIXED)
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
    kern_ms = [s["kernel_ms"] for s in stats]
    avg_kern_s = sum(kern_ms) / len(kern_ms) / 1e3
    units = nd * (sum(s["inner_iters"] for s in stats) / len(stats))   # DoF-iterations per launch
    flops_unit = MG_FLOPS_PER_DOF_ITER if prob.info.precond == L.MQ_PRECOND_MULTIGRID else CG_FLOPS_PER_DOF_ITER
    achieved_tflops = flops_unit * units / avg_kern_s / 1e12
    traffic = measured_traffic("ie_resident_mlmc3_129_hbm_counters.md")

    # QoI error of the mixed path against FP64 references
    q_mixed = [q.cpu().numpy() for q in qfs]
    qc_mixed = [q.cpu().numpy() if q is not None else None for q in qcs]
    result = {}
    fp64 = None
    if not args.no_fp64_baseline:
        # plain FP64 GPU path: one sample per launch, FP64 CG (streaming kernel, S = 1)
        p64 = mq.Problem(w.problem, L.MQ_PREC_FP64)
        lv = w.levels[0]
        nb = 4
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
                "samples": nb, "path": "FP64 CG, one sample per launch, streaming kernel",
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
                   "launch": [stats[-1]["grid"], stats[-1]["block"]]},
        "p50_latency_ms": st["lat_p50_ms"],
        "p99_latency_ms": st["lat_p99_ms"],
        "qoi_max_rel_err_vs_fp64_oracle": qerr_oracle,
        "mlmc_estimate": float(e),
        "cg_iters_per_sample_step": stats[-1]["inner_iters"] / stats[-1]["sample_steps"],
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": traffic,
                     "kernel": "k_ie_resident<float,128,16,8,64,multigrid>",
                     "avg_launch_ms": 1e3 * avg_kern_s,
                     "flops_per_dof_iter": flops_unit,
                     "precond": "multigrid" if prob.info.precond == L.MQ_PRECOND_MULTIGRID else "jacobi",
                     "dof_iters_per_launch": units,
                     "hbm_equivalent_gbs": CG_BYTES_PER_DOF_ITER_FP32 * units / avg_kern_s / 1e9},
        "cpu_baseline": cpu,
    }
    res.update(result)
    if fp64:
        res["speedup_vs_plain_fp64"] = value / fp64["value"]
    prob.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
