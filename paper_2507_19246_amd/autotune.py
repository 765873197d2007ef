"""Measured selection of the launch and solver knobs of one problem (autotuner).

For a mesh/material/precision the tuner times short level runs that fill the
device (two instances per compute unit, a few steps each) under every
candidate of:

* ``tile``: the workgroup shape (resident: 16 or 32 rows per thread where both
  exist; streaming: one 1024-thread or two 512-thread workgroups per CU),
* ``precond``: Jacobi scaling alone or the multigrid V-cycle,
* ``mg_omega``: the damped-Jacobi weight of the multigrid smoother,
* ``inner_rtol``: the relative tolerance of the inner CG (mixed precision),

then, for the best multigrid candidate, the depth of the coarse hierarchy
(``mg_levels``) and the damped-Jacobi sweeps at its coarsest level
(``mg_coarse_sweeps``), then the smoother weight and the inner tolerance again
with that hierarchy, and keeps the fastest candidate whose QoIs agree with the default
configuration's within the precision's tolerance (1e-6 mixed, 1e-10 FP64).
The outer tolerance, and so the accuracy of every result, is never tuned.

Results are cached in a JSON file keyed by device name, mesh, material and
precision (``MQ_AUTOTUNE_CACHE``, default ``tuned.json`` beside this module).
"""
from __future__ import annotations

import itertools
import json
import os
from typing import Dict, List, Optional

from . import _lib as L

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuned.json")

QOI_AGREEMENT = {L.MQ_PREC_MIXED: 1e-6, L.MQ_PREC_FP64: 1e-10}
# a candidate replaces the defaults only when it is this much faster
NOISE_MARGIN = 1.02


def cache_path() -> str:
    return os.environ.get("MQ_AUTOTUNE_CACHE", DEFAULT_CACHE)


def device_id() -> str:
    """Cache identity of device 0: architecture and compute-unit count (the
    marketing name depends on the host's device table and is not stable)."""
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = (getattr(p, "gcnArchName", "") or "").split(":")[0] or torch.cuda.get_device_name(0)
    return f"{arch}-{p.multi_processor_count}cu"


def cache_key(device: str, problem, precision: int) -> str:
    m = problem.material
    return f"{device}|n{problem.n_nodes}|mat{m.kind}|prec{precision}"


def _is_pow2_mesh(n_nodes: int) -> bool:
    n = n_nodes - 2
    return n >= 1 and ((n + 1) & n) == 0


def candidates(problem, precision: int) -> List[Dict]:
    """Knob combinations worth timing for this problem (host logic only)."""
    n = problem.n_nodes - 2
    # tile 2: 32 rows per thread on the resident path (64..127 interior nodes per
    # side), 512-thread workgroups (two per compute unit) on the streaming path
    tiles = [1, 2] if (64 <= n <= 127 or n > 127) else [1]
    preconds = [L.MQ_PRECOND_JACOBI]
    if _is_pow2_mesh(problem.n_nodes):
        # Jacobi CG needs O(n) iterations per step: on the streaming meshes
        # (n > 127) it is never competitive and only lengthens the tuning run
        preconds = [L.MQ_PRECOND_MULTIGRID] if n > 127 else preconds + [L.MQ_PRECOND_MULTIGRID]
    rtols = [1e-5, 3e-6, 1e-6] if precision == L.MQ_PREC_MIXED else [1e-10]
    out = []
    for tile, pc, rt in itertools.product(tiles, preconds, rtols):
        omegas = [0.7, 0.8, 0.9] if pc == L.MQ_PRECOND_MULTIGRID else [0.0]
        for om in omegas:
            out.append({"tile": tile, "precond": pc, "mg_omega": om, "inner_rtol": rt})
    return out


# second stage: coarse-hierarchy variants (levels in use, coarsest sweeps); the
# deeper ones only where the hierarchy has more levels than that
COARSE_VARIANTS = [(3, 4), (3, 6), (3, 8), (4, 2), (4, 4), (5, 2), (5, 4)]


def coarse_candidates(best_knobs: Dict, resolved_precond: int, n_nodes: int = 0) -> List[Dict]:
    if resolved_precond != L.MQ_PRECOND_MULTIGRID:
        return []
    n, depth = n_nodes - 2, 0
    while n > 1:  # levels below the fine one: n -> (n - 1) / 2 down to one node
        n = (n - 1) // 2
        depth += 1
    return [dict(best_knobs, mg_levels=lv, mg_coarse_sweeps=sw) for lv, sw in COARSE_VARIANTS
            if n_nodes == 0 or lv < depth]


def refine_candidates(best_knobs: Dict, resolved_precond: int, precision: int) -> List[Dict]:
    """Third stage: smoother weight x inner tolerance around a chosen coarse
    hierarchy (multigrid with an explicit hierarchy only)."""
    if resolved_precond != L.MQ_PRECOND_MULTIGRID or "mg_levels" not in best_knobs:
        return []
    rtols = [1e-5, 3e-6, 1e-6] if precision == L.MQ_PREC_MIXED else [1e-10]
    out = []
    for om, rt in itertools.product([0.7, 0.8, 0.9], rtols):
        k = dict(best_knobs, mg_omega=om, inner_rtol=rt)
        if k != best_knobs:
            out.append(k)
    return out


def _load(path: str) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(problem, precision: int, device: Optional[str] = None, path: Optional[str] = None) -> Optional[Dict]:
    """Cached knobs for this problem, or None."""
    import torch
    device = device or device_id()
    return _load(path or cache_path()).get(cache_key(device, problem, precision), {}).get("knobs")


def autotune(problem, precision: int, steps_per_period: int = 32, n_periods: int = 1,
             n_samples: Optional[int] = None, force: bool = False, path: Optional[str] = None,
             verbose: bool = False) -> Dict:
    """Return the fastest agreeing knobs (from the cache unless force)."""
    import numpy as np
    import torch

    from . import api as mq

    path = path or cache_path()
    device = device_id()
    key = cache_key(device, problem, precision)
    db = _load(path)
    if not force and key in db:
        return db[key]["knobs"]
    base = mq.Problem(problem, precision)
    n_xi = base.n_xi
    base.close()
    if n_samples is None:
        # fill the device: two instances per compute unit (the most slots any shape has)
        n_samples = 2 * torch.cuda.get_device_properties(0).multi_processor_count
    gen = torch.Generator().manual_seed(99)
    xi = torch.randn(n_samples, n_xi, generator=gen, dtype=torch.float64).to("cuda")
    tol = QOI_AGREEMENT[precision]
    ref_q = [None]
    trials = []

    def trial(knobs):
        try:
            p = mq.Problem(problem, precision, **knobs)
        except L.MQError:
            return  # this combination does not exist for the mesh (e.g. no room in LDS)
        mq.mlmc_level_run(p, steps_per_period, 0, n_periods, xi[:8])  # warm-up (code objects)
        dt = float("inf")
        for _ in range(2):  # best kernel time of two runs
            q, _, _, rc, st = mq.mlmc_level_run(p, steps_per_period, 0, n_periods, xi)
            dt = min(dt, st["kernel_ms"] / 1e3)
        qh = q.cpu().numpy()
        info = {"tile": p.info.tile, "precond": p.info.precond, "block": p.info.block}
        p.close()
        if ref_q[0] is None:
            ref_q[0] = qh
        agree = bool(np.all(np.abs(qh - ref_q[0]) <= tol * np.abs(ref_q[0]))) and rc == 0
        rate = st["sample_steps"] / dt
        trials.append({"knobs": knobs, "rate": rate, "agree": agree, "resolved": info})
        if verbose:
            print(f"autotune {key} {knobs} -> {rate:.0f} sample-steps/s agree={agree}", flush=True)

    for knobs in [{}] + candidates(problem, precision):
        trial(knobs)
    best = max((t for t in trials if t["agree"]), key=lambda t: t["rate"])
    for knobs in coarse_candidates(best["knobs"], best["resolved"]["precond"], problem.n_nodes):
        trial(knobs)
    best = max((t for t in trials if t["agree"]), key=lambda t: t["rate"])
    # third stage: the smoother weight and the inner tolerance again, with the
    # chosen coarse hierarchy (the first stage timed them with the default one,
    # and the best weight depends on how many coarsest sweeps follow)
    for knobs in refine_candidates(best["knobs"], best["resolved"]["precond"], precision):
        trial(knobs)
    best = max((t for t in trials if t["agree"]), key=lambda t: t["rate"])
    if best["rate"] < NOISE_MARGIN * trials[0]["rate"]:
        best = trials[0]  # within the timing noise of the defaults: keep them
    db = _load(path)
    db[key] = {"knobs": best["knobs"], "rate": best["rate"], "default_rate": trials[0]["rate"],
               "resolved": best["resolved"], "trials": len(trials),
               "probe": {"samples": n_samples, "steps_per_period": steps_per_period, "n_periods": n_periods}}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return best["knobs"]


def tuned_problem(problem, precision: int, tune: bool = False, **override):
    """A Problem with the cached knobs (tuning first when asked and not cached)."""
    from . import api as mq
    knobs = autotune(problem, precision) if tune else (lookup(problem, precision) or {})
    knobs = dict(knobs)
    knobs.update(override)
    return mq.Problem(problem, precision, **knobs), knobs
