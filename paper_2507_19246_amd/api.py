"""Thin torch-facing wrappers of the libmq C ABI (marshalling only)."""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import torch

from . import _lib as L

# Solver defaults per precision: (outer FP64 tolerance on ||b - A d|| / ||b||,
# inner CG relative tolerance, inner iteration cap, refinement sweep cap).
SOLVER_DEFAULTS = {
    L.MQ_PREC_FP64: dict(tol=1e-13, inner_rtol=1e-10, max_iter=20000, max_sweeps=10),
    L.MQ_PREC_MIXED: dict(tol=1e-7, inner_rtol=1e-5, max_iter=20000, max_sweeps=10),
}


def default_desc(problem, precision: int, path: int = L.MQ_PATH_AUTO, **solver) -> L.ProblemDesc:
    """Fill the C problem description from a `workloads.Problem`."""
    m = problem.material
    d = L.ProblemDesc()
    d.n_nodes = problem.n_nodes
    d.material = m.kind
    d.precision = precision
    d.path = path
    for i, v in enumerate(problem.conductor):
        d.conductor[i] = v
    d.strip[0], d.strip[1] = problem.strip
    d.J0, d.freq = problem.J0, problem.freq
    d.sigma0, d.nu_cond, d.nu_air = m.sigma0, m.nu_cond, m.nu_air
    d.s_sigma, d.s_nu = m.s_sigma, m.s_nu
    d.n_modes, d.corr_len, d.s_kl = m.n_modes, m.corr_len, m.s_kl
    d.k1, d.k2, d.k3, d.s_k = m.k1, m.k2, m.k3, m.s_k
    d.picard_tol, d.picard_max = m.picard_tol, m.picard_max
    sv = dict(SOLVER_DEFAULTS[precision])
    sv.update(solver)
    d.tol, d.inner_rtol = sv["tol"], sv["inner_rtol"]
    d.max_iter, d.max_sweeps = sv["max_iter"], sv["max_sweeps"]
    d.precond = sv.get("precond", L.MQ_PRECOND_AUTO)
    d.tile = sv.get("tile", 0)
    d.mg_levels = sv.get("mg_levels", 0)
    d.mg_coarse_sweeps = sv.get("mg_coarse_sweeps", 0)
    d.split_steps = sv.get("split_steps", 0)
    d.mg_block_min = sv.get("mg_block_min", 0)
    d.mg_omega = sv.get("mg_omega", 0.0)
    d.mem_kind = sv.get("mem_kind", L.MQ_MEM_DEVICE)
    d.mass = sv.get("mass", L.MQ_MASS_CONSISTENT)
    return d


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f64(x, shape=None) -> torch.Tensor:
    t = torch.as_tensor(x, dtype=torch.float64)
    if shape is not None:
        t = t.reshape(shape)
    return t.to("cuda").contiguous()


class Problem:
    """Handle of one mesh/material/solver set-up (fem_setup)."""

    def __init__(self, problem, precision: int, path: int = L.MQ_PATH_AUTO, **solver):
        self.lib = L.load()
        self.spec = problem
        self.desc = default_desc(problem, precision, path, **solver)
        h = C.c_void_p()
        L.check(self.lib.fem_setup(C.byref(self.desc), _stream(), C.byref(h)))
        self.h = h
        info = L.ProblemInfo()
        L.check(self.lib.mq_problem_info_get(self.h, C.byref(info)))
        self.info = info
        self.n_dof = info.n_dof
        self.n_xi = info.n_xi

    def close(self):
        if getattr(self, "h", None):
            self.lib.mq_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_initial_state(self, a0=None):
        """a(t_0) of every later run on this handle (interior DoF order); None: zeros."""
        if a0 is None:
            L.check(self.lib.mq_set_initial_state(self.h, None))
            return
        a = _dev_f64(a0).reshape(-1)
        if a.numel() != self.n_dof:
            raise ValueError(f"a0 has {a.numel()} values, the problem has {self.n_dof} DoF")
        L.check(self.lib.mq_set_initial_state(self.h, _ptr(a)))

    @property
    def path(self) -> int:
        if self.desc.path == L.MQ_PATH_WIDE:
            return L.MQ_PATH_WIDE
        return L.MQ_PATH_RESIDENT if (self.desc.path != L.MQ_PATH_STREAMING and self.info.resident_ok) else L.MQ_PATH_STREAMING


def mlmc_level_run(prob: Problem, steps_per_period: int, coarse_steps_per_period: int, n_periods: int,
                   xi, want_state: bool = False):
    """Returns (q_fine, q_coarse or None, final_state or None, status, stats dict)."""
    xi_d = _dev_f64(xi).reshape(-1, prob.n_xi).contiguous()
    n = xi_d.shape[0]
    qf = torch.empty(n, dtype=torch.float64, device="cuda")
    qc = torch.empty(n, dtype=torch.float64, device="cuda") if coarse_steps_per_period > 0 else None
    fs = torch.empty((n, prob.n_dof), dtype=torch.float64, device="cuda") if want_state else None
    lv = L.LevelDesc(steps_per_period, coarse_steps_per_period, n_periods, 0)
    st = L.RunStats()
    rc = L.check(prob.lib.mlmc_level_run(prob.h, C.byref(lv), n, _ptr(xi_d), _ptr(qf), _ptr(qc),
                                         _ptr(fs), C.byref(st)))
    return qf, qc, fs, rc, st.as_dict()


def mlmc_multilevel_run(prob: Problem, levels: Sequence, xis: Sequence):
    """All levels in one persistent launch.  levels: (spp, coarse_spp, n_periods) tuples.
    Returns (list of q_fine, list of q_coarse or None, status, stats)."""
    nl = len(levels)
    lvs = (L.LevelDesc * nl)()
    ns = (C.c_int32 * nl)()
    xs, qfs, qcs = [], [], []
    for l, (spp, cspp, nper) in enumerate(levels):
        lvs[l] = L.LevelDesc(spp, cspp, nper, 0)
        x = _dev_f64(xis[l]).reshape(-1, prob.n_xi).contiguous()
        ns[l] = x.shape[0]
        xs.append(x)
        qfs.append(torch.empty(x.shape[0], dtype=torch.float64, device="cuda"))
        qcs.append(torch.empty(x.shape[0], dtype=torch.float64, device="cuda") if cspp > 0 else None)
    px = (C.c_void_p * nl)(*[x.data_ptr() for x in xs])
    pf = (C.c_void_p * nl)(*[q.data_ptr() for q in qfs])
    pc = (C.c_void_p * nl)(*[(q.data_ptr() if q is not None else None) for q in qcs])
    st = L.RunStats()
    rc = L.check(prob.lib.mlmc_multilevel_run(prob.h, nl, lvs, ns, px, pf, pc, C.byref(st)))
    return qfs, qcs, rc, st.as_dict()


def mlmc_multimesh_run(probs: Sequence[Problem], levels: Sequence, xis: Sequence):
    """Level l on the mesh of probs[l], its coupled coarse run on probs[l - 1]'s mesh.
    Returns (list of q_fine, list of q_coarse or None, status, stats)."""
    nl = len(levels)
    lib = probs[0].lib
    hs = (C.c_void_p * nl)(*[p.h.value for p in probs])
    lvs = (L.LevelDesc * nl)(*[L.LevelDesc(a, b, c, 0) for a, b, c in levels])
    xs = [_dev_f64(x).reshape(-1, probs[0].n_xi).contiguous() for x in xis]
    ns = (C.c_int32 * nl)(*[x.shape[0] for x in xs])
    qfs = [torch.empty(x.shape[0], dtype=torch.float64, device="cuda") for x in xs]
    qcs = [torch.empty(x.shape[0], dtype=torch.float64, device="cuda") if l > 0 else None
           for l, x in enumerate(xs)]
    px = (C.c_void_p * nl)(*[x.data_ptr() for x in xs])
    pf = (C.c_void_p * nl)(*[q.data_ptr() for q in qfs])
    pc = (C.c_void_p * nl)(*[(q.data_ptr() if q is not None else None) for q in qcs])
    st = L.RunStats()
    rc = L.check(lib.mlmc_multimesh_run(nl, hs, lvs, ns, px, pf, pc, C.byref(st)))
    return qfs, qcs, rc, st.as_dict()


def mlmc_adaptive_run(prob: Problem, levels: Sequence, xi_pools: Sequence, target_rmse: float,
                      n_pilot: int = 32, var_fraction: float = 0.5, max_rounds: int = 10):
    """Adaptive MLMC (Eq. (11)) over per-level input pools xi_pools[l] ([n_max_l, n_xi]).
    Returns (E, level means, level variances, samples used per level, q_fine, q_coarse, status, stats)."""
    nl = len(levels)
    lvs = (L.LevelDesc * nl)(*[L.LevelDesc(a, b, c, 0) for a, b, c in levels])
    xs = [_dev_f64(x).reshape(-1, prob.n_xi).contiguous() for x in xi_pools]
    nmax = (C.c_int32 * nl)(*[x.shape[0] for x in xs])
    qfs = [torch.empty(x.shape[0], dtype=torch.float64, device="cuda") for x in xs]
    qcs = [torch.empty(x.shape[0], dtype=torch.float64, device="cuda") for x in xs]
    px = (C.c_void_p * nl)(*[x.data_ptr() for x in xs])
    pf = (C.c_void_p * nl)(*[q.data_ptr() for q in qfs])
    pc = (C.c_void_p * nl)(*[q.data_ptr() for q in qcs])
    ad = L.AdaptiveDesc(target_rmse, var_fraction, n_pilot, max_rounds)
    used = (C.c_int32 * nl)()
    out = (C.c_double * (1 + 2 * nl))()
    st = L.RunStats()
    rc = L.check(prob.lib.mlmc_adaptive_run(prob.h, nl, lvs, nmax, px, pf, pc, C.byref(ad), used, out,
                                            C.byref(st)))
    n = [used[i] for i in range(nl)]
    return (out[0], list(out[1:1 + nl]), list(out[1 + nl:]), n, [q[:k] for q, k in zip(qfs, n)],
            [q[:k] if l > 0 else None for l, (q, k) in enumerate(zip(qcs, n))], rc, st.as_dict())


def mlmc_combined_run(prob: Problem, levels: Sequence, xis: Sequence, n_slices: int = 0,
                      coarse_steps_per_period: int = 0, k_max: int = 0, tol: float = 1e-8):
    """MLMC with Parareal on the finest level (mlmc_combined_run).  Returns (list of
    q_fine, list of q_coarse (None at level 0), Parareal K per finest-level sample,
    status, run stats, combined-run stats)."""
    nl = len(levels)
    lvs = (L.LevelDesc * nl)(*[L.LevelDesc(a, b, c, 0) for a, b, c in levels])
    xs = [_dev_f64(x).reshape(-1, prob.n_xi).contiguous() for x in xis]
    ns = (C.c_int32 * nl)(*[x.shape[0] for x in xs])
    qfs = [torch.empty(x.shape[0], dtype=torch.float64, device="cuda") for x in xs]
    qcs = [torch.empty(x.shape[0], dtype=torch.float64, device="cuda") if l > 0 else None
           for l, x in enumerate(xs)]
    it = torch.zeros(xs[-1].shape[0], dtype=torch.int32, device="cuda")
    px = (C.c_void_p * nl)(*[x.data_ptr() for x in xs])
    pf = (C.c_void_p * nl)(*[q.data_ptr() for q in qfs])
    pc = (C.c_void_p * nl)(*[(q.data_ptr() if q is not None else None) for q in qcs])
    cd = L.CombinedDesc(n_slices, coarse_steps_per_period, k_max, 0, tol)
    st, cs = L.RunStats(), L.CombinedStats()
    rc = L.check(prob.lib.mlmc_combined_run(prob.h, nl, lvs, ns, px, C.byref(cd), pf, pc, _ptr(it),
                                            C.byref(st), C.byref(cs)))
    return qfs, qcs, it, rc, st.as_dict(), cs.as_dict()


def plan_split(steps: Sequence[int], slots: int, split_steps: int = 0) -> dict:
    """The tail-splitting plan of a launch (mq_plan_split, host arithmetic): lists
    orig, first, len, dep per launch entry and the simulated makespans (steps)."""
    lib = L.load()
    n = len(steps)
    st = (C.c_int32 * max(n, 1))(*steps)
    m = C.c_int32()
    mk = (C.c_double * 2)()
    L.check(lib.mq_plan_split(n, st, slots, split_steps, 0, None, None, None, None, mk, C.byref(m)))
    cap = m.value
    arrs = [(C.c_int32 * max(cap, 1))() for _ in range(4)]
    L.check(lib.mq_plan_split(n, st, slots, split_steps, cap, *arrs, mk, C.byref(m)))
    o, f, ln, d = ([int(x) for x in a[:cap]] for a in arrs)
    return {"orig": o, "first": f, "len": ln, "dep": d, "makespan": (mk[0], mk[1])}


def cost_model(C_l: Sequence[float], N_l: Sequence[float], K: int, M: int, n_cores: int) -> dict:
    """The combined method's cost model (mq_cost_model): Eqs. (15)-(19), (21)-(25)."""
    lib = L.load()
    ci = L.CostIn()
    ci.n_levels, ci.K, ci.M, ci.n_cores = len(C_l), K, M, n_cores
    for i, (c, n) in enumerate(zip(C_l, N_l)):
        ci.C[i], ci.N[i] = float(c), float(n)
    co = L.CostOut()
    L.check(lib.mq_cost_model(C.byref(ci), C.byref(co)))
    out = {f: getattr(co, f) for f, _ in co._fields_ if f != "batches"}
    out["batches"] = list(co.batches[:len(C_l)])
    return out


def parareal_run(prob: Problem, n_periods: int, n_slices: int, fine_steps_per_slice: int,
                 coarse_steps_per_slice: int, k_max: int, tol: float, xi, fixed_k: int = 0,
                 want_state: bool = False):
    """Returns (q, iters, final_state or None, status, stats)."""
    xi_d = _dev_f64(xi).reshape(-1, prob.n_xi).contiguous()
    n = xi_d.shape[0]
    q = torch.empty(n, dtype=torch.float64, device="cuda")
    it = torch.empty(n, dtype=torch.int32, device="cuda")
    fs = torch.empty((n, prob.n_dof), dtype=torch.float64, device="cuda") if want_state else None
    pd = L.PararealDesc(n_periods, n_slices, fine_steps_per_slice, coarse_steps_per_slice, k_max,
                        fixed_k, tol)
    st = L.RunStats()
    rc = L.check(prob.lib.parareal_run(prob.h, C.byref(pd), n, _ptr(xi_d), _ptr(q), _ptr(it),
                                       _ptr(fs), C.byref(st)))
    return q, it, fs, rc, st.as_dict()


def last_flags():
    """Per-instance MQ_FLAG_* bits of this thread's last level, multilevel or
    Parareal run (numpy int32; order as documented for mq_last_flags)."""
    import numpy as np
    lib = L.load()
    n = C.c_int64()
    L.check(lib.mq_last_flags(None, 0, C.byref(n)))
    out = np.zeros(n.value, dtype=np.int32)
    if n.value:
        L.check(lib.mq_last_flags(out.ctypes.data_as(C.POINTER(C.c_int32)), n.value, C.byref(n)))
    return out


def mlmc_estimate(q_fine: Sequence[torch.Tensor], q_coarse: Sequence[Optional[torch.Tensor]]):
    """Eq. (9) on the device: returns (E, level means, level variances) as a float64 tensor split."""
    lib = L.load()
    nl = len(q_fine)
    ns = (C.c_int32 * nl)(*[int(q.numel()) for q in q_fine])
    pf = (C.c_void_p * nl)(*[q.data_ptr() for q in q_fine])
    pc = (C.c_void_p * nl)(*[(q.data_ptr() if q is not None else None) for q in q_coarse])
    out = torch.empty(1 + 2 * nl, dtype=torch.float64, device="cuda")
    L.check(lib.mlmc_estimate(nl, ns, pf, pc, _ptr(out), _stream()))
    return out[0], out[1:1 + nl], out[1 + nl:]


def debug_apply(prob: Problem, which: int, dt: float, xi, x) -> torch.Tensor:
    xi_d = _dev_f64(xi).reshape(-1, prob.n_xi).contiguous()
    n = xi_d.shape[0]
    x_d = _dev_f64(x).reshape(n, prob.n_dof).contiguous()
    y = torch.empty_like(x_d)
    L.check(prob.lib.mq_debug_apply(prob.h, which, dt, n, _ptr(xi_d), _ptr(x_d), _ptr(y)))
    return y


class Server:
    """Continuous-batching request server (mq_server_*)."""

    def __init__(self, base_problem, precision: int, hbm_budget_bytes: int, max_inflight: int = 1024,
                 n_streams: int = 2, max_batch: int = 0, chunk_steps: int = 0, wide_min_nodes: int = 0,
                 wide_queue: int = 0, wide_load_limit: int = 0, **solver):
        self.lib = L.load()
        sd = L.ServerDesc()
        sd.base = default_desc(base_problem, precision, **solver)
        sd.hbm_budget_bytes = int(hbm_budget_bytes)
        sd.max_inflight = max_inflight
        sd.n_streams = n_streams
        sd.max_batch = max_batch
        sd.chunk_steps = chunk_steps
        sd.wide_min_nodes = wide_min_nodes
        sd.wide_queue = wide_queue
        sd.wide_load_limit = wide_load_limit
        self.desc = sd
        h = C.c_void_p()
        L.check(self.lib.mq_server_create(C.byref(sd), _stream(), C.byref(h)))
        self.h = h

    def submit(self, n_nodes: int, steps_per_period: int, n_periods: int, xi, user_id: int = 0) -> int:
        rq = L.Request()
        rq.n_nodes, rq.steps_per_period, rq.n_periods = n_nodes, steps_per_period, n_periods
        rq.n_xi = len(xi)
        for i, v in enumerate(xi):
            rq.xi[i] = float(v)
        rq.user_id = user_id
        t = C.c_uint64()
        L.check(self.lib.mq_submit(self.h, C.byref(rq), C.byref(t)))
        return t.value

    def poll(self, cap: int = 256):
        buf = (L.Result * cap)()
        n = C.c_int32()
        L.check(self.lib.mq_poll(self.h, buf, cap, C.byref(n)))
        return [buf[i] for i in range(n.value)]

    def pending(self) -> int:
        n = C.c_int32()
        L.check(self.lib.mq_server_pending(self.h, C.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.mq_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
