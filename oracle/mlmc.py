"""Monte Carlo and Multi-Level Monte Carlo estimators (oracle).

Section II-B.  Plain MC, Eq. (8): E_MC = (1/N) sum_k Q^(k).
MLMC over time levels, Eq. (9): every sample drawn for level l is solved
on level l and on level l-1 with the same input xi (Q_{-1} = 0), and
    E_MLMC = sum_l (1/N_l) sum_k [Q_l^(k,l) - Q_{l-1}^(k,l)].
Level variances V_l (needed by Eq. (11)) use the unbiased N_l - 1 form.
Sums run left to right in sample order.
"""
from __future__ import annotations

import numpy as np

from . import mesh as meshmod, picard, timestep


def level_run(problem, steps_per_period: int, coarse_steps_per_period: int, n_periods: int,
              xi: np.ndarray, m=None):
    """Coupled (l, l-1) QoIs for every row of xi; q_coarse is None at level 0."""
    if m is None:
        m = meshmod.build(problem.n_nodes)
    tab = timestep.kl_table_for(problem, m)
    solve = picard.solve_sample if problem.material.kind == 2 else timestep.solve_sample
    qf = np.empty(len(xi))
    qc = np.empty(len(xi)) if coarse_steps_per_period > 0 else None
    for k, x in enumerate(xi):
        qf[k] = solve(problem, x, steps_per_period, n_periods, m=m, kl_table=tab)[0]
        if qc is not None:
            qc[k] = solve(problem, x, coarse_steps_per_period, n_periods, m=m, kl_table=tab)[0]
    return qf, qc


def estimate(q_fine, q_coarse):
    """Eq. (9): returns (E, level means Y_l, level variances V_l)."""
    means, var = [], []
    for l, qf in enumerate(q_fine):
        qf = np.asarray(qf, dtype=np.float64)
        qc = q_coarse[l]
        dq = qf.copy() if (l == 0 or qc is None) else qf - np.asarray(qc, dtype=np.float64)
        s = 0.0
        for v in dq:
            s += v
        y = s / len(dq)
        ss = 0.0
        for v in dq:
            ss += (v - y) * (v - y)
        means.append(y)
        var.append(ss / (len(dq) - 1) if len(dq) > 1 else 0.0)
    e = 0.0
    for y in means:
        e += y
    return e, np.asarray(means), np.asarray(var)


def optimal_samples(V, C, eps: float, theta: float = 0.5):
    """Eq. (11): N_l proportional to sqrt(V_l / C_l).

    The constant comes from the optimisation the paper cites: minimise the
    cost sum_l N_l C_l subject to the estimator variance sum_l V_l / N_l =
    theta eps^2 (theta: share of the squared RMSE eps^2 given to the
    statistical error).  The Lagrange conditions give
        N_l = sqrt(V_l / C_l) * sum_k sqrt(V_k C_k) / (theta eps^2),
    returned rounded up (0 where V_l = 0)."""
    V = np.asarray(V, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    s = 0.0
    for v, c in zip(V, C):
        s += np.sqrt(v * c)
    return np.array([int(np.ceil(np.sqrt(v / c) * s / (theta * eps * eps))) if v > 0 else 0
                     for v, c in zip(V, C)], dtype=np.int64)


def adaptive(q_of, C, eps: float, n_pilot: int, n_max, theta: float = 0.5, max_rounds: int = 10):
    """Adaptive MLMC (Section II-B): the level variances are estimated at run
    time.  Start with n_pilot samples per level; each round adds, on every
    level at once, the samples that Eq. (11) asks for given the current
    variance estimates (never fewer than already taken, at most n_max[l]);
    stop when no level asks for more.

    q_of(l, k0, k1) returns (q_fine, q_coarse or None) for samples k0..k1-1 of
    level l.  Returns (E, Y, V, N, rounds)."""
    L = len(C)
    qf = [np.empty(0) for _ in range(L)]
    qc = [None if l == 0 else np.empty(0) for l in range(L)]
    have = [0] * L
    need = [min(n_pilot, n_max[l]) for l in range(L)]
    rounds = 0
    while True:
        rounds += 1
        for l in range(L):
            if need[l] > have[l]:
                f, c = q_of(l, have[l], need[l])
                qf[l] = np.concatenate([qf[l], f])
                if l > 0:
                    qc[l] = np.concatenate([qc[l], c])
                have[l] = need[l]
        e, y, v = estimate(qf, qc)
        opt = optimal_samples(v, C, eps, theta)
        need = [max(have[l], min(int(opt[l]), n_max[l])) for l in range(L)]
        if need == have or rounds >= max_rounds:
            return e, y, v, np.array(have), rounds
