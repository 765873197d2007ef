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
