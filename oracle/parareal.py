"""Sequential Parareal for one sample (oracle).

Section II-C, Eq. (12):
    U_n^(k+1) = F(T_n, T_{n-1}, U_{n-1}^(k))
                + [C(T_n, T_{n-1}, U_{n-1}^(k+1)) - C(T_n, T_{n-1}, U_{n-1}^(k))],
with the active window of the paper: in iteration j the fine propagator
runs on slices j..M and the coarse one on slices j..M-1 (the first j-1
slices are already exact).  The correction is bracketed as F + (C_new -
C_old) so that an unchanged input gives exactly F.

Sweep order, for j = 1, 2, ...:
  1. fine: for n = j..M, F_n = F(U_{n-1}) and the slice's Joule-loss sum q_n;
  2. jump: J_j = max_{n=j..M-1} ||F_n - U_n||_2 / ||F_n||_2; stop when
     J_j <= tol, j = k_max or j = M (K = j);
  3. correct: for n = j..M-1 in order, U_n <- F_n + (C(U_{n-1}^new) - C_old[n]),
     where C(U_{j-1}) is unchanged and reused, so the coarse propagator is
     evaluated M-j-1 times (the initial coarse pass, M-1 evaluations, is the
     coarse work of iteration 1): the counts of Eqs. (13)-(14).
Q = sum_n q_n / T with q_n from each slice's latest fine run.
F and C are implicit Euler (``timestep.Stepper``) with dt_F and dt_C; the
source is evaluated at global times.
"""
from __future__ import annotations

import numpy as np

from . import mesh as meshmod, timestep


def run(problem, xi, n_periods: int, n_slices: int, fine_steps_per_slice: int,
        coarse_steps_per_slice: int, k_max: int, tol: float, fixed_k: int = 0,
        m=None, kl_table=None, trace=None, a0=None):
    """Returns dict(Q, K, state=U_M, jumps=[...], U=[U_0..U_M], fine_evals, coarse_evals)."""
    if m is None:
        m = meshmod.build(problem.n_nodes)
    if kl_table is None:
        kl_table = timestep.kl_table_for(problem, m)
    sysm = timestep.build_system(problem, xi, m, kl_table)
    T = n_periods * problem.period
    Ms = n_slices
    dt_f = T / (Ms * fine_steps_per_slice)
    dt_c = T / (Ms * coarse_steps_per_slice)
    Fst = timestep.Stepper(sysm, dt_f)
    Cst = timestep.Stepper(sysm, dt_c)

    def F(n, u):       # slice n = 1..M, from T_{n-1}
        return Fst.run(u, fine_steps_per_slice, (n - 1) * fine_steps_per_slice)

    def C(n, u):
        return Cst.run(u, coarse_steps_per_slice, (n - 1) * coarse_steps_per_slice)[0]

    nd = m.n_dof
    U = [np.zeros(nd) if a0 is None else np.array(a0, dtype=np.float64)] + [None] * Ms
    # U[n] is the initial value of slice n+1 (U[0] = a(T_0))
    c_old = [None] * (Ms + 1)                 # c_old[n] = C(n, U[n-1])
    coarse_evals = 0
    for n in range(1, Ms):
        c_old[n] = C(n, U[n - 1])
        coarse_evals += 1
        U[n] = c_old[n]
    q = np.zeros(Ms + 1)
    Fend = [None] * (Ms + 1)
    jumps = []
    fine_evals = 0
    K = 0
    kcap = min(k_max, Ms)
    if fixed_k:
        kcap = min(fixed_k, Ms)
    for j in range(1, kcap + 1):
        for n in range(j, Ms + 1):
            Fend[n], q[n] = F(n, U[n - 1])
            fine_evals += 1
        J = 0.0
        for n in range(j, Ms):
            J = max(J, float(np.linalg.norm(Fend[n] - U[n]) / np.linalg.norm(Fend[n])))
        jumps.append(J)
        K = j
        if trace is not None:
            trace.append([u.copy() if u is not None else None for u in U])
        if (not fixed_k and J <= tol) or j == kcap:
            break
        # correction sweep; slice j's input is unchanged, so C(j, U[j-1]) = c_old[j]
        newU = list(U)
        newU[j] = Fend[j] + (c_old[j] - c_old[j])
        for n in range(j + 1, Ms):
            c_new = C(n, newU[n - 1])
            coarse_evals += 1
            newU[n] = Fend[n] + (c_new - c_old[n])
            c_old[n] = c_new
        U = newU
    s = 0.0
    for n in range(1, Ms + 1):
        s += q[n]
    return dict(Q=s / T, K=K, state=Fend[Ms], jumps=jumps, U=U, fine_evals=fine_evals,
                coarse_evals=coarse_evals, q_slices=q[1:].copy())


def serial_fine(problem, xi, n_periods, n_slices, fine_steps_per_slice, m=None, kl_table=None,
                a0=None):
    """Serial fine solution with the Joule-loss sum grouped by slice exactly as
    Parareal groups it."""
    if m is None:
        m = meshmod.build(problem.n_nodes)
    if kl_table is None:
        kl_table = timestep.kl_table_for(problem, m)
    sysm = timestep.build_system(problem, xi, m, kl_table)
    T = n_periods * problem.period
    dt_f = T / (n_slices * fine_steps_per_slice)
    st = timestep.Stepper(sysm, dt_f)
    a = np.zeros(m.n_dof) if a0 is None else np.array(a0, dtype=np.float64)
    states = [a]
    qs = []
    for n in range(1, n_slices + 1):
        a, qn = st.run(a, fine_steps_per_slice, (n - 1) * fine_steps_per_slice)
        states.append(a)
        qs.append(qn)
    s = 0.0
    for v in qs:
        s += v
    return dict(Q=s / T, state=a, states=states)
