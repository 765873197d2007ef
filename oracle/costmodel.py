"""Time-to-solution / effort model of MLMC + Parareal (oracle).

Section II-C, Eqs. (13)-(16) and Section II-D, Eqs. (17)-(25) plus the
finite-core speedup expression that follows Eq. (25).  tau_F, tau_C are the
sequential costs of the fine and coarse propagators over the whole
interval; M slices; K Parareal iterations; C_l per-level sample costs.
"""
from __future__ import annotations

import math


def tau_para_iter(k: int, M: int, tau_f: float, tau_c: float) -> float:
    """Eq. (13): wall time of iteration k."""
    return tau_f / M + (M - k) / M * tau_c


def effort_para_iter(k: int, M: int, tau_f: float, tau_c: float) -> float:
    """Eq. (14): effort (core-time) of iteration k."""
    return (M - k + 1) / M * tau_f + (M - k) / M * tau_c


def tau_para(K: int, M: int, tau_f: float, tau_c: float) -> float:
    """Eq. (15)."""
    return K / M * (tau_f + (M - (K + 1) / 2) * tau_c)


def effort_para(K: int, M: int, tau_f: float, tau_c: float) -> float:
    """Eq. (16)."""
    return K / M * (M - (K + 1) / 2) * (tau_f + tau_c) + K / M * tau_f


def ref_cost(C, N):
    """Eq. (17): (tau_ref, E_ref) of MLMC with unlimited cores."""
    return sum(C), sum(n * c for n, c in zip(N, C))


def comb_cost(C, N, tau_p: float, effort_p: float):
    """Eqs. (18)-(19): combined method, Parareal on level L only."""
    L = len(C) - 1
    return (sum(C[:L]) + tau_p, sum(N[l] * C[l] for l in range(L)) + N[L] * effort_p)


def exp_cost(C0: float, r: float, L: int):
    """Eq. (20): C_l = C0 r^l."""
    return [C0 * r ** l for l in range(L + 1)]


def s_inf(r: float, L: int) -> float:
    """Eq. (21) closed form of the maximum speedup."""
    return (r ** (L + 1) - 1) / (2 * r ** L - r ** (L - 1) - 1)


def s_inf_ratio(C) -> float:
    """Eq. (21) as the ratio of sums (tau_para reduced to C_{L-1})."""
    L = len(C) - 1
    return sum(C) / (sum(C[:L]) + C[L - 1])


def kappa(r: float, n_para: int) -> int:
    """Eq. (22): largest K with tau_para <= C_{L-1} (coarse = level L-2)."""
    b = 2 * r * r + 2 * n_para - 1
    return math.floor((b - math.sqrt(b * b - 8 * n_para * r)) / 2)


def effort_ratio(C, N, K: int, M: int) -> float:
    """Eq. (23): eps_inf = E_comb / E_ref with tau_F = C_L, tau_C = C_{L-2}."""
    L = len(C) - 1
    ep = effort_para(K, M, C[L], C[L - 2])
    return comb_cost(C, N, 0.0, ep)[1] / ref_cost(C, N)[1]


def batches(C, N, n_c: int):
    """Eq. (24): b_l = ceil(N_l (1 + C_{l-1}/C_l) / n_c), C_{-1}/C_0 = 0."""
    out = []
    for l in range(len(C)):
        ratio = 0.0 if l == 0 else C[l - 1] / C[l]
        out.append(math.ceil(N[l] * (1 + ratio) / n_c))
    return out


def cores_per_parareal_sample(C, N, n_c: int) -> int:
    """Eq. (25)."""
    L = len(C) - 1
    return math.floor(n_c / (N[L] * (1 + C[L - 1] / C[L])))


def speedup_finite(C, N, n_c: int, K: int, r: float) -> float:
    """Finite-core speedup (expression after Eq. (25)); its bracket mixes C_l
    with r^L, which is consistent only for C_0 = 1 (C_l = r^l)."""
    L = len(C) - 1
    b = batches(C, N, n_c)
    n_p = cores_per_parareal_sample(C, N, n_c)
    num = sum(bl * cl for bl, cl in zip(b, C))
    den = sum(b[l] * C[l] for l in range(L)) + K / n_p * (r ** L + (n_p - (K + 1) / 2) * r ** (L - 2))
    return num / den
