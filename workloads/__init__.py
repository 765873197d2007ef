"""Seeded synthetic inputs shared by the HIP path and the FP64 oracle.

This module holds no arithmetic of the method: it only describes the
problems (mesh size, material parameters, time grids, sample counts) and
draws the random inputs xi that every solver call takes as an argument.
Both the oracle and the GPU library consume the same xi arrays, so the
two never need to re-implement the same random stream.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
hash of (seed, stream, level, sample, dim), 53-bit uniforms, then the
Box-Muller transform (Box and Muller, 1958) for standard normals.

Workloads follow the paper's FE example (Section III-B): a transient 2-D
eddy-current model driven over several electrical periods, uncertain
conductivity, mean Joule loss as the quantity of interest.  The paper's
own machine model and its mesh files are not available, so a unit-square
model with a conducting square and a source strip stands in for it.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

_M64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15

MU0 = 4.0e-7 * math.pi            # vacuum permeability [H/m]
NU_AIR = 1.0 / MU0                # reluctivity of air [m/H]
NU_COND = 1.0 / (1000.0 * MU0)    # nominal conductor reluctivity (mu_r = 1000)


# ---------------------------------------------------------------------------
# counter-based generator
# ---------------------------------------------------------------------------
def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser applied to z + golden gamma (vectorised, uint64)."""
    with np.errstate(over="ignore"):
        z = (z + np.uint64(_GOLDEN)).astype(np.uint64)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def _key(seed: int, stream: int, level: int, sample: np.ndarray) -> np.ndarray:
    k = _mix64(np.asarray([seed & _M64], dtype=np.uint64))
    k = _mix64(k ^ np.uint64(stream & _M64))
    k = _mix64(k ^ np.uint64(level & _M64))
    return _mix64(k ^ np.asarray(sample, dtype=np.uint64))


def uniforms(seed: int, stream: int, level: int, sample, n_dim: int, which: int = 0) -> np.ndarray:
    """53-bit uniforms in (0, 1); shape [len(sample), n_dim]."""
    sample = np.atleast_1d(np.asarray(sample, dtype=np.uint64))
    key = _key(seed, stream, level, sample)[:, None]
    d = np.arange(n_dim, dtype=np.uint64)[None, :]
    bits = _mix64(key ^ (np.uint64(2) * d + np.uint64(which)))
    return ((bits >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)


def normals(seed: int, stream: int, level: int, sample, n_dim: int) -> np.ndarray:
    """Standard normals xi[sample, dim] (Box-Muller, cosine branch)."""
    u1 = uniforms(seed, stream, level, sample, n_dim, which=0)
    u2 = uniforms(seed, stream, level, sample, n_dim, which=1)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


# ---------------------------------------------------------------------------
# problem descriptions
# ---------------------------------------------------------------------------
MAT_LOGNORMAL_SCALAR = 0   # one sigma and one nu per sample for the whole conductor
MAT_KL = 1                 # lognormal KL random field for sigma, nu fixed
MAT_NONLINEAR = 2          # nu(|B|) = k1 exp(k2 |B|^2) + k3, per-sample scaled k's

PREC_FP64 = 0
PREC_MIXED = 1


@dataclass(frozen=True)
class Material:
    kind: int = MAT_LOGNORMAL_SCALAR
    sigma0: float = 5.0e6          # median conductor conductivity [S/m]
    nu_cond: float = NU_COND       # median / fixed conductor reluctivity
    nu_air: float = NU_AIR
    s_sigma: float = 0.2           # lognormal std of sigma (scalar model)
    s_nu: float = 0.2              # lognormal std of nu (scalar model)
    n_modes: int = 8               # KL modes
    corr_len: float = 0.2          # KL correlation length
    s_kl: float = 0.3              # KL log-field std
    k1: float = 3.8                # nonlinear curve
    k2: float = 2.17
    k3: float = 396.2
    s_k: float = 0.1               # lognormal std of each k scale
    picard_tol: float = 1e-8
    picard_max: int = 50

    @property
    def n_xi(self) -> int:
        if self.kind == MAT_LOGNORMAL_SCALAR:
            return 2
        if self.kind == MAT_KL:
            return self.n_modes
        return 3


@dataclass(frozen=True)
class Problem:
    n_nodes: int                                     # nodes per side of the unit square
    material: Material = Material()
    conductor: Tuple[float, float, float, float] = (0.3, 0.7, 0.3, 0.7)  # x0, x1, y0, y1
    strip: Tuple[float, float] = (0.1, 0.2)          # source strip x-range (all y)
    J0: float = 1.0e6                                # source amplitude [A/m^2]
    freq: float = 50.0                               # [Hz]

    @property
    def n_dof(self) -> int:
        return (self.n_nodes - 2) ** 2

    @property
    def period(self) -> float:
        return 1.0 / self.freq


@dataclass(frozen=True)
class Level:
    steps_per_period: int
    coarse_steps_per_period: int  # 0 for level 0 (Q_{-1} = 0)
    n_periods: int
    n_samples: int


@dataclass(frozen=True)
class PararealSpec:
    n_periods: int
    n_slices: int
    fine_steps_per_slice: int
    coarse_steps_per_slice: int
    k_max: int
    tol: float


@dataclass(frozen=True)
class Workload:
    name: str
    problem: Problem
    precision: int
    levels: Tuple[Level, ...] = ()
    parareal: Optional[PararealSpec] = None
    n_parareal_samples: int = 0
    seed: int = 0
    stream: int = 0


def plain_fp64_33() -> Workload:
    """Plain MC, FP64, 33x33 nodes, scalar lognormal sigma/nu, 16 samples, 64 steps."""
    return Workload(
        name="plain-fp64-33x33-16samples-64steps",
        problem=Problem(33, Material(kind=MAT_LOGNORMAL_SCALAR)),
        precision=PREC_FP64,
        levels=(Level(64, 0, 1, 16),),
        stream=0,
    )


def mlmc3_mixed_129() -> Workload:
    """MLMC with 3 time levels (64/128/256 steps per period, 4 periods), 129x129,
    8-mode KL sigma, 512/128/32 samples, FP32 PCG inside FP64 refinement."""
    return Workload(
        name="mlmc3-mixed-129x129-kl8-512/128/32",
        problem=Problem(129, Material(kind=MAT_KL)),
        precision=PREC_MIXED,
        levels=(Level(64, 0, 4, 512), Level(128, 64, 4, 128), Level(256, 128, 4, 32)),
        stream=1,
    )


def parareal_257() -> Workload:
    """Parareal on the finest level: 257x257, 1024 fine steps over 4 periods in 32
    slices, coarse = 1 IE step per slice, K <= 8, tol 1e-8, 64 samples."""
    return Workload(
        name="parareal-mixed-257x257-kl8-64samples-32slices",
        problem=Problem(257, Material(kind=MAT_KL)),
        precision=PREC_MIXED,
        parareal=PararealSpec(n_periods=4, n_slices=32, fine_steps_per_slice=32,
                              coarse_steps_per_slice=1, k_max=8, tol=1e-8),
        n_parareal_samples=64,
        stream=2,
    )


def nonlinear_mlmc4_129() -> Workload:
    """Nonlinear iron, MLMC 4 levels (32/64/128/256 steps per period, 2 periods),
    129x129, 1024/256/64/16 samples, Picard tolerance 1e-8."""
    return Workload(
        name="nonlinear-mlmc4-129x129-1024/256/64/16",
        problem=Problem(129, Material(kind=MAT_NONLINEAR, sigma0=5.0e6)),
        precision=PREC_MIXED,
        levels=(Level(32, 0, 2, 1024), Level(64, 32, 2, 256), Level(128, 64, 2, 64),
                Level(256, 128, 2, 16)),
        stream=3,
    )


SERVING_MESHES = (65, 129, 257, 513)
SERVING_MESH_WEIGHTS = (0.4, 0.3, 0.2, 0.1)
SERVING_STEPS = (64, 128, 256, 512, 1024)


@dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    n_nodes: int
    steps_per_period: int
    n_periods: int
    xi: Tuple[float, ...]


def serving_stream(n_requests: int = 4096, rate_hz: float = 200.0, seed: int = 0,
                   stream: int = 4, meshes=SERVING_MESHES, weights=SERVING_MESH_WEIGHTS,
                   steps=SERVING_STEPS, n_periods: int = 2, n_modes: int = 8):
    """Poisson arrivals of sample-solve requests with a mixed mesh/level mix."""
    idx = np.arange(n_requests)
    u = uniforms(seed, stream, 1000, idx, 3)
    gaps = -np.log(u[:, 0]) / rate_hz
    arrivals = np.cumsum(gaps) - gaps[0]
    cw = np.cumsum(np.asarray(weights, dtype=np.float64))
    cw /= cw[-1]
    mesh_i = np.searchsorted(cw, u[:, 1], side="right")
    step_i = np.minimum((u[:, 2] * len(steps)).astype(np.int64), len(steps) - 1)
    xi = normals(seed, stream, 0, idx, n_modes)
    return [Request(int(i), float(arrivals[i]), int(meshes[mesh_i[i]]), int(steps[step_i[i]]),
                    n_periods, tuple(float(v) for v in xi[i])) for i in idx]


def level_xi(w: Workload, level: int, n: Optional[int] = None, first: int = 0) -> np.ndarray:
    """xi[n, n_xi] for `level` of workload `w`; samples on different levels are
    independent, the coupled (l, l-1) pair of one sample shares its row."""
    if n is None:
        n = w.levels[level].n_samples if w.levels else w.n_parareal_samples
    return normals(w.seed, w.stream, level, np.arange(first, first + n), w.problem.material.n_xi)


def with_nodes(w: Workload, n_nodes: int) -> Workload:
    return dataclasses.replace(w, problem=dataclasses.replace(w.problem, n_nodes=n_nodes))
