"""Batched MLMC + Parareal eddy-current UQ on MI355X (Python binding of libmq).

The binding only marshals arguments: torch CUDA/HIP tensors provide device
memory and streams; every step of the hot path (assembly, implicit Euler with
CG, Joule-loss accumulation, Parareal, MLMC sums) runs in the HIP library.
"""
from .api import (  # noqa: F401
    Problem, cost_model, default_desc, mlmc_adaptive_run, mlmc_combined_run, mlmc_estimate, mlmc_level_run,
    mlmc_multilevel_run, mlmc_multimesh_run, parareal_run, plan_split,
    debug_apply, last_flags, Server,
)
from ._lib import MQError, load  # noqa: F401
