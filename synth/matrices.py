"""Seeded control and interaction matrices.

R (n_act x n_slopes) has entries N(0, 1/n_slopes), drawn in float64 and stored
once as float32; that float32 array is the reference control matrix.
D (n_slopes x n_act) has entries N(0, 0.25/n_act) in float64, so that the
implicit pseudo-open-loop operator R.D has spectral radius near 0.5 and the
closed loop (1-leak-gain) I + gain R.D stays stable.
"""
from __future__ import annotations

import numpy as np

from .workloads import Workload, seed_for

__all__ = ["control_matrix", "interaction_matrix", "gaussian_matrix"]

_RMAT, _DMAT = 2, 3


def gaussian_matrix(rows: int, cols: int, sigma: float, seed, dtype=np.float32,
                    block_rows: int = 256) -> np.ndarray:
    """rows x cols matrix of N(0, sigma^2), drawn in float64 row blocks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((rows, cols), dtype)
    for r0 in range(0, rows, block_rows):
        r1 = min(rows, r0 + block_rows)
        out[r0:r1] = sigma * rng.standard_normal((r1 - r0, cols))
    return out


def control_matrix(wl: Workload, inst_index: int) -> np.ndarray:
    inst = wl.instances[inst_index]
    ns = inst.n_slopes
    return gaussian_matrix(inst.n_act, ns, 1.0 / np.sqrt(ns),
                           seed_for(wl.index, inst_index, 99, _RMAT), np.float32)


def interaction_matrix(wl: Workload, inst_index: int) -> np.ndarray:
    inst = wl.instances[inst_index]
    return gaussian_matrix(inst.n_slopes, inst.n_act, 0.5 / np.sqrt(inst.n_act),
                           seed_for(wl.index, inst_index, 99, _DMAT), np.float64)
