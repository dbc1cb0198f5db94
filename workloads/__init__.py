"""Seeded synthetic workloads shared by the oracle tests and the HIP path.

This module holds problem definitions (grid sizes, shifts, block sizes) and
seeded random draws only.  It contains none of the eigensolver's arithmetic:
no operator application, no preconditioner, no projection.  Both the CPU
oracle tests and the GPU path import it so that they see bit-identical
inputs; neither side imports the other.

Random draws use ``numpy.random.default_rng`` seeded with fixed integer
tuples, in FP64 on the host.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np


def rng(*seed: int) -> np.random.Generator:
    return np.random.default_rng(list(seed))


def start_block(n: int, k: int, seed: Tuple[int, ...], dtype=np.float64) -> np.ndarray:
    """Seeded N(0,1) start block, point-major (n rows, k contiguous columns)."""
    g = rng(*seed)
    if np.dtype(dtype).kind == "c":
        re = g.standard_normal((n, k))
        im = g.standard_normal((n, k))
        return (re + 1j * im).astype(dtype)
    return g.standard_normal((n, k)).astype(dtype)


@dataclass
class Workload:
    """A problem instance: operator kind, grid, shift, block size, start seed."""

    name: str
    kind: str                    # "fd5_2d" | "fd7_3d" | "bloch7_3d" | ...
    dims: Tuple[int, ...]        # interior points per dimension
    h: float                     # grid spacing
    scale: float                 # multiplies the negative discrete Laplacian
    sigma: float
    k: int                       # wanted pairs
    k_extra: int                 # extra block columns (real problems: 1)
    precond: str                 # "identity" | "mg"
    v0_seed: Tuple[int, ...]
    mg_levels: int = 5
    mg_pre: int = 2
    mg_post: int = 2
    mg_omega: float = 2.0 / 3.0
    potential: Optional[np.ndarray] = None
    notes: str = ""

    @property
    def n(self) -> int:
        return int(np.prod(self.dims))

    @property
    def k_int(self) -> int:
        return self.k + self.k_extra

    def v0(self) -> np.ndarray:
        return start_block(self.n, self.k_int, self.v0_seed)


def fd_lambda_max(N: int, h: float, d: int) -> float:
    """Largest eigenvalue of the d-dim 5/7-point Dirichlet Laplacian (problem setup)."""
    return d * (4.0 / h**2) * math.sin(N * math.pi * h / 2.0) ** 2


def config1() -> Workload:
    """2-D 5-point Dirichlet Laplacian, 32x32 interior, h=1/33, B=I, T=I, k=4
    nearest sigma = 0.4*lambda_max."""
    N, h = 32, 1.0 / 33.0
    lmax = fd_lambda_max(N, h, 2)
    return Workload(
        name="fd5_2d_32x32_k4", kind="fd5_2d", dims=(N, N), h=h, scale=1.0,
        sigma=0.4 * lmax, k=4, k_extra=1, precond="identity", v0_seed=(1, 0),
    )


def config2(N: int = 64) -> Workload:
    """3-D 7-point Dirichlet Laplacian on N^3 (N=64: n=262144), h=1/(N+1),
    B=I, k=16 nearest sigma = 0.25*lambda_max, T = one MG V-cycle on the
    unshifted Laplacian (5 levels, 2+2 weighted Jacobi, omega=2/3)."""
    h = 1.0 / (N + 1)
    lmax = fd_lambda_max(N, h, 3)
    levels = max(1, int(round(math.log2(N))) - 1)   # 64 -> 4^3 coarsest
    return Workload(
        name=f"fd7_3d_{N}cubed_k16", kind="fd7_3d", dims=(N, N, N), h=h, scale=1.0,
        sigma=0.25 * lmax, k=16, k_extra=1, precond="mg", v0_seed=(2, 0),
        mg_levels=min(5, levels),
    )


def small_fd7(N: int, k: int, frac: float, seed=(9, 0), precond="mg", levels=None) -> Workload:
    """Reduced 3-D FD problem with sigma at a given fraction of lambda_max."""
    h = 1.0 / (N + 1)
    lmax = fd_lambda_max(N, h, 3)
    lv = levels if levels is not None else max(1, int(round(math.log2(N))) - 1)
    return Workload(
        name=f"fd7_3d_{N}cubed_k{k}", kind="fd7_3d", dims=(N, N, N), h=h, scale=1.0,
        sigma=frac * lmax, k=k, k_extra=1, precond=precond, v0_seed=seed,
        mg_levels=lv,
    )


def small_fd5(N: int, k: int, frac: float, seed=(8, 0), precond="identity", levels=None) -> Workload:
    h = 1.0 / (N + 1)
    lmax = fd_lambda_max(N, h, 2)
    lv = levels if levels is not None else max(1, int(round(math.log2(N))) - 1)
    return Workload(
        name=f"fd5_2d_{N}sq_k{k}", kind="fd5_2d", dims=(N, N), h=h, scale=1.0,
        sigma=frac * lmax, k=k, k_extra=1, precond=precond, v0_seed=seed,
        mg_levels=lv,
    )
