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
    lock: bool = True            # soft locking of converged columns
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


def fd7_closed_form(N: int, h: float) -> np.ndarray:
    """Sorted eigenvalues of the 3-D 7-point Dirichlet Laplacian (N^3)."""
    s = (4.0 / h**2) * np.sin(np.arange(1, N + 1) * np.pi / (2 * (N + 1))) ** 2
    return np.sort(np.add.outer(np.add.outer(s, s), s).ravel())


def shift_between(ev: np.ndarray, nbelow: int, frac: float = 0.4) -> float:
    """A shift with about `nbelow` eigenvalues below it, placed `frac` of the
    way between two consecutive distinct eigenvalues (so that it is not an
    eigenvalue and the two neighbouring clusters are not equidistant)."""
    u = np.unique(np.round(ev, 8))
    i = int(np.searchsorted(u, ev[nbelow]))
    return float(u[i - 1] + frac * (u[i] - u[i - 1]))


def bench_workload(N: int = 64, nbelow: int = 121) -> Workload:
    """The benchmark workload: the 3-D Laplacian of the second configuration
    (64^3, h = 1/65, k = 16, 5-level V-cycle) with the shift about 125
    eigenvalues into the spectrum (sigma ~ 485.22 for N = 64), where the 16
    nearest eigenvalues form whole clusters of the cube's degenerate
    spectrum (1 + 6 + 6 + 3), so that the wanted set is unambiguous.  The
    block carries 4 guard columns and soft locking is off: with a V-cycle
    for the Laplacian (not for |A - sigma I|) one guard column, or locking,
    lets the block settle on clusters below the shift.  The design notes
    explain why the quarter-of-lambda_max shift of the configuration is not
    used for the throughput number."""
    w = config2(N)
    w.sigma = shift_between(fd7_closed_form(N, w.h), nbelow)
    w.k_extra = 4
    w.lock = False
    w.name = f"fd7_3d_{N}cubed_k16_below{nbelow}"
    return w


def gaussian_potential(N: int, ngauss: int, seed: Tuple[int, ...], d: int = 2) -> np.ndarray:
    """Sum of negative Gaussians on an N^d grid (grid units, points at
    1..N): depth U(1, 4), width U(0.5, 1.5), centres U(1, N)^d.  Returned
    x-fastest, length N^d."""
    g = rng(*seed)
    depth = g.uniform(1.0, 4.0, ngauss)
    width = g.uniform(0.5, 1.5, ngauss)
    centres = g.uniform(1.0, float(N), (ngauss, d))
    axes = [np.arange(1, N + 1, dtype=np.float64)] * d
    mesh = np.meshgrid(*axes[::-1], indexing="ij")[::-1]   # mesh[0] = x (fastest)
    V = np.zeros((N,) * d)
    for a in range(ngauss):
        r2 = sum((mesh[i] - centres[a, i]) ** 2 for i in range(d))
        V -= depth[a] * np.exp(-r2 / (2.0 * width[a] ** 2))
    return V.ravel()


def periodic_gaussian_potential(N: int, ngauss: int, seed: Tuple[int, ...],
                                d: int = 3) -> np.ndarray:
    """Sum of negative Gaussians on an N^d periodic box (grid units, points
    at 0..N-1): depth U(1, 4), width U(0.5, 1.5), centres U[0, N)^d, each
    coordinate difference taken to its nearest periodic image.  Returned
    x-fastest, length N^d."""
    g = rng(*seed)
    depth = g.uniform(1.0, 4.0, ngauss)
    width = g.uniform(0.5, 1.5, ngauss)
    centres = g.uniform(0.0, float(N), (ngauss, d))
    axes = [np.arange(N, dtype=np.float64)] * d
    mesh = np.meshgrid(*axes[::-1], indexing="ij")[::-1]   # mesh[0] = x (fastest)
    V = np.zeros((N,) * d)
    for a in range(ngauss):
        r2 = np.zeros((N,) * d)
        for i in range(d):
            dx = np.abs(mesh[i] - centres[a, i])
            dx = np.minimum(dx, N - dx)
            r2 += dx * dx
        V -= depth[a] * np.exp(-r2 / (2.0 * width[a] ** 2))
    return V.ravel()


def bloch_thetas() -> Tuple[float, float, float]:
    """Bloch phases per period of the periodic model: 2 pi (0.1, 0.2, 0.3)."""
    return (2.0 * math.pi * 0.1, 2.0 * math.pi * 0.2, 2.0 * math.pi * 0.3)


def mass_density(N: int, seed: Tuple[int, ...], d: int = 2, contrast: float = 4.0) -> np.ndarray:
    """A positive, smoothly varying diagonal mass b on an N^d grid (a
    membrane or medium of variable density): 1 plus (contrast - 1) times
    a sum of 3 positive Gaussian bumps scaled to peak 1, so that
    1 <= b <= contrast.  Returned x-fastest, length N^d."""
    bump = -gaussian_potential(N, 3, seed, d)
    return 1.0 + (contrast - 1.0) * bump / bump.max()


def batched_problem(b: int, sizes=(64, 96, 128, 160)):
    """Problem b of the batched set: grid size N_b, potential, targets."""
    g = rng(5, 2)
    Ns = g.choice(np.array(sizes), 256)
    N = int(Ns[b])
    pot = gaussian_potential(N, 16, (5, 1, b))
    targets = np.sort(rng(5, 3, b).uniform(1.5, 2.5, 8))
    return N, pot, targets


def perturbed_abs_inverse(A: np.ndarray, B: np.ndarray, sigma: float, eps: float,
                          seed: Tuple[int, ...]) -> np.ndarray:
    """The preconditioners of the small finite-element experiment of
    Section 6.1: T = |A - sigma B|^-1 + E, with |.| the matrix absolute
    value of the symmetric matrix A - sigma B (from its eigendecomposition)
    and E = G G^T (G seeded standard normal) scaled to spectral norm
    eps ||(A - sigma B)^-1||.  A, B dense; returns a dense SPD matrix."""
    d, U = np.linalg.eigh(A - sigma * B)
    T = (U / np.abs(d)) @ U.T
    G = rng(*seed).standard_normal(A.shape)
    E = G @ G.T
    E *= eps / np.abs(d).min() / np.linalg.norm(E, 2)
    T = T + E
    return 0.5 * (T + T.T)
