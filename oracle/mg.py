"""Geometric multigrid V-cycle used as the HPD preconditioner T (oracle).

The paper requires T to be Hermitian positive definite (Section 5) and uses
a multigrid V-cycle in its Laplacian experiments (Appendix A, Algorithm 4
with B_l = L_l on the fine levels).  This module builds the plain V-cycle on
the Laplacian part of the operator:

* levels: the finest grid has N points per dimension; each coarser level
  pairs neighbouring points (N -> N/2), cell-centred, down to the coarsest
  level, which is solved exactly with a dense inverse;
* level operators: the same stencil re-discretised with spacing 2^l h
  (no potential);
* prolongation: d-linear interpolation, 3/4 from the parent and 1/4 from the
  parent's neighbour in each direction; a neighbour outside a Dirichlet box
  is zero, a neighbour across a Bloch-periodic face is the wrapped value
  times the phase;
* restriction: R = P^H / 2^d;
* smoothing: nu_pre and nu_post sweeps of weighted Jacobi,
  w <- w + omega * D^-1 (r - A_l w), starting from w = 0.

With R proportional to P^H, a symmetric smoother (Jacobi), the same number
of pre- and post-sweeps and Hermitian positive definite level operators,
the V-cycle is a Hermitian linear operator; it is positive definite because
weighted Jacobi with omega = 2/3 satisfies 2D/omega - A_l > 0 for these
stencils.  Both facts are checked by the tests on small grids.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import operators as ops


def _prolong1d(Nc: int, bc: str, theta: float = 0.0) -> sp.csr_matrix:
    Nf = 2 * Nc
    P = sp.lil_matrix((Nf, Nc), dtype=np.complex128 if bc == "bloch" else np.float64)
    for c in range(Nc):
        for a, nb in ((0, c - 1), (1, c + 1)):
            f = 2 * c + a
            P[f, c] += 0.75
            if 0 <= nb < Nc:
                P[f, nb] += 0.25
            elif bc == "bloch":
                if nb < 0:
                    P[f, nb + Nc] += 0.25 * np.exp(-1j * theta)
                else:
                    P[f, nb - Nc] += 0.25 * np.exp(1j * theta)
            # Dirichlet: neighbour outside the box is zero
    return P.tocsr()


def _kron_x_fastest(mats):
    out = None
    for m in reversed(mats):
        out = m if out is None else sp.kron(out, m, format="csr")
    return out.tocsr()


class VCycle:
    """T ~ A_lap^{-1} by one V-cycle; ``apply`` works on an (n, k) block."""

    def __init__(self, kind: str, dims, h: float, scale: float, levels: int,
                 nu_pre: int = 2, nu_post: int = 2, omega: float = 2.0 / 3.0,
                 thetas=None):
        self.kind = kind
        self.nu_pre, self.nu_post, self.omega = nu_pre, nu_post, omega
        self.d = len(dims)
        self.A, self.Dinv, self.P = [], [], []
        dims = tuple(dims)
        hl = h
        for lev in range(levels):
            if kind == "bloch":
                A = ops.bloch_periodic(dims, hl, thetas, scale=scale)
            else:
                A = ops.fd_dirichlet(dims, hl, scale=scale)
            self.A.append(A)
            self.Dinv.append(1.0 / A.diagonal())
            if lev == levels - 1:
                break
            if any(N % 2 for N in dims):
                raise ValueError(f"grid {dims} cannot be coarsened")
            cdims = tuple(N // 2 for N in dims)
            mats = [_prolong1d(Nc, "bloch" if kind == "bloch" else "dirichlet",
                               0.0 if thetas is None else thetas[a])
                    for a, Nc in enumerate(cdims)]
            self.P.append(_kron_x_fastest(mats))
            dims = cdims
            hl = 2.0 * hl
        self.coarse_inv = np.linalg.inv(self.A[-1].toarray())

    def _cycle(self, lev: int, r: np.ndarray) -> np.ndarray:
        if lev == len(self.A) - 1:
            return self.coarse_inv @ r
        A, Dinv, om = self.A[lev], self.Dinv[lev][:, None], self.omega
        w = np.zeros_like(r)
        for _ in range(self.nu_pre):
            w = w + om * Dinv * (r - A @ w)
        P = self.P[lev]
        rc = (P.conj().T @ (r - A @ w)) / (2 ** self.d)
        w = w + P @ self._cycle(lev + 1, rc)
        for _ in range(self.nu_post):
            w = w + om * Dinv * (r - A @ w)
        return w

    def apply(self, R: np.ndarray) -> np.ndarray:
        R = np.asarray(R)
        one = R.ndim == 1
        Rb = R[:, None] if one else R
        dt = np.result_type(Rb.dtype, self.A[0].dtype, np.float64)
        out = self._cycle(0, Rb.astype(dt))
        return out[:, 0] if one else out

    __call__ = apply


def dense_matrix(T, n: int, dtype=np.float64) -> np.ndarray:
    """Columns T e_j, for checking symmetry and definiteness on small grids."""
    return T(np.eye(n, dtype=dtype))
