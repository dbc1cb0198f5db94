"""Brute-force dense reference (oracle; test infrastructure only).

The plain definition of what block PLHR computes: the k eigenpairs of the
Hermitian pencil (A, B) whose eigenvalues are nearest sigma (eq. 1.1 and the
ordering of Section 4), from a dense LAPACK eigendecomposition.  Usable for
n up to a few thousand.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def nearest_pairs(A, B, sigma: float, k: int):
    """Eigenvalues (ordered by |lam - sigma|, ties to the smaller) and
    B-orthonormal eigenvectors of the k pairs nearest sigma."""
    Ad = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    if B is None:
        lam, X = np.linalg.eigh(Ad)
    else:
        Bd = B.toarray() if hasattr(B, "toarray") else np.asarray(B)
        lam, X = sla.eigh(Ad, Bd)
    order = np.lexsort((lam, np.abs(lam - sigma)))[:k]
    return lam[order], X[:, order]


def cluster_basis(A, B, sigma: float, k: int, rtol: float = 1e-9):
    """B-orthonormal basis of the union of the eigenspaces of every
    eigenvalue among the k nearest sigma.  When the k-th value is part of a
    multiple eigenvalue, any k-dimensional subspace of that union made of
    eigenvectors is a correct answer, so subspaces are compared with it."""
    Ad = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    if B is None:
        lam, X = np.linalg.eigh(Ad)
    else:
        Bd = B.toarray() if hasattr(B, "toarray") else np.asarray(B)
        lam, X = sla.eigh(Ad, Bd)
    order = np.lexsort((lam, np.abs(lam - sigma)))[:k]
    sel = lam[order]
    scale = max(np.abs(lam).max(), 1.0)
    mask = np.zeros(len(lam), dtype=bool)
    for v in sel:
        mask |= np.abs(lam - v) <= rtol * scale
    return lam[mask], X[:, mask]


def all_eigenvalues(A, B=None):
    Ad = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    if B is None:
        return np.linalg.eigvalsh(Ad)
    Bd = B.toarray() if hasattr(B, "toarray") else np.asarray(B)
    return sla.eigh(Ad, Bd, eigvals_only=True)


def subspace_sine(Vref, V, B=None) -> float:
    """sin of the largest principal angle between span(Vref) and span(V)
    in the B-inner product, || (I - Q Q^* B) Qv ||_B, with B-orthonormal
    bases Q of span(Vref) and Qv of span(V); accurate for small angles."""
    def mulB(X):
        return X if B is None else B @ X

    def borth(X):
        G = X.conj().T @ mulB(X)
        L = np.linalg.cholesky(0.5 * (G + G.conj().T))
        return X @ np.linalg.inv(L).conj().T

    Q = borth(np.asarray(Vref))
    Qv = borth(np.asarray(V))
    Rm = Qv - Q @ (Q.conj().T @ mulB(Qv))
    G = Rm.conj().T @ mulB(Rm)
    return float(np.sqrt(max(np.linalg.eigvalsh(0.5 * (G + G.conj().T)).max(), 0.0)))
