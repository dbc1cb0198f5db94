"""Sparse assembly of the model operators (oracle; test infrastructure only).

Every operator here is a scipy.sparse CSR matrix in FP64 (complex128 for the
Bloch operator).  Grid points are numbered x-fastest: p = i + Nx*(j + Ny*l).

* ``fd_dirichlet``: the standard (2d+1)-point finite-difference negative
  Laplacian on the interior points of a box with zero Dirichlet data, spacing
  h, times ``scale``, plus an optional diagonal potential.  This is the model
  operator of Section 6.2 of the paper (5-point, h = 2^-7).
* ``bloch_periodic``: the same stencil on a periodic box where the unknown
  picks up the phase exp(i*theta_d) when it wraps around in direction d
  (a Bloch/k-point condition); Hermitian.
* ``fe_q1``: stiffness and consistent mass matrices of bilinear (2-D) or
  trilinear (3-D) elements on a uniform mesh of the unit box, Dirichlet
  (interior nodes only) or natural (all nodes).  Section 6.1 of the paper uses
  the 2-D Dirichlet case with 50 elements per side.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _lap1d_dirichlet(N: int, h: float) -> sp.csr_matrix:
    main = np.full(N, 2.0)
    off = np.full(N - 1, -1.0)
    return sp.diags([off, main, off], [-1, 0, 1], shape=(N, N), format="csr") / h**2


def _kron_sum(ops):
    """Kronecker sum for x-fastest numbering: ops[0] acts on x (fastest)."""
    d = len(ops)
    sizes = [o.shape[0] for o in ops]
    total = None
    for a in range(d):
        term = None
        for b in reversed(range(d)):          # slowest index first in kron
            m = ops[b] if b == a else sp.identity(sizes[b], format="csr")
            term = m if term is None else sp.kron(term, m, format="csr")
        total = term if total is None else total + term
    return total.tocsr()


def fd_dirichlet(dims, h: float, scale: float = 1.0, potential=None) -> sp.csr_matrix:
    """scale * (-Laplacian_h) + diag(potential) with zero Dirichlet boundary."""
    L = _kron_sum([_lap1d_dirichlet(N, h) for N in dims]) * scale
    if potential is not None:
        L = L + sp.diags(np.asarray(potential, dtype=np.float64).ravel())
    return L.tocsr()


def _lap1d_bloch(N: int, h: float, theta: float) -> sp.csr_matrix:
    """1-D periodic second difference with Bloch phase exp(i*theta) on wrap."""
    M = sp.lil_matrix((N, N), dtype=np.complex128)
    ph = np.exp(1j * theta)
    for i in range(N):
        M[i, i] += 2.0
        if N == 1:
            M[i, i] -= ph + np.conj(ph)
            continue
        if i + 1 < N:
            M[i, i + 1] += -1.0
        else:
            M[i, 0] += -ph            # x_{N} = e^{i theta} x_0
        if i - 1 >= 0:
            M[i, i - 1] += -1.0
        else:
            M[i, N - 1] += -np.conj(ph)   # x_{-1} = e^{-i theta} x_{N-1}
    return (M.tocsr() / h**2)


def bloch_periodic(dims, h: float, thetas, scale: float = 0.5, potential=None) -> sp.csr_matrix:
    """scale * (-Laplacian_theta) + diag(potential), Bloch-periodic box."""
    L = _kron_sum([_lap1d_bloch(N, h, t) for N, t in zip(dims, thetas)]) * scale
    if potential is not None:
        L = L + sp.diags(np.asarray(potential, dtype=np.float64).ravel().astype(np.complex128))
    return L.tocsr()


# ---------------------------------------------------------------- finite elements
def _fe1d(Nel: int, h: float):
    """1-D linear-element stiffness and mass on all Nel+1 nodes of [0, Nel*h]."""
    n = Nel + 1
    K = sp.lil_matrix((n, n))
    M = sp.lil_matrix((n, n))
    ke = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    me = np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6.0
    for e in range(Nel):
        idx = [e, e + 1]
        for a in range(2):
            for b in range(2):
                K[idx[a], idx[b]] += ke[a, b]
                M[idx[a], idx[b]] += me[a, b]
    return K.tocsr(), M.tocsr()


def fe_q1(Nel: int, d: int, bc: str = "dirichlet", potential=None):
    """Stiffness K (+ lumped-mass potential) and consistent mass M of tensor
    bilinear/trilinear elements on the unit box with Nel elements per side.

    For tensor-product elements on a uniform mesh the element matrices are
    Kronecker products of the 1-D ones, so the global matrices are
    K = sum_a (M1 x .. x K1(a) x .. x M1) and M = M1 x .. x M1.
    bc = "dirichlet" keeps interior nodes only; "natural" keeps all nodes.
    The potential (one value per kept node) enters as diag(m_L * V), where
    m_L is the row sum of M (lumped mass).
    Returns (A, B) with A = K + M_L V and B = M.
    """
    h = 1.0 / Nel
    K1, M1 = _fe1d(Nel, h)
    if bc == "dirichlet":
        keep = np.arange(1, Nel)
        K1 = K1[keep][:, keep]
        M1 = M1[keep][:, keep]
    elif bc != "natural":
        raise ValueError(bc)
    n1 = K1.shape[0]
    K = None
    for a in range(d):
        term = None
        for b in reversed(range(d)):
            m = K1 if b == a else M1
            term = m if term is None else sp.kron(term, m, format="csr")
        K = term if K is None else K + term
    M = None
    for b in range(d):
        M = M1 if M is None else sp.kron(M, M1, format="csr")
    K = K.tocsr()
    M = M.tocsr()
    if potential is not None:
        mL = np.asarray(M.sum(axis=1)).ravel()
        K = K + sp.diags(mL * np.asarray(potential, dtype=np.float64).ravel())
    assert K.shape == (n1**d, n1**d)
    return K.tocsr(), M


def norm1(M) -> float:
    """Exact matrix 1-norm (largest absolute column sum)."""
    return float(np.abs(M).sum(axis=0).max())
