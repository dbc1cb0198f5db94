"""Hellmann-Feynman eigenvalue gradient (oracle; test infrastructure only).

For a Hermitian pencil A(p) v = lam B v whose A depends on a potential p
through A = L + diag(w * p) (w = 1 for finite differences, the lumped mass
for finite elements) and a simple eigenvalue lam with eigenvector v,
first-order perturbation theory gives

    d lam / d p_x = w_x |v(x)|^2 / (v^* B v).

For a loss L(lam_1..lam_k) the chain rule sums this over j with weights
dL/dlam_j.  This is not part of the paper; it is the standard first-order
eigenvalue perturbation formula.
"""
from __future__ import annotations

import numpy as np


def eigval_grad(V: np.ndarray, dL_dlam: np.ndarray, B=None, w=None) -> np.ndarray:
    V = np.asarray(V)
    BV = V if B is None else B @ V
    vbv = np.real(np.sum(np.conj(V) * BV, axis=0))
    g = (np.abs(V) ** 2) @ (np.asarray(dL_dlam) / vbv)
    if w is not None:
        g = g * np.asarray(w)
    return g


def loss_and_grad_targets(lam: np.ndarray, targets: np.ndarray):
    """L = sum_j (lam_j - t_j)^2 and dL/dlam."""
    d = np.asarray(lam) - np.asarray(targets)
    return float(np.sum(d * d)), 2.0 * d
