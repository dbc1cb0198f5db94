"""Pins of the oracle's multigrid V-cycle (CPU only): T must be Hermitian
positive definite (Section 5 of the paper) and a good approximation of the
inverse Laplacian."""
import numpy as np
import pytest

from oracle import mg, operators as ops


def _dense_T(V, n, dtype=np.float64):
    return V.apply(np.eye(n, dtype=dtype))


@pytest.mark.parametrize("dims,levels", [((8, 8), 3), ((16, 8), 3), ((4, 4, 4), 2),
                                         ((8, 8, 8), 3)])
def test_vcycle_symmetric_positive_definite(dims, levels):
    h = 1.0 / (dims[0] + 1)
    V = mg.VCycle("fd", dims, h, 1.0, levels)
    n = int(np.prod(dims))
    T = _dense_T(V, n)
    assert np.linalg.norm(T - T.T) <= 1e-12 * np.linalg.norm(T)
    assert np.linalg.eigvalsh(0.5 * (T + T.T)).min() > 0.0


def test_vcycle_single_level_is_exact_inverse():
    dims, h = (6, 5), 0.1
    V = mg.VCycle("fd", dims, h, 1.0, levels=1)
    A = ops.fd_dirichlet(dims, h).toarray()
    T = _dense_T(V, 30)
    assert np.allclose(T @ A, np.eye(30), atol=1e-12)


@pytest.mark.parametrize("dims,levels", [((16, 16), 3), ((32, 32), 4), ((8, 8, 8), 3)])
def test_vcycle_spectral_equivalence(dims, levels):
    """kappa(T A) is small and stays small as the grid is refined; a
    dropped coarse correction or a wrong restriction scale blows it up."""
    h = 1.0 / (dims[0] + 1)
    V = mg.VCycle("fd", dims, h, 1.0, levels)
    A = ops.fd_dirichlet(dims, h).toarray()
    T = _dense_T(V, A.shape[0])
    ev = np.linalg.eigvals(T @ A).real
    assert ev.min() > 0.0
    assert ev.max() / ev.min() < 3.0


def test_vcycle_reduces_error_like_a_solver():
    dims, h = (32, 32), 1 / 33
    V = mg.VCycle("fd", dims, h, 1.0, 4)
    A = ops.fd_dirichlet(dims, h)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(A.shape[0])
    b = A @ x
    e = x.copy()
    y = np.zeros_like(x)
    for _ in range(12):
        y = y + V.apply(b - A @ y)
    # a stationary iteration with T converges at a grid-independent rate
    assert np.linalg.norm(y - x) <= 1e-3 * np.linalg.norm(e)


def test_bloch_vcycle_hermitian_positive_definite():
    dims = (8, 8, 4)
    V = mg.VCycle("bloch", dims, 1.0, 0.5, 3, thetas=(0.6, 1.2, 1.8))
    n = int(np.prod(dims))
    T = _dense_T(V, n, np.complex128)
    assert np.linalg.norm(T - T.conj().T) <= 1e-12 * np.linalg.norm(T)
    assert np.linalg.eigvalsh(0.5 * (T + T.conj().T)).min() > 0.0


def test_restriction_is_scaled_transpose_of_prolongation():
    V = mg.VCycle("fd", (8, 8, 8), 1 / 9, 1.0, 2)
    P = V.P[0].toarray()
    # every interior fine point interpolates with weights summing to one
    rows = P.sum(axis=1)
    assert np.isclose(rows.max(), 1.0)
    # each coarse column's weights sum to 2^d away from the boundary
    assert np.isclose(P.sum(axis=0).max(), 8.0)
