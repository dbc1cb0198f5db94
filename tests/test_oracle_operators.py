"""Pins of the oracle's operator assembly against closed forms and the
values the paper prints (CPU only)."""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import operators as ops
from tests import closed_forms as cf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("dims,h,scale", [((6, 7), 1 / 8, 1.0), ((4, 5, 3), 0.3, 0.5),
                                          ((32, 32), 1 / 33, 1.0)])
def test_fd_dirichlet_spectrum_closed_form(dims, h, scale):
    A = ops.fd_dirichlet(dims, h, scale)
    ev = np.linalg.eigvalsh(A.toarray())
    ref = cf.fd_dirichlet_eigs(dims, h, scale)
    assert np.allclose(ev, ref, rtol=1e-12, atol=1e-9 * ref.max())


def test_fd_dirichlet_eigenvector_is_sine_product():
    dims, h = (5, 6, 4), 0.25
    A = ops.fd_dirichlet(dims, h)
    idx = (2, 5, 3)
    v = cf.fd_dirichlet_mode(dims, idx)
    lam = sum((4 / h**2) * math.sin(i * math.pi / (2 * (N + 1))) ** 2 for N, i in zip(dims, idx))
    assert np.linalg.norm(A @ v - lam * v) <= 1e-12 * lam * np.linalg.norm(v)


def test_fd_config1_targets():
    # the four eigenvalues nearest sigma = 0.4 lambda_max of the 32x32 problem
    h = 1 / 33
    ev = cf.fd_dirichlet_eigs((32, 32), h)
    sigma = 0.4 * ev.max()
    near = np.sort(ev[np.argsort(np.abs(ev - sigma), kind="stable")[:4]])
    assert np.allclose(near, [3480.72324640789, 3480.72324640789, 3492.06128911250,
                              3492.06128911250], rtol=1e-13)


def test_potential_is_diagonal_shift():
    dims, h = (5, 4), 0.2
    pot = np.linspace(-1, 2, 20)
    A0 = ops.fd_dirichlet(dims, h)
    A1 = ops.fd_dirichlet(dims, h, potential=pot)
    assert np.allclose((A1 - A0).toarray(), np.diag(pot))


def test_norm1_fd():
    h = 1 / 17
    assert ops.norm1(ops.fd_dirichlet((16, 16), h)) == pytest.approx(8 / h**2, rel=1e-14)
    assert ops.norm1(ops.fd_dirichlet((8, 8, 8), h)) == pytest.approx(12 / h**2, rel=1e-14)


def test_bloch_hermitian_and_closed_form():
    dims, thetas = (5, 4, 3), (0.7, -1.3, 2.1)
    A = ops.bloch_periodic(dims, 1.0, thetas, scale=0.5)
    Ad = A.toarray()
    assert np.allclose(Ad, Ad.conj().T)
    ev = np.linalg.eigvalsh(Ad)
    assert np.allclose(ev, cf.bloch_eigs(dims, 1.0, thetas, 0.5), atol=1e-12)


@pytest.mark.parametrize("d,Nel,bc", [(2, 6, "dirichlet"), (2, 5, "natural"), (3, 4, "dirichlet"),
                                      (3, 3, "natural")])
def test_fe_q1_closed_form(d, Nel, bc):
    K, M = ops.fe_q1(Nel, d, bc)
    ev = sla.eigh(K.toarray(), M.toarray(), eigvals_only=True)
    ref = cf.fe_q1_eigs(Nel, d, bc)
    assert np.allclose(ev, ref, rtol=1e-10, atol=1e-9)


def _golden_fe():
    rows = []
    with open(os.path.join(GOLDEN, "paper_fe_eigenvalues.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            lab, sig, val, dig = line.split()
            rows.append((lab, float(sig), float(val), int(dig)))
    return rows


@pytest.mark.parametrize("lab,sigma,printed,digits", _golden_fe())
def test_fe_paper_printed_eigenvalues(lab, sigma, printed, digits):
    """Section 6.1: 50x50 bilinear elements, the eigenvalue closest to
    sigma matches the paper's printed value to all printed digits."""
    K, M = ops.fe_q1(50, 2, "dirichlet")
    assert K.shape[0] == 2401
    vals = spla.eigsh(K.tocsc(), k=6, M=M.tocsc(), sigma=sigma, which="LM",
                      return_eigenvectors=False)
    near = vals[np.argmin(np.abs(vals - sigma))]
    assert abs(near - printed) <= 0.5 * 10.0 ** (-digits)
    # and the closed form agrees with the assembly
    ref = cf.fe_q1_eigs(50, 2)
    assert np.min(np.abs(ref - near)) <= 1e-9 * near
