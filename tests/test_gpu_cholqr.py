"""Complex Cholesky-QR (plhr_cholqr_c128) against the oracle's
orthonormalisation (Gram-Schmidt with one reorthogonalisation, whose
result with positive real diagonal is the unique QR factor): Q element by
element and R = Q^H Z for 1 to 64 columns; Q^H Q = I and Q R = Z at the
periodic model's size (n = 96^3, m = 64); dependent columns reported."""
import numpy as np
import pytest

import workloads as wl
from oracle import plhr as alg

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,m", [(5000, 1), (5000, 7), (4099, 33), (20000, 64)])
def test_complex_cholqr_matches_oracle(n, m):
    from paper_1408_0042_amd.plhr import cholqr_c128
    from tests.gpu_util import dev, host
    Z = wl.start_block(n, m, (160, n, m), dtype=np.complex128)
    Qd, Rd = cholqr_c128(dev(Z))
    Q, R = host(Qd), host(Rd)
    Qo, labels = alg.b_orthonormalize([("V", Z)], None)
    assert len(labels) == m
    assert np.abs(Q - Qo).max() <= 1e-12 * np.abs(Qo).max(), (n, m)
    Ro = Qo.conj().T @ Z
    assert np.abs(np.tril(R, -1)).max() == 0.0
    assert np.all(np.diag(R).real > 0) and np.all(np.diag(R).imag == 0)
    assert np.abs(R - np.triu(Ro)).max() <= 1e-12 * np.abs(Ro).max()
    assert np.abs(Q.conj().T @ Q - np.eye(m)).max() <= 1e-13


def test_complex_cholqr_reports_dependent_columns():
    from paper_1408_0042_amd import _lib as L
    from paper_1408_0042_amd.plhr import cholqr_c128
    from tests.gpu_util import dev
    Z = wl.start_block(3000, 6, (161, 0), dtype=np.complex128)
    Z[:, 4] = (2.0 - 1.0j) * Z[:, 1]
    with pytest.raises(L.PLHRError) as e:
        cholqr_c128(dev(Z))
    assert e.value.code == L.ERR_NOT_HPD


def test_complex_cholqr_at_the_periodic_model_size():
    from paper_1408_0042_amd.plhr import cholqr_c128
    from tests.gpu_util import dev, host
    n, m = 96 ** 3, 64
    Z = wl.start_block(n, m, (3, 5), dtype=np.complex128)
    Qd, Rd = cholqr_c128(dev(Z))
    Q, R = host(Qd), host(Rd)
    assert np.abs(Q.conj().T @ Q - np.eye(m)).max() <= 1e-13
    rows = np.random.default_rng(162).choice(n, 3000, replace=False)
    assert np.abs(Q[rows] @ R - Z[rows]).max() <= 1e-13 * np.abs(Z).max()
