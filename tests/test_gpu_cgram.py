"""Complex Hermitian Gram products (plhr_gram_c128) against their
definition X^H Y in FP64 on the host: odd and ragged column counts,
several column chunks, X = Y (Hermitian result), no rows, and the periodic
model's size (n = 96^3, m = 128 = 4 (k + k_extra) for k = 32), with the
elementwise bound c eps |X|^T |Y| of a summation over rows."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _check(n, mx, my, same=False, seed=0):
    from paper_1408_0042_amd.plhr import gram_c128
    from tests.gpu_util import dev, host
    X = wl.start_block(n, mx, (150, n, mx, seed), dtype=np.complex128)
    Y = X if same else wl.start_block(n, my, (151, n, my, seed), dtype=np.complex128)
    Xd = dev(X)
    G = host(gram_c128(Xd, None if same else dev(Y)))
    ref = X.conj().T @ Y
    bound = 1e-13 * (np.abs(X).T @ np.abs(Y))
    assert np.all(np.abs(G - ref) <= bound + 1e-300), (n, mx, my)
    return G


@pytest.mark.parametrize("n,mx,my", [(1000, 5, 7), (4099, 64, 100), (3000, 70, 200),
                                     (257, 1, 1), (20000, 128, 128)])
def test_complex_gram_matches_definition(n, mx, my):
    _check(n, mx, my)


def test_complex_gram_of_a_block_with_itself_is_hermitian():
    G = _check(5000, 84, 84, same=True)
    assert np.abs(G - G.conj().T).max() <= 1e-13 * np.abs(G).max()
    assert np.all(np.diag(G).real > 0)


def test_complex_gram_without_rows_is_zero():
    import torch
    from paper_1408_0042_amd.plhr import gram_c128
    X = torch.empty((0, 6), dtype=torch.complex128, device="cuda")
    G = gram_c128(X, torch.empty((0, 4), dtype=torch.complex128, device="cuda"))
    assert G.shape == (6, 4) and not bool(G.abs().max() > 0)


def test_complex_gram_at_the_periodic_model_size():
    _check(96 ** 3, 128, 128, same=True, seed=1)
