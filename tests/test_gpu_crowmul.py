"""Complex block products Y = Z M (plhr_rowmul_c128), the block updates of
the complex iteration, against their definition in FP64 on the host under
the elementwise bound c eps |Z||M|: odd, ragged and full column counts,
no rows, and the periodic model's size (n = 96^3, m = 64, k = 32) on
sampled rows."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,m,k", [(5000, 7, 5), (4099, 64, 64), (1000, 1, 1), (3001, 33, 17),
                                   (77, 64, 3)])
def test_complex_block_product_matches_definition(n, m, k):
    from paper_1408_0042_amd.plhr import rowmul_c128
    from tests.gpu_util import dev, host
    Z = wl.start_block(n, m, (170, n, m), dtype=np.complex128)
    M = wl.start_block(m, k, (171, m, k), dtype=np.complex128)
    Y = host(rowmul_c128(dev(Z), dev(M)))
    ref = Z @ M
    assert np.all(np.abs(Y - ref) <= 1e-14 * (np.abs(Z) @ np.abs(M)) + 1e-300), (n, m, k)


def test_complex_block_product_without_rows():
    import torch
    from paper_1408_0042_amd.plhr import rowmul_c128
    Z = torch.empty((0, 5), dtype=torch.complex128, device="cuda")
    M = torch.ones((5, 3), dtype=torch.complex128, device="cuda")
    assert rowmul_c128(Z, M).shape == (0, 3)


def test_complex_block_product_at_the_periodic_model_size():
    from paper_1408_0042_amd.plhr import rowmul_c128
    from tests.gpu_util import dev, host
    n, m, k = 96 ** 3, 64, 32
    Z = wl.start_block(n, m, (3, 6), dtype=np.complex128)
    M = wl.start_block(m, k, (3, 7), dtype=np.complex128)
    Y = host(rowmul_c128(dev(Z), dev(M)))
    rows = np.random.default_rng(172).choice(n, 4000, replace=False)
    ref = Z[rows] @ M
    assert np.all(np.abs(Y[rows] - ref) <= 1e-14 * (np.abs(Z[rows]) @ np.abs(M)) + 1e-300)
