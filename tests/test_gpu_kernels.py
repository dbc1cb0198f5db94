"""Element-wise parity of the HIP operator and preconditioner kernels with
the oracle (sparse stencil products, multigrid V-cycle)."""
import numpy as np
import pytest

import workloads as wl
from oracle import mg, operators as ops

pytestmark = pytest.mark.gpu


def _solver(kind, dims, h, sigma, k, precond=None, scale=1.0, pot=None, k_extra=1,
            precision="fp64"):
    from paper_1408_0042_amd.plhr import Solver
    from tests.gpu_util import dev
    return Solver(kind, dims, h, sigma, k, scale=scale, precond=precond,
                  potential=None if pot is None else dev(pot), k_extra=k_extra,
                  precision=precision)


@pytest.mark.parametrize("kind,dims,ncols", [("fd5_2d", (33, 17), 5), ("fd7_3d", (12, 9, 7), 6),
                                             ("fd7_3d", (64, 64, 64), 34)])
def test_stencil_parity(kind, dims, ncols):
    from tests.gpu_util import dev, host
    h, sigma = 0.05, 123.25
    pot = np.random.default_rng(1).uniform(-3, 3, int(np.prod(dims)))
    S = _solver(kind, dims, h, sigma, (ncols + 1) // 2 - 1 or 1, scale=0.7, pot=pot)
    A = ops.fd_dirichlet(dims, h, 0.7, potential=pot)
    X = wl.start_block(A.shape[0], ncols, (31, ncols))
    for which, ref in (("A", A @ X), ("A-sigma", A @ X - sigma * X)):
        Y = host(S.apply(which, dev(X)))
        err = np.abs(Y - ref).max() / np.abs(ref).max()
        assert err < 1e-14, (which, err)
    S.close()


@pytest.mark.parametrize("kind,dims,levels,ncols", [("fd5_2d", (32, 32), 4, 5),
                                                    ("fd5_2d", (16, 16), 3, 6),
                                                    ("fd7_3d", (16, 16, 8), 3, 4),
                                                    ("fd7_3d", (64, 64, 64), 5, 34)])
def test_vcycle_parity(kind, dims, levels, ncols):
    from tests.gpu_util import dev, host
    h = 1.0 / (dims[0] + 1)
    S = _solver(kind, dims, h, 10.0, (ncols + 1) // 2 - 1 or 1,
                precond={"levels": levels, "nu": 2, "omega": 2 / 3})
    V = mg.VCycle("fd", dims, h, 1.0, levels)
    X = wl.start_block(int(np.prod(dims)), ncols, (32, ncols))
    Y = host(S.apply("T", dev(X)))
    ref = V.apply(X)
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    assert err < 1e-13, err
    S.close()


@pytest.mark.parametrize("kind,dims,levels,ncols", [("fd5_2d", (32, 32), 4, 5),
                                                    ("fd7_3d", (16, 16, 8), 3, 4),
                                                    ("fd7_3d", (64, 64, 64), 5, 34)])
def test_vcycle_parity_mixed(kind, dims, levels, ncols):
    """The FP32 V-cycle of the mixed mode against the FP64 oracle V-cycle:
    every level rounds to FP32 (unit roundoff 6e-8), and the error of a few
    dozen stencil sweeps and transfers stays below 2e-6 of the output."""
    from tests.gpu_util import dev, host
    h = 1.0 / (dims[0] + 1)
    S = _solver(kind, dims, h, 10.0, (ncols + 1) // 2 - 1 or 1,
                precond={"levels": levels, "nu": 2, "omega": 2 / 3}, precision="mixed")
    V = mg.VCycle("fd", dims, h, 1.0, levels)
    X = wl.start_block(int(np.prod(dims)), ncols, (33, ncols))
    Y = host(S.apply("T", dev(X)))
    ref = V.apply(X)
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    assert 1e-12 < err < 2e-6, err   # FP32 really used, and accurate to FP32
    S.close()
