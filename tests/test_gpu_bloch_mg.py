"""The multigrid preconditioner of the complex Bloch operator
(plhr_bloch_prec_*) against the oracle's Bloch V-cycle, element by element:
cubic and non-cubic boxes (a coarsest grid with one point in a direction),
one to three levels, one and two sweeps, ragged column counts, a block
whose rows exceed the LDS staging of the transfers, the
periodic model's full grid (96^3, 5 levels); T Hermitian and positive
definite on random blocks; an empty block."""
import numpy as np
import pytest

import workloads as wl
from oracle import mg

pytestmark = pytest.mark.gpu

THETAS = wl.bloch_thetas()


def _gpu_T(X, dims, h, scale, levels, nu, omega):
    from paper_1408_0042_amd.plhr import BlochPrecond
    from tests.gpu_util import dev, host
    T = BlochPrecond(dims, h=h, thetas=THETAS, scale=scale, levels=levels, nu=nu, omega=omega,
                     max_cols=max(1, X.shape[1]))
    Y = host(T.apply(dev(X)))
    T.close()
    return Y


@pytest.mark.parametrize("dims,h,scale,levels,nu,omega,ncols", [
    ((8, 8, 8), 1.0, 0.5, 3, 2, 2 / 3, 5),
    ((16, 8, 4), 0.8, 1.0, 3, 1, 0.6, 33),
    ((6, 4, 2), 1.0, 0.5, 1, 2, 2 / 3, 3),
    ((12, 12, 12), 1.0, 0.5, 2, 2, 2 / 3, 1),
    ((16, 4, 4), 1.0, 0.5, 2, 2, 2 / 3, 600),   # rows over 64 KB: gathering transfers
])
def test_bloch_vcycle_matches_oracle(dims, h, scale, levels, nu, omega, ncols):
    n = int(np.prod(dims))
    X = wl.start_block(n, ncols, (140, n, ncols), dtype=np.complex128)
    V = mg.VCycle("bloch", dims, h, scale, levels, nu_pre=nu, nu_post=nu, omega=omega,
                  thetas=THETAS)
    ref = V.apply(X)
    Y = _gpu_T(X, dims, h, scale, levels, nu, omega)
    assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max(), (dims, levels)


def test_bloch_vcycle_hermitian_positive_definite():
    import torch
    from paper_1408_0042_amd.plhr import BlochPrecond
    from tests.gpu_util import dev, host
    dims = (16, 16, 16)
    n = 16 ** 3
    T = BlochPrecond(dims, thetas=THETAS, levels=3, max_cols=6)
    X1 = dev(wl.start_block(n, 6, (141, 0), dtype=np.complex128))
    X2 = dev(wl.start_block(n, 6, (141, 1), dtype=np.complex128))
    Y1, Y2 = T.apply(X1), T.apply(X2)
    lhs = host((X2.conj() * Y1).sum(0))
    rhs = host((Y2.conj() * X1).sum(0))
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(lhs).max()
    q = host((X1.conj() * Y1).sum(0))
    assert np.all(q.real > 0) and np.abs(q.imag).max() <= 1e-12 * q.real.max()
    Z = torch.empty((n, 0), dtype=torch.complex128, device="cuda")
    assert T.apply(Z).shape == (n, 0)
    T.close()


def test_bloch_vcycle_full_grid_matches_oracle():
    """96^3 (n = 884,736), 5 levels down to 6^3, 8 columns (the kernels
    take the same path at every column count)."""
    N, ncols = 96, 8
    dims = (N, N, N)
    X = wl.start_block(N ** 3, ncols, (3, 3), dtype=np.complex128)
    V = mg.VCycle("bloch", dims, 1.0, 0.5, 5, thetas=THETAS)
    ref = V.apply(X)
    Y = _gpu_T(X, dims, 1.0, 0.5, 5, 2, 2 / 3)
    assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max()


def test_bloch_vcycle_in_a_caller_workspace_is_bitwise_equal():
    """With a caller workspace (no device allocation by the handle) the
    V-cycle is the same arithmetic on the same level sizes: bitwise equal
    to the one in the library's own buffers."""
    import torch
    from paper_1408_0042_amd.plhr import BlochPrecond
    from tests.gpu_util import dev, host
    dims, cols = (16, 8, 8), 7
    kw = dict(thetas=THETAS, levels=3, nu=2, max_cols=cols)
    nbytes = BlochPrecond.workspace_bytes(dims, **kw)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    ws = ws[off:off + nbytes]
    X = dev(wl.start_block(16 * 8 * 8, cols, (142, 0), dtype=np.complex128))
    T1 = BlochPrecond(dims, workspace=ws, **kw)
    T0 = BlochPrecond(dims, **kw)
    Y1, Y0 = host(T1.apply(X)), host(T0.apply(X))
    T1.close()
    T0.close()
    assert np.array_equal(Y1, Y0)
