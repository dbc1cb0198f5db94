"""Bloch-periodic complex block products (plhr_op_apply) against the
oracle's sparse Bloch Hamiltonian: element by element on small boxes
(ragged and wide column counts, one- and two-point directions,
potential and shift), an empty block, and at the periodic model's full
size (96^3, 32 columns) on sampled rows, face and corner points
included, plus Hermitian symmetry of the product there."""
import numpy as np
import pytest

import workloads as wl
from oracle import operators as ops

pytestmark = pytest.mark.gpu

THETAS = wl.bloch_thetas()


def _apply(X, dims, **kw):
    from paper_1408_0042_amd.plhr import bloch_apply
    from tests.gpu_util import dev, host
    pot = kw.pop("potential", None)
    Y = bloch_apply(dev(X), dims, potential=None if pot is None else dev(pot), **kw)
    return host(Y)


@pytest.mark.parametrize("dims,ncols", [((8, 6, 5), 1), ((8, 6, 5), 7), ((12, 10, 9), 33),
                                        ((1, 4, 3), 5), ((2, 2, 2), 3), ((16, 16, 16), 32),
                                        ((5, 1, 1), 2), ((160, 3, 2), 12), ((40, 3, 2), 50)])
def test_bloch_block_product_matches_oracle(dims, ncols):
    n = int(np.prod(dims))
    pot = wl.periodic_gaussian_potential(max(dims), 4, (130, n), d=3)
    pot = pot.reshape((max(dims),) * 3)[:dims[2], :dims[1], :dims[0]].ravel().copy()
    X = wl.start_block(n, ncols, (131, n, ncols), dtype=np.complex128)
    for h, scale, shift, p in ((1.0, 0.5, 0.0, None), (0.7, 1.3, 2.25, pot)):
        A = ops.bloch_periodic(dims, h, THETAS, scale=scale, potential=p)
        ref = A @ X - shift * X
        Y = _apply(X, dims, h=h, thetas=THETAS, scale=scale, potential=p, shift=shift)
        assert np.abs(Y - ref).max() <= 1e-14 * np.abs(ref).max(), (dims, ncols, h, shift)


def test_bloch_empty_block_is_a_no_op():
    import torch
    from paper_1408_0042_amd.plhr import bloch_apply
    X = torch.empty((4 * 4 * 4, 0), dtype=torch.complex128, device="cuda")
    Y = bloch_apply(X, (4, 4, 4), thetas=THETAS)
    assert Y.shape == (64, 0)


def test_bloch_full_size_sampled_rows_and_hermitian():
    """The periodic model at 96^3 (n = 884,736) with 64 Gaussian wells and
    32 columns: sampled rows against the oracle's sparse rows, and
    <X2, A X1> = <A X2, X1> over the whole box."""
    import torch
    from paper_1408_0042_amd.plhr import bloch_apply
    from tests.gpu_util import dev, host
    N, ncols = 96, 32
    dims = (N, N, N)
    n = N ** 3
    pot = wl.periodic_gaussian_potential(N, 64, (3, 1))
    A = ops.bloch_periodic(dims, 1.0, THETAS, scale=0.5, potential=pot)
    X = wl.start_block(n, ncols, (3, 0), dtype=np.complex128)
    Xd, potd = dev(X), dev(pot)
    Y = bloch_apply(Xd, dims, thetas=THETAS, potential=potd, shift=1.5)
    g = np.random.default_rng(132)
    corners = [i + N * (j + N * l) for i in (0, N - 1) for j in (0, N - 1) for l in (0, N - 1)]
    faces = [int(g.integers(N)) + N * (int(g.integers(N)) + N * l) for l in (0, N - 1)
             for _ in range(64)]
    rows = np.unique(np.concatenate([g.choice(n, 2000, replace=False), corners, faces]))
    ref = A[rows] @ X - 1.5 * X[rows]
    Ys = host(Y[torch.from_numpy(rows).cuda()])
    assert np.abs(Ys - ref).max() <= 1e-14 * np.abs(ref).max()
    # Hermitian: sum conj(X2) (A X1) equals sum conj(A X2) X1 column by column
    X2d = dev(wl.start_block(n, ncols, (3, 2), dtype=np.complex128))
    Y2 = bloch_apply(X2d, dims, thetas=THETAS, potential=potd, shift=1.5)
    lhs = host((X2d.conj() * Y).sum(0))
    rhs = host((Y2.conj() * Xd).sum(0))
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(lhs).max()
