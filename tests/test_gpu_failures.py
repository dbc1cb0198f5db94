"""Failure paths of the solver (raised from the host side inputs, every
kernel exits normally) and run-to-run reproducibility."""
import numpy as np
import pytest

import workloads as wl
from oracle import dense, operators as ops
from tests import closed_forms as cf
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _solver(**kw):
    from paper_1408_0042_amd.plhr import Solver
    return Solver(**kw)


def _small(**kw):
    N, h = 12, 1 / 13
    ev = cf.fd_dirichlet_eigs((N, N), h)
    u = np.unique(np.round(ev, 8))
    sigma = float(u[10] + 0.4 * (u[11] - u[10]))
    args = dict(kind="fd5_2d", dims=(N, N), h=h, sigma=sigma, k=3, k_extra=2, tol=1e-10,
                max_iters=3000, precond={"levels": 2, "nu": 2, "omega": 2 / 3})
    args.update(kw)
    return args, ev


def test_rank_deficient_start_block_is_a_breakdown():
    from paper_1408_0042_amd import _lib as L
    args, _ = _small()
    V0 = wl.start_block(144, 5, (80, 0))
    V0[:, 3] = V0[:, 1]
    S = _solver(**args)
    with pytest.raises(L.PLHRError) as e:
        S.solve(dev(V0))
    assert e.value.code == L.ERR_BREAKDOWN
    S.close()


def test_non_finite_start_block_is_a_breakdown():
    from paper_1408_0042_amd import _lib as L
    args, _ = _small()
    V0 = wl.start_block(144, 5, (81, 0))
    V0[7, 2] = np.nan
    S = _solver(**args)
    with pytest.raises(L.PLHRError) as e:
        S.solve(dev(V0))
    assert e.value.code == L.ERR_BREAKDOWN
    S.close()


def test_max_iters_returns_not_converged_with_the_best_iterate():
    from paper_1408_0042_amd import _lib as L
    args, ev = _small(max_iters=3)
    S = _solver(**args)
    r = S.solve(dev(wl.start_block(144, 5, (82, 0))), allow_unconverged=True)
    assert not r.converged and r.iters == 3
    assert np.all(np.isfinite(host(r.eigvals))) and np.all(np.isfinite(r.rel_res))
    assert np.all(r.rel_res > 0)
    with pytest.raises(L.PLHRError) as e:
        S.solve(dev(wl.start_block(144, 5, (82, 0))))
    assert e.value.code == L.ERR_NOT_CONVERGED
    S.close()


def test_start_block_of_exact_eigenvectors_converges_at_once():
    """V0 holding the k + k_extra nearest sine modes: the residual check
    before the first step is already met."""
    args, ev = _small()
    N = 12
    sigma = args["sigma"]
    modes = [(i, j) for i in range(1, N + 1) for j in range(1, N + 1)]
    lam = np.array([(4 * 169.0) * (np.sin(i * np.pi / 26) ** 2 + np.sin(j * np.pi / 26) ** 2)
                    for i, j in modes])
    pick = np.lexsort((lam, np.abs(lam - sigma)))[:5]
    V0 = np.column_stack([cf.fd_dirichlet_mode((N, N), modes[p]) for p in pick])
    S = _solver(**args)
    r = S.solve(dev(np.ascontiguousarray(V0)))
    assert r.converged and r.iters == 0
    ref = np.sort(ev[np.lexsort((ev, np.abs(ev - sigma)))][:3])
    assert np.allclose(np.sort(host(r.eigvals)), ref, rtol=1e-12)
    S.close()


def test_shift_on_an_eigenvalue():
    """sigma exactly on a (double) eigenvalue: (A - sigma B) annihilates
    the wanted eigenvectors, so G_L and G_R of eq. (3.5) lose rank along
    them and the T-harmonic extraction cannot single them out; the oracle
    stalls near relative residual 1e-3 here as well.  The GPU must come
    back cleanly: converged or PLHR_ERR_NOT_CONVERGED with finite outputs
    no farther from sigma than the nearest other eigenvalue (the pairs the
    extraction can see; which of these it returns depends on rounding),
    never a breakdown or a non-finite value."""
    from paper_1408_0042_amd import _lib as L
    args, ev = _small(max_iters=400)
    u = np.unique(np.round(ev, 8))
    sigma = float(ev[np.argmin(np.abs(ev - u[10]))])     # a double eigenvalue
    args.update(sigma=sigma, k=2, k_extra=3)
    S = _solver(**args)
    r = S.solve(dev(wl.start_block(144, 5, (83, 0))), allow_unconverged=True)
    lam = host(r.eigvals)
    assert np.all(np.isfinite(lam)) and np.all(np.isfinite(host(r.V)))
    assert np.all(np.isfinite(r.rel_res))
    gap = np.min(np.abs(u[np.abs(u - sigma) > 1e-6 * sigma] - sigma))
    assert np.all(np.abs(lam - sigma) <= gap * (1.0 + 1e-6)), (lam, sigma, gap)
    S.close()


def test_repeated_solves_are_bitwise_identical():
    """No atomics and fixed reduction orders: two solves from the same
    start block give the same bits (eigenvalues, vectors, residuals and
    iteration count)."""
    args, _ = _small()
    V0 = dev(wl.start_block(144, 5, (84, 0)))
    S = _solver(**args)
    r1 = S.solve(V0)
    a = (host(r1.eigvals).copy(), host(r1.V).copy(), r1.rel_res.copy(), r1.iters)
    r2 = S.solve(V0)
    b = (host(r2.eigvals), host(r2.V), r2.rel_res, r2.iters)
    assert a[3] == b[3]
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    S.close()
    S2 = _solver(**args)
    r3 = S2.solve(V0)
    assert r3.iters == a[3] and np.array_equal(host(r3.V), a[1])
    S2.close()


def test_a_smaller_context_does_not_break_a_larger_one():
    """Kernel LDS limits are process-wide: creating a context with a
    narrower trial subspace after a wider one must leave the wider one
    working."""
    from tests.gpu_util import dev
    N, h = 32, 1 / 33
    ev = cf.fd_dirichlet_eigs((N, N), h)
    u = np.unique(np.round(ev, 8))
    sigma = float(u[32] + 0.4 * (u[33] - u[32]))
    big = _solver(kind="fd5_2d", dims=(N, N), h=h, sigma=sigma, k=16, k_extra=5, tol=1e-8,
                  max_iters=3, precond={"levels": 3, "nu": 2, "omega": 2 / 3})
    small = _solver(kind="fd5_2d", dims=(N, N), h=h, sigma=sigma, k=1, k_extra=1, tol=1e-8,
                    max_iters=3)
    small.solve(dev(wl.start_block(N * N, 2, (85, 0))), allow_unconverged=True)
    r = big.solve(dev(wl.start_block(N * N, 21, (86, 0))), allow_unconverged=True)
    assert r.iters == 3 and np.all(np.isfinite(r.rel_res))
    big.close()
    small.close()


def test_caller_workspace_is_bitwise_equal():
    """plhr_create with a caller workspace (no device allocation by the
    context, multigrid hierarchy included) gives the same bits as the
    library-allocated context."""
    import torch
    args, _ = _small()
    V0 = dev(wl.start_block(144, 5, (84, 0)))
    S1 = _solver(**args)
    r1 = S1.solve(V0)
    nbytes = S1.workspace_bytes
    S1.close()
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-raw.data_ptr()) % 256
    S2 = _solver(workspace=raw[off:off + nbytes], **args)
    r2 = S2.solve(V0)
    S2.close()
    assert r1.converged and r2.converged and r1.iters == r2.iters
    assert np.array_equal(host(r1.eigvals), host(r2.eigvals))
    assert np.array_equal(host(r1.V), host(r2.V))
