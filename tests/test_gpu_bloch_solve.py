"""The block iteration in complex arithmetic (Algorithm 2) on the complex
Hermitian Bloch operator, on the GPU: per-step Rayleigh quotients against
the oracle's Algorithm 2 (T = I and the Bloch V-cycle), converged pairs
against the dense eigenvalues and eigenvectors, and graph replay against
eager launches."""
import numpy as np
import pytest

import workloads as wl
from oracle import mg, operators as ops, plhr

pytestmark = pytest.mark.gpu

THETAS = wl.bloch_thetas()

# (box, eigenvalues below sigma, k, V-cycle levels or 0 for T = I)
CASES = {
    "8x8x4_vcycle": ((8, 8, 4), 3, 2, 3),
    "8x8x8_identity": ((8, 8, 8), 3, 2, 0),
    "6x6x6_vcycle": ((6, 6, 6), 4, 2, 2),
    "4x4x8_identity": ((4, 4, 8), 3, 2, 0),
}


def _problem(name):
    dims, nb, k, lev = CASES[name]
    n = int(np.prod(dims))
    pot = wl.rng(150, 1).uniform(-2.0, 0.0, n)
    A = ops.bloch_periodic(dims, 1.0, THETAS, scale=0.5, potential=pot)
    ev = np.linalg.eigvalsh(A.toarray())
    sigma = wl.shift_between(ev, nb, 0.4)
    T = mg.VCycle("bloch", dims, 1.0, 0.5, lev, nu_pre=2, nu_post=2,
                  thetas=THETAS).apply if lev else None
    prob = plhr.Problem(A=A, T=T, sigma=sigma)
    pre = {"levels": lev, "nu": 2, "omega": 2 / 3} if lev else None
    return dims, n, k, pot, A, ev, sigma, prob, pre


def _solver(dims, pot, sigma, k, pre, **kw):
    from paper_1408_0042_amd.plhr import Solver
    from tests.gpu_util import dev
    return Solver("bloch7_3d", dims, 1.0, sigma, k, scale=0.5, potential=dev(pot), precond=pre,
                  thetas=THETAS, lock=False, **kw)


@pytest.mark.parametrize("name", ["8x8x4_vcycle", "8x8x8_identity", "6x6x6_vcycle"])
def test_bloch_block_steps_match_oracle(name):
    from tests.gpu_util import dev, host
    dims, n, k, pot, A, ev, sigma, prob, pre = _problem(name)
    print(f"case {name} n={n} k={k} sigma={sigma:.6f}", flush=True)
    V0 = wl.start_block(n, k + 1, (151, 0), dtype=np.complex128)
    o = plhr.BPLHR(prob, V0, k, real=False, lock=False)
    S = _solver(dims, pot, sigma, k, pre)
    S.start(dev(V0))
    lam, V = S.state()
    assert np.array_equal(lam[0::2], lam[1::2])
    assert np.allclose(lam[0::2], o.lam, rtol=1e-12)
    # the start block is held as given (complex128, interleaved)
    assert np.array_equal(host(V), V0)
    for it in range(10):
        o.step()
        S.iterate(1)
        lam, _ = S.state()
        assert np.array_equal(lam[0::2], lam[1::2]), it
        assert np.allclose(np.sort(lam[0::2]), np.sort(o.lam), rtol=1e-9, atol=1e-11), \
            (it, lam[0::2], o.lam)
    S.close()


def test_bloch_block_soft_locking_matches_oracle():
    """Soft locking in the complex block iteration: a column whose relative
    residual is at or below tol generates no W, S or P (both of its real
    columns).  At tol = 1e-6 the 8 x 8 x 4 case locks its first column
    after 29 steps and stops after 39 (measured on the oracle); every step's
    Rayleigh quotients and number of active columns equal the oracle's."""
    from paper_1408_0042_amd.plhr import Solver
    from tests.gpu_util import dev
    dims, n, k, pot, A, ev, sigma, prob, pre = _problem("8x8x4_vcycle")
    tol = 1e-6
    V0 = wl.start_block(n, k + 1, (151, 0), dtype=np.complex128)
    o = plhr.BPLHR(prob, V0, k, real=False, lock=True)
    o.tol = tol
    S = Solver("bloch7_3d", dims, 1.0, sigma, k, scale=0.5, potential=dev(pot), precond=pre,
               thetas=THETAS, lock=True, tol=tol, max_iters=200)
    S.start(dev(V0))
    locked_steps = 0
    for it in range(60):
        act = int(np.sum(o.residuals() > tol))
        info = S.iterate(1)
        if info.converged:
            wanted = plhr.wanted_columns(o.lam, sigma, k)
            assert np.all(o.residuals()[wanted] <= tol), it
            break
        assert info.n_active == 2 * act, (it, info.n_active, act)
        locked_steps += act < k + 1
        o.step()
        lam, _ = S.state()
        assert np.allclose(np.sort(lam[0::2]), np.sort(o.lam), rtol=1e-9, atol=1e-11), \
            (it, lam[0::2], o.lam)
    else:
        raise AssertionError("no convergence in 60 steps")
    assert locked_steps >= 5, locked_steps
    S.close()


# (with T = I the 8 x 8 x 8 case stalls near 1e-8 in the oracle as well)
@pytest.mark.parametrize("name", ["8x8x4_vcycle", "6x6x6_vcycle", "4x4x8_identity"])
def test_bloch_block_converges_to_the_dense_pairs(name):
    from tests.gpu_util import dev, host
    dims, n, k, pot, A, ev, sigma, prob, pre = _problem(name)
    print(f"case {name} n={n} k={k} sigma={sigma:.6f}", flush=True)
    V0 = wl.start_block(n, k + 1, (152, 0), dtype=np.complex128)
    S = _solver(dims, pot, sigma, k, pre, tol=1e-10, max_iters=2000)
    r = S.solve(dev(V0))
    assert r.converged
    lam = host(r.eigvals)
    V = host(r.V)
    assert V.dtype == np.complex128 and V.shape == (n, k)
    near = ev[np.argsort(np.abs(ev - sigma))[:k]]
    scale = np.abs(ev).max()
    # the returned order: nearest sigma first
    assert np.all(np.diff(np.abs(lam - sigma)) >= 0)
    assert np.abs(np.sort(lam) - np.sort(near)).max() < 1e-10 * scale
    assert np.all(r.rel_res <= 1e-10)
    Ad = A.toarray()
    res = Ad @ V - V * lam[None, :]
    assert np.abs(res).max() < 1e-7 * scale
    # orthonormal complex vectors in the eigenspace of the k values
    assert np.abs(V.conj().T @ V - np.eye(k)).max() < 1e-10
    w, U = np.linalg.eigh(Ad)
    Uk = U[:, np.argsort(np.abs(w - sigma))[:k]]
    sine = np.linalg.norm(V - Uk @ (Uk.conj().T @ V), axis=0)
    assert sine.max() < 1e-6
    assert np.abs(V.imag).max() > 0.1
    S.close()


def test_bloch_block_graph_replay_matches_eager():
    from tests.gpu_util import dev
    dims, n, k, pot, A, ev, sigma, prob, pre = _problem("8x8x4_vcycle")
    V0 = dev(wl.start_block(n, k + 1, (153, 0), dtype=np.complex128))
    lams = []
    for g in (False, True):
        S = _solver(dims, pot, sigma, k, pre, use_graph=g)
        S.start(V0)
        for _ in range(3):
            S.iterate(5)
            lams.append(S.state()[0])
        S.close()
    for a, b in zip(lams[:3], lams[3:]):
        assert np.array_equal(a, b)


def test_bloch_block_full_size_residuals_by_the_oracle_operator():
    """The periodic model at full size (96^3, n = 884736, 64 Gaussian wells,
    k = 8 + 2 complex columns, the Bloch V-cycle, sigma below the spectrum)
    as the benchmark runs it: every returned pair's relative residual,
    recomputed on the host with the oracle's sparse Bloch operator, meets
    the tolerance, and the vectors are orthonormal.  (That they are the 8
    lowest pairs is not checked: no dense or shift-invert solve of this
    size fits the host.)"""
    import torch
    from paper_1408_0042_amd.plhr import Solver
    from tests.gpu_util import host
    N, k, kx, sigma = 96, 8, 2, -4.0
    n = N ** 3
    potn = wl.periodic_gaussian_potential(N, 64, (3, 1))
    print(f"case bloch 96^3 k={k}+{kx} sigma={sigma}", flush=True)
    pot = torch.from_numpy(potn).cuda()
    V0 = torch.from_numpy(wl.start_block(n, k + kx, (3, 2), dtype=np.complex128)).cuda()
    S = Solver("bloch7_3d", (N, N, N), 1.0, sigma, k, scale=0.5, potential=pot,
               thetas=THETAS, precond={"levels": 5, "nu": 2, "omega": 2 / 3}, tol=1e-8,
               max_iters=3000, k_extra=kx, lock=False, check_every=25, use_graph=True)
    r = S.solve(V0)
    S.close()
    lam, V = host(r.eigvals), host(r.V)
    assert r.converged and np.all(np.diff(lam) >= 0)
    A = ops.bloch_periodic((N, N, N), 1.0, THETAS, scale=0.5, potential=potn)
    nA = abs(A).sum(axis=1).max()
    R = A @ V - V * lam[None, :]
    rel = np.linalg.norm(R, axis=0) / ((nA + np.abs(lam)) * np.linalg.norm(V, axis=0))
    assert rel.max() <= 1.5e-8, rel
    assert np.abs(V.conj().T @ V - np.eye(k)).max() < 1e-10
    assert np.all(lam > sigma) and np.all(lam < 0.0)   # bound states of the wells


def test_bloch_block_in_a_caller_workspace_is_bitwise_equal():
    """plhr_create with a caller workspace (the context and its Bloch
    V-cycle carve everything from it, no device allocation) gives the same
    bits as the library-allocated context."""
    import torch
    from tests.gpu_util import dev, host
    dims, n, k, pot, A, ev, sigma, prob, pre = _problem("8x8x4_vcycle")
    V0 = dev(wl.start_block(n, k + 1, (154, 0), dtype=np.complex128))
    S1 = _solver(dims, pot, sigma, k, pre, tol=1e-10, max_iters=2000)
    r1 = S1.solve(V0)
    nbytes = S1.workspace_bytes
    S1.close()
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-raw.data_ptr()) % 256
    ws = raw[off:off + nbytes]
    S2 = _solver(dims, pot, sigma, k, pre, tol=1e-10, max_iters=2000, workspace=ws)
    r2 = S2.solve(V0)
    S2.close()
    assert r1.converged and r2.converged and r1.iters == r2.iters
    assert np.array_equal(host(r1.eigvals), host(r2.eigvals))
    assert np.array_equal(host(r1.V), host(r2.V))
