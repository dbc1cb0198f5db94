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


def test_bloch_vcycle_spectrally_equivalent():
    """kappa(T A_theta) stays small at nonzero phases: the transfer must
    pick up exp(-+i theta) across a periodic face in the right direction
    (the opposite sign keeps T Hermitian positive definite but lets the
    coarse correction point the wrong way, kappa ~ 10)."""
    dims, th = (8, 8, 8), (0.6, 1.2, 1.8)
    V = mg.VCycle("bloch", dims, 1.0, 0.5, 3, thetas=th)
    A = ops.bloch_periodic(dims, 1.0, th, scale=0.5).toarray()
    T = _dense_T(V, 512, np.complex128)
    ev = np.linalg.eigvals(T @ A).real
    assert ev.min() > 0.0
    assert ev.max() / ev.min() < 3.0


# -------------------------------------------------------------- AV-MG
def test_abs_polynomial_positive_and_convergent():
    """The damped Chebyshev series of |x| on [a, b] (a < 0 < b) is positive
    on the whole interval (so p(L - sigma I) is SPD) and its error shrinks
    with the degree."""
    a, b = -3.0, 9.0
    x = np.linspace(a, b, 40001)
    errs = []
    for deg in (4, 10, 20, 40):
        c = mg.abs_polynomial(a, b, deg)
        p = mg.cheb_eval(c, a, b, x)
        assert p.min() > 0.0
        errs.append(np.abs(p - np.abs(x)).max())
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    assert errs[-1] < 0.35 * (b - a) / 40 * 4


def test_chebyshev_recurrence_matches_spectral_evaluation():
    """p(S) X by the three-term recurrence equals U p(Lambda) U^T X from
    the eigendecomposition of S."""
    dims, h = (6, 5), 0.1
    L = ops.fd_dirichlet(dims, h)
    sigma = 300.0
    S = L.toarray() - sigma * np.eye(30)
    ev, U = np.linalg.eigh(S)
    a, b = -sigma, 8.0 / h**2 - sigma
    c = mg.abs_polynomial(a, b, 9)
    X = np.random.default_rng(30).standard_normal((30, 3))
    got = mg.cheb_apply(c, a, b, S, X)
    want = U @ (mg.cheb_eval(c, a, b, ev)[:, None] * (U.T @ X))
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_avmg_without_shift_is_the_plain_vcycle():
    """sigma = 0: every level takes B_l = L_l (sqrt(sigma) h_l < delta),
    Richardson with alpha = omega / diag is weighted Jacobi and the
    coarsest |L_0|^-1 = L_0^-1, so Algorithm 4 is the V-cycle."""
    dims, h = (16, 8), 1 / 17
    V = mg.VCycle("fd", dims, h, 1.0, 3)
    W = mg.AVMG(dims, h, 1.0, 3, 0.0)
    X = np.random.default_rng(31).standard_normal((128, 4))
    assert W.kind == ["laplacian", "laplacian", "laplacian"]
    assert np.allclose(W.apply(X), V.apply(X), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("mode,absval", [("av", True), ("inv", False)])
def test_single_level_is_the_exact_coarse_solve(mode, absval):
    """One level: Algorithm 4 is |L - sigma I|^-1 and Algorithm 5 is
    (L - sigma I)^-1; |S| is computed here as the square root of S^2."""
    import scipy.linalg as sla
    dims, h = (7, 6), 0.1
    L = ops.fd_dirichlet(dims, h).toarray()
    sigma = 401.0
    S = L - sigma * np.eye(42)
    W = mg.AVMG(dims, h, 1.0, 1, sigma, mode=mode)
    T = W.apply(np.eye(42))
    ref = np.linalg.inv(np.real(sla.sqrtm(S @ S)) if absval else S)
    assert np.allclose(T, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_avmg_two_level_closed_form():
    """One V-cycle of Algorithm 4 over two levels is
    T = (I - E^2) B^-1 + E P |L_c - sigma|^-1 P^T E / 2^d,  E = (I - alpha B)^nu,
    with B = p_m(L - sigma I) here (a deep shift)."""
    dims, h = (8, 8), 1 / 9
    L = ops.fd_dirichlet(dims, h)
    sigma = 0.3 * 8 / h**2
    W = mg.AVMG(dims, h, 1.0, 2, sigma, nu=2)
    assert W.kind[0] == "poly"
    n = 64
    B = W.level_op(0, np.eye(n))
    ev, U = np.linalg.eigh(L.toarray() - sigma * np.eye(n))
    c, a, b = W.poly[0]
    assert np.allclose(B, U @ np.diag(mg.cheb_eval(c, a, b, ev)) @ U.T, atol=1e-10 * np.abs(B).max())
    E = np.linalg.matrix_power(np.eye(n) - W.alpha[0] * B, 2)
    Lc = W.L[1].toarray()
    evc, Uc = np.linalg.eigh(Lc - sigma * np.eye(Lc.shape[0]))
    Tc = Uc @ np.diag(1.0 / np.abs(evc)) @ Uc.T
    P = W.P[0].toarray()
    ref = (np.eye(n) - E @ E) @ np.linalg.inv(B) + E @ P @ Tc @ P.T @ E / 4.0
    T = W.apply(np.eye(n))
    assert np.allclose(T, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("d,N,frac,levels", [(2, 32, 0.05, 4), (2, 32, 0.2, 4), (3, 8, 0.25, 3),
                                             (2, 31, 0.05, 3)])
def test_avmg_spd_and_better_than_vcycle_at_deep_shifts(d, N, frac, levels):
    """Algorithm 4 is SPD and approximates |L - sigma I|^-1 far better than
    the V-cycle of L does: kappa(T |L - sigma I|) drops by >= 8x."""
    h = 1.0 / (N + 1)
    dims = (N,) * d
    Ld = ops.fd_dirichlet(dims, h).toarray()
    n = Ld.shape[0]
    ev, U = np.linalg.eigh(Ld)
    sigma = frac * ev.max()
    absS = (U * np.abs(ev - sigma)) @ U.T
    kap = {}
    for name, T in (("vc", mg.VCycle("fd", dims, h, 1.0, levels)),
                    ("av", mg.AVMG(dims, h, 1.0, levels, sigma))):
        Tm = T.apply(np.eye(n))
        if name == "av":
            assert np.linalg.norm(Tm - Tm.T) <= 1e-12 * np.linalg.norm(Tm)
            assert np.linalg.eigvalsh(0.5 * (Tm + Tm.T)).min() > 0.0
        e = np.linalg.eigvals(Tm @ absS).real
        kap[name] = e.max() / e.min()
    assert kap["av"] * 8.0 < kap["vc"]


@pytest.mark.parametrize("dims,levels", [((15, 15), 3), ((31, 31), 4), ((7, 7, 7), 2),
                                         ((15, 15, 15), 3)])
def test_vertex_centred_vcycle_spd_and_spectrally_equivalent(dims, levels):
    """Odd grids coarsen vertex-centred (N -> (N-1)/2, linear interpolation,
    full weighting R = P^T / 2^d): T stays SPD and kappa(T A) small."""
    h = 1.0 / (dims[0] + 1)
    V = mg.VCycle("fd", dims, h, 1.0, levels)
    A = ops.fd_dirichlet(dims, h).toarray()
    T = _dense_T(V, A.shape[0])
    assert np.linalg.norm(T - T.T) <= 1e-12 * np.linalg.norm(T)
    ev = np.linalg.eigvals(T @ A).real
    assert ev.min() > 0.0
    assert ev.max() / ev.min() < 3.0


def test_vertex_centred_transfer_is_exact_on_linear_functions():
    """Linear interpolation reproduces a linear function on the shared and
    the halfway points; the coarse grid of 2^j - 1 points has spacing 2h."""
    cd, how = mg.coarsen((15, 7))
    assert cd == (7, 3) and how == "vertex"
    P = mg._prolong1d_vertex(7).toarray()
    xc = np.arange(1, 8) * 2.0          # coarse points at fine positions 2, 4, .., 14
    xf = np.arange(1, 16) * 1.0
    f = P @ (3.0 * xc)
    # exact inside; the first and last fine points see the zero boundary
    assert np.allclose(f[1:-1], 3.0 * xf[1:-1])
    assert np.isclose(f[0], 0.5 * 3.0 * 2.0) and np.isclose(f[-1], 0.5 * 3.0 * 14.0)
    with pytest.raises(ValueError):
        mg.coarsen((15, 8))


def test_avmg_acts_on_complex_vectors_as_a_real_operator():
    """Algorithm 1 runs in complex arithmetic with a real T: applied to a
    complex block, AV-MG must equal its dense matrix (assembled from real
    unit vectors) times that block."""
    dims, h = (15, 15), 1 / 16
    T = mg.AVMG(dims, h, 1.0, 3, 300.0)
    n = 225
    Td = mg.dense_matrix(T.apply, n)
    rng = np.random.default_rng(7)
    Z = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    assert np.allclose(T.apply(Z), Td @ Z, rtol=1e-12, atol=1e-12 * np.abs(Td @ Z).max())
    assert np.abs((T.apply(Z)).imag).max() > 0.0
