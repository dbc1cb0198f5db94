"""Pins of the oracle's block PLHR (Algorithms 1-3 of the paper) against
the plain definition (the k eigenpairs nearest sigma), reductions to
textbook procedures, the Petrov-Galerkin condition eq. (3.3) and
identities the paper states (CPU only)."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import dense, hf, mg, operators as ops, plhr
from tests import closed_forms as cf


def _dense(M):
    return M.toarray() if hasattr(M, "toarray") else np.asarray(M)


def _abs_inv(A, B, sigma):
    """|A - sigma B|^{-1} (matrix absolute value of the shifted matrix)."""
    S = _dense(A) - sigma * (np.eye(A.shape[0]) if B is None else _dense(B))
    d, U = np.linalg.eigh(S)
    return U @ np.diag(1.0 / np.abs(d)) @ U.T


def _small_problem(N=10, d=2, seed=0):
    dims = (N,) * d
    h = 1.0 / (N + 1)
    A = ops.fd_dirichlet(dims, h)
    rng = np.random.default_rng(seed)
    pot = rng.uniform(-50, 50, A.shape[0])
    return ops.fd_dirichlet(dims, h, potential=pot)


# ------------------------------------------------ T-harmonic projection (3.5)
def test_tharmonic_with_inverse_preconditioner_is_standard_rr():
    """T = (A - sigma B)^{-1} gives G_R = Z^* B Z and G_L = Z^*(A - sigma B) Z,
    so xi + sigma are the ordinary Ritz values of (A, B) on span(Z)."""
    A = _small_problem()
    n = A.shape[0]
    sigma = 900.0
    Tm = np.linalg.inv(_dense(A) - sigma * np.eye(n))
    prob = plhr.Problem(A=A, T=lambda X: Tm @ X, sigma=sigma)
    Z = np.random.default_rng(3).standard_normal((n, 12))
    GL, GR = plhr.tharmonic_matrices(prob, Z)
    xi, Y, _ = plhr.sorted_tharmonic(GL, GR)
    ritz = sla.eigh(Z.T @ (A @ Z), Z.T @ Z, eigvals_only=True)
    assert np.allclose(np.sort(xi.real + sigma), np.sort(ritz), rtol=1e-9)
    assert np.max(np.abs(xi.imag)) < 1e-6 * np.max(np.abs(xi))


def test_tharmonic_identity_preconditioner_is_harmonic_rr():
    """T = I, B = I: eq. (3.5) is the standard harmonic Rayleigh-Ritz
    (Section 3.1), a Hermitian-definite problem with real xi."""
    A = _small_problem(seed=1)
    n = A.shape[0]
    sigma = 700.0
    prob = plhr.Problem(A=A, sigma=sigma)
    Z = np.random.default_rng(4).standard_normal((n, 10))
    S = A @ Z - sigma * Z
    xi_ref = 1.0 / sla.eigh(Z.T @ S, S.T @ S, eigvals_only=True)   # harmonic Ritz
    GL, GR = plhr.tharmonic_matrices(prob, Z)
    xi, _, _ = plhr.sorted_tharmonic(GL, GR, real_pairs=True)
    assert np.all(xi.imag == 0.0)
    assert np.allclose(np.sort(xi.real), np.sort(xi_ref), rtol=1e-8)


def test_tharmonic_full_space_gives_exact_eigenvalues():
    A = _small_problem(N=6)
    n = A.shape[0]
    sigma = 300.0
    V = mg.VCycle("fd", (6, 6), 1 / 7, 1.0, 2)
    prob = plhr.Problem(A=A, T=V.apply, sigma=sigma)
    Z = np.random.default_rng(5).standard_normal((n, n))
    GL, GR = plhr.tharmonic_matrices(prob, Z)
    xi, _, _ = plhr.sorted_tharmonic(GL, GR, real_pairs=True)
    ev = np.linalg.eigvalsh(_dense(A))
    assert np.allclose(np.sort(xi.real + sigma), ev, rtol=1e-8, atol=1e-8)


def test_petrov_galerkin_condition_and_basis_invariance():
    """Every pair returned satisfies (A - theta B) v  perp_T  (A - sigma B) Z
    (eq. 3.3) with theta = sigma + xi, v = Z y; and xi does not depend on the
    basis of span(Z)."""
    dims, h = (8, 8), 1 / 9
    A = ops.fd_dirichlet(dims, h, potential=np.random.default_rng(6).uniform(-20, 20, 64))
    sigma = 400.0
    V = mg.VCycle("fd", dims, h, 1.0, 3)
    Tm = V.apply(np.eye(64))
    prob = plhr.Problem(A=A, T=V.apply, sigma=sigma)
    Z = np.random.default_rng(7).standard_normal((64, 9))
    GL, GR = plhr.tharmonic_matrices(prob, Z)
    xi, Y, _ = plhr.sorted_tharmonic(GL, GR, real_pairs=True)
    Ad = _dense(A)
    for j in range(4):
        v = Z @ Y[:, j]
        theta = sigma + xi[j]
        lhs = (Z.T @ (Ad - sigma * np.eye(64))) @ Tm @ ((Ad - theta * np.eye(64)) @ v)
        assert np.linalg.norm(lhs) <= 1e-9 * np.linalg.norm(Ad) ** 2 * np.linalg.norm(Tm) * np.linalg.norm(v)
    M = np.random.default_rng(8).standard_normal((9, 9)) + 3 * np.eye(9)
    GL2, GR2 = plhr.tharmonic_matrices(prob, Z @ M)
    xi2, _, _ = plhr.sorted_tharmonic(GL2, GR2, real_pairs=True)
    assert np.allclose(xi2[:5], xi[:5], rtol=1e-7)


def test_conjugate_pairs_are_adjacent_and_ordered():
    rng = np.random.default_rng(9)
    GL = rng.standard_normal((12, 12))
    GL = GL @ GL.T + 12 * np.eye(12)
    GR = rng.standard_normal((12, 12))   # non-symmetric: complex pairs appear
    xi, Y, unit = plhr.sorted_tharmonic(GL, GR, real_pairs=True)
    mags = np.abs(xi)
    assert np.all(np.diff(mags) >= -1e-12 * mags.max())
    ncplx = 0
    for j in range(12):
        if xi[j].imag != 0.0 and unit[j] == j:
            ncplx += 1
            assert xi[j].imag > 0 and np.isclose(xi[j + 1], np.conj(xi[j]), rtol=1e-10)
            assert np.allclose(GL @ Y[:, j], xi[j] * (GR @ Y[:, j]), atol=1e-8 * np.abs(GL).max())
    assert ncplx > 0


def test_pair_rayleigh_quotient_equals_complex_rq():
    """eq. (4.1): for v = vR + i vI, lambda(v) = (vR'AvR + vI'AvI)/(vR'BvR + vI'BvI)."""
    K, M = ops.fe_q1(6, 2)
    rng = np.random.default_rng(10)
    vR, vI = rng.standard_normal((2, K.shape[0]))
    v = vR + 1j * vI
    cplx = np.real(np.vdot(v, K @ v) / np.vdot(v, M @ v))
    prob = plhr.Problem(A=K, B=M, sigma=0.0)
    lam = plhr.real_rayleigh(prob, np.column_stack([vR, vI]), ["R", "I"], [1, 0])
    assert np.allclose(lam, cplx, rtol=1e-13)


def test_b_orthonormalize_and_drop():
    K, M = ops.fe_q1(6, 2)
    n = K.shape[0]
    rng = np.random.default_rng(11)
    V = rng.standard_normal((n, 3))
    W = np.column_stack([V[:, 0] + V[:, 1], rng.standard_normal(n)])   # first W column dependent
    Zh, labels = plhr.b_orthonormalize([("V", V), ("W", W)], M)
    assert labels == [("V", 0), ("V", 1), ("V", 2), ("W", 1)]
    assert np.linalg.norm(Zh.T @ (M @ Zh) - np.eye(4)) <= 1e-12
    # a dependent V column is dropped as well; the span is unchanged
    Zh2, lab2 = plhr.b_orthonormalize([("V", np.column_stack([V[:, 0], 2 * V[:, 0]]))], M)
    assert lab2 == [("V", 0)] and Zh2.shape[1] == 1


# ---------------------------------------------------- one step from scratch
def _ritz_rqs_from_subspace(A, T, sigma, Z, k):
    """Independent dense T-harmonic step: orthonormal basis by QR, eq. (3.5),
    k smallest |xi|, RQs of the (complex) Ritz vectors."""
    Q, _ = np.linalg.qr(Z)
    Ad = _dense(A)
    S = Ad @ Q - sigma * Q
    GL = S.T @ T @ S
    GR = S.T @ T @ Q
    xi, Y = sla.eig(GL, GR)
    order = np.argsort(np.abs(xi), kind="stable")[:k]
    X = Q @ Y[:, order]
    return np.sort(np.real(np.sum(np.conj(X) * (Ad @ X), axis=0) / np.sum(np.abs(X) ** 2, axis=0)))


def test_first_two_steps_match_dense_construction():
    """Steps 3-11 of Algorithm 3 against an independent dense build of the
    trial subspace span{V, T(AV - BV Lam), T(AW - BW Lam), V_prev}."""
    dims, h = (10, 10), 1 / 11
    A = ops.fd_dirichlet(dims, h, potential=np.random.default_rng(12).uniform(0, 80, 100))
    sigma = 600.0
    V = mg.VCycle("fd", dims, h, 1.0, 2)
    Tm = V.apply(np.eye(100))
    prob = plhr.Problem(A=A, T=V.apply, sigma=sigma)
    V0 = np.random.default_rng(13).standard_normal((100, 4))
    s = plhr.BPLHR(prob, V0, 3, real=True, lock=False)
    Ad = _dense(A)
    Vc = plhr.b_normalize(None, V0)
    lam0 = np.sum(Vc * (Ad @ Vc), axis=0)
    W = Tm @ (Ad @ Vc - Vc * lam0)
    S = Tm @ (Ad @ W - W * lam0)
    ref1 = _ritz_rqs_from_subspace(A, Tm, sigma, np.column_stack([Vc, W, S]), 4)
    s.step()
    assert np.allclose(np.sort(s.lam), ref1, rtol=1e-9)
    V1, lam1 = s.V.copy(), s.lam.copy()
    W1 = Tm @ (Ad @ V1 - V1 * lam1)
    S1 = Tm @ (Ad @ W1 - W1 * lam1)
    ref2 = _ritz_rqs_from_subspace(A, Tm, sigma, np.column_stack([V1, W1, S1, Vc]), 4)
    s.step()
    assert np.allclose(np.sort(s.lam), ref2, rtol=1e-8)


# ------------------------------------------------------- whole iterations
def test_converges_to_brute_force_with_av_preconditioner():
    A = _small_problem(N=16, seed=2)
    sigma = 1500.0
    Tm = _abs_inv(A, None, sigma)
    prob = plhr.Problem(A=A, T=lambda X: Tm @ X, sigma=sigma)
    V0 = wl.start_block(A.shape[0], 6, (20, 0))
    res = plhr.bplhr(prob, V0, 5, tol=1e-13, maxit=200)
    lam_ref, X_ref = dense.nearest_pairs(A, None, sigma, 5)
    assert res.converged
    assert np.allclose(res.lam, lam_ref, rtol=1e-12)
    assert dense.subspace_sine(X_ref, res.V) < 1e-8
    # final Ritz vectors are B-orthonormal
    assert np.linalg.norm(res.V.T @ res.V - np.eye(5)) < 1e-12


def test_config1_shape_with_identity_preconditioner():
    """2-D Dirichlet Laplacian with T = I (configuration shape of the small
    benchmark case, on a 12x12 grid): converges to the closed-form nearest
    eigenvalues.  Two extra block columns are needed to catch both copies of
    the double eigenvalues of the square (one extra column converges to a
    farther eigenvalue instead)."""
    N, h = 12, 1 / 13
    A = ops.fd_dirichlet((N, N), h)
    ev = cf.fd_dirichlet_eigs((N, N), h)
    sigma = 0.4 * ev.max()
    prob = plhr.Problem(A=A, sigma=sigma)
    res = plhr.bplhr(prob, wl.start_block(N * N, 6, (1, 0)), 4, tol=1e-10, maxit=3000)
    ref = ev[np.lexsort((ev, np.abs(ev - sigma)))][:4]
    assert res.converged
    assert np.allclose(res.lam, ref, rtol=1e-12)


def test_mg_preconditioned_3d_converges():
    w = wl.small_fd7(8, 4, 0.1, seed=(21, 0), levels=2)
    w.k_extra = 3           # guard columns: the cube has 3-fold eigenvalues
    A = ops.fd_dirichlet(w.dims, w.h)
    T = mg.VCycle("fd", w.dims, w.h, 1.0, w.mg_levels)
    prob = plhr.Problem(A=A, T=T.apply, sigma=w.sigma)
    res = plhr.bplhr(prob, w.v0(), w.k, tol=1e-11, maxit=500)
    lam_ref, X_ref = dense.nearest_pairs(A, None, w.sigma, w.k)
    assert res.converged
    assert np.allclose(res.lam, lam_ref, rtol=1e-12)


def test_generalized_fe_reproduces_paper_eigenvalue():
    """Section 6.1: the FE pencil (K, M) on 50x50 elements; single-vector
    PLHR with T = |A - sigma B|^{-1} at sigma = 497 returns the printed
    lambda_31 = 497.5521."""
    K, M = ops.fe_q1(50, 2)
    sigma = 497.0
    Tm = _abs_inv(K, M, sigma)
    prob = plhr.Problem(A=K, B=M, T=lambda X: Tm @ X, sigma=sigma)
    v0 = wl.start_block(K.shape[0], 1, (22, 0))[:, 0]
    lams, v = plhr.plhr_single(prob, v0, maxit=60, tol=1e-12)
    assert abs(lams[-1] - 497.5521) < 5e-5


@pytest.mark.parametrize("sigma,printed", [(497.0, 497.5521), (980.0, 979.7072)])
def test_single_vector_with_perturbed_av_preconditioner_reproduces_paper(sigma, printed):
    """Section 6.1: Algorithm 1 on the FE pencil (K, M), 50 x 50 elements,
    with T = |A - sigma B|^-1 + E, ||E|| = 1e-5 ||(A - sigma B)^-1||,
    converges to the printed eigenvalue nearest sigma, and to the dense
    generalized eigenvalue to rounding."""
    K, M = ops.fe_q1(50, 2)
    Kd, Md = K.toarray(), M.toarray()
    T = wl.perturbed_abs_inverse(Kd, Md, sigma, 1e-5, (25, int(sigma)))
    prob = plhr.Problem(A=K, B=M, T=lambda X: T @ X, sigma=sigma)
    v0 = wl.start_block(K.shape[0], 1, (22, 0))[:, 0]
    lams, v = plhr.plhr_single(prob, v0, maxit=30, tol=1e-11)
    assert len(lams) <= 12                      # a strong preconditioner: a few steps
    assert abs(lams[-1] - printed) < 5e-5
    w = sla.eigh(Kd, Md, eigvals_only=True)
    assert abs(lams[-1] - w[np.argmin(np.abs(w - sigma))]) < 1e-9 * sigma


def test_algorithm3_equals_algorithm2_when_all_xi_real():
    """With T = I and B = I every xi is real (harmonic RR), so the real
    version follows the complex one (Section 4.1, last paragraph)."""
    A = _small_problem(N=10, seed=3)
    prob = plhr.Problem(A=A, sigma=500.0)
    V0 = wl.start_block(100, 4, (23, 0))
    r = plhr.BPLHR(prob, V0, 4, real=True, lock=False)
    c = plhr.BPLHR(prob, V0, 4, real=False, lock=False)
    for _ in range(10):
        r.step()
        c.step()
        assert np.allclose(np.sort(r.lam), np.sort(c.lam), rtol=1e-9)


def test_algorithm1_equals_block_algorithm_for_k1():
    A = _small_problem(N=10, seed=4)
    sigma = 650.0
    V = mg.VCycle("fd", (10, 10), 1 / 11, 1.0, 1)
    prob = plhr.Problem(A=A, T=V.apply, sigma=sigma)
    v0 = wl.start_block(100, 1, (24, 0))
    lams1, _ = plhr.plhr_single(prob, v0[:, 0], maxit=6)
    b = plhr.BPLHR(prob, v0, 1, real=False, lock=False)
    for i in range(6):
        b.step()
        assert np.isclose(b.lam[0], lams1[i + 1], rtol=1e-9)


def test_rank_deficient_start_block_is_an_error():
    A = _small_problem(N=8)
    prob = plhr.Problem(A=A, sigma=300.0)
    V0 = wl.start_block(64, 3, (25, 0))
    V0[:, 2] = V0[:, 0]
    with pytest.raises(plhr.Breakdown):
        plhr.BPLHR(prob, V0, 2)


def test_residual_trend_and_ritz_values_approach_exact():
    A = _small_problem(N=12, seed=5)
    sigma = 250.0
    V = mg.VCycle("fd", (12, 12), 1 / 13, 1.0, 2)
    prob = plhr.Problem(A=A, T=V.apply, sigma=sigma)
    res = plhr.bplhr(prob, wl.start_block(144, 6, (26, 0)), 3, tol=1e-11, maxit=400)
    lam_ref, _ = dense.nearest_pairs(A, None, sigma, 3)
    rr = [np.max(r[plhr.wanted_columns(l, sigma, 3)])
          for r, l in zip(res.history.rel_res, res.history.lam)]
    assert res.converged
    assert np.allclose(res.lam, lam_ref, rtol=1e-12)
    assert rr[-1] <= 1e-3 * rr[0]
    win = 20
    peaks = [max(rr[i:i + win]) for i in range(0, len(rr) - win, win)]
    assert all(b <= a * 1.0001 for a, b in zip(peaks, peaks[1:]))


# --------------------------------------------------------- HF gradient
def test_hf_gradient_matches_finite_differences_and_sum_rule():
    N, h = 8, 1.0
    rng = np.random.default_rng(27)
    pot = rng.uniform(-1, 1, N * N)
    sigma = 2.0
    k = 3
    targets = np.array([1.9, 2.0, 2.2])

    def lams(p):
        A = ops.fd_dirichlet((N, N), h, 0.5, potential=p)
        return dense.nearest_pairs(A, None, sigma, k)

    lam, X = lams(pot)
    L0, dl = hf.loss_and_grad_targets(lam, targets)
    g = hf.eigval_grad(X, dl)
    # sum rule: a constant shift of the potential moves every lambda by it
    assert np.isclose(np.sum(hf.eigval_grad(X, np.ones(k))), k, rtol=1e-12)
    eps = 1e-6
    for x in rng.choice(N * N, 6, replace=False):
        pp, pm = pot.copy(), pot.copy()
        pp[x] += eps
        pm[x] -= eps
        fd = (hf.loss_and_grad_targets(lams(pp)[0], targets)[0]
              - hf.loss_and_grad_targets(lams(pm)[0], targets)[0]) / (2 * eps)
        assert abs(fd - g[x]) <= 1e-7 * max(1.0, abs(g[x]))


# ------------------------------------------------- harmonic extraction
def test_harmonic_extraction_ignores_T_in_the_projection():
    """extraction="harmonic": eq. (3.5) with T -> I inside the projection
    (Section 6.2, "harm."): with B = I the values are the standard harmonic
    Ritz values 1/eig(Z^T S, S^T S), S = (A - sigma) Z, whatever T is."""
    A = _small_problem(seed=7)
    n = A.shape[0]
    sigma = 700.0
    V = mg.VCycle("fd", (10, 10), 1 / 11, 1.0, 2)
    prob = plhr.Problem(A=A, T=V.apply, sigma=sigma, extraction="harmonic")
    Z = np.random.default_rng(14).standard_normal((n, 10))
    S = A @ Z - sigma * Z
    xi_ref = 1.0 / sla.eigh(Z.T @ S, S.T @ S, eigvals_only=True)
    GL, GR = plhr.tharmonic_matrices(prob, Z)
    xi, _, _ = plhr.sorted_tharmonic(GL, GR, real_pairs=True)
    assert np.all(xi.imag == 0.0)
    assert np.allclose(np.sort(xi.real), np.sort(xi_ref), rtol=1e-8)
    # the T-harmonic values of the same basis differ
    prob.extraction = "tharmonic"
    GL2, GR2 = plhr.tharmonic_matrices(prob, Z)
    xi2, _, _ = plhr.sorted_tharmonic(GL2, GR2, real_pairs=True)
    assert not np.allclose(np.sort(np.abs(xi2)), np.sort(np.abs(xi_ref)), rtol=1e-3)


def test_bplhr_with_avmg_and_both_extractions_converges():
    """Block PLHR with the AV-MG preconditioner (Algorithm 4), T-harmonic
    and harmonic extraction, on a 2-D Laplacian (vertex-centred 31 x 31
    grid, 3 levels) at an interior shift: both reach the brute-force
    nearest pairs."""
    N = 31
    h = 1.0 / (N + 1)
    A = ops.fd_dirichlet((N, N), h)
    ev = cf.fd_dirichlet_eigs((N, N), h)
    sigma = wl.shift_between(ev, 30)
    T = mg.AVMG((N, N), h, 1.0, 3, sigma)
    lam_ref, _ = dense.nearest_pairs(A, None, sigma, 4)
    for ex in ("tharmonic", "harmonic"):
        prob = plhr.Problem(A=A, T=T.apply, sigma=sigma, extraction=ex)
        res = plhr.bplhr(prob, wl.start_block(N * N, 6, (27, 0)), 4, tol=1e-10, maxit=600)
        assert res.converged, ex
        assert np.allclose(np.sort(res.lam), np.sort(lam_ref), rtol=1e-10), ex


def test_refined_extraction_minimises_the_T_norm_residual():
    """Section 3.3: the refined vector is the B-unit vector of span(Z) with
    the smallest ||A v - lam B v||_T.  Checked against an independent route:
    the smallest singular value of T^{1/2}(A - lam B) Zhat (Zhat
    B-orthonormal) and its right singular vector, and random trial
    vectors never doing better."""
    K, M = ops.fe_q1(8, 2)
    n = K.shape[0]
    T = mg.VCycle("fd", (7, 7), 1 / 8, 1.0, 2)
    prob = plhr.Problem(A=K, B=M, T=T.apply, sigma=300.0)
    Z = np.random.default_rng(71).standard_normal((n, 4))
    Zh, _ = plhr.b_orthonormalize([("V", Z)], M)
    lam_t = 280.0
    th2, y = plhr.refined_vector(prob, Zh, lam_t)
    Td = mg.dense_matrix(T.apply, n)
    d, U = np.linalg.eigh(0.5 * (Td + Td.T))
    Th = (U * np.sqrt(d)) @ U.T
    Kmat = Th @ ((K.toarray() - lam_t * M.toarray()) @ Zh)
    _, sv, Vt = np.linalg.svd(Kmat)
    assert np.isclose(th2, sv[-1] ** 2, rtol=1e-10)
    assert abs(abs(np.dot(Vt[-1], y)) - 1.0) < 1e-10
    R = np.random.default_rng(72).standard_normal((4, 200))
    vals = np.sum((Kmat @ R) ** 2, axis=0) / np.sum(R ** 2, axis=0)
    assert vals.min() >= th2 * (1 - 1e-12)


def test_plmr_converges_to_the_eigenpair_its_start_approximates():
    """PLMR refines toward the eigenpair near the current Rayleigh quotient:
    from a perturbed eigenvector it converges to that eigenpair, quickly
    with T close to |A - sigma|^-1 and more slowly with a V-cycle; from the
    exact eigenvector the refined residual is zero and nothing moves."""
    A = _small_problem(N=12, seed=7)
    n = A.shape[0]
    lam, X = np.linalg.eigh(A.toarray())
    gaps = np.minimum(lam[10:41] - lam[9:40], lam[11:42] - lam[10:41])
    j = 10 + int(np.argmax(gaps))              # a well separated interior pair
    r = np.random.default_rng(73).standard_normal(n)
    v0 = X[:, j] + 0.05 * r / np.linalg.norm(r)
    Tabs = _abs_inv(A, None, lam[j] - 1.0)
    prob = plhr.Problem(A=A, T=lambda Y: Tabs @ Y, sigma=lam[j])
    lams, v = plhr.plmr_single(prob, v0, maxit=20, tol=1e-12)
    assert len(lams) <= 12
    assert abs(lams[-1] - lam[j]) <= 1e-12 * abs(lam[j])
    assert dense.subspace_sine(X[:, [j]], v[:, None]) < 1e-8
    T = mg.VCycle("fd", (12, 12), 1 / 13, 1.0, 2)
    prob = plhr.Problem(A=A, T=T.apply, sigma=lam[j])
    lams, v = plhr.plmr_single(prob, v0, maxit=200)
    assert abs(lams[-1] - lam[j]) <= 1e-10 * abs(lam[j])
    lams2, v2 = plhr.plmr_single(prob, X[:, j], maxit=2)
    assert np.allclose(lams2, lam[j], rtol=1e-12)
    assert dense.subspace_sine(X[:, [j]], v2[:, None]) < 1e-10


def test_algorithm2_on_the_bloch_operator_reaches_the_dense_eigenvalues():
    """Algorithm 2 (complex arithmetic) with the Bloch V-cycle on a complex
    Hermitian periodic operator (8 x 8 x 4 box, phases 2 pi (0.1, 0.2, 0.3),
    a random potential): the two eigenvalues nearest sigma equal those of
    the dense matrix, and the vectors are complex eigenvectors of it."""
    dims, th = (8, 8, 4), wl.bloch_thetas()
    n = 256
    pot = wl.rng(150, 1).uniform(-2.0, 0.0, n)
    A = ops.bloch_periodic(dims, 1.0, th, scale=0.5, potential=pot)
    Ad = A.toarray()
    ev = np.linalg.eigvalsh(Ad)
    sigma = wl.shift_between(ev, 3, 0.4)
    T = mg.VCycle("bloch", dims, 1.0, 0.5, 3, nu_pre=2, nu_post=2, thetas=th)
    prob = plhr.Problem(A=A, T=T.apply, sigma=sigma)
    V0 = wl.start_block(n, 3, (151, 0), dtype=np.complex128)
    r = plhr.bplhr(prob, V0, 2, tol=1e-10, maxit=300, real=False, lock=False)
    assert r.converged
    near = np.sort(ev[np.argsort(np.abs(ev - sigma))[:2]])
    assert np.abs(np.sort(r.lam) - near).max() < 1e-12 * np.abs(ev).max()
    res = Ad @ r.V - r.V * r.lam[None, :]
    assert np.abs(res).max() < 1e-8
    assert np.abs(r.V.imag).max() > 0.1            # genuinely complex vectors
