"""Further pins of the oracle (CPU only): the subspace-angle measure on
known angles, the selection of Algorithm 3 on hand-built projected
pencils with a prescribed spectrum (including a conjugate pair cut by the
block size, the unpaired column of Y' = [Y0 YR ytilde_R YI]), the
lumped-mass potential of the finite-element pencil and the
Hellmann-Feynman gradient with a mass matrix and point weights."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import dense, hf, operators as ops, plhr
from tests.pencils import projected_pencil


# ------------------------------------------------------------ subspace_sine
def _rotated_pair(n, angles, rng):
    """Orthonormal U (n x k) and W whose principal angles with U are
    exactly `angles`: w_j = cos(a_j) u_j + sin(a_j) u'_j, with u'_j
    orthonormal and orthogonal to U."""
    k = len(angles)
    Q, _ = np.linalg.qr(rng.standard_normal((n, 2 * k)))
    U, Up = Q[:, :k], Q[:, k:]
    W = U * np.cos(angles)[None, :] + Up * np.sin(angles)[None, :]
    return U, W


@pytest.mark.parametrize("angles", [[1e-9, 0.0], [3e-5, 1e-7, 0.0], [0.3, 0.1], [1.2, 0.5, 0.0]])
def test_subspace_sine_known_angles_euclidean(angles):
    rng = np.random.default_rng(70)
    U, W = _rotated_pair(40, np.array(angles), rng)
    want = np.sin(max(angles))
    # the measure depends on the spans only: mix the columns of both sides
    Mu = rng.standard_normal((len(angles),) * 2) + 3 * np.eye(len(angles))
    Mw = rng.standard_normal((len(angles),) * 2) + 3 * np.eye(len(angles))
    got = dense.subspace_sine(U @ Mu, W @ Mw)
    assert abs(got - want) <= 1e-12 + 1e-9 * want


@pytest.mark.parametrize("angles", [[2e-9, 1e-10], [0.25, 0.05]])
def test_subspace_sine_known_angles_b_inner_product(angles):
    """With B = C C^T, the map x -> C^-T x turns Euclidean angles into
    B-angles, so the B-measure of the mapped pair is the known angle."""
    rng = np.random.default_rng(71)
    n = 30
    G = rng.standard_normal((n, n))
    B = G @ G.T + n * np.eye(n)
    C = np.linalg.cholesky(B)
    U, W = _rotated_pair(n, np.array(angles), rng)
    Ub = sla.solve_triangular(C.T, U, lower=False)
    Wb = sla.solve_triangular(C.T, W, lower=False)
    got = dense.subspace_sine(Ub, Wb, B)
    want = np.sin(max(angles))
    assert abs(got - want) <= 1e-12 + 1e-7 * want
    # and the Euclidean measure of the same pair is a different number
    assert abs(dense.subspace_sine(Ub, Wb) - want) > 1e-3 * want


# ---------------------------------------------- selection on a known pencil
def _in_span(y, S):
    c, *_ = np.linalg.lstsq(S, y, rcond=None)
    return np.linalg.norm(y - S @ c) / np.linalg.norm(y)


def test_selection_cuts_a_pair_into_ytilde():
    """k_int = 3 with the third unit a conjugate pair: Y' = [y0 y1 ytilde_R]."""
    xis = [0.1, 0.2, 0.3 + 0.05j, 1.0, 2.0, -3.0]
    GL, GR, m, Yb = projected_pencil(xis, 72)
    xi, Y, unit = plhr.sorted_tharmonic(GL, GR, real_pairs=True)
    assert np.allclose(xi[:4], [0.1, 0.2, 0.3 + 0.05j, 0.3 - 0.05j], rtol=1e-10)
    Yp, kinds, pair_of = plhr.real_selection(xi, Y, unit, 3)
    assert kinds == ["real", "real", "tilde"] and pair_of == [-1, -1, -1]
    assert Yp.shape == (m, 3) and np.isrealobj(Yp)
    for j in range(2):
        r = GL @ Yp[:, j] - xi[j].real * (GR @ Yp[:, j])
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(GL) * np.linalg.norm(Yp[:, j])
    # ytilde_R is the real part of the pair's eigenvector: it lies in the
    # pair's real invariant subspace (and is not in either real eigenvector's)
    assert _in_span(Yp[:, 2], Yb[2]) < 1e-10
    assert _in_span(Yp[:, 2], np.column_stack([Yb[0], Yb[1]])) > 1e-3


def test_selection_layout_pairs_and_ytilde():
    """k_int = 5 over units (real, pair, real, pair, ...): Y' = [Y0 YR
    ytilde_R YI] = [y(0.1) y(0.3) Re y(0.2+i/20) ytilde Im y(0.2+i/20)];
    the I column follows the ytilde column."""
    xis = [0.1, 0.2 + 0.05j, 0.3, 0.4 + 0.1j, 1.0, 2.0, 3.0, 4.0]
    GL, GR, m, Yb = projected_pencil(xis, 73)
    xi, Y, unit = plhr.sorted_tharmonic(GL, GR, real_pairs=True)
    Yp, kinds, pair_of = plhr.real_selection(xi, Y, unit, 5)
    assert kinds == ["real", "real", "R", "tilde", "I"]
    assert pair_of == [-1, -1, 4, -1, 2]
    assert _in_span(Yp[:, 0], Yb[0]) < 1e-10
    assert _in_span(Yp[:, 1], Yb[2]) < 1e-10
    y = Yp[:, 2] + 1j * Yp[:, 4]
    r = GL @ y - (0.2 + 0.05j) * (GR @ y)
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(GL) * np.linalg.norm(y)
    assert _in_span(Yp[:, 3], Yb[3]) < 1e-10


def test_sort_order_equal_modulus():
    """Units sorted by |xi|, a conjugate pair kept together with the
    Im xi > 0 member first.  Equal moduli (0.5, -0.5 and the pair
    0.3 +- 0.4i) come out of QZ rounded differently, so among them any
    order is a correct one: only the grouping and the moduli are fixed."""
    xis = [0.5, -0.5, 0.3 + 0.4j, 2.0]
    GL, GR, m, _ = projected_pencil(xis, 74)
    xi, Y, unit = plhr.sorted_tharmonic(GL, GR, real_pairs=True)
    assert np.allclose(np.abs(xi), [0.5, 0.5, 0.5, 0.5, 2.0], rtol=1e-10)
    assert np.allclose(xi[4], 2.0, rtol=1e-10)
    j = int(np.flatnonzero(np.abs(xi.imag) > 0.1)[0])
    assert np.allclose(xi[j:j + 2], [0.3 + 0.4j, 0.3 - 0.4j], rtol=1e-10)
    assert unit[j] == j and unit[j + 1] == j
    assert sorted(np.round(xi[[q for q in range(4) if q not in (j, j + 1)]].real, 9)) == [-0.5, 0.5]


def test_ytilde_rayleigh_quotient_is_its_own():
    """Algorithm 3: the unpaired column takes its own Rayleigh quotient,
    a pair the quotient of eq. (4.1) on both columns."""
    K, M = ops.fe_q1(5, 2)
    rng = np.random.default_rng(75)
    V = rng.standard_normal((K.shape[0], 4))
    prob = plhr.Problem(A=K, B=M)
    lam = plhr.real_rayleigh(prob, V, ["real", "R", "tilde", "I"], [-1, 3, -1, 1])
    own = np.array([V[:, j] @ (K @ V[:, j]) / (V[:, j] @ (M @ V[:, j])) for j in range(4)])
    pair = ((V[:, 1] @ (K @ V[:, 1]) + V[:, 3] @ (K @ V[:, 3]))
            / (V[:, 1] @ (M @ V[:, 1]) + V[:, 3] @ (M @ V[:, 3])))
    assert np.allclose(lam, [own[0], pair, own[2], pair], rtol=1e-14)


# ------------------------------------------------ finite-element potential
@pytest.mark.parametrize("d,Nel", [(2, 6), (3, 4)])
def test_fe_lumped_potential_constant_mode(d, Nel):
    """Natural boundary, constant potential c: the constant vector is in
    the null space of K and sum_i phi_i = 1, so with the lumped mass its
    Rayleigh quotient for (K + M_L c, M) is c exactly (the unit box has
    volume 1); a potential weighted by anything but the row sums of M
    would give another value."""
    c = 3.7
    n = (Nel + 1) ** d
    A, M = ops.fe_q1(Nel, d, bc="natural", potential=np.full(n, c))
    K, _ = ops.fe_q1(Nel, d, bc="natural")
    one = np.ones(n)
    assert np.linalg.norm(K @ one) <= 1e-12 * Nel**2
    assert abs(one @ (A @ one) / (one @ (M @ one)) - c) <= 1e-13 * c
    assert abs((A - K).diagonal().sum() - c) <= 1e-13 * c


# ---------------------------------------------- HF gradient with B and w
def test_hf_gradient_with_mass_and_weights_matches_finite_differences():
    """A = K + diag(m_L p), B = M: d lambda / d p_x = m_x v(x)^2 / v^T M v,
    against central differences of dense generalized eigenvalues."""
    Nel = 7
    K, M = ops.fe_q1(Nel, 2)
    n = K.shape[0]
    mL = np.asarray(M.sum(axis=1)).ravel()
    rng = np.random.default_rng(76)
    p = rng.uniform(-20, 20, n)
    sigma, k = 200.0, 2

    def pairs(pp):
        A, _ = ops.fe_q1(Nel, 2, potential=pp)
        return dense.nearest_pairs(A, M, sigma, k)

    lam, X = pairs(p)
    X = X * rng.uniform(0.5, 2.0, k)[None, :]        # any normalisation
    dl = np.array([1.3, -0.7])
    g = hf.eigval_grad(X, dl, B=M, w=mL)
    eps = 1e-6
    for x in rng.choice(n, 5, replace=False):
        pp, pm = p.copy(), p.copy()
        pp[x] += eps
        pm[x] -= eps
        fd = (dl @ pairs(pp)[0] - dl @ pairs(pm)[0]) / (2 * eps)
        assert abs(fd - g[x]) <= 1e-6 * max(1.0, np.abs(g).max())
