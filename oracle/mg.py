"""Geometric multigrid V-cycle used as the HPD preconditioner T (oracle).

The paper requires T to be Hermitian positive definite (Section 5) and uses
a multigrid V-cycle in its Laplacian experiments (Appendix A, Algorithm 4
with B_l = L_l on the fine levels).  This module builds the plain V-cycle on
the Laplacian part of the operator:

* levels: the finest grid has N points per dimension; each coarser level
  pairs neighbouring points (N -> N/2, cell-centred) when N is even, or
  keeps every other point (N -> (N-1)/2, vertex-centred) when N is odd,
  down to the coarsest level, which is solved exactly with a dense inverse;
* level operators: the same stencil re-discretised with spacing 2^l h
  (no potential);
* prolongation: d-linear interpolation; cell-centred, 3/4 from the parent
  and 1/4 from the parent's neighbour in each direction; vertex-centred,
  the coarse value on the points the grids share and the mean of the two
  coarse neighbours halfway between them; a neighbour outside a Dirichlet
  box is zero, a neighbour across a Bloch-periodic face is the wrapped
  value times the phase;
* restriction: R = P^H / 2^d;
* smoothing: nu_pre and nu_post sweeps of weighted Jacobi,
  w <- w + omega * D^-1 (r - A_l w), starting from w = 0.

With R proportional to P^H, a symmetric smoother (Jacobi), the same number
of pre- and post-sweeps and Hermitian positive definite level operators,
the V-cycle is a Hermitian linear operator; it is positive definite because
weighted Jacobi with omega = 2/3 satisfies 2D/omega - A_l > 0 for these
stencils.  Both facts are checked by the tests on small grids.

``AVMG`` is Algorithm 4 of Appendix A (the absolute-value preconditioner
T ~ |L - sigma I|^-1, polynomial level operators where the grid does not
resolve the shift, exact |L_0 - sigma I_0|^-1 on the coarsest level) and,
with mode="inv", Algorithm 5 (INV-MG, T ~ (L - sigma I)^-1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import operators as ops


def _prolong1d(Nc: int, bc: str, theta: float = 0.0) -> sp.csr_matrix:
    Nf = 2 * Nc
    P = sp.lil_matrix((Nf, Nc), dtype=np.complex128 if bc == "bloch" else np.float64)
    for c in range(Nc):
        for a, nb in ((0, c - 1), (1, c + 1)):
            f = 2 * c + a
            P[f, c] += 0.75
            if 0 <= nb < Nc:
                P[f, nb] += 0.25
            elif bc == "bloch":
                if nb < 0:
                    P[f, nb + Nc] += 0.25 * np.exp(-1j * theta)
                else:
                    P[f, nb - Nc] += 0.25 * np.exp(1j * theta)
            # Dirichlet: neighbour outside the box is zero
    return P.tocsr()


def _prolong1d_vertex(Nc: int) -> sp.csr_matrix:
    """Vertex-centred linear interpolation, Nc coarse points to 2 Nc + 1
    fine points (Dirichlet): fine point 2c+1 sits on coarse point c, fine
    point 2c halfway between coarse points c-1 and c (zero outside)."""
    Nf = 2 * Nc + 1
    P = sp.lil_matrix((Nf, Nc))
    for c in range(Nc):
        P[2 * c + 1, c] = 1.0
        P[2 * c, c] += 0.5
        P[2 * c + 2, c] += 0.5
    return P.tocsr()


def coarsen(dims):
    """Coarse grid and transfer kind of one level: every dimension even
    pairs neighbouring points (cell-centred, N -> N/2); every dimension
    odd keeps every other point (vertex-centred, N -> (N-1)/2)."""
    if all(N % 2 == 0 for N in dims):
        return tuple(N // 2 for N in dims), "cell"
    if all(N % 2 == 1 and N >= 3 for N in dims):
        return tuple((N - 1) // 2 for N in dims), "vertex"
    raise ValueError(f"grid {dims} cannot be coarsened")


def _kron_x_fastest(mats):
    out = None
    for m in reversed(mats):
        out = m if out is None else sp.kron(out, m, format="csr")
    return out.tocsr()


class VCycle:
    """T ~ A_lap^{-1} by one V-cycle; ``apply`` works on an (n, k) block."""

    def __init__(self, kind: str, dims, h: float, scale: float, levels: int,
                 nu_pre: int = 2, nu_post: int = 2, omega: float = 2.0 / 3.0,
                 thetas=None):
        self.kind = kind
        self.nu_pre, self.nu_post, self.omega = nu_pre, nu_post, omega
        self.d = len(dims)
        self.A, self.Dinv, self.P = [], [], []
        dims = tuple(dims)
        hl = h
        for lev in range(levels):
            if kind == "bloch":
                A = ops.bloch_periodic(dims, hl, thetas, scale=scale)
            else:
                A = ops.fd_dirichlet(dims, hl, scale=scale)
            self.A.append(A)
            self.Dinv.append(1.0 / A.diagonal())
            if lev == levels - 1:
                break
            cdims, how = coarsen(dims)
            if how == "vertex":
                if kind == "bloch":
                    raise ValueError("a periodic grid needs an even number of points")
                mats = [_prolong1d_vertex(Nc) for Nc in cdims]
            else:
                mats = [_prolong1d(Nc, "bloch" if kind == "bloch" else "dirichlet",
                                   0.0 if thetas is None else thetas[a])
                        for a, Nc in enumerate(cdims)]
            self.P.append(_kron_x_fastest(mats))
            dims = cdims
            hl = 2.0 * hl
        self.coarse_inv = np.linalg.inv(self.A[-1].toarray())

    def _cycle(self, lev: int, r: np.ndarray) -> np.ndarray:
        if lev == len(self.A) - 1:
            return self.coarse_inv @ r
        A, Dinv, om = self.A[lev], self.Dinv[lev][:, None], self.omega
        w = np.zeros_like(r)
        for _ in range(self.nu_pre):
            w = w + om * Dinv * (r - A @ w)
        P = self.P[lev]
        rc = (P.conj().T @ (r - A @ w)) / (2 ** self.d)
        w = w + P @ self._cycle(lev + 1, rc)
        for _ in range(self.nu_post):
            w = w + om * Dinv * (r - A @ w)
        return w

    def apply(self, R: np.ndarray) -> np.ndarray:
        R = np.asarray(R)
        one = R.ndim == 1
        Rb = R[:, None] if one else R
        dt = np.result_type(Rb.dtype, self.A[0].dtype, np.float64)
        out = self._cycle(0, Rb.astype(dt))
        return out[:, 0] if one else out

    __call__ = apply


def dense_matrix(T, n: int, dtype=np.float64) -> np.ndarray:
    """Columns T e_j, for checking symmetry and definiteness on small grids."""
    return T(np.eye(n, dtype=dtype))


# ------------------------------------------------------------------ AV-MG
def _cheb_coeffs(f, a: float, b: float, deg: int, nodes: int = 8192) -> np.ndarray:
    """Chebyshev coefficients c_0..c_deg of f on [a, b] by the discrete
    cosine sums over `nodes` Chebyshev points (first kind)."""
    j = np.arange(nodes)
    t = np.cos(np.pi * (j + 0.5) / nodes)
    fx = f(0.5 * (b - a) * t + 0.5 * (a + b))
    c = np.array([2.0 / nodes * np.sum(fx * np.cos(i * np.pi * (j + 0.5) / nodes))
                  for i in range(deg + 1)])
    c[0] *= 0.5
    return c


def _jackson(deg: int) -> np.ndarray:
    """Jackson damping factors g_0..g_deg (kernel polynomial method): the
    damped Chebyshev series is a convolution with a nonnegative kernel, so
    it keeps a nonnegative function nonnegative."""
    N = deg + 1
    i = np.arange(N)
    q = np.pi / (N + 1)
    return ((N - i + 1) * np.cos(i * q) + np.sin(i * q) / np.tan(q)) / (N + 1)


def abs_polynomial(a: float, b: float, deg: int) -> np.ndarray:
    """Coefficients (Chebyshev basis on [a, b]) of p_m ~ |x|: the Jackson-
    damped Chebyshev series of |x| of degree deg.  It is positive on [a, b]
    (a nonnegative kernel applied to |x|), so p_m(L - sigma I) is SPD."""
    return _cheb_coeffs(np.abs, a, b, deg) * _jackson(deg)


def cheb_eval(c: np.ndarray, a: float, b: float, x: np.ndarray) -> np.ndarray:
    t = (2.0 * np.asarray(x) - (a + b)) / (b - a)
    t0, t1 = np.ones_like(t), t
    out = c[0] * t0 + (c[1] * t1 if len(c) > 1 else 0.0)
    for i in range(2, len(c)):
        t0, t1 = t1, 2.0 * t * t1 - t0
        out = out + c[i] * t1
    return out


def cheb_apply(c: np.ndarray, a: float, b: float, S, X: np.ndarray) -> np.ndarray:
    """p(S) X for p = sum_i c_i T_i((2x - a - b)/(b - a)), by the three-term
    recurrence (one product with S per degree)."""
    def tmap(Y):
        return (2.0 * (S @ Y) - (a + b) * Y) / (b - a)
    t0 = X
    out = c[0] * t0
    if len(c) == 1:
        return out
    t1 = tmap(X)
    out = out + c[1] * t1
    for i in range(2, len(c)):
        t0, t1 = t1, 2.0 * tmap(t1) - t0
        out = out + c[i] * t1
    return out


class AVMG:
    """Appendix A, Algorithm 4 (AV-MG): one V-cycle for |L - sigma I| w = r
    on the Laplacian part L of the operator, T ~ |L - sigma I|^{-1}.

    * levels and transfers as in VCycle (cell-centred, L_l re-discretised at
      spacing 2^l h, R = P^T / 2^d);
    * level operator B_l = L_l where sqrt(sigma / scale) h_l < delta (the
      grid resolves the wanted oscillations, and the smoother only sees
      the components well above sigma, for which |L - sigma| ~ L); on the
      other levels B_l = p_m(L_l - sigma I_l), the Jackson-damped Chebyshev
      series of |x| of degree m on the spectral interval [-sigma,
      lambda_max(L_l) - sigma] (Gershgorin bound 4 d scale / h_l^2);
    * smoothing: nu Richardson steps w <- w + alpha_l (r - B_l w) before and
      after the coarse correction, alpha_l = omega / (2 d scale / h_l^2)
      for B_l = L_l (weighted Jacobi of a constant diagonal) and
      alpha_l = 1 / max p_m for the polynomial levels;
    * coarsest level: the exact |L_0 - sigma I_0|^{-1} (dense
      eigendecomposition).

    With these choices T = (I - E^2) B_l^{-1} + E P T_c R E per level, E =
    (I - alpha_l B_l)^nu, which is symmetric positive definite whenever
    B_l is and 0 < alpha_l lambda(B_l) < 2 (no Galerkin condition needed).

    mode="inv" gives Algorithm 5 (INV-MG): B_l = L_l - sigma I_l on every
    level, the same smoother and transfers, coarsest (L_0 - sigma I_0)^{-1};
    indefinite.
    """

    def __init__(self, dims, h: float, scale: float, levels: int, sigma: float,
                 delta: float = 0.6, degree: int = 10, nu: int = 2,
                 omega: float = 2.0 / 3.0, mode: str = "av"):
        if mode not in ("av", "inv"):
            raise ValueError(mode)
        self.mode, self.sigma, self.nu = mode, float(sigma), nu
        self.d = len(dims)
        self.L, self.P, self.kind, self.alpha, self.poly = [], [], [], [], []
        dims = tuple(dims)
        hl = h
        for lev in range(levels):
            L = ops.fd_dirichlet(dims, hl, scale=scale)
            self.L.append(L)
            diag = 2.0 * self.d * scale / hl**2
            lmax = 2.0 * diag                       # Gershgorin bound
            if mode == "inv":
                self.kind.append("shifted")
                self.alpha.append(omega / diag)
                self.poly.append(None)
            elif np.sqrt(self.sigma / scale) * hl < delta:
                self.kind.append("laplacian")
                self.alpha.append(omega / diag)
                self.poly.append(None)
            else:
                a, b = -self.sigma, lmax - self.sigma
                c = abs_polynomial(a, b, degree)
                pmax = float(cheb_eval(c, a, b, np.linspace(a, b, 20001)).max())
                self.kind.append("poly")
                self.alpha.append(1.0 / pmax)
                self.poly.append((c, a, b))
            if lev == levels - 1:
                break
            cdims, how = coarsen(dims)
            self.P.append(_kron_x_fastest([_prolong1d_vertex(Nc) if how == "vertex"
                                           else _prolong1d(Nc, "dirichlet") for Nc in cdims]))
            dims = cdims
            hl = 2.0 * hl
        S = self.L[-1].toarray() - self.sigma * np.eye(self.L[-1].shape[0])
        if mode == "av":
            ev, U = np.linalg.eigh(S)
            self.coarse = (U / np.abs(ev)[None, :]) @ U.T
        else:
            self.coarse = np.linalg.inv(S)

    def level_op(self, lev: int, X: np.ndarray) -> np.ndarray:
        """B_l X."""
        L = self.L[lev]
        kd = self.kind[lev]
        if kd == "laplacian":
            return L @ X
        if kd == "shifted":
            return L @ X - self.sigma * X
        c, a, b = self.poly[lev]
        n = L.shape[0]
        Ls = L - self.sigma * sp.identity(n, format="csr")
        return cheb_apply(c, a, b, Ls, X)

    def _cycle(self, lev: int, r: np.ndarray) -> np.ndarray:
        if lev == len(self.L) - 1:
            return self.coarse @ r
        al = self.alpha[lev]
        w = np.zeros_like(r)
        for _ in range(self.nu):
            w = w + al * (r - self.level_op(lev, w))
        P = self.P[lev]
        rc = (P.T @ (r - self.level_op(lev, w))) / (2 ** self.d)
        w = w + P @ self._cycle(lev + 1, rc)
        for _ in range(self.nu):
            w = w + al * (r - self.level_op(lev, w))
        return w

    def apply(self, R: np.ndarray) -> np.ndarray:
        R = np.asarray(R)
        one = R.ndim == 1
        Rb = R[:, None] if one else R
        if np.iscomplexobj(Rb):
            # a real operator: applied to the real and imaginary parts
            out = (self._cycle(0, np.ascontiguousarray(Rb.real, dtype=np.float64))
                   + 1j * self._cycle(0, np.ascontiguousarray(Rb.imag, dtype=np.float64)))
        else:
            out = self._cycle(0, Rb.astype(np.float64))
        return out[:, 0] if one else out

    __call__ = apply
