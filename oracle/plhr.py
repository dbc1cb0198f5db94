"""Block PLHR in FP64 on the CPU (oracle; test infrastructure only).

Follows the paper step by step:

* Algorithm 1 (Section 3.2): single-vector PLHR on the raw basis
  Z = [v, w, s, p];
* Algorithm 2 (Section 4): block PLHR in complex arithmetic;
* Algorithm 3 (Section 4.1): block PLHR in real arithmetic for real
  symmetric A, B and T, with complex-conjugate T-harmonic Ritz vectors
  replaced by their real and imaginary parts;
* the PLMR variant (Section 3.3): Algorithm 1's trial subspace with the
  refinement extraction (minimal T-norm residual at the current Rayleigh
  quotient).

The projected problem of every iteration is eq. (3.5),

    Z^*(A - sigma B) T (A - sigma B) Z y = xi Z^*(A - sigma B) T B Z y,

posed on the B-orthonormalised basis Zhat = [Vhat What Shat Phat]
(the blocks are B-orthonormalised in that order, Section 4) and solved with
LAPACK's QZ (scipy.linalg.eig).  The k eigenvectors with the smallest |xi|
give the new block (Definition 3.1); the harmonic values are discarded and
replaced by Rayleigh quotients (Section 3.2), with eq. (4.1) for the real and
imaginary parts of a conjugate pair.  After the loop a standard Rayleigh-Ritz
step on V returns B-orthonormal Ritz vectors (Section 4).

Readings of points the paper leaves open (all listed with their reasons in
the design notes of the repository):
* relative residual: ||A v - lam B v||_2 / ((||A||_1 + |lam| ||B||_1) ||v||_2);
* soft locking: a column whose relative residual is at or below tol
  contributes no w, s, p columns to the next trial subspace; the set is
  recomputed every iteration;
* the iteration stops when the k columns nearest sigma (by current Rayleigh
  quotient) are all converged; the extra column of the real variant is not
  required to converge;
* B-orthonormalisation: classical Gram-Schmidt run twice per column in the
  B-inner product; a column whose norm falls below drop_tol times its norm
  before projection adds nothing to span(Z) and is dropped (the start block
  itself must have full rank);
* sort key for xi: (|xi|, Re xi, -Im xi), so a conjugate pair is adjacent
  with the positive-imaginary member first.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla


class Breakdown(RuntimeError):
    pass


def _mul(M, X):
    return X if M is None else M @ X


def _prec(T, X):
    return X if T is None else T(X)


def _norm1(M) -> float:
    if M is None:
        return 1.0
    return float(np.abs(M).sum(axis=0).max())


@dataclass
class Problem:
    A: object                       # sparse or dense, Hermitian
    B: object = None                # None means identity
    T: Optional[Callable] = None    # None means identity; must be HPD
    sigma: float = 0.0
    normA1: Optional[float] = None
    normB1: Optional[float] = None
    # "tharmonic": eq. (3.5); "harmonic": the same with T replaced by I
    # inside the projection only (the search directions still use T), the
    # "harm." variant of the experiments in Section 6.2
    extraction: str = "tharmonic"

    def __post_init__(self):
        if self.normA1 is None:
            self.normA1 = _norm1(self.A)
        if self.normB1 is None:
            self.normB1 = _norm1(self.B)


def rel_residuals(prob: Problem, V: np.ndarray, lam: np.ndarray) -> np.ndarray:
    R = prob.A @ V - _mul(prob.B, V) * lam[None, :]
    rn = np.linalg.norm(R, axis=0)
    vn = np.linalg.norm(V, axis=0)
    return rn / ((prob.normA1 + np.abs(lam) * prob.normB1) * vn)


def b_normalize(B, V):
    BV = _mul(B, V)
    nr = np.sqrt(np.real(np.sum(np.conj(V) * BV, axis=0)))
    return V / nr[None, :]


def rayleigh(prob: Problem, V: np.ndarray) -> np.ndarray:
    num = np.real(np.sum(np.conj(V) * (prob.A @ V), axis=0))
    den = np.real(np.sum(np.conj(V) * _mul(prob.B, V), axis=0))
    return num / den


def b_orthonormalize(blocks, B, drop_tol: float = 1e-10):
    """B-orthonormalise the columns of the blocks in the given order.

    ``blocks`` is a list of (name, X).  Returns (Zhat, labels) where labels
    lists (name, column) of the kept columns in order.
    """
    cols, bcols, labels = [], [], []
    for name, X in blocks:
        if X is None or X.shape[1] == 0:
            continue
        for j in range(X.shape[1]):
            x = X[:, j].copy()
            n0 = np.sqrt(abs(np.vdot(x, _mul(B, x))))
            if n0 == 0.0:
                continue
            for _ in range(2):
                if cols:
                    Q = np.column_stack(cols)
                    BQ = np.column_stack(bcols)
                    x = x - Q @ (BQ.conj().T @ x)
            bx = _mul(B, x)
            nrm = np.sqrt(abs(np.vdot(x, bx)))
            if nrm <= drop_tol * n0:
                # a numerically dependent column adds nothing to the span
                # of Z, which is all the projection uses (Section 4)
                continue
            cols.append(x / nrm)
            bcols.append(bx / nrm)
            labels.append((name, j))
    if not any(lb[0] == "V" for lb in labels):
        raise Breakdown("the V block vanished")
    return np.column_stack(cols), labels


def tharmonic_matrices(prob: Problem, Zh: np.ndarray):
    """Left and right matrices of eq. (3.5) for the basis Zh (with T = I
    when prob.extraction is "harmonic")."""
    Q = prob.A @ Zh - prob.sigma * _mul(prob.B, Zh)      # (A - sigma B) Z
    if prob.extraction == "harmonic":
        TQ = Q                                          # T -> I in the projection
    elif prob.extraction == "tharmonic":
        TQ = _prec(prob.T, Q)                           # T (A - sigma B) Z
    else:
        raise ValueError(prob.extraction)
    GL = Q.conj().T @ TQ                                # Z^*(A-sB) T (A-sB) Z
    GR = TQ.conj().T @ _mul(prob.B, Zh)                 # Z^*(A-sB) T B Z  (T = T^*)
    return GL, GR


def sorted_tharmonic(GL, GR, real_pairs: bool = False):
    """Eigenpairs (xi, Y) of GL y = xi GR y sorted by (|xi|, Re xi, -Im xi).

    With real_pairs=True (real pencils, Algorithm 3) LAPACK returns each
    complex-conjugate pair as two consecutive eigenvalues, the one with
    positive imaginary part first; the pair is kept together as one unit in
    the sort, so a complex xi is always immediately followed by its
    conjugate.  Returns (xi, Y, unit) where unit[j] is the index of the first
    column of j's unit (unit[j] == j for a single eigenvalue or the first
    member of a pair).
    """
    xi, Y = sla.eig(GL, GR)
    xi = np.asarray(xi, dtype=np.complex128)
    m = len(xi)
    groups = []
    j = 0
    while j < m:
        if real_pairs and np.isfinite(xi[j]) and xi[j].imag != 0.0:
            if j + 1 >= m or not (xi[j].imag > 0 > xi[j + 1].imag):
                raise Breakdown("LAPACK conjugate pair layout not found")
            groups.append([j, j + 1])
            j += 2
        else:
            groups.append([j])
            j += 1

    def key(g):
        z = xi[g[0]]
        if not np.isfinite(z):
            return (np.inf, np.inf, 0.0)
        return (abs(z), z.real, -z.imag)

    groups.sort(key=key)
    order, unit = [], []
    for g in groups:
        first = len(order)
        for idx in g:
            order.append(idx)
            unit.append(first)
    order = np.array(order)
    return xi[order], Y[:, order], np.array(unit)


def real_selection(xi: np.ndarray, Y: np.ndarray, unit: np.ndarray, kk: int):
    """Algorithm 3, selection step: from the sorted (xi, Y) take kk columns
    and build the real Y' = [Y0 YR ytilR YI].  Returns (Yp, kinds, pair_of)
    where kinds[j] is 'real', 'R', 'tilde' or 'I' for column j of Y' and
    pair_of[j] is the partner column index for 'R'/'I' columns."""
    Y0, YR, YI = [], [], []
    ytil = None
    i = 0
    while i < kk:
        if xi[i].imag == 0.0 or not np.isfinite(xi[i]):
            Y0.append(np.real(Y[:, i]))
            i += 1
            continue
        assert unit[i] == i and i + 1 < len(xi) and unit[i + 1] == i
        if i + 1 < kk:
            y = Y[:, i]                      # the member with Im xi > 0
            YR.append(y.real)
            YI.append(y.imag)
            i += 2
        else:                                # its conjugate is number kk+1
            ytil = Y[:, i].real
            i += 1
    cols = Y0 + YR + ([ytil] if ytil is not None else []) + YI
    kinds = (["real"] * len(Y0) + ["R"] * len(YR)
             + (["tilde"] if ytil is not None else []) + ["I"] * len(YI))
    pair_of = [-1] * len(cols)
    base_R = len(Y0)
    base_I = len(Y0) + len(YR) + (1 if ytil is not None else 0)
    for a in range(len(YR)):
        pair_of[base_R + a] = base_I + a
        pair_of[base_I + a] = base_R + a
    return np.column_stack(cols), kinds, pair_of


def real_rayleigh(prob: Problem, V: np.ndarray, kinds, pair_of) -> np.ndarray:
    """Algorithm 3, Rayleigh-quotient step, with eq. (4.1) for pairs."""
    AV = prob.A @ V
    BV = _mul(prob.B, V)
    vav = np.sum(V * AV, axis=0)
    vbv = np.sum(V * BV, axis=0)
    lam = vav / vbv
    for j, kd in enumerate(kinds):
        if kd in ("R", "I"):
            q = pair_of[j]
            lam[j] = (vav[j] + vav[q]) / (vbv[j] + vbv[q])
    return lam


@dataclass
class History:
    lam: List[np.ndarray] = field(default_factory=list)
    rel_res: List[np.ndarray] = field(default_factory=list)
    m: List[int] = field(default_factory=list)


@dataclass
class Result:
    lam: np.ndarray
    V: np.ndarray
    rel_res: np.ndarray
    iters: int
    converged: bool
    history: History


def wanted_columns(lam: np.ndarray, sigma: float, k: int) -> np.ndarray:
    """Indices of the k columns whose values are nearest sigma (ties: smaller)."""
    order = np.lexsort((lam, np.abs(lam - sigma)))
    return order[:k]


class BPLHR:
    """State of Algorithm 2 (real=False) or Algorithm 3 (real=True)."""

    def __init__(self, prob: Problem, V0: np.ndarray, k: int, real: bool = True,
                 lock: bool = True, drop_tol: float = 1e-10):
        self.prob, self.k, self.real, self.lock = prob, k, real, lock
        self.drop_tol = drop_tol
        V = np.array(V0, dtype=np.float64 if real else np.complex128)
        # the start block must have full rank
        _, labels = b_orthonormalize([("V", V)], prob.B, drop_tol)
        if len(labels) < V.shape[1]:
            raise Breakdown("the start block is rank deficient")
        # step 1-2: B-normalise, Lambda = diag(V^* A V)
        V = b_normalize(prob.B, V)
        self.V = V
        self.lam = np.real(np.sum(np.conj(V) * (prob.A @ V), axis=0))
        self.P = None
        self.iters = 0
        self.last_labels = None

    # ---- one pass through the body of the while-loop
    def residuals(self):
        return rel_residuals(self.prob, self.V, self.lam)

    def step(self, rel_res=None):
        prob = self.prob
        V, lam = self.V, self.lam
        kk = V.shape[1]
        if rel_res is None:
            rel_res = self.residuals()
        tol = getattr(self, "tol", 0.0)
        active = np.ones(kk, dtype=bool)
        if self.lock:
            active = rel_res > tol
        # W = T (A V - B V Lambda) and S = T (A W - B W Lambda), active columns
        Va, la = V[:, active], lam[active]
        W = _prec(prob.T, prob.A @ Va - _mul(prob.B, Va) * la[None, :])
        S = _prec(prob.T, prob.A @ W - _mul(prob.B, W) * la[None, :])
        Pa = None if self.P is None else self.P[:, active]
        blocks = [("V", V), ("W", W), ("S", S), ("P", Pa)]
        Zh, labels = b_orthonormalize(blocks, prob.B, self.drop_tol)
        self.last_labels = labels
        GL, GR = tharmonic_matrices(prob, Zh)
        xi, Y, unit = sorted_tharmonic(GL, GR, real_pairs=self.real)
        isV = np.array([lb[0] == "V" for lb in labels])
        if self.real:
            Yp, kinds, pair_of = real_selection(xi, Y, unit, kk)
            Pn = Zh[:, ~isV] @ Yp[~isV, :]
            Vn = Zh[:, isV] @ Yp[isV, :] + Pn
            lamn = real_rayleigh(prob, Vn, kinds, pair_of)
        else:
            Ys = Y[:, :kk]
            Pn = Zh[:, ~isV] @ Ys[~isV, :]
            Vn = Zh[:, isV] @ Ys[isV, :] + Pn
            lamn = rayleigh(prob, Vn)
        self.V = b_normalize(prob.B, Vn)
        self.P = Pn
        self.lam = lamn
        self.xi = xi
        self.iters += 1
        return Zh.shape[1]

    def final_rr(self):
        """Standard Rayleigh-Ritz on span(V); k Ritz pairs nearest sigma."""
        prob = self.prob
        V = self.V
        H = V.conj().T @ (prob.A @ V)
        M = V.conj().T @ _mul(prob.B, V)
        H = 0.5 * (H + H.conj().T)
        M = 0.5 * (M + M.conj().T)
        theta, X = sla.eigh(H, M)
        Vr = V @ X
        sel = wanted_columns(theta, prob.sigma, self.k)
        order = sel[np.lexsort((theta[sel], np.abs(theta[sel] - prob.sigma)))]
        return theta[order], Vr[:, order]


def bplhr(prob: Problem, V0: np.ndarray, k: int, tol: float = 1e-8, maxit: int = 1000,
          real: bool = True, lock: bool = True, drop_tol: float = 1e-10,
          record: bool = True) -> Result:
    """Run Algorithm 3 (real=True) or Algorithm 2 (real=False) to convergence."""
    s = BPLHR(prob, V0, k, real=real, lock=lock, drop_tol=drop_tol)
    s.tol = tol
    hist = History()
    converged = False
    for it in range(maxit + 1):
        rr = s.residuals()
        if record:
            hist.lam.append(s.lam.copy())
            hist.rel_res.append(rr.copy())
        want = wanted_columns(s.lam, prob.sigma, k)
        if np.all(rr[want] <= tol):
            converged = True
            break
        if it == maxit:
            break
        m = s.step(rr)
        if record:
            hist.m.append(m)
    lam, V = s.final_rr()
    return Result(lam=lam, V=V, rel_res=rel_residuals(prob, V, lam), iters=s.iters,
                  converged=converged, history=hist)


def plhr_single(prob: Problem, v0: np.ndarray, maxit: int = 50, tol: float = 0.0):
    """Algorithm 1: single-vector PLHR in complex arithmetic on the raw basis
    Z = [v, w, s, p] (no orthonormalisation).  Returns the list of Rayleigh
    quotients (one per iteration, starting with the initial one) and v."""
    v = np.array(v0, dtype=np.complex128).ravel()
    v = v / np.sqrt(np.real(np.vdot(v, _mul(prob.B, v))))
    lam = np.real(np.vdot(v, prob.A @ v))
    p = None
    lams = [lam]
    for _ in range(maxit):
        r = prob.A @ v - lam * _mul(prob.B, v)
        w = _prec(prob.T, r)
        s = _prec(prob.T, prob.A @ w - lam * _mul(prob.B, w))
        cols = [v, w, s] + ([p] if p is not None else [])
        Z = np.column_stack(cols)
        GL, GR = tharmonic_matrices(prob, Z)
        xi, Y, _ = sorted_tharmonic(GL, GR)
        y = Y[:, 0]
        p = y[1] * w + y[2] * s + (y[3] * p if p is not None else 0.0)
        v = y[0] * v + p
        v = v / np.sqrt(np.real(np.vdot(v, _mul(prob.B, v))))
        lam = np.real(np.vdot(v, prob.A @ v))
        lams.append(lam)
        if tol > 0:
            rr = np.linalg.norm(prob.A @ v - lam * _mul(prob.B, v)) / (
                (prob.normA1 + abs(lam) * prob.normB1) * np.linalg.norm(v))
            if rr <= tol:
                break
    return np.array(lams), v


def refined_vector(prob: Problem, Zh: np.ndarray, lam_t: float):
    """The refinement extraction of Section 3.3: over span(Zh) (Zh
    B-orthonormal), the B-unit vector v = Zh y minimising the T-norm of
    A v - lam_t B v, i.e. the eigenvector of the smallest eigenvalue of
    Zh^*(A - lam_t B) T (A - lam_t B) Zh y = theta^2 y.  Returns (theta^2, y)."""
    Rl = prob.A @ Zh - lam_t * _mul(prob.B, Zh)          # (A - lam_t B) Z
    F = Rl.conj().T @ _prec(prob.T, Rl)
    F = 0.5 * (F + F.conj().T)
    th, Y = np.linalg.eigh(F)
    return th[0], Y[:, 0]


def plmr_single(prob: Problem, v0: np.ndarray, maxit: int = 50, tol: float = 0.0):
    """The PLMR method of Section 3.3: the trial subspace of Algorithm 1,
    span{v, w, s, p}, with the refinement extraction at the current Rayleigh
    quotient (lam_t = lam) in place of the T-harmonic one; the conjugate
    direction is p = beta w + gamma s + delta p as in Algorithm 1.  The
    basis is B-orthonormalised in the order v, w, s, p (the same span).
    Real arithmetic for real A, B, T (the projected problem is Hermitian).
    Returns the Rayleigh quotients (the initial one first) and v."""
    v = np.array(v0, dtype=np.float64).ravel()
    v = v / np.sqrt(np.vdot(v, _mul(prob.B, v)))
    lam = float(np.vdot(v, prob.A @ v))
    p = None
    lams = [lam]
    for _ in range(maxit):
        w = _prec(prob.T, prob.A @ v - lam * _mul(prob.B, v))
        s = _prec(prob.T, prob.A @ w - lam * _mul(prob.B, w))
        blocks = [("V", v[:, None]), ("W", w[:, None]), ("S", s[:, None]),
                  ("P", None if p is None else p[:, None])]
        Zh, labels = b_orthonormalize(blocks, prob.B)
        _, y = refined_vector(prob, Zh, lam)
        isV = np.array([lb[0] == "V" for lb in labels])
        p = Zh[:, ~isV] @ y[~isV]
        v = Zh[:, isV] @ y[isV] + p
        v = v / np.sqrt(np.vdot(v, _mul(prob.B, v)))
        lam = float(np.vdot(v, prob.A @ v))
        lams.append(lam)
        if tol > 0:
            rr = np.linalg.norm(prob.A @ v - lam * _mul(prob.B, v)) / (
                (prob.normA1 + abs(lam) * prob.normB1) * np.linalg.norm(v))
            if rr <= tol:
                break
    return np.array(lams), v
