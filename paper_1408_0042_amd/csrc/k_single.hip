// Small kernels of the single-vector iteration (Algorithm 1) in complex
// arithmetic, and the dense preconditioner product.
//
// Algorithm 1 works with one complex vector v and its directions w, s, p:
// the T-harmonic problem eq. (3.5) of Z = [v w s p] is not Hermitian and
// can have complex eigenpairs even for real A, B and T, so the iteration
// runs in complex arithmetic (Section 3.2).  On the device a complex
// column is two real columns (real part, imaginary part), which is the
// interleaved layout of a complex128 vector: the real operators, the
// preconditioner, the Gram products and the block transforms of the
// block path act on them unchanged.  Only the two small steps differ:
//
//   k_single_ortho  z_a^H B z_b = G(2a,2b) + G(2a+1,2b+1)
//                                 + i (G(2a,2b+1) - G(2a+1,2b))
//                   from the real Gram G of the 8 real columns; Cholesky
//                   of the column-scaled complex Gram in slot order with
//                   the dropping rule of the block path; M = D R^-1 is
//                   written as the real 8 x 8 matrix that multiplies the
//                   interleaved columns, [[Re, Im], [-Im, Re]] per entry
//   k_single_tharm  complex G_L, G_R from the real [G_L | G_R]; G_L = L L^H,
//                   C = L^-1 G_R L^-H, complex Schur form of C by
//                   Hessenberg reduction and single-shift QR with Givens
//                   rotations (Golub & Van Loan, Sec. 7.5), the eigenvalue
//                   tau of largest modulus (xi = 1/tau of smallest modulus;
//                   ties by (Re xi, -Im xi)), its eigenvector by back
//                   substitution in the Schur form, y = L^-H u of unit
//                   2-norm with its largest entry real and positive, and
//                   the coefficients Y' (8 x 2 real) of v <- Z y
//
// The projected problems are at most 4 x 4: one thread does the
// arithmetic.  The refinement step of PLMR (Section 3.3, real arithmetic,
// one real column) is here too.
#include <cmath>

#include "common.cuh"

namespace plhr {

namespace {

struct cd {
  double re, im;
};
__device__ __forceinline__ cd mk(double r, double i) { return cd{r, i}; }
__device__ __forceinline__ cd operator+(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd operator*(cd a, cd b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cd operator*(double s, cd a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ cd cj(cd a) { return {a.re, -a.im}; }
__device__ __forceinline__ double ab(cd a) { return hypot(a.re, a.im); }
__device__ __forceinline__ cd dv(cd a, cd b) {  // a / b, scaled against overflow
  const double s = fmax(fabs(b.re), fabs(b.im));
  const cd bs = {b.re / s, b.im / s};
  const double d = bs.re * bs.re + bs.im * bs.im;
  const cd n = a * cj(bs);
  return {n.re / (d * s), n.im / (d * s)};
}
__device__ cd csqrt_(cd z) {
  const double r = ab(z);
  if (r == 0.0) return {0.0, 0.0};
  const double t = sqrt(0.5 * (r + fabs(z.re)));
  if (z.re >= 0.0) return {t, z.im / (2.0 * t)};
  return {fabs(z.im) / (2.0 * t), copysign(t, z.im)};
}

constexpr int kN = 4;  // complex slots v, w, s, p

// Rotation [[c, s], [-conj(s), c]] (c real) with -conj(s) a + c b = 0.
__device__ void givens(cd a, cd b, double& c, cd& s) {
  const double aa = ab(a), bb = ab(b);
  if (bb == 0.0) {
    c = 1.0;
    s = {0.0, 0.0};
    return;
  }
  if (aa == 0.0) {
    c = 0.0;
    s = (1.0 / bb) * cj(b);
    return;
  }
  const double r = hypot(aa, bb);
  c = aa / r;
  s = (1.0 / (aa * r)) * (a * cj(b));
}

// H <- G H G^H on rows/columns (p, q) of an n x n matrix; Q <- Q G^H.
__device__ void rot_sim(cd* H, cd* Q, int n, int p, int q, double c, cd s) {
  for (int j = 0; j < n; ++j) {  // rows p, q
    const cd x = H[p * kN + j], y = H[q * kN + j];
    H[p * kN + j] = c * x + s * y;
    H[q * kN + j] = c * y - cj(s) * x;
  }
  for (int r = 0; r < n; ++r) {  // columns p, q
    const cd x = H[r * kN + p], y = H[r * kN + q];
    H[r * kN + p] = c * x + cj(s) * y;
    H[r * kN + q] = c * y - s * x;
    const cd u = Q[r * kN + p], v = Q[r * kN + q];
    Q[r * kN + p] = c * u + cj(s) * v;
    Q[r * kN + q] = c * v - s * u;
  }
}

// Complex Schur form H = Q T Q^H of an n x n matrix (n <= 4) in place;
// returns false when the QR iteration does not converge.
__device__ bool schur(cd* H, cd* Q, int n) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Q[i * kN + j] = mk(i == j ? 1.0 : 0.0, 0.0);
  // Hessenberg form by rotations
  for (int j = 0; j + 2 < n; ++j)
    for (int i = n - 1; i >= j + 2; --i) {
      double c;
      cd s;
      givens(H[(i - 1) * kN + j], H[i * kN + j], c, s);
      rot_sim(H, Q, n, i - 1, i, c, s);
      H[i * kN + j] = mk(0.0, 0.0);
    }
  const double eps = 2.220446049250313e-16;
  int hi = n - 1, its = 0, total = 0;
  while (hi > 0) {
    // deflation
    int lo = hi;
    while (lo > 0) {
      const double sub = ab(H[lo * kN + lo - 1]);
      const double dia = ab(H[lo * kN + lo]) + ab(H[(lo - 1) * kN + lo - 1]);
      if (sub <= eps * dia || sub == 0.0) {
        H[lo * kN + lo - 1] = mk(0.0, 0.0);
        break;
      }
      --lo;
    }
    if (lo == hi) {
      --hi;
      its = 0;
      continue;
    }
    if (++total > 60 * n) return false;
    // Wilkinson shift from the trailing 2 x 2 of the active window, an
    // exceptional shift after 10 and 20 steps without deflation
    const cd a = H[(hi - 1) * kN + hi - 1], b = H[(hi - 1) * kN + hi];
    const cd c2 = H[hi * kN + hi - 1], d = H[hi * kN + hi];
    cd mu;
    if (its == 10 || its == 20) {
      mu = d + mk(0.75 * ab(c2), 0.0);
    } else {
      const cd half = 0.5 * (a - d);
      const cd disc = csqrt_(half * half + b * c2);
      const cd m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
      mu = (ab(m1 - d) <= ab(m2 - d)) ? m1 : m2;
    }
    ++its;
    // one explicit-shift QR step on the window [lo, hi]
    double cs[kN];
    cd sn[kN];
    for (int k = lo; k <= hi; ++k) H[k * kN + k] = H[k * kN + k] - mu;
    for (int k = lo; k < hi; ++k) {
      givens(H[k * kN + k], H[(k + 1) * kN + k], cs[k], sn[k]);
      for (int j = k; j < n; ++j) {
        const cd x = H[k * kN + j], y = H[(k + 1) * kN + j];
        H[k * kN + j] = cs[k] * x + sn[k] * y;
        H[(k + 1) * kN + j] = cs[k] * y - cj(sn[k]) * x;
      }
      H[(k + 1) * kN + k] = mk(0.0, 0.0);
    }
    for (int k = lo; k < hi; ++k) {
      for (int r = 0; r <= hi; ++r) {
        const cd x = H[r * kN + k], y = H[r * kN + k + 1];
        H[r * kN + k] = cs[k] * x + cj(sn[k]) * y;
        H[r * kN + k + 1] = cs[k] * y - sn[k] * x;
      }
      for (int r = 0; r < n; ++r) {
        const cd u = Q[r * kN + k], v = Q[r * kN + k + 1];
        Q[r * kN + k] = cs[k] * u + cj(sn[k]) * v;
        Q[r * kN + k + 1] = cs[k] * v - sn[k] * u;
      }
    }
    for (int k = lo; k <= hi; ++k) H[k * kN + k] = H[k * kN + k] + mu;
  }
  return true;
}

// ordering of xi = 1/tau: (|xi|, Re xi, -Im xi), tau = 0 last
__device__ bool xi_before(cd ta, cd tb) {
  const double aa = ab(ta), bb = ab(tb);
  if (aa == 0.0 || bb == 0.0) return aa > bb;
  const double ma = 1.0 / aa, mb = 1.0 / bb;
  if (ma != mb) return ma < mb;
  const double ra = ta.re / (aa * aa), rb = tb.re / (bb * bb);
  if (ra != rb) return ra < rb;
  const double ia = -ta.im / (aa * aa), ib = -tb.im / (bb * bb);
  return -ia < -ib;
}

constexpr double kOrthoRedoC = 1e-4;  // as the block path's Cholesky-QR

}  // namespace

// ----------------------------------------------------- complex Cholesky-QR
__global__ __launch_bounds__(64) void k_single_ortho(SmallParams p, SmallBufs b, DevStatus* st) {
  if (halted(st)) {
    if (p.pass == 1 && b.gate && threadIdx.x == 0) b.gate->done = 1;
    return;
  }
  if (p.pass == 2 && b.gate && b.gate->done) return;
  if (threadIdx.x != 0) return;
  const int m = p.m;  // 8 real columns
  const int have_p = st->have_p;
  cd G[kN * kN], R[kN * kN], X[kN * kN];
  double d[kN];
  int valid[kN];
  for (int a = 0; a < kN; ++a)
    for (int c = 0; c < kN; ++c) {
      const double* g0 = b.G + (size_t)(2 * a) * m;
      const double* g1 = b.G + (size_t)(2 * a + 1) * m;
      G[a * kN + c] = mk(g0[2 * c] + g1[2 * c + 1], g0[2 * c + 1] - g1[2 * c]);
    }
  for (int a = 0; a < kN; ++a) {
    int v = (a == 3) ? have_p : (a == 0 ? 1 : (b.active[0] | b.active[1]));
    const double g = G[a * kN + a].re;
    if (v && !(g > 0.0 && g < INFINITY)) v = 0;
    valid[a] = v;
    d[a] = v ? 1.0 / sqrt(g) : 0.0;
  }
  if (!valid[0]) {
    st->error = PLHR_ERR_BREAKDOWN;
    st->reason = kReasonVVanished;
    return;
  }
  for (int a = 0; a < kN; ++a)
    for (int c = 0; c < kN; ++c) {
      G[a * kN + c] = (valid[a] && valid[c]) ? (d[a] * d[c]) * G[a * kN + c] : mk(0.0, 0.0);
      R[a * kN + c] = mk(0.0, 0.0);
      X[a * kN + c] = mk(a == c ? 1.0 : 0.0, 0.0);
    }
  // G = R^H R in slot order; a numerically dependent column is dropped
  double minpiv = INFINITY;
  for (int j = 0; j < kN; ++j) {
    if (!valid[j]) continue;
    double piv = G[j * kN + j].re;
    for (int q = 0; q < j; ++q)
      if (valid[q]) piv -= R[q * kN + j].re * R[q * kN + j].re + R[q * kN + j].im * R[q * kN + j].im;
    if (!(piv > p.drop_tol)) {
      if (j == 0) {
        st->error = PLHR_ERR_BREAKDOWN;
        st->reason = kReasonVVanished;
        return;
      }
      valid[j] = 0;
      continue;
    }
    minpiv = fmin(minpiv, piv);
    const double r = sqrt(piv);
    R[j * kN + j] = mk(r, 0.0);
    for (int l = j + 1; l < kN; ++l) {
      if (!valid[l]) continue;
      cd s = G[j * kN + l];
      for (int q = 0; q < j; ++q)
        if (valid[q]) s = s - cj(R[q * kN + j]) * R[q * kN + l];
      R[j * kN + l] = (1.0 / r) * s;
    }
  }
  // X = R^-1 (upper) on the kept slots
  for (int i = kN - 1; i >= 0; --i) {
    if (!valid[i]) continue;
    for (int c = i; c < kN; ++c) {
      if (!valid[c]) continue;
      cd s = mk(c == i ? 1.0 : 0.0, 0.0);
      for (int q = i + 1; q <= c; ++q)
        if (valid[q]) s = s - R[i * kN + q] * X[q * kN + c];
      X[i * kN + c] = (1.0 / R[i * kN + i].re) * s;
    }
  }
  // M = D R^-1 as the real matrix of the interleaved columns
  for (int a = 0; a < kN; ++a)
    for (int c = 0; c < kN; ++c) {
      const bool on = valid[a] && valid[c] && c >= a;
      const cd v = on ? d[a] * X[a * kN + c] : mk(0.0, 0.0);
      b.M[(size_t)(2 * a) * m + 2 * c] = v.re;
      b.M[(size_t)(2 * a) * m + 2 * c + 1] = v.im;
      b.M[(size_t)(2 * a + 1) * m + 2 * c] = -v.im;
      b.M[(size_t)(2 * a + 1) * m + 2 * c + 1] = v.re;
    }
  int nk = 0, nd = 0;
  for (int a = 0; a < kN; ++a) {
    b.keep[2 * a] = b.keep[2 * a + 1] = valid[a];
    nk += valid[a];
    const int wanted = (a == 3) ? have_p : 1;
    if (!valid[a] && wanted) ++nd;
  }
  st->m_kept = 2 * nk;
  st->n_dropped = 2 * nd;
  if (p.pass == 1 && b.gate) {
    b.gate->error = 0;
    b.gate->done = (minpiv < kOrthoRedoC) ? 0 : 1;
  }
}

// ------------------------------------------- complex projected problem
__global__ __launch_bounds__(64) void k_single_tharm(SmallParams p, SmallBufs b, DevStatus* st) {
  if (halted(st)) return;
  if (threadIdx.x != 0) return;
  const int m = p.m, ld2 = 2 * m;
  int idx[kN];
  int n = 0;
  for (int a = 0; a < kN; ++a)
    if (b.keep[2 * a]) idx[n++] = a;
  if (n < 1) {
    st->error = PLHR_ERR_BREAKDOWN;
    st->reason = kReasonVVanished;
    return;
  }
  cd GL[kN * kN], GR[kN * kN], L[kN * kN], C[kN * kN], Q[kN * kN];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const int a = idx[i], c = idx[j];
      const double* r0 = b.GLR + (size_t)(2 * a) * ld2;
      const double* r1 = b.GLR + (size_t)(2 * a + 1) * ld2;
      GL[i * kN + j] = mk(r0[2 * c] + r1[2 * c + 1], r0[2 * c + 1] - r1[2 * c]);
      GR[i * kN + j] = mk(r0[m + 2 * c] + r1[m + 2 * c + 1], r0[m + 2 * c + 1] - r1[m + 2 * c]);
    }
  // Hermitian part of G_L
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      const cd h = 0.5 * (GL[i * kN + j] + cj(GL[j * kN + i]));
      GL[i * kN + j] = h;
      GL[j * kN + i] = cj(h);
    }
  // G_L = L L^H; pivots as in the block path (raised to 1e-15 max diag, a
  // clearly negative one leaves its slot out: tau = 0, never selected)
  double maxd = 0.0;
  for (int j = 0; j < n; ++j) maxd = fmax(maxd, GL[j * kN + j].re);
  const double floor_ = fmax(1e-15 * maxd, 1e-300);
  int dead[kN], ndead = 0;
  for (int i = 0; i < kN * kN; ++i) L[i] = mk(0.0, 0.0);
  for (int j = 0; j < n; ++j) {
    double p0 = GL[j * kN + j].re;
    for (int q = 0; q < j; ++q)
      p0 -= L[j * kN + q].re * L[j * kN + q].re + L[j * kN + q].im * L[j * kN + q].im;
    dead[j] = (p0 < -1e-10 * maxd) ? 1 : 0;
    if (dead[j]) {
      ++ndead;
      for (int q = 0; q < j; ++q) L[j * kN + q] = mk(0.0, 0.0);
      L[j * kN + j] = mk(1.0, 0.0);
      continue;
    }
    const double r = sqrt(fmax(p0, floor_));
    L[j * kN + j] = mk(r, 0.0);
    for (int i = j + 1; i < n; ++i) {
      cd s = GL[i * kN + j];
      for (int q = 0; q < j; ++q) s = s - L[i * kN + q] * cj(L[j * kN + q]);
      L[i * kN + j] = (1.0 / r) * s;
    }
  }
  if (ndead) st->n_excluded += ndead;
  if (ndead == n) {
    st->error = PLHR_ERR_BREAKDOWN;
    st->reason = kReasonVVanished;
    return;
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (dead[i] || dead[j]) GR[i * kN + j] = mk(0.0, 0.0);
  // X = L^-1 G_R (into C), then C = X L^-H = (L^-1 X^H)^H
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      cd s = GR[i * kN + c];
      for (int q = 0; q < i; ++q) s = s - L[i * kN + q] * C[q * kN + c];
      C[i * kN + c] = dv(s, L[i * kN + i]);
    }
  for (int c = 0; c < n; ++c)  // GR <- L^-1 C^H, column c
    for (int i = 0; i < n; ++i) {
      cd s = cj(C[c * kN + i]);
      for (int q = 0; q < i; ++q) s = s - L[i * kN + q] * GR[q * kN + c];
      GR[i * kN + c] = dv(s, L[i * kN + i]);
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) C[i * kN + j] = cj(GR[j * kN + i]);
  if (!schur(C, Q, n)) {
    st->error = PLHR_ERR_BREAKDOWN;
    st->reason = kReasonQR;
    return;
  }
  // eigenvalues in xi order (diagnostics) and the selected one
  int ord[kN];
  for (int i = 0; i < n; ++i) ord[i] = i;
  for (int i = 1; i < n; ++i)
    for (int j = i; j > 0 && xi_before(C[ord[j] * kN + ord[j]], C[ord[j - 1] * kN + ord[j - 1]]);
         --j) {
      const int t = ord[j];
      ord[j] = ord[j - 1];
      ord[j - 1] = t;
    }
  for (int r = 0; r < m; ++r) {
    b.xi[r] = 0.0;
    b.xi[m + r] = 0.0;
  }
  for (int r = 0; r < n; ++r) {
    const cd t = C[ord[r] * kN + ord[r]];
    const double a2 = t.re * t.re + t.im * t.im;
    b.xi[r] = (a2 > 0.0) ? t.re / a2 : INFINITY;
    b.xi[m + r] = (a2 > 0.0) ? -t.im / a2 : 0.0;
  }
  const int ks = ord[0];
  const cd tau = C[ks * kN + ks];
  if (!(ab(tau) > 0.0)) {
    st->error = PLHR_ERR_BREAKDOWN;
    st->reason = kReasonQR;
    return;
  }
  // eigenvector of the triangular factor (z_ks = 1), then u = Q z
  cd z[kN], u[kN], y[kN];
  double cn = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) cn = fmax(cn, ab(C[i * kN + j]));
  const double small = 2.220446049250313e-16 * fmax(cn, 1e-300);
  for (int i = 0; i < n; ++i) z[i] = mk(0.0, 0.0);
  z[ks] = mk(1.0, 0.0);
  for (int i = ks - 1; i >= 0; --i) {
    cd s = mk(0.0, 0.0);
    for (int j = i + 1; j <= ks; ++j) s = s + C[i * kN + j] * z[j];
    cd den = C[i * kN + i] - tau;
    if (ab(den) < small) den = mk(small, 0.0);
    z[i] = dv(mk(-s.re, -s.im), den);
  }
  for (int i = 0; i < n; ++i) {
    cd s = mk(0.0, 0.0);
    for (int j = 0; j < n; ++j) s = s + Q[i * kN + j] * z[j];
    u[i] = s;
  }
  // y = L^-H u
  for (int i = n - 1; i >= 0; --i) {
    cd s = u[i];
    for (int q = i + 1; q < n; ++q) s = s - cj(L[q * kN + i]) * y[q];
    y[i] = dv(s, L[i * kN + i]);
  }
  double nr2 = 0.0, big = -1.0;
  int im = 0;
  for (int i = 0; i < n; ++i) {
    const double a2 = y[i].re * y[i].re + y[i].im * y[i].im;
    nr2 += a2;
    if (a2 > big) big = a2, im = i;
  }
  // unit 2-norm, largest entry real and positive
  const double ay = ab(y[im]);
  const cd ph = (ay > 0.0) ? mk(y[im].re / ay, -y[im].im / ay) : mk(1.0, 0.0);
  const double sc = (nr2 > 0.0) ? 1.0 / sqrt(nr2) : 0.0;
  const int kint = p.kint;  // 2
  for (int e = 0; e < m * kint; ++e) b.Y[e] = 0.0;
  for (int i = 0; i < n; ++i) {
    const cd v = sc * (y[i] * ph);
    const int a = idx[i];
    b.Y[(size_t)(2 * a) * kint + 0] = v.re;
    b.Y[(size_t)(2 * a) * kint + 1] = v.im;
    b.Y[(size_t)(2 * a + 1) * kint + 0] = -v.im;
    b.Y[(size_t)(2 * a + 1) * kint + 1] = v.re;
  }
  b.kinds[0] = 1;
  b.kinds[1] = 3;
  b.pair[0] = 1;
  b.pair[1] = 0;
}

// ------------------------------------------------ PLMR refinement step
// F = Zhat^T (A - lam B) T (A - lam B) Zhat on the kept slots from the
// Gram [G_1 | G_2] = (T(A - lam B)Zhat)^T [(A - sigma B)Zhat | B Zhat]:
// F(i, j) = G_1(j, i) + (sigma - lam) G_2(j, i), symmetrised.  Its
// eigenpairs by cyclic Jacobi (Golub & Van Loan, Sec. 8.5); the vector of
// the smallest eigenvalue theta^2 (ties: lower slot) is y, unit 2-norm,
// largest entry positive (Zhat is B-orthonormal, so v = Zhat y has
// ||v||_B = 1).
__global__ __launch_bounds__(64) void k_plmr_small(SmallParams p, SmallBufs b, DevStatus* st) {
  if (halted(st)) return;
  if (threadIdx.x != 0) return;
  const int m = p.m, ld2 = 2 * m;
  int idx[kN];
  int n = 0;
  for (int a = 0; a < m && a < kN; ++a)
    if (b.keep[a]) idx[n++] = a;
  if (n < 1) {
    st->error = PLHR_ERR_BREAKDOWN;
    st->reason = kReasonVVanished;
    return;
  }
  const double lam = b.lam[0];
  double F[kN * kN], V[kN * kN];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const int a = idx[i], c = idx[j];
      const double fij = b.GLR[(size_t)c * ld2 + a] + (p.sigma - lam) * b.GLR[(size_t)c * ld2 + m + a];
      const double fji = b.GLR[(size_t)a * ld2 + c] + (p.sigma - lam) * b.GLR[(size_t)a * ld2 + m + c];
      F[i * kN + j] = 0.5 * (fij + fji);
      V[i * kN + j] = (i == j) ? 1.0 : 0.0;
    }
  double a2 = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) a2 += F[i * kN + j] * F[i * kN + j];
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += F[i * kN + j] * F[i * kN + j];
    if (!(off > 1e-30 * a2)) break;
    for (int pp = 0; pp < n; ++pp)
      for (int q = pp + 1; q < n; ++q) {
        const double apq = F[pp * kN + q];
        if (apq == 0.0) continue;
        const double th = (F[q * kN + q] - F[pp * kN + pp]) / (2.0 * apq);
        const double t = copysign(1.0, th) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int r = 0; r < n; ++r) {  // columns pp, q
          const double x = F[r * kN + pp], y = F[r * kN + q];
          F[r * kN + pp] = c * x - sn * y;
          F[r * kN + q] = sn * x + c * y;
          const double u = V[r * kN + pp], w = V[r * kN + q];
          V[r * kN + pp] = c * u - sn * w;
          V[r * kN + q] = sn * u + c * w;
        }
        for (int r = 0; r < n; ++r) {  // rows pp, q
          const double x = F[pp * kN + r], y = F[q * kN + r];
          F[pp * kN + r] = c * x - sn * y;
          F[q * kN + r] = sn * x + c * y;
        }
      }
  }
  int js = 0;
  for (int j = 1; j < n; ++j)
    if (F[j * kN + j] < F[js * kN + js]) js = j;
  double nr2 = 0.0, big = -1.0;
  int im = 0;
  for (int i = 0; i < n; ++i) {
    const double v = V[i * kN + js];
    nr2 += v * v;
    if (fabs(v) > big) big = fabs(v), im = i;
  }
  double sc = (nr2 > 0.0) ? 1.0 / sqrt(nr2) : 0.0;
  if (V[im * kN + js] < 0.0) sc = -sc;
  for (int e = 0; e < m * p.kint; ++e) b.Y[e] = 0.0;
  for (int i = 0; i < n; ++i) b.Y[(size_t)idx[i] * p.kint] = V[i * kN + js] * sc;
  for (int r = 0; r < 2 * m; ++r) b.xi[r] = 0.0;
  b.xi[0] = F[js * kN + js];  // theta^2, the squared T-norm of the refined residual
  b.kinds[0] = 0;
  b.pair[0] = -1;
}

void launch_plmr_small(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s) {
  prof_begin(KC_THARM_QR, 2.0 * p.m * p.m * 8.0, 2000.0, s);
  hipLaunchKernelGGL(k_plmr_small, dim3(1), dim3(64), 0, s, p, b, st);
  prof_end(KC_THARM_QR, s);
}

void launch_single_ortho(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s) {
  prof_begin(KC_ORTHO, (double)p.m * p.m * 8.0, 64.0 * 4 * 4 * 4, s);
  hipLaunchKernelGGL(k_single_ortho, dim3(1), dim3(64), 0, s, p, b, st);
  prof_end(KC_ORTHO, s);
}

void launch_single_tharm(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s) {
  prof_begin(KC_THARM_QR, 2.0 * p.m * p.m * 8.0, 4000.0, s);
  hipLaunchKernelGGL(k_single_tharm, dim3(1), dim3(64), 0, s, p, b, st);
  prof_end(KC_THARM_QR, s);
}

// ------------------------------------------------ dense preconditioner
// One wavefront per row of T: lanes stride over the row (coalesced), four
// columns of X at a time, then a butterfly sum over the wavefront (a
// fixed order: deterministic).
__global__ __launch_bounds__(256) void k_dense_prec(size_t n, const double* __restrict__ T,
                                                    const double* __restrict__ X, int ldx,
                                                    double* o0, int ld0, double* o1, int ld1,
                                                    int split, int ncols, const DevStatus* st) {
  if (halted(st)) return;
  const int lane = threadIdx.x & 63;
  const size_t row = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const double* tr = T + row * n;
  for (int c0 = 0; c0 < ncols; c0 += 4) {
    const int nc = min(4, ncols - c0);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (size_t j = lane; j < n; j += 64) {
      const double t = tr[j];
      const double* x = X + j * ldx + c0;
      a0 += t * x[0];
      if (nc > 1) a1 += t * x[1];
      if (nc > 2) a2 += t * x[2];
      if (nc > 3) a3 += t * x[3];
    }
    for (int off = 32; off > 0; off >>= 1) {
      a0 += __shfl_xor(a0, off);
      a1 += __shfl_xor(a1, off);
      a2 += __shfl_xor(a2, off);
      a3 += __shfl_xor(a3, off);
    }
    if (lane < nc) {
      const double v = (lane == 0) ? a0 : (lane == 1) ? a1 : (lane == 2) ? a2 : a3;
      const int c = c0 + lane;
      if (c < split)
        o0[row * ld0 + c] = v;
      else
        o1[row * ld1 + (c - split)] = v;
    }
  }
}

void launch_dense_prec(size_t n, const double* T, const double* X, int ldx, Blk o0, Blk o1,
                       int split, int ncols, const DevStatus* st, hipStream_t s) {
  const double nn = (double)n;
  prof_begin(KC_COARSE, 8.0 * nn * nn + 16.0 * nn * ncols, 2.0 * nn * nn * ncols, s);
  const unsigned nb = (unsigned)((n + 3) / 4);
  hipLaunchKernelGGL(k_dense_prec, dim3(nb), dim3(256), 0, s, n, T, X, ldx, o0.ptr, o0.ld,
                     o1.ptr, o1.ld, split, ncols, st);
  prof_end(KC_COARSE, s);
}

}  // namespace plhr
