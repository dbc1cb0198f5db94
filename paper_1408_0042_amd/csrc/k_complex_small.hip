// Small kernels of the iterations in complex arithmetic: Algorithm 1 (one
// complex vector) and Algorithm 2 (a block of k_int complex vectors).
//
// A complex column is stored as two adjacent real columns (real part,
// imaginary part), the interleaved layout of a complex128 block, so the
// trial basis Z = [V W S P] of N = 4 k_int complex columns is a real block
// of m = 2N columns, and the Gram products, block transforms and updates of
// the real path act on it unchanged.  The complex Gram products follow from
// the real ones:
//     z_a^H Y z_b = G(2a,2b) + G(2a+1,2b+1) + i (G(2a,2b+1) - G(2a+1,2b))
// for G = Z^T [Y Z] of the interleaved real views (Y real symmetric or the
// Hermitian operator's interleaved product), and a complex matrix M acting
// on the columns is the real 2N x 2N matrix with the 2 x 2 blocks
// [[Re, Im], [-Im, Re]].
//
//   k_cplx_ortho   Cholesky of the column-scaled complex Gram in slot order
//                  with the dropping rule of the real path (a column whose
//                  pivot is at most drop_tol adds nothing and is left out),
//                  M = D R^-1 as the real matrix of the interleaved columns;
//                  the same gate as the real Cholesky-QR for the automatic
//                  second pass
//   k_cplx_tharm   eq. (3.5) in complex arithmetic: G_L = L L^H, C = L^-1 G_R
//                  L^-H, the complex Schur form C = Q T Q^H (Hessenberg by
//                  Householder reflections, then single-shift QR with Wilkinson
//                  shifts, Golub & Van Loan Sec. 7.5), the k_int eigenvalues
//                  tau of largest modulus (xi = 1/tau of smallest modulus,
//                  ties by (Re xi, -Im xi)), their eigenvectors by back
//                  substitution in T, y = L^-H Q z of unit 2-norm with the
//                  largest entry real and positive, and the coefficients Y'
//                  (2N x 2 k_int real)
//   k_cplx_final   the final Rayleigh-Ritz step on span(V) in complex
//                  arithmetic: V^H (A - sigma) V x = theta V^H V x with the
//                  dropping rule, the k pairs nearest sigma
//
// One wavefront per kernel: the loops over rows or columns of a matrix
// step are spread over the lanes, the steps are separated by barriers
// (free for a single wavefront).  The matrices are held in LDS.
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

constexpr int kW = 64;          // one wavefront
constexpr int kMaxN = kMaxM / 2;  // complex columns of the widest basis

// 1/sqrt(x) from the hardware estimate and two Newton steps
__device__ __forceinline__ double crsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}

// |re| + |im|: the modulus surrogate of the deflation tests
__device__ __forceinline__ double ab1(cd a) { return fabs(a.re) + fabs(a.im); }

// Rotation [[c, s], [-conj(s), c]] (c real) with -conj(s) a + c b = 0:
// c = |a| / r, s = (a / |a|) conj(b) / r, r = sqrt(|a|^2 + |b|^2), from
// squared moduli and reciprocal square roots (the entries are far from
// the overflow and underflow thresholds of their squares).
__device__ void givens(cd a, cd b, double& c, cd& s) {
  const double bb2 = b.re * b.re + b.im * b.im;
  if (bb2 == 0.0) {
    c = 1.0;
    s = {0.0, 0.0};
    return;
  }
  const double aa2 = a.re * a.re + a.im * a.im;
  if (aa2 == 0.0) {
    c = 0.0;
    s = crsq(bb2) * cj(b);
    return;
  }
  const double ia = crsq(aa2), ir = crsq(aa2 + bb2);
  c = aa2 * ia * ir;
  s = (ia * ir) * (a * cj(b));
}

// Complex Schur form H = Q T Q^H of an n x n matrix (stride ld) in place,
// by the whole wavefront; every lane keeps the same control flow (all its
// decisions read the matrix after a barrier).  Returns false when the QR
// iteration does not converge.  `stamp` (may be null) takes the shader
// clock after the Hessenberg reduction.
__device__ bool schur_w(cd* H, cd* Q, int ld, int n, long long* stamp = nullptr) {
  for (int e = threadIdx.x; e < n * n; e += kW) {
    const int i = e / n, j = e - i * n;
    Q[i * ld + j] = mk(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // Hessenberg form by Householder reflections P = I - tau v v^H (Golub &
  // Van Loan, Sec. 7.4.3, complex): step j maps column j below the
  // diagonal, x = H[j+1.., j], to alpha e_1 with alpha = -(x_0 / |x_0|)
  // ||x||, v = x - alpha e_1, tau = 2 / v^H v; then H <- P H P, Q <- Q P.
  // n - 2 steps of three lane-parallel phases (each lane one column for
  // P H, one row of H and of Q for H P and Q P) instead of one
  // rotation per subdiagonal entry.
  static_assert(kMaxN <= kW, "one lane per row or column");
  __shared__ cd hv[kMaxN];
  const int lane = threadIdx.x;
  for (int j = 0; j + 2 < n; ++j) {
    const int len = n - j - 1;  // rows j+1 .. n-1
    cd xl = mk(0.0, 0.0);
    if (lane < len) xl = H[(j + 1 + lane) * ld + j];
    double s2 = (lane >= 1 && lane < len) ? xl.re * xl.re + xl.im * xl.im : 0.0;
    for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off);
    s2 = __shfl(s2, 0);  // one value for every lane
    if (s2 == 0.0) continue;  // uniform: the column is already reduced
    const cd x0 = H[(j + 1) * ld + j];
    const double a2 = x0.re * x0.re + x0.im * x0.im;
    const double nrm = sqrt(a2 + s2);
    const double ia = (a2 > 0.0) ? crsq(a2) : 0.0;
    const cd alpha = mk((a2 > 0.0) ? -nrm * (ia * x0.re) : -nrm, -nrm * (ia * x0.im));
    const cd v0 = x0 - alpha;
    const double tau = 2.0 / (v0.re * v0.re + v0.im * v0.im + s2);
    if (lane == 0)
      hv[0] = v0;
    else if (lane < len)
      hv[lane] = xl;
    __syncthreads();
    // P H on columns j+1 ..; column j becomes alpha e_1
    for (int c = j + 1 + lane; c < n; c += kW) {
      cd w = mk(0.0, 0.0);
      for (int r = 0; r < len; ++r) w = w + cj(hv[r]) * H[(j + 1 + r) * ld + c];
      const cd tw = tau * w;
      for (int r = 0; r < len; ++r) H[(j + 1 + r) * ld + c] = H[(j + 1 + r) * ld + c] - hv[r] * tw;
    }
    if (lane == 0)
      H[(j + 1) * ld + j] = alpha;
    else if (lane < len)
      H[(j + 1 + lane) * ld + j] = mk(0.0, 0.0);
    __syncthreads();
    // H P and Q P on rows, columns j+1 ..
    for (int r = lane; r < n; r += kW) {
      cd zh = mk(0.0, 0.0), zq = mk(0.0, 0.0);
      for (int c = 0; c < len; ++c) {
        zh = zh + H[r * ld + j + 1 + c] * hv[c];
        zq = zq + Q[r * ld + j + 1 + c] * hv[c];
      }
      const cd th = tau * zh, tq = tau * zq;
      for (int c = 0; c < len; ++c) {
        const cd vc = cj(hv[c]);
        H[r * ld + j + 1 + c] = H[r * ld + j + 1 + c] - th * vc;
        Q[r * ld + j + 1 + c] = Q[r * ld + j + 1 + c] - tq * vc;
      }
    }
    __syncthreads();
  }
  if (stamp && threadIdx.x == 0) *stamp = clock64();
  const double eps = 2.220446049250313e-16;
  int hi = n - 1, its = 0, total = 0;
  // a step's rotations, kept for its right-hand sweep (LDS, not per-lane
  // arrays: those would be indexed dynamically and live in scratch)
  __shared__ double cs[kMaxN];
  __shared__ cd sn[kMaxN];
  while (hi > 0) {
    int lo = hi;
    while (lo > 0) {  // deflation test with |re| + |im| moduli
      const double sub = ab1(H[lo * ld + lo - 1]);
      const double dia = ab1(H[lo * ld + lo]) + ab1(H[(lo - 1) * ld + lo - 1]);
      if (sub <= eps * dia || sub == 0.0) break;
      --lo;
    }
    __syncthreads();
    if (lo > 0 && threadIdx.x == 0) H[lo * ld + lo - 1] = mk(0.0, 0.0);
    if (lo == hi) {
      __syncthreads();
      --hi;
      its = 0;
      continue;
    }
    if (++total > 60 * n) return false;
    const cd a = H[(hi - 1) * ld + hi - 1], b = H[(hi - 1) * ld + hi];
    const cd c2 = H[hi * ld + hi - 1], d = H[hi * ld + hi];
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
    __syncthreads();
    // one explicit-shift QR step on the window [lo, hi]: H - mu I = QR by
    // rotations from the left, then RQ + mu I
    for (int k = lo + (int)threadIdx.x; k <= hi; k += kW) H[k * ld + k] = H[k * ld + k] - mu;
    __syncthreads();
    // Left sweep: lane j owns column j.  The row being rotated down (row k
    // after rotation k - 1) stays in a register of each lane; rotation k
    // comes from its diagonal entry (lane k's register, by shuffle) and
    // the untouched subdiagonal entry below it, and the rotated upper row
    // is stored as row k of R.  No lane reads what another lane wrote, so
    // the sweep needs no barrier; the values are those of applying the
    // rotations one row pair at a time.
    {
      cd cr = mk(0.0, 0.0);
      if (lane >= lo && lane < n) cr = H[lo * ld + lane];
      for (int k = lo; k < hi; ++k) {
        const cd a = mk(__shfl(cr.re, k), __shfl(cr.im, k));
        double c;
        cd sk;
        givens(a, H[(k + 1) * ld + k], c, sk);
        if (lane == 0) {
          cs[k] = c;
          sn[k] = sk;
        }
        if (lane >= k && lane < n) {
          const cd x = cr, y = H[(k + 1) * ld + lane];
          H[k * ld + lane] = c * x + sk * y;
          cr = c * y - cj(sk) * x;
        }
      }
      if (lane >= hi && lane < n) H[hi * ld + lane] = cr;
      if (lane >= lo && lane < hi) H[(lane + 1) * ld + lane] = mk(0.0, 0.0);
    }
    __syncthreads();
    // Right sweep (R Q^H and the Schur vectors): lane r owns row r of H
    // (r <= hi) or of Q, and applies every rotation along it in order, the
    // column between two rotations kept in a register.
    for (int r = lane; r < hi + 1 + n; r += kW) {
      cd* row = (r <= hi) ? H + r * ld : Q + (r - hi - 1) * ld;
      cd x = row[lo];
      for (int k = lo; k < hi; ++k) {
        const double c = cs[k];
        const cd sk = sn[k];
        const cd y = row[k + 1];
        row[k] = c * x + cj(sk) * y;
        x = c * y - sk * x;
      }
      row[hi] = x;
    }
    __syncthreads();
    for (int k = lo + (int)threadIdx.x; k <= hi; k += kW) H[k * ld + k] = H[k * ld + k] + mu;
    __syncthreads();
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

constexpr double kOrthoRedoC = 1e-4;  // as the real path's Cholesky-QR

// complex Gram entry (a, b) of the interleaved real Gram G (row stride ld)
__device__ __forceinline__ cd cgram(const double* G, int ld, int a, int b) {
  const double* r0 = G + (size_t)(2 * a) * ld;
  const double* r1 = G + (size_t)(2 * a + 1) * ld;
  return mk(r0[2 * b] + r1[2 * b + 1], r0[2 * b + 1] - r1[2 * b]);
}

}  // namespace

// ----------------------------------------------------- complex Cholesky-QR
// LDS: G (N x N, R in its upper triangle) | X (N x N, R^-1)
__global__ __launch_bounds__(kW) void k_cplx_ortho(SmallParams p, SmallBufs b, DevStatus* st) {
  if (halted(st)) {
    if (p.pass == 1 && b.gate && threadIdx.x == 0) b.gate->done = 1;
    return;
  }
  if (p.pass == 2 && b.gate && b.gate->done) return;
  extern __shared__ __attribute__((aligned(16))) double smem[];
  __shared__ int valid[kMaxN];
  __shared__ double d[kMaxN];
  const int m = p.m, N = m / 2, kc = p.kint / 2, t = threadIdx.x;
  const int ld = N;
  cd* G = reinterpret_cast<cd*>(smem);
  cd* X = G + N * ld;
  const int have_p = st->have_p;
  for (int a = t; a < N; a += kW) {
    const int slot = a / kc, col = a - slot * kc;
    // a locked column (active 0) generates no W, S or P
    int v = (slot == 0) ? 1 : (b.active[2 * col] && (slot != 3 || have_p));
    const double g = cgram(b.G, m, a, a).re;
    if (v && !(g > 0.0 && g < INFINITY)) v = 0;
    valid[a] = v;
    d[a] = v ? 1.0 / sqrt(g) : 0.0;
  }
  __syncthreads();
  for (int e = t; e < N * N; e += kW) {
    const int a = e / N, c = e - a * N;
    G[a * ld + c] = (valid[a] && valid[c]) ? (d[a] * d[c]) * cgram(b.G, m, a, c) : mk(0.0, 0.0);
    X[a * ld + c] = mk(a == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // right-looking Cholesky G = R^H R in slot order on the upper triangle;
  // a numerically dependent column is dropped (the decision is uniform)
  double minpiv = INFINITY;
  for (int j = 0; j < N; ++j) {
    if (!valid[j]) continue;
    const double piv = G[j * ld + j].re;
    if (!(piv > p.drop_tol)) {
      __syncthreads();
      if (t == 0) valid[j] = 0;
      __syncthreads();
      continue;
    }
    minpiv = fmin(minpiv, piv);
    const double r = sqrt(piv), ir = 1.0 / r;
    __syncthreads();
    for (int l = j + t; l < N; l += kW) G[j * ld + l] = (l == j) ? mk(r, 0.0) : ir * G[j * ld + l];
    __syncthreads();
    const int rem = N - j - 1;
    for (int e = t; e < rem * rem; e += kW) {
      const int i = j + 1 + e / rem, l = j + 1 + e % rem;
      if (l >= i) G[i * ld + l] = G[i * ld + l] - cj(G[j * ld + i]) * G[j * ld + l];
    }
    __syncthreads();
  }
  // rows and columns of dropped or absent columns of R are zero
  for (int e = t; e < N * N; e += kW) {
    const int a = e / N, c = e - a * N;
    if (!(valid[a] && valid[c] && c >= a)) G[a * ld + c] = mk(0.0, 0.0);
  }
  __syncthreads();
  // X = R^-1 (upper) by right-looking back substitution on the kept columns
  for (int i = N - 1; i >= 0; --i) {
    if (!valid[i]) continue;
    const double ir = 1.0 / G[i * ld + i].re;
    for (int c = i + t; c < N; c += kW) X[i * ld + c] = ir * X[i * ld + c];
    __syncthreads();
    for (int e = t; e < i * (N - i); e += kW) {
      const int r = e / (N - i), c = i + e % (N - i);
      X[r * ld + c] = X[r * ld + c] - G[r * ld + i] * X[i * ld + c];
    }
    __syncthreads();
  }
  // M = D R^-1 as the real matrix of the interleaved columns
  for (int e = t; e < N * N; e += kW) {
    const int a = e / N, c = e - a * N;
    const bool on = valid[a] && valid[c] && c >= a;
    const cd v = on ? d[a] * X[a * ld + c] : mk(0.0, 0.0);
    b.M[(size_t)(2 * a) * m + 2 * c] = v.re;
    b.M[(size_t)(2 * a) * m + 2 * c + 1] = v.im;
    b.M[(size_t)(2 * a + 1) * m + 2 * c] = -v.im;
    b.M[(size_t)(2 * a + 1) * m + 2 * c + 1] = v.re;
  }
  for (int a = t; a < N; a += kW) b.keep[2 * a] = b.keep[2 * a + 1] = valid[a];
  if (t == 0) {
    int nk = 0, nd = 0, anyv = 0;
    for (int a = 0; a < N; ++a) {
      const int slot = a / kc, col = a - slot * kc;
      nk += valid[a];
      if (slot == 0) anyv |= valid[a];
      const int wanted = (slot == 0) ? 1 : (b.active[2 * col] && (slot != 3 || have_p));
      if (!valid[a] && wanted) ++nd;
    }
    st->m_kept = 2 * nk;
    st->n_dropped = 2 * nd;
    if (!anyv) {
      st->error = PLHR_ERR_BREAKDOWN;
      st->reason = kReasonVVanished;
    }
    if (p.pass == 1 && b.gate) {
      b.gate->error = 0;
      b.gate->done = (minpiv < kOrthoRedoC) ? 0 : 1;
    }
  }
}

// -------------------------------------------- complex projected problem
// LDS: GL (-> L) | GR (-> C -> T) | Q | Z (n x kc eigenvectors of T, then
// y) | ord, idx
__global__ __launch_bounds__(kW) void k_cplx_tharm(SmallParams p, SmallBufs b, DevStatus* st) {
  if (halted(st)) return;
  if (threadIdx.x == 0) st->tphase[0] = clock64();
  extern __shared__ __attribute__((aligned(16))) double smem[];
  __shared__ int idx[kMaxN], dead[kMaxN], ord[kMaxN];
  __shared__ int n_s, ndead_s, ok_s;
  const int m = p.m, N = m / 2, kc = p.kint / 2, ld2 = 2 * m, t = threadIdx.x;
  if (t == 0) {
    int c = 0;
    for (int a = 0; a < N; ++a)
      if (b.keep[2 * a]) idx[c++] = a;
    n_s = c;
    ndead_s = 0;
  }
  __syncthreads();
  const int n = n_s, ld = N;
  if (n < kc) {
    if (t == 0) {
      st->error = PLHR_ERR_BREAKDOWN;
      st->reason = kReasonVVanished;
    }
    return;
  }
  cd* L = reinterpret_cast<cd*>(smem);
  cd* C = L + N * ld;
  cd* Q = C + N * ld;
  cd* Zv = Q + N * ld;  // n x kc
  for (int e = t; e < n * n; e += kW) {
    const int i = e / n, j = e - i * n;
    const int a = idx[i], c = idx[j];
    // Hermitian part of G_L (its lower triangle is what the Cholesky reads)
    const cd gij = cgram(b.GLR, ld2, a, c), gji = cgram(b.GLR, ld2, c, a);
    L[i * ld + j] = 0.5 * (gij + cj(gji));
    const double* r0 = b.GLR + (size_t)(2 * a) * ld2 + m;
    const double* r1 = b.GLR + (size_t)(2 * a + 1) * ld2 + m;
    C[i * ld + j] = mk(r0[2 * c] + r1[2 * c + 1], r0[2 * c + 1] - r1[2 * c]);
  }
  for (int j = t; j < n; j += kW) dead[j] = 0;
  __syncthreads();
  double maxd = 0.0;
  for (int j = 0; j < n; ++j) maxd = fmax(maxd, L[j * ld + j].re);
  const double floor_ = fmax(1e-15 * maxd, 1e-300);
  // G_L = L L^H, right-looking on the lower triangle; pivots as in the real
  // path (raised to 1e-15 max diag; a clearly negative one leaves its
  // column out: tau = 0, never selected)
  for (int j = 0; j < n; ++j) {
    const double p0 = L[j * ld + j].re;
    __syncthreads();
    if (p0 < -1e-10 * maxd) {
      if (t == 0) {
        dead[j] = 1;
        ++ndead_s;
      }
      for (int i = j + 1 + t; i < n; i += kW) L[i * ld + j] = mk(0.0, 0.0);
      __syncthreads();
      continue;
    }
    const double r = sqrt(fmax(p0, floor_)), ir = 1.0 / r;
    for (int i = j + t; i < n; i += kW) L[i * ld + j] = (i == j) ? mk(r, 0.0) : ir * L[i * ld + j];
    __syncthreads();
    const int rem = n - j - 1;
    for (int e = t; e < rem * rem; e += kW) {
      const int i = j + 1 + e / rem, l = j + 1 + e % rem;
      if (l <= i) L[i * ld + l] = L[i * ld + l] - L[i * ld + j] * cj(L[l * ld + j]);
    }
    __syncthreads();
  }
  // L: zero above the diagonal, rows and columns of dead columns e_j; G_R
  // rows and columns of dead columns zero
  for (int e = t; e < n * n; e += kW) {
    const int i = e / n, c = e - i * n;
    if (dead[i] || dead[c]) {
      L[i * ld + c] = mk(i == c ? 1.0 : 0.0, 0.0);
      C[i * ld + c] = mk(0.0, 0.0);
    } else if (c > i) {
      L[i * ld + c] = mk(0.0, 0.0);
    }
  }
  __syncthreads();
  if (t == 0 && ndead_s) st->n_excluded += ndead_s;
  if (ndead_s && n - ndead_s < kc) {
    if (t == 0) {
      st->error = PLHR_ERR_BREAKDOWN;
      st->reason = kReasonVVanished;
    }
    return;
  }
  if (t == 0) st->tphase[1] = clock64();
  // C <- L^-1 C (rows, unscaled right-looking), then C <- C L^-H (columns).
  // Each lane owns one column (then one row) of C and runs every step on
  // it in order: the updates of an entry are those of the step-by-step
  // elimination, with no barrier between steps.
  for (int c = t; c < n; c += kW)
    for (int r = 0; r + 1 < n; ++r) {
      const double ir = 1.0 / L[r * ld + r].re;
      const cd xr = C[r * ld + c];
      for (int i = r + 1; i < n; ++i)
        C[i * ld + c] = C[i * ld + c] - (ir * L[i * ld + r]) * xr;
    }
  __syncthreads();
  for (int e = t; e < n * n; e += kW) {
    const int i = e / n, c = e - i * n;
    C[i * ld + c] = (1.0 / L[i * ld + i].re) * C[i * ld + c];
  }
  __syncthreads();
  for (int i = t; i < n; i += kW)
    for (int r = 0; r + 1 < n; ++r) {
      const double ir = 1.0 / L[r * ld + r].re;
      const cd xr = C[i * ld + r];
      for (int c = r + 1; c < n; ++c)
        C[i * ld + c] = C[i * ld + c] - (ir * cj(L[c * ld + r])) * xr;
    }
  __syncthreads();
  for (int e = t; e < n * n; e += kW) {
    const int i = e / n, c = e - i * n;
    C[i * ld + c] = (1.0 / L[c * ld + c].re) * C[i * ld + c];
  }
  __syncthreads();
  if (t == 0) st->tphase[2] = clock64();
  const bool ok = schur_w(C, Q, ld, n, &st->tphase[3]);
  if (t == 0) st->tphase[4] = clock64();
  __syncthreads();
  if (!ok) {
    if (t == 0) {
      st->error = PLHR_ERR_BREAKDOWN;
      st->reason = kReasonQR;
    }
    return;
  }
  // eigenvalues in xi order (diagnostics) and the selection: each lane
  // ranks one eigenvalue by counting those before it (ties by index), the
  // order of a stable sort by xi_before
  for (int i = t; i < n; i += kW) {
    const cd ti = C[i * ld + i];
    int r = 0;
    for (int o = 0; o < n; ++o) {
      if (o == i) continue;
      const cd to = C[o * ld + o];
      r += (xi_before(to, ti) || (o < i && !xi_before(ti, to))) ? 1 : 0;
    }
    ord[r] = i;
  }
  __syncthreads();
  if (t == 0) {
    ok_s = 1;
    for (int j = 0; j < kc; ++j)
      if (!(ab(C[ord[j] * ld + ord[j]]) > 0.0)) ok_s = 0;
  }
  __syncthreads();
  for (int r = t; r < m; r += kW) {
    b.xi[r] = 0.0;
    b.xi[m + r] = 0.0;
  }
  for (int r = t; r < n; r += kW) {
    const cd tv = C[ord[r] * ld + ord[r]];
    const double a2 = tv.re * tv.re + tv.im * tv.im;
    b.xi[r] = (a2 > 0.0) ? tv.re / a2 : INFINITY;
    b.xi[m + r] = (a2 > 0.0) ? -tv.im / a2 : 0.0;
  }
  if (!ok_s) {
    if (t == 0) {
      st->error = PLHR_ERR_BREAKDOWN;
      st->reason = kReasonQR;
    }
    return;
  }
  // eigenvector z of T for each selected tau (z_ks = 1, back substitution),
  // one lane per eigenvector
  double cn = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) cn = fmax(cn, ab(C[i * ld + j]));
  const double small = 2.220446049250313e-16 * fmax(cn, 1e-300);
  for (int j = t; j < kc; j += kW) {
    const int ks = ord[j];
    const cd tau = C[ks * ld + ks];
    for (int i = 0; i < n; ++i) Zv[i * kc + j] = mk(i == ks ? 1.0 : 0.0, 0.0);
    for (int i = ks - 1; i >= 0; --i) {
      cd s = mk(0.0, 0.0);
      for (int q = i + 1; q <= ks; ++q) s = s + C[i * ld + q] * Zv[q * kc + j];
      cd den = C[i * ld + i] - tau;
      if (ab(den) < small) den = mk(small, 0.0);
      Zv[i * kc + j] = dv(mk(-s.re, -s.im), den);
    }
  }
  __syncthreads();
  // u = Q z, n x kc, stored in the region of T (no longer read)
  for (int e = t; e < n * kc; e += kW) {
    const int i = e / kc, j = e - i * kc;
    cd s = mk(0.0, 0.0);
    for (int q = 0; q < n; ++q) s = s + Q[i * ld + q] * Zv[q * kc + j];
    C[i * kc + j] = s;
  }
  __syncthreads();
  if (t == 0) st->tphase[5] = clock64();
  // y = L^-H u (one lane per vector), unit 2-norm, largest entry real and
  // positive, scattered into Y' as real 2 x 2 blocks
  for (int e = t; e < m * p.kint; e += kW) b.Y[e] = 0.0;
  __syncthreads();
  for (int j = t; j < kc; j += kW) {
    for (int i = n - 1; i >= 0; --i) {
      cd s = C[i * kc + j];
      for (int q = i + 1; q < n; ++q) s = s - cj(L[q * ld + i]) * Zv[q * kc + j];
      Zv[i * kc + j] = (1.0 / L[i * ld + i].re) * s;
    }
    double nr2 = 0.0, big = -1.0;
    int im = 0;
    for (int i = 0; i < n; ++i) {
      const cd y = Zv[i * kc + j];
      const double a2 = y.re * y.re + y.im * y.im;
      nr2 += a2;
      if (a2 > big) big = a2, im = i;
    }
    const cd ym = Zv[im * kc + j];
    const double ay = ab(ym);
    const cd ph = (ay > 0.0) ? mk(ym.re / ay, -ym.im / ay) : mk(1.0, 0.0);
    const double sc = (nr2 > 0.0) ? 1.0 / sqrt(nr2) : 0.0;
    const int kint = p.kint;
    for (int i = 0; i < n; ++i) {
      const cd v = sc * (Zv[i * kc + j] * ph);
      const int a = idx[i];
      b.Y[(size_t)(2 * a) * kint + 2 * j] = v.re;
      b.Y[(size_t)(2 * a) * kint + 2 * j + 1] = v.im;
      b.Y[(size_t)(2 * a + 1) * kint + 2 * j] = -v.im;
      b.Y[(size_t)(2 * a + 1) * kint + 2 * j + 1] = v.re;
    }
    b.kinds[2 * j] = 1;
    b.kinds[2 * j + 1] = 3;
    b.pair[2 * j] = 2 * j + 1;
    b.pair[2 * j + 1] = 2 * j;
  }
  __syncthreads();
  if (t == 0) st->tphase[6] = clock64();
}

// ------------------------------------------------ final Rayleigh-Ritz
// V^H (A - sigma) V x = theta V^H V x on the kc = kint/2 complex columns of
// V: V^H V scaled to unit diagonal and factored with the trial-space
// dropping rule (a dependent column is left out), C = L^-1 H L^-H, its
// eigenpairs from the Schur form (C is Hermitian: T is diagonal to rounding
// and the columns of Q are the eigenvectors), the k values nearest sigma
// (ties: smaller), x = D L^-H q.  LDS: H (-> C -> T) | L | Q.
__global__ __launch_bounds__(kW) void k_cplx_final(SmallParams p, const double* __restrict__ HM,
                                                   SmallBufs b, DevStatus* st) {
  extern __shared__ __attribute__((aligned(16))) double smem[];
  __shared__ int keep[kMaxN], ord[kMaxN];
  __shared__ double dsc[kMaxN];
  __shared__ int nk_s;
  const int kint = p.kint, kc = kint / 2, k = p.k / 2, t = threadIdx.x, ld = kc;
  const int ldh = 2 * kint;  // HM row stride
  cd* H = reinterpret_cast<cd*>(smem);
  cd* L = H + kc * ld;
  cd* Q = L + kc * ld;
  // when at least k columns met the tolerance, the others (guard columns
  // still converging) are left out too, as in the real final step
  if (t == 0) {
    int cnv = 0;
    for (int a = 0; a < kc; ++a) cnv += (b.relres[2 * a] <= p.tol) ? 1 : 0;
    nk_s = cnv;
  }
  __syncthreads();
  for (int a = t; a < kc; a += kW) {
    const double g = cgram(HM + kint, ldh, a, a).re;
    const bool excl = nk_s >= k && !(b.relres[2 * a] <= p.tol);
    keep[a] = (g > 0.0 && g < INFINITY && !excl) ? 1 : 0;
    dsc[a] = (g > 0.0 && g < INFINITY) ? 1.0 / sqrt(g) : 0.0;
  }
  __syncthreads();
  for (int e = t; e < kc * kc; e += kW) {
    const int i = e / kc, j = e - i * kc;
    const double s2 = dsc[i] * dsc[j];
    H[i * ld + j] = s2 * cgram(HM, ldh, i, j);
    L[i * ld + j] = s2 * cgram(HM + kint, ldh, i, j);
  }
  __syncthreads();
  // scaled V^H V = L L^H with dropping, right-looking on the lower triangle
  for (int j = 0; j < kc; ++j) {
    const double piv = L[j * ld + j].re;
    const bool drop = !(keep[j] && piv > p.drop_tol);
    __syncthreads();
    if (drop) {
      if (t == 0) keep[j] = 0;
      for (int i = j + t; i < kc; i += kW) L[i * ld + j] = mk(i == j ? 1.0 : 0.0, 0.0);
      __syncthreads();
      continue;
    }
    const double r = sqrt(piv), ir = 1.0 / r;
    for (int i = j + t; i < kc; i += kW) L[i * ld + j] = (i == j) ? mk(r, 0.0) : ir * L[i * ld + j];
    __syncthreads();
    const int rem = kc - j - 1;
    for (int e = t; e < rem * rem; e += kW) {
      const int i = j + 1 + e / rem, l = j + 1 + e % rem;
      if (l <= i) L[i * ld + l] = L[i * ld + l] - L[i * ld + j] * cj(L[l * ld + j]);
    }
    __syncthreads();
  }
  for (int e = t; e < kc * kc; e += kW) {
    const int i = e / kc, c = e - i * kc;
    if (c > i || (!keep[i] && i != c) || (!keep[c] && i != c)) L[i * ld + c] = mk(0.0, 0.0);
    if (!keep[i] || !keep[c]) H[i * ld + c] = mk(0.0, 0.0);
  }
  if (t == 0) {
    int nk = 0;
    for (int a = 0; a < kc; ++a) nk += keep[a];
    nk_s = nk;
  }
  __syncthreads();
  if (nk_s < k) {
    if (t == 0) {
      st->error = PLHR_ERR_BREAKDOWN;
      st->reason = kReasonFinalGram;
    }
    return;
  }
  // C = L^-1 H L^-H as in the projected problem
  for (int r = 0; r + 1 < kc; ++r) {
    const double ir = 1.0 / L[r * ld + r].re;
    for (int e = t; e < (kc - r - 1) * kc; e += kW) {
      const int i = r + 1 + e / kc, c = e % kc;
      H[i * ld + c] = H[i * ld + c] - (ir * L[i * ld + r]) * H[r * ld + c];
    }
    __syncthreads();
  }
  for (int e = t; e < kc * kc; e += kW) {
    const int i = e / kc, c = e - i * kc;
    H[i * ld + c] = (1.0 / L[i * ld + i].re) * H[i * ld + c];
  }
  __syncthreads();
  for (int r = 0; r + 1 < kc; ++r) {
    const double ir = 1.0 / L[r * ld + r].re;
    for (int e = t; e < (kc - r - 1) * kc; e += kW) {
      const int c = r + 1 + e / kc, i = e % kc;
      H[i * ld + c] = H[i * ld + c] - (ir * cj(L[c * ld + r])) * H[i * ld + r];
    }
    __syncthreads();
  }
  for (int e = t; e < kc * kc; e += kW) {
    const int i = e / kc, c = e - i * kc;
    H[i * ld + c] = (1.0 / L[c * ld + c].re) * H[i * ld + c];
  }
  __syncthreads();
  // Hermitian part (rounding), then the Schur form
  for (int e = t; e < kc * kc; e += kW) {
    const int i = e / kc, c = e - i * kc;
    if (c < i) {
      const cd h = 0.5 * (H[i * ld + c] + cj(H[c * ld + i]));
      H[i * ld + c] = h;
      H[c * ld + i] = cj(h);
    } else if (c == i) {
      H[i * ld + i] = mk(H[i * ld + i].re, 0.0);
    }
  }
  __syncthreads();
  const bool ok = schur_w(H, Q, ld, kc);
  __syncthreads();
  if (!ok) {
    if (t == 0) {
      st->error = PLHR_ERR_BREAKDOWN;
      st->reason = kReasonQR;
    }
    return;
  }
  // order by |theta| (theta = lambda - sigma), ties smaller theta; the
  // eigenvalues of dropped columns (their rows and columns are zero) last
  if (t == 0) {
    int c = 0;
    for (int i = 0; i < kc; ++i) ord[c++] = i;
    for (int i = 1; i < kc; ++i)
      for (int j = i; j > 0; --j) {
        const int a = ord[j], bb = ord[j - 1];
        const double ta = H[a * ld + a].re, tb = H[bb * ld + bb].re;
        // a column of Q that lies in the span of dropped columns has a zero
        // eigenvalue that is not a Ritz value: push it last
        double wa = 0.0, wb = 0.0;
        for (int r = 0; r < kc; ++r) {
          if (keep[r]) continue;
          wa += ab(Q[r * ld + a]);
          wb += ab(Q[r * ld + bb]);
        }
        const bool da = wa > 0.5, db = wb > 0.5;
        const bool before = (da != db) ? db : (fabs(ta) < fabs(tb) || (fabs(ta) == fabs(tb) && ta < tb));
        if (!before) break;
        ord[j] = bb;
        ord[j - 1] = a;
      }
  }
  __syncthreads();
  // x = D L^-H q for the k selected, one lane each; final_C expands it
  for (int e = t; e < kint * 2 * k; e += kW) b.final_C[e] = 0.0;
  __syncthreads();
  for (int j = t; j < k; j += kW) {
    const int col = ord[j];
    cd x[kMaxN];
    for (int i = kc - 1; i >= 0; --i) {
      cd s = Q[i * ld + col];
      for (int q = i + 1; q < kc; ++q) s = s - cj(L[q * ld + i]) * x[q];
      x[i] = (1.0 / L[i * ld + i].re) * s;
    }
    for (int i = 0; i < kc; ++i) {
      const cd v = keep[i] ? dsc[i] * x[i] : mk(0.0, 0.0);
      b.final_C[(size_t)(2 * i) * (2 * k) + 2 * j] = v.re;
      b.final_C[(size_t)(2 * i) * (2 * k) + 2 * j + 1] = v.im;
      b.final_C[(size_t)(2 * i + 1) * (2 * k) + 2 * j] = -v.im;
      b.final_C[(size_t)(2 * i + 1) * (2 * k) + 2 * j + 1] = v.re;
    }
    const double th = p.sigma + H[col * ld + col].re;
    b.final_theta[2 * j] = th;
    b.final_theta[2 * j + 1] = th;
  }
}

static size_t cplx_ortho_lds(int m) {
  const size_t N = (size_t)m / 2;
  return 2 * N * N * sizeof(cd);
}
static size_t cplx_tharm_lds(int m, int kint) {
  const size_t N = (size_t)m / 2, kc = (size_t)kint / 2;
  return (3 * N * N + N * kc) * sizeof(cd);
}

hipError_t cplx_set_attributes() {
  hipError_t e = set_lds_limit((const void*)k_cplx_ortho);
  if (e == hipSuccess) e = set_lds_limit((const void*)k_cplx_tharm);
  if (e == hipSuccess) e = set_lds_limit((const void*)k_cplx_final);
  return e;
}

void launch_cplx_final(const SmallParams& p, const double* HM, SmallBufs b, DevStatus* st,
                       hipStream_t s) {
  const size_t kc = (size_t)p.kint / 2;
  hipLaunchKernelGGL(k_cplx_final, dim3(1), dim3(kW), 3 * kc * kc * sizeof(cd), s, p, HM, b, st);
}

void launch_cplx_ortho(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s) {
  const double N = p.m / 2.0;
  prof_begin(KC_ORTHO, (double)p.m * p.m * 8.0, 8.0 * N * N * N / 3.0, s);
  hipLaunchKernelGGL(k_cplx_ortho, dim3(1), dim3(kW), cplx_ortho_lds(p.m), s, p, b, st);
  prof_end(KC_ORTHO, s);
}

void launch_cplx_tharm(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s) {
  const double N = p.m / 2.0;
  prof_begin(KC_THARM_QR, 2.0 * p.m * p.m * 8.0, 4.0 * 25.0 * N * N * N, s);
  hipLaunchKernelGGL(k_cplx_tharm, dim3(1), dim3(kW), cplx_tharm_lds(p.m, p.kint), s, p, b, st);
  prof_end(KC_THARM_QR, s);
}

}  // namespace plhr
