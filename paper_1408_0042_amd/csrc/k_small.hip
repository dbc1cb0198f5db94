// Small dense kernels of the PLHR iteration, each one workgroup with all
// operands in LDS (m = 4 (k + k_extra) slots, m <= 100).
//
//   k_init_lam     Rayleigh quotients of the start block (Algorithm 3, step 2)
//   k_conv_check   relative residuals, soft locking, stopping test
//   k_ortho_small  Cholesky of the Gram matrix of Z = [V W S P] with column
//                  scaling and dropping of dependent W/S/P columns; returns
//                  M with Zhat = Z M B-orthonormal (Section 4: V, W, S, P
//                  are orthonormalised in this order, which is what a
//                  Cholesky factorisation of the Gram matrix in slot order
//                  computes)
//   k_tharm_small  the projected problem eq. (3.5), G_L y = xi G_R y, via
//                  G_L = L L^T, C = L^-1 G_R L^-T, Hessenberg reduction,
//                  Francis double-shift QR (real Schur form), eigenvectors
//                  by back substitution; selection of the kint smallest
//                  |xi| with conjugate pairs kept adjacent and the real
//                  basis Y' = [Y0 YR ytilde_R YI] of Algorithm 3
//   k_rq_small     Rayleigh quotients of the new block, eq. (4.1) for pairs
//   k_final_rr     standard Rayleigh-Ritz on span(V) (the last step of
//                  Algorithms 2 and 3): Cholesky + cyclic Jacobi
//   k_final_res    relative residuals of the returned pairs
#include <cmath>

#include "common.cuh"

namespace plhr {

__device__ __forceinline__ int slot_valid(int s, int kint, const int* active, int have_p) {
  if (s < kint) return 1;
  const int j = s % kint;
  const int blk = s / kint;  // 1 = W, 2 = S, 3 = P
  if (!active[j]) return 0;
  if (blk == 3 && !have_p) return 0;
  return 1;
}

// Sum of per-workgroup partials: out[v] = sum_q part[q * nv + v] for
// v < nv (nv <= 128), using every thread of the block in a fixed order.
// Must be called by all threads; `red` is LDS scratch of blockDim doubles.
__device__ void sum_partials(const double* __restrict__ part, int nblk, int nv, double* out,
                             double* red) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = nt / nv;           // threads per value
  const int v = t % nv, s = t / nv;
  double acc = 0.0;
  if (s < per)
    for (int q = s; q < nblk; q += per) acc += part[(size_t)q * nv + v];
  red[t] = acc;
  __syncthreads();
  if (t < nv) {
    double a = 0.0;
    for (int q = 0; q < per; ++q) a += red[q * nv + t];
    out[t] = a;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- init
__global__ void k_init_lam(SmallParams p, const double* __restrict__ part, int nblk,
                           SmallBufs b, DevStatus* st) {
  __shared__ double red[256], sums[128];
  sum_partials(part, nblk, 2 * p.kint, sums, red);
  const int c = threadIdx.x;
  if (c < p.kint) {
    const double vv = sums[c], vq = sums[p.kint + c];
    b.lam[c] = p.sigma + vq / vv;
    b.kinds[c] = 0;
    b.pair[c] = -1;
    b.active[c] = 1;
  }
  if (c == 0) {
    st->done = 0;
    st->error = 0;
    st->iter = 0;
    st->have_p = 0;
    st->n_active = p.kint;
    st->m_kept = 0;
    st->n_dropped = 0;
    st->max_rel_res = 0.0;
  }
}

// Rank test of the start block: scaled Cholesky of G = V0^T B V0 (kint x
// kint, in b.G); a pivot below drop_tol means linearly dependent columns.
__global__ void k_start_check(SmallParams p, SmallBufs b, DevStatus* st) {
  if (threadIdx.x != 0) return;
  const int n = p.kint;  // <= 25 (4 kint <= 100)
  __shared__ double G[25 * 25];
  __shared__ double d[25];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) G[i * n + j] = b.G[i * n + j];
  for (int i = 0; i < n; ++i) {
    if (!(G[i * n + i] > 0.0 && G[i * n + i] < INFINITY)) {
      st->error = PLHR_ERR_BREAKDOWN;
      st->reason = kReasonStartRank;
      return;
    }
    d[i] = 1.0 / sqrt(G[i * n + i]);
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) G[i * n + j] *= d[i] * d[j];
  for (int j = 0; j < n; ++j) {
    double piv = G[j * n + j];
    for (int q = 0; q < j; ++q) piv -= G[j * n + q] * G[j * n + q];
    if (!(piv > p.drop_tol)) {
      st->error = PLHR_ERR_BREAKDOWN;
      st->reason = kReasonStartRank;
      return;
    }
    const double r = sqrt(piv);
    G[j * n + j] = r;
    for (int i = j + 1; i < n; ++i) {
      double s = G[i * n + j];
      for (int q = 0; q < j; ++q) s -= G[i * n + q] * G[j * n + q];
      G[i * n + j] = s / r;
    }
  }
}

// ------------------------------------------------------- convergence test
__global__ void k_conv_check(SmallParams p, const double* __restrict__ part, int nblk,
                             SmallBufs b, DevStatus* st) {
  if (halted(st)) return;
  __shared__ double rel[128];
  __shared__ double red[256], sums[128];
  const int c = threadIdx.x;
  const int kint = p.kint;
  sum_partials(part, nblk, 2 * kint, sums, red);
  if (c < kint) {
    const double rr = sums[c], vv = sums[kint + c];
    const double lam = b.lam[c];
    const double den = (p.normA1 + fabs(lam) * p.normB1) * sqrt(vv);
    const double r = (den > 0.0) ? sqrt(rr) / den : INFINITY;
    rel[c] = (r == r) ? r : INFINITY;  // NaN counts as not converged
    b.relres[c] = rel[c];
  }
  __syncthreads();
  if (c < kint) {
    // wanted: the k columns nearest sigma (ties: smaller lambda, then index)
    const double lc = b.lam[c];
    const double dc = fabs(lc - p.sigma);
    int rank = 0;
    for (int q = 0; q < kint; ++q) {
      const double lq = b.lam[q];
      const double dq = fabs(lq - p.sigma);
      if (dq < dc || (dq == dc && (lq < lc || (lq == lc && q < c)))) ++rank;
    }
    rel[64 + c] = (rank < p.k) ? 1.0 : 0.0;  // wanted flag
    b.active[c] = p.lock ? (rel[c] > p.tol ? 1 : 0) : 1;
  }
  __syncthreads();
  if (c == 0) {
    int done = 1, nact = 0;
    double mx = 0.0;
    for (int q = 0; q < kint; ++q) {
      if (rel[64 + q] > 0.5) {
        if (!(rel[q] <= p.tol)) done = 0;
        mx = fmax(mx, rel[q]);
      }
      nact += b.active[q];
    }
    st->max_rel_res = mx;
    st->n_active = nact;
    if (done) st->done = 1;
    for (int q = 0; q < kint; ++q)
      if (!(rel[q] < INFINITY) && rel[64 + q] > 0.5) {
        st->error = PLHR_ERR_BREAKDOWN;
        st->reason = kReasonNonFinite;
      }
  }
}

// --------------------------------------------- Cholesky-QR in slot order
// LDS: Gs (m x m), d (m), valid (m)
__global__ __launch_bounds__(256) void k_ortho_small(SmallParams p, SmallBufs b, DevStatus* st) {
  if (halted(st)) return;
  extern __shared__ double sm[];
  const int m = p.m, kint = p.kint;
  double* Gs = sm;
  double* d = Gs + m * m;
  __shared__ int valid[256];
  __shared__ int flag;
  const int t = threadIdx.x, nt = blockDim.x;
  const int have_p = st->have_p;
  for (int s = t; s < m; s += nt) {
    int v = slot_valid(s, kint, b.active, have_p);
    const double g = b.G[(size_t)s * m + s];
    if (v && !(g > 0.0 && g < INFINITY)) v = 0;
    valid[s] = v;
    d[s] = v ? 1.0 / sqrt(g) : 0.0;
  }
  if (t == 0) flag = 0;
  __syncthreads();
  for (int e = t; e < m * m; e += nt) {
    const int i = e / m, j = e - i * m;
    Gs[e] = (valid[i] && valid[j]) ? b.G[e] * d[i] * d[j] : 0.0;
  }
  __syncthreads();
  if (t < kint && valid[t]) flag = 1;
  __syncthreads();
  if (!flag) {  // every V column vanished
    if (t == 0) {
      st->error = PLHR_ERR_BREAKDOWN;
      st->reason = kReasonVVanished;
    }
    return;
  }
  for (int j = 0; j < m; ++j) {
    if (!valid[j]) continue;
    const double piv = Gs[j * m + j];
    // a numerically dependent column (V included) adds nothing to span(Z)
    if (!(piv > p.drop_tol)) {
      __syncthreads();
      if (t == 0) valid[j] = 0;
      __syncthreads();
      continue;
    }
    const double rjj = sqrt(piv);
    __syncthreads();
    for (int l = j + 1 + t; l < m; l += nt)
      if (valid[l]) Gs[j * m + l] /= rjj;
    if (t == 0) Gs[j * m + j] = rjj;
    __syncthreads();
    // trailing update of the upper triangle
    const int rem = m - j - 1;
    for (int e = t; e < rem * rem; e += nt) {
      const int i = j + 1 + e / rem, l = j + 1 + e % rem;
      if (i <= l && valid[i] && valid[l]) Gs[i * m + l] -= Gs[j * m + i] * Gs[j * m + l];
    }
    __syncthreads();
  }
  // M = D R^-1: column c of R^-1 by back substitution (thread per column)
  for (int c = t; c < m; c += nt) {
    for (int i = 0; i < m; ++i) b.M[(size_t)i * m + c] = 0.0;
    if (!valid[c]) continue;
    // x_i for i <= c, stored directly into M column c (scaled by d at end)
    b.M[(size_t)c * m + c] = 1.0 / Gs[c * m + c];
    for (int i = c - 1; i >= 0; --i) {
      if (!valid[i]) continue;
      double s = 0.0;
      for (int q = i + 1; q <= c; ++q)
        if (valid[q]) s += Gs[i * m + q] * b.M[(size_t)q * m + c];
      b.M[(size_t)i * m + c] = -s / Gs[i * m + i];
    }
    for (int i = 0; i <= c; ++i) b.M[(size_t)i * m + c] *= d[i];
  }
  __syncthreads();
  for (int s = t; s < m; s += nt) b.keep[s] = valid[s];
  if (t == 0) {
    int nk = 0, nd = 0;
    for (int s = 0; s < m; ++s) {
      nk += valid[s];
      if (s >= kint && !valid[s] && slot_valid(s, kint, b.active, have_p)) ++nd;
    }
    st->m_kept = nk;
    st->n_dropped = nd;
  }
}

// ------------------------------------------------ T-harmonic eigensolver
struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, den = b.re + b.im * r;
    return {(a.re + a.im * r) / den, (a.im - a.re * r) / den};
  }
  const double r = b.re / b.im, den = b.im + b.re * r;
  return {(a.re * r + a.im) / den, (a.im * r - a.re) / den};
}
__device__ __forceinline__ double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }

static constexpr int kTh = 64;  // one wavefront

// Francis double-shift QR on the upper Hessenberg H (n x n, ld n) with
// Schur vectors accumulated into Zs (Zs <- Zs * Q).  Leaves H in real
// Schur form: 1x1 blocks and 2x2 blocks with complex eigenvalues; 2x2
// blocks with real eigenvalues are split by a rotation.  Returns false if
// the iteration limit is hit.
__device__ bool francis_qr(double* H, double* Zs, int n, double hnorm) {
  const int t = threadIdx.x;
  const double ulp = 2.220446049250313e-16;
  const double small = 1e-300;
  int hi = n - 1;
  int its = 0, total = 0;
  while (hi >= 0) {
    // Deflation: the usual relative test, a normwise one (a subdiagonal
    // below ulp*||H|| is a backward-stable perturbation), and a threshold
    // that widens by 10x every 10 sweeps without deflation, up to
    // 1e8*ulp.  Degenerate eigenvalues of the pencil (symmetric grids)
    // make clusters of three or more equal tau, on which double-shift
    // sweeps make no progress; the widened test accepts the tiny coupling
    // inside such a cluster, whose eigenvalues are equal to that accuracy.
    const double mult = (its >= 10) ? pow(10.0, (double)min(its / 10, 8)) : 1.0;
    int l = hi;
    for (; l > 0; --l) {
      const double h = fabs(H[l * n + l - 1]);
      double tst = fabs(H[(l - 1) * n + l - 1]) + fabs(H[l * n + l]);
      if (tst == 0.0) tst = hnorm;
      if (h <= mult * ulp * tst || h <= ulp * hnorm || h <= small) break;
    }
    __syncthreads();
    if (l > 0) {
      if (t == 0) H[l * n + l - 1] = 0.0;
      __syncthreads();
    }
    if (l == hi) {
      --hi;
      its = 0;
      continue;
    }
    if (l == hi - 1) {
      // 2x2 block: split it if its eigenvalues are real
      const int q = hi - 1;
      const double a = H[q * n + q], bb = H[q * n + q + 1], c = H[(q + 1) * n + q],
                   dd = H[(q + 1) * n + q + 1];
      const double pq = 0.5 * (a - dd);
      const double disc = pq * pq + bb * c;
      if (c != 0.0 && disc >= 0.0) {
        const double sq = sqrt(disc);
        const double lam = dd + (pq >= 0.0 ? pq + sq : pq - sq);
        double e1 = lam - dd, e2 = c;
        const double r = hypot(e1, e2);
        const double cs = e1 / r, sn = e2 / r;
        __syncthreads();
        for (int j = q + t; j < n; j += kTh) {
          const double h0 = H[q * n + j], h1 = H[(q + 1) * n + j];
          H[q * n + j] = cs * h0 + sn * h1;
          H[(q + 1) * n + j] = -sn * h0 + cs * h1;
        }
        __syncthreads();
        for (int i = t; i <= q + 1; i += kTh) {
          const double h0 = H[i * n + q], h1 = H[i * n + q + 1];
          H[i * n + q] = cs * h0 + sn * h1;
          H[i * n + q + 1] = -sn * h0 + cs * h1;
        }
        for (int i = t; i < n; i += kTh) {
          const double z0 = Zs[i * n + q], z1 = Zs[i * n + q + 1];
          Zs[i * n + q] = cs * z0 + sn * z1;
          Zs[i * n + q + 1] = -sn * z0 + cs * z1;
        }
        __syncthreads();
        if (t == 0) H[(q + 1) * n + q] = 0.0;
        __syncthreads();
      }
      hi -= 2;
      its = 0;
      continue;
    }
    if (total >= 60 * n) return false;
    ++its;
    ++total;
    double h11, h12, h21, h22;
    if (its % 10 == 0) {
      const double s = fabs(H[hi * n + hi - 1]) + fabs(H[(hi - 1) * n + hi - 2]);
      h11 = 0.75 * s + H[hi * n + hi];
      h12 = -0.4375 * s;
      h21 = s;
      h22 = h11;
    } else {
      h11 = H[(hi - 1) * n + hi - 1];
      h12 = H[(hi - 1) * n + hi];
      h21 = H[hi * n + hi - 1];
      h22 = H[hi * n + hi];
    }
    const double tr = h11 + h22, det = h11 * h22 - h12 * h21;
    double x = H[l * n + l] * H[l * n + l] + H[l * n + l + 1] * H[(l + 1) * n + l] -
               tr * H[l * n + l] + det;
    double y = H[(l + 1) * n + l] * (H[l * n + l] + H[(l + 1) * n + l + 1] - tr);
    double z = H[(l + 1) * n + l] * H[(l + 2) * n + l + 1];
    for (int k = l; k <= hi - 1; ++k) {
      const int nr = (k < hi - 1) ? 3 : 2;
      if (k > l) {
        x = H[k * n + k - 1];
        y = H[(k + 1) * n + k - 1];
        z = (nr == 3) ? H[(k + 2) * n + k - 1] : 0.0;
      }
      const double s = fabs(x) + fabs(y) + fabs(z);
      __syncthreads();
      if (s == 0.0) continue;
      const double xs = x / s, ys = y / s, zs = z / s;
      const double nrm = sqrt(xs * xs + ys * ys + zs * zs);
      const double beta = (xs >= 0.0) ? -nrm : nrm;
      const double tau = (beta - xs) / beta;
      const double v0d = xs - beta;
      const double v1 = ys / v0d, v2 = zs / v0d;
      const int jlo = (k > l) ? k - 1 : l;
      for (int j = jlo + t; j < n; j += kTh) {
        const double a0 = H[k * n + j], a1 = H[(k + 1) * n + j];
        const double a2 = (nr == 3) ? H[(k + 2) * n + j] : 0.0;
        const double sm = tau * (a0 + v1 * a1 + v2 * a2);
        H[k * n + j] = a0 - sm;
        H[(k + 1) * n + j] = a1 - sm * v1;
        if (nr == 3) H[(k + 2) * n + j] = a2 - sm * v2;
      }
      __syncthreads();
      const int ihi = (k + 3 < hi) ? k + 3 : hi;
      for (int i = t; i <= ihi; i += kTh) {
        const double a0 = H[i * n + k], a1 = H[i * n + k + 1];
        const double a2 = (nr == 3) ? H[i * n + k + 2] : 0.0;
        const double sm = tau * (a0 + v1 * a1 + v2 * a2);
        H[i * n + k] = a0 - sm;
        H[i * n + k + 1] = a1 - sm * v1;
        if (nr == 3) H[i * n + k + 2] = a2 - sm * v2;
      }
      for (int i = t; i < n; i += kTh) {
        const double a0 = Zs[i * n + k], a1 = Zs[i * n + k + 1];
        const double a2 = (nr == 3) ? Zs[i * n + k + 2] : 0.0;
        const double sm = tau * (a0 + v1 * a1 + v2 * a2);
        Zs[i * n + k] = a0 - sm;
        Zs[i * n + k + 1] = a1 - sm * v1;
        if (nr == 3) Zs[i * n + k + 2] = a2 - sm * v2;
      }
      __syncthreads();
      if (k > l && t == 0) {
        H[(k + 1) * n + k - 1] = 0.0;
        if (nr == 3) H[(k + 2) * n + k - 1] = 0.0;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  return true;
}

// LDS layout (doubles): L n*n | H n*n | Zs n*n | Xre n*ks | Xim n*ks |
// per-eigenvalue arrays 8*n
__global__ __launch_bounds__(kTh) void k_tharm_small(SmallParams p, SmallBufs b, DevStatus* st) {
  if (halted(st)) return;
  if (threadIdx.x == 0) st->tphase[0] = clock64();
  extern __shared__ double sm[];
  __shared__ int idx[256];
  __shared__ int nks;
  __shared__ double hn;
  const int m = p.m, kint = p.kint;
  const int t = threadIdx.x;
  if (t == 0) {
    int c = 0;
    for (int s = 0; s < m; ++s)
      if (b.keep[s]) idx[c++] = s;
    nks = c;
  }
  __syncthreads();
  const int n = nks;
  const int ks = kint;
  double* L = sm;
  double* H = L + n * n;
  double* Zs = H + n * n;
  double* Xre = Zs + n * n;
  double* Xim = Xre + n * ks;
  double* tre = Xim + n * ks;      // tau re (n)
  double* tim = tre + n;           // tau im (n)
  double* kya = tim + n;           // sort key |xi|
  double* kyb = kya + n;           // Re xi
  double* kyc = kyb + n;           // -Im xi
  int* unitsz = (int*)(kyc + n);   // unit size at leader position (0 for members)
  int* rnk = unitsz + n;           // rank of unit (by leader)
  int* selcol = rnk + n;           // output column for leader (-1 if not selected)
  int* selkind = selcol + n;       // kind for selected unit
  int* order = selkind + n;        // unit leader position for each sorted rank
  const int ld2 = 2 * m;
  // 1. load G_L (symmetrised) and G_R on the kept slots
  for (int e = t; e < n * n; e += kTh) {
    const int a = e / n, c = e - a * n;
    const int ia = idx[a], ic = idx[c];
    L[e] = 0.5 * (b.GLR[(size_t)ia * ld2 + ic] + b.GLR[(size_t)ic * ld2 + ia]);
    H[e] = b.GLR[(size_t)ia * ld2 + m + ic];
  }
  __syncthreads();
  if (t == 0) st->tphase[1] = clock64();
  // 2. Cholesky G_L = L L^T (lower, in place)
  double maxd = 0.0;
  for (int j = 0; j < n; ++j) maxd = fmax(maxd, L[j * n + j]);
  for (int j = 0; j < n; ++j) {
    double piv = L[j * n + j];
    const double floor_ = 1e-15 * maxd;
    if (!(piv > floor_)) piv = floor_ > 0.0 ? floor_ : 1e-300;
    const double djj = sqrt(piv);
    __syncthreads();
    for (int i = j + 1 + t; i < n; i += kTh) L[i * n + j] /= djj;
    if (t == 0) L[j * n + j] = djj;
    __syncthreads();
    const int rem = n - j - 1;
    for (int e = t; e < rem * rem; e += kTh) {
      const int i = j + 1 + e / rem, c = j + 1 + e % rem;
      if (c <= i) L[i * n + c] -= L[i * n + j] * L[c * n + j];
    }
    __syncthreads();
  }
  for (int e = t; e < n * n; e += kTh) {
    const int i = e / n, c = e - i * n;
    if (c > i) L[e] = 0.0;
  }
  __syncthreads();
  if (t == 0) st->tphase[2] = clock64();
  // 3. C = L^-1 G_R L^-T in H: columns (forward substitution), then rows
  for (int c = t; c < n; c += kTh) {
    for (int i = 0; i < n; ++i) {
      double s = H[i * n + c];
      for (int q = 0; q < i; ++q) s -= L[i * n + q] * H[q * n + c];
      H[i * n + c] = s / L[i * n + i];
    }
  }
  __syncthreads();
  for (int r = t; r < n; r += kTh) {
    for (int i = 0; i < n; ++i) {
      double s = H[r * n + i];
      for (int q = 0; q < i; ++q) s -= L[i * n + q] * H[r * n + q];
      H[r * n + i] = s / L[i * n + i];
    }
  }
  __syncthreads();
  if (t == 0) st->tphase[3] = clock64();
  // 4. Hessenberg reduction with accumulation of Zs
  for (int e = t; e < n * n; e += kTh) Zs[e] = ((e / n) == (e % n)) ? 1.0 : 0.0;
  __syncthreads();
  double* u = tre;  // scratch vector (n) during the reduction
  for (int k = 0; k + 2 < n; ++k) {
    // x = H[k+1:, k]
    double ss = 0.0;
    for (int i = k + 2; i < n; ++i) ss += H[i * n + k] * H[i * n + k];
    const double x0 = H[(k + 1) * n + k];
    if (ss == 0.0) continue;  // already reduced (uniform)
    const double nrm = sqrt(x0 * x0 + ss);
    const double alpha = (x0 >= 0.0) ? -nrm : nrm;
    __syncthreads();
    for (int i = k + 1 + t; i < n; i += kTh) u[i] = (i == k + 1) ? x0 - alpha : H[i * n + k];
    __syncthreads();
    const double uu = (x0 - alpha) * (x0 - alpha) + ss;
    const double beta = 2.0 / uu;
    // left: rows k+1.., columns k..n-1
    for (int j = k + t; j < n; j += kTh) {
      double s = 0.0;
      for (int i = k + 1; i < n; ++i) s += u[i] * H[i * n + j];
      s *= beta;
      for (int i = k + 1; i < n; ++i) H[i * n + j] -= s * u[i];
    }
    __syncthreads();
    // right: columns k+1.., all rows; and Zs
    for (int i = t; i < n; i += kTh) {
      double s = 0.0;
      for (int q = k + 1; q < n; ++q) s += H[i * n + q] * u[q];
      s *= beta;
      for (int q = k + 1; q < n; ++q) H[i * n + q] -= s * u[q];
      double sz = 0.0;
      for (int q = k + 1; q < n; ++q) sz += Zs[i * n + q] * u[q];
      sz *= beta;
      for (int q = k + 1; q < n; ++q) Zs[i * n + q] -= sz * u[q];
    }
    __syncthreads();
    if (t == 0) {
      H[(k + 1) * n + k] = alpha;
      for (int i = k + 2; i < n; ++i) H[i * n + k] = 0.0;
    }
    __syncthreads();
  }
  if (t == 0) {
    double s = 0.0;
    for (int e = 0; e < n * n; ++e) s += H[e] * H[e];
    hn = sqrt(s);
  }
  __syncthreads();
  if (t == 0) st->tphase[4] = clock64();
  // 5. Francis QR
  const bool ok = francis_qr(H, Zs, n, hn > 0.0 ? hn : 1.0);
  if (!ok) {
    if (t == 0) {
      st->error = PLHR_ERR_BREAKDOWN;
      st->reason = kReasonQR;
    }
    return;
  }
  if (t == 0) st->tphase[5] = clock64();
  // 6. eigenvalues tau, units, xi = 1/tau, sort keys
  if (t == 0) {
    int q = 0;
    while (q < n) {
      if (q + 1 < n && H[(q + 1) * n + q] != 0.0) {
        const double a = H[q * n + q], bb = H[q * n + q + 1], c = H[(q + 1) * n + q],
                     dd = H[(q + 1) * n + q + 1];
        const double pq = 0.5 * (a - dd);
        const double disc = pq * pq + bb * c;
        const double mu = 0.5 * (a + dd);
        const double nu = sqrt(fmax(-disc, 0.0));
        // leader: Im tau < 0 (its xi has Im > 0)
        tre[q] = mu;
        tim[q] = -nu;
        tre[q + 1] = mu;
        tim[q + 1] = nu;
        unitsz[q] = 2;
        unitsz[q + 1] = 0;
        q += 2;
      } else {
        tre[q] = H[q * n + q];
        tim[q] = 0.0;
        unitsz[q] = 1;
        q += 1;
      }
    }
  }
  __syncthreads();
  for (int q = t; q < n; q += kTh) {
    const double a2 = tre[q] * tre[q] + tim[q] * tim[q];
    if (a2 == 0.0) {
      kya[q] = INFINITY;
      kyb[q] = INFINITY;
      kyc[q] = 0.0;
    } else {
      const double xr = tre[q] / a2, xi_ = -tim[q] / a2;  // 1/tau
      kya[q] = sqrt(xr * xr + xi_ * xi_);
      kyb[q] = xr;
      kyc[q] = -xi_;
    }
    selcol[q] = -1;
  }
  __syncthreads();
  // rank units by (|xi|, Re xi, -Im xi, position)
  for (int q = t; q < n; q += kTh) {
    if (unitsz[q] == 0) {
      rnk[q] = -1;
      continue;
    }
    int r = 0;
    for (int o = 0; o < n; ++o) {
      if (unitsz[o] == 0 || o == q) continue;
      bool less = kya[o] < kya[q] ||
                  (kya[o] == kya[q] &&
                   (kyb[o] < kyb[q] || (kyb[o] == kyb[q] && (kyc[o] < kyc[q] ||
                                                             (kyc[o] == kyc[q] && o < q)))));
      r += less ? 1 : 0;
    }
    rnk[q] = r;
  }
  __syncthreads();
  if (t == 0) {
    int nu = 0;
    for (int q = 0; q < n; ++q)
      if (unitsz[q]) order[rnk[q]] = q, ++nu;
    // selection: count kinds first
    int cnt = 0, nreal = 0, npair = 0, ntil = 0;
    for (int r = 0; r < nu && cnt < kint; ++r) {
      const int q = order[r];
      if (unitsz[q] == 1) {
        selkind[q] = 0;
        ++nreal;
        cnt += 1;
      } else if (cnt + 2 <= kint) {
        selkind[q] = 1;
        ++npair;
        cnt += 2;
      } else {
        selkind[q] = 2;
        ++ntil;
        cnt += 1;
      }
      selcol[q] = r;  // provisional: sorted position
    }
    // assign output columns: [Y0 | YR | ytilde | YI]
    int cr = 0, cp = 0;
    for (int r = 0; r < nu; ++r) {
      const int q = order[r];
      if (selcol[q] < 0) continue;
      if (selkind[q] == 0) {
        selcol[q] = cr++;
      } else if (selkind[q] == 1) {
        selcol[q] = nreal + cp;
        ++cp;
      } else {
        selcol[q] = nreal + npair;
      }
    }
    for (int c = 0; c < kint; ++c) {
      b.kinds[c] = 0;
      b.pair[c] = -1;
    }
    for (int q = 0; q < n; ++q) {
      if (selcol[q] < 0 || unitsz[q] == 0) continue;
      const int c = selcol[q];
      if (selkind[q] == 1) {
        const int ci = nreal + npair + ntil + (c - nreal);
        b.kinds[c] = 1;
        b.kinds[ci] = 3;
        b.pair[c] = ci;
        b.pair[ci] = c;
      } else if (selkind[q] == 2) {
        b.kinds[c] = 2;
      }
    }
    // diagnostics: sorted xi
    for (int r = 0; r < nu && r < m; ++r) {
      const int q = order[r];
      b.xi[r] = (kya[q] < INFINITY) ? kyb[q] : INFINITY;
      b.xi[m + r] = -kyc[q];
    }
  }
  __syncthreads();
  if (t == 0) st->tphase[6] = clock64();
  // 7. Zs <- L^-T Zs (so that y = Zs x directly): back substitution per column
  for (int c = t; c < n; c += kTh) {
    for (int i = n - 1; i >= 0; --i) {
      double s = Zs[i * n + c];
      for (int q = i + 1; q < n; ++q) s -= L[q * n + i] * Zs[q * n + c];
      Zs[i * n + c] = s / L[i * n + i];
    }
  }
  __syncthreads();
  if (t == 0) st->tphase[7] = clock64();
  // 8. eigenvectors of the quasi-triangular H by back substitution, one
  //    selected unit per thread; x stored in column u of Xre/Xim where u
  //    is the unit's selection slot (0..ks-1, provisional = output column)
  const double smin = fmax(2.220446049250313e-16 * hn, 1e-290);
  for (int q = 0; q < n; ++q) {
    // uniform loop over leaders; the thread with lane == slot does the work
    if (unitsz[q] == 0 || selcol[q] < 0) continue;
    const int u = selcol[q];
    if ((u % kTh) != t) continue;
    const cplx tau = {tre[q], tim[q]};
    const int sz = unitsz[q];
    for (int i = 0; i < n; ++i) {
      Xre[i * ks + u] = 0.0;
      Xim[i * ks + u] = 0.0;
    }
    int pend;
    int i;
    if (sz == 1) {
      Xre[q * ks + u] = 1.0;
      pend = q;
      i = q - 1;
    } else {
      const double a = H[q * n + q], bb = H[q * n + q + 1];
      Xre[q * ks + u] = bb;
      Xim[q * ks + u] = 0.0;
      Xre[(q + 1) * ks + u] = tau.re - a;
      Xim[(q + 1) * ks + u] = tau.im;
      pend = q + 1;
      i = q - 1;
    }
    while (i >= 0) {
      if (i > 0 && H[i * n + i - 1] != 0.0) {
        cplx r1 = {0, 0}, r2 = {0, 0};
        for (int j = i + 1; j <= pend; ++j) {
          const cplx xj = {Xre[j * ks + u], Xim[j * ks + u]};
          r1.re -= H[(i - 1) * n + j] * xj.re;
          r1.im -= H[(i - 1) * n + j] * xj.im;
          r2.re -= H[i * n + j] * xj.re;
          r2.im -= H[i * n + j] * xj.im;
        }
        const cplx a11 = {H[(i - 1) * n + i - 1] - tau.re, -tau.im};
        const cplx a12 = {H[(i - 1) * n + i], 0.0};
        const cplx a21 = {H[i * n + i - 1], 0.0};
        const cplx a22 = {H[i * n + i] - tau.re, -tau.im};
        cplx det = cmul(a11, a22);
        const cplx bc = cmul(a12, a21);
        det.re -= bc.re;
        det.im -= bc.im;
        if (cabs2(det) < smin * smin) det = {smin, 0.0};
        cplx n1 = cmul(r1, a22), t1 = cmul(a12, r2);
        n1.re -= t1.re;
        n1.im -= t1.im;
        cplx n2 = cmul(a11, r2), t2 = cmul(a21, r1);
        n2.re -= t2.re;
        n2.im -= t2.im;
        const cplx x1 = cdiv(n1, det), x2 = cdiv(n2, det);
        Xre[(i - 1) * ks + u] = x1.re;
        Xim[(i - 1) * ks + u] = x1.im;
        Xre[i * ks + u] = x2.re;
        Xim[i * ks + u] = x2.im;
        i -= 2;
      } else {
        cplx r = {0, 0};
        for (int j = i + 1; j <= pend; ++j) {
          r.re -= H[i * n + j] * Xre[j * ks + u];
          r.im -= H[i * n + j] * Xim[j * ks + u];
        }
        cplx den = {H[i * n + i] - tau.re, -tau.im};
        if (cabs2(den) < smin * smin) den = {smin, 0.0};
        const cplx x = cdiv(r, den);
        Xre[i * ks + u] = x.re;
        Xim[i * ks + u] = x.im;
        i -= 1;
      }
      // rescale on growth
      double big = 0.0;
      for (int j = (i + 1 > 0 ? i + 1 : 0); j <= pend; ++j)
        big = fmax(big, fabs(Xre[j * ks + u]) + fabs(Xim[j * ks + u]));
      if (big > 1e100) {
        for (int j = 0; j <= pend; ++j) {
          Xre[j * ks + u] *= 1e-100;
          Xim[j * ks + u] *= 1e-100;
        }
      }
    }
  }
  __syncthreads();
  if (t == 0) st->tphase[8] = clock64();
  // 9. y = Zs x into the L (re) and H (im) regions (both free now)
  double* Yre = L;
  double* Yim = H;
  for (int e = t; e < n * ks; e += kTh) {
    const int i = e / ks, u = e - i * ks;
    double sr = 0.0, si = 0.0;
    for (int q = 0; q < n; ++q) {
      sr += Zs[i * n + q] * Xre[q * ks + u];
      si += Zs[i * n + q] * Xim[q * ks + u];
    }
    Yre[e] = sr;
    Yim[e] = si;
  }
  __syncthreads();
  if (t == 0) st->tphase[9] = clock64();
  // 10. normalise and scatter into Y' (m x kint, slot rows)
  for (int e = t; e < m * kint; e += kTh) b.Y[e] = 0.0;
  __syncthreads();
  for (int q = 0; q < n; ++q) {
    if (unitsz[q] == 0 || selcol[q] < 0) continue;
    const int u = selcol[q];
    if ((u % kTh) != t) continue;
    double nr2 = 0.0;
    for (int i = 0; i < n; ++i) nr2 += Yre[i * ks + u] * Yre[i * ks + u] + Yim[i * ks + u] * Yim[i * ks + u];
    double sc = (nr2 > 0.0) ? 1.0 / sqrt(nr2) : 0.0;
    const int kind = (unitsz[q] == 1) ? 0 : selkind[q];
    if (kind == 0) {
      // real vector: sign so that the largest entry is positive
      int im = 0;
      for (int i = 1; i < n; ++i)
        if (fabs(Yre[i * ks + u]) > fabs(Yre[im * ks + u])) im = i;
      if (Yre[im * ks + u] < 0.0) sc = -sc;
      for (int i = 0; i < n; ++i) b.Y[(size_t)idx[i] * kint + u] = Yre[i * ks + u] * sc;
    } else if (kind == 1) {
      const int ci = b.pair[u];
      for (int i = 0; i < n; ++i) {
        b.Y[(size_t)idx[i] * kint + u] = Yre[i * ks + u] * sc;
        b.Y[(size_t)idx[i] * kint + ci] = Yim[i * ks + u] * sc;
      }
    } else {
      for (int i = 0; i < n; ++i) b.Y[(size_t)idx[i] * kint + u] = Yre[i * ks + u] * sc;
    }
  }
}

// --------------------------------------------------- Rayleigh quotients
// part: nblk x 2kint, [v.v | v.(A - sigma B) v]
__global__ void k_rq_small(SmallParams p, const double* __restrict__ part, int nblk,
                           SmallBufs b, DevStatus* st) {
  if (halted(st)) return;
  __shared__ double red[256], sums[128];
  const int c = threadIdx.x, kint = p.kint;
  sum_partials(part, nblk, 2 * kint, sums, red);
  const double* vv = sums;
  const double* vq = sums + kint;
  if (c < kint) {
    const int kd = b.kinds[c];
    double lam;
    if (kd == 1 || kd == 3) {
      const int o = b.pair[c];
      lam = p.sigma + (vq[c] + vq[o]) / (vv[c] + vv[o]);
    } else {
      lam = p.sigma + vq[c] / vv[c];
    }
    b.lam[c] = lam;
  }
  if (c == 0) {
    st->iter += 1;
    st->have_p = 1;
  }
}

// ------------------------------------------------- final Rayleigh-Ritz
// HM: kint x 2kint = [V^T (A - sigma B) V | V^T B V]
__global__ __launch_bounds__(kTh) void k_final_rr(SmallParams p, const double* __restrict__ HM,
                                                  SmallBufs b, DevStatus* st) {
  extern __shared__ double sm[];
  const int n = p.kint, k = p.k, t = threadIdx.x;
  double* L = sm;           // n x n
  double* C = L + n * n;    // n x n
  double* U = C + n * n;    // n x n
  double* ev = U + n * n;   // n
  for (int e = t; e < n * n; e += kTh) {
    const int i = e / n, j = e - i * n;
    L[e] = 0.5 * (HM[(size_t)i * 2 * n + n + j] + HM[(size_t)j * 2 * n + n + i]);
    C[e] = 0.5 * (HM[(size_t)i * 2 * n + j] + HM[(size_t)j * 2 * n + i]);
    U[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  // Cholesky of M
  for (int j = 0; j < n; ++j) {
    const double piv = L[j * n + j];
    if (!(piv > 0.0)) {
      if (t == 0) {
        st->error = PLHR_ERR_NOT_HPD;
        st->reason = kReasonFinalGram;
      }
      return;
    }
    const double d = sqrt(piv);
    __syncthreads();
    for (int i = j + 1 + t; i < n; i += kTh) L[i * n + j] /= d;
    if (t == 0) L[j * n + j] = d;
    __syncthreads();
    const int rem = n - j - 1;
    for (int e = t; e < rem * rem; e += kTh) {
      const int i = j + 1 + e / rem, c = j + 1 + e % rem;
      if (c <= i) L[i * n + c] -= L[i * n + j] * L[c * n + j];
    }
    __syncthreads();
  }
  // C <- L^-1 C L^-T
  for (int c = t; c < n; c += kTh)
    for (int i = 0; i < n; ++i) {
      double s = C[i * n + c];
      for (int q = 0; q < i; ++q) s -= L[i * n + q] * C[q * n + c];
      C[i * n + c] = s / L[i * n + i];
    }
  __syncthreads();
  for (int r = t; r < n; r += kTh)
    for (int i = 0; i < n; ++i) {
      double s = C[r * n + i];
      for (int q = 0; q < i; ++q) s -= L[i * n + q] * C[r * n + q];
      C[r * n + i] = s / L[i * n + i];
    }
  __syncthreads();
  for (int e = t; e < n * n; e += kTh) {
    const int i = e / n, j = e - i * n;
    if (i < j) {
      const double a = 0.5 * (C[i * n + j] + C[j * n + i]);
      C[i * n + j] = a;
      C[j * n + i] = a;
    }
  }
  __syncthreads();
  // cyclic Jacobi
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        if (i != j) off += C[i * n + j] * C[i * n + j];
        else dia += C[i * n + j] * C[i * n + j];
      }
    if (off <= 1e-32 * dia || off == 0.0) break;
    for (int pp = 0; pp < n - 1; ++pp)
      for (int qq = pp + 1; qq < n; ++qq) {
        const double apq = C[pp * n + qq];
        if (apq == 0.0) continue;
        const double app = C[pp * n + pp], aqq = C[qq * n + qq];
        const double theta = (aqq - app) / (2.0 * apq);
        const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(tt * tt + 1.0), s = tt * c;
        __syncthreads();
        // columns p, q
        for (int i = t; i < n; i += kTh) {
          const double cip = C[i * n + pp], ciq = C[i * n + qq];
          C[i * n + pp] = c * cip - s * ciq;
          C[i * n + qq] = s * cip + c * ciq;
          const double uip = U[i * n + pp], uiq = U[i * n + qq];
          U[i * n + pp] = c * uip - s * uiq;
          U[i * n + qq] = s * uip + c * uiq;
        }
        __syncthreads();
        for (int j = t; j < n; j += kTh) {
          const double cpj = C[pp * n + j], cqj = C[qq * n + j];
          C[pp * n + j] = c * cpj - s * cqj;
          C[qq * n + j] = s * cpj + c * cqj;
        }
        __syncthreads();
      }
  }
  for (int i = t; i < n; i += kTh) ev[i] = C[i * n + i];
  __syncthreads();
  // X = L^-T U (in U): back substitution per column
  for (int c = t; c < n; c += kTh)
    for (int i = n - 1; i >= 0; --i) {
      double s = U[i * n + c];
      for (int q = i + 1; q < n; ++q) s -= L[q * n + i] * U[q * n + c];
      U[i * n + c] = s / L[i * n + i];
    }
  __syncthreads();
  if (t == 0) {
    // order by |theta - sigma| (= |ev|), ties to the smaller theta
    int used[128];
    for (int i = 0; i < n; ++i) used[i] = 0;
    for (int r = 0; r < k; ++r) {
      int best = -1;
      for (int i = 0; i < n; ++i) {
        if (used[i]) continue;
        if (best < 0 || fabs(ev[i]) < fabs(ev[best]) ||
            (fabs(ev[i]) == fabs(ev[best]) && ev[i] < ev[best]))
          best = i;
      }
      used[best] = 1;
      b.final_theta[r] = p.sigma + ev[best];
      for (int i = 0; i < n; ++i) b.final_C[(size_t)i * k + r] = U[i * n + best];
    }
  }
}

// relative residuals of the returned pairs from column sums
__global__ void k_final_res(SmallParams p, const double* __restrict__ part, int nblk,
                            SmallBufs b) {
  __shared__ double red[256], sums[128];
  const int c = threadIdx.x, k = p.k;
  sum_partials(part, nblk, 2 * k, sums, red);
  if (c < k) {
    const double rr = sums[c], vv = sums[k + c];
    const double lam = b.final_theta[c];
    b.relres[c] = sqrt(rr) / ((p.normA1 + fabs(lam) * p.normB1) * sqrt(vv));
    b.vbv[c] = vv;
  }
}

// ------------------------------------------------------------ launchers
static size_t tharm_lds(int m, int kint) {
  const size_t n = m;
  return (3 * n * n + 2 * n * kint + 5 * n) * sizeof(double) + 5 * n * sizeof(int);
}

void launch_init_lam(const SmallParams& p, const double* part, int nblk, SmallBufs b,
                     DevStatus* st, hipStream_t s) {
  hipLaunchKernelGGL(k_init_lam, dim3(1), dim3(256), 0, s, p, part, nblk, b, st);
}
void launch_start_check(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s) {
  hipLaunchKernelGGL(k_start_check, dim3(1), dim3(64), 0, s, p, b, st);
}
void launch_conv_check(const SmallParams& p, const double* part, int nblk, SmallBufs b,
                       DevStatus* st, int, hipStream_t s) {
  prof_begin(KC_SMALL, 0.0, 0.0, s);
  hipLaunchKernelGGL(k_conv_check, dim3(1), dim3(256), 0, s, p, part, nblk, b, st);
  prof_end(KC_SMALL, s);
}
void launch_ortho_small(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s) {
  const size_t lds = ((size_t)p.m * p.m + p.m) * sizeof(double);
  prof_begin(KC_SMALL, 0.0, 0.0, s);
  hipLaunchKernelGGL(k_ortho_small, dim3(1), dim3(256), lds, s, p, b, st);
  prof_end(KC_SMALL, s);
}
void launch_tharm_small(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s) {
  prof_begin(KC_SMALL, 0.0, 0.0, s);
  hipLaunchKernelGGL(k_tharm_small, dim3(1), dim3(kTh), tharm_lds(p.m, p.kint), s, p, b, st);
  prof_end(KC_SMALL, s);
}
void launch_rq_small(const SmallParams& p, const double* part, int nblk, SmallBufs b,
                     DevStatus* st, hipStream_t s) {
  prof_begin(KC_SMALL, 0.0, 0.0, s);
  hipLaunchKernelGGL(k_rq_small, dim3(1), dim3(256), 0, s, p, part, nblk, b, st);
  prof_end(KC_SMALL, s);
}
void launch_final_rr(const SmallParams& p, const double* HM, SmallBufs b, DevStatus* st,
                     hipStream_t s) {
  const size_t lds = (3 * (size_t)p.kint * p.kint + p.kint) * sizeof(double);
  hipLaunchKernelGGL(k_final_rr, dim3(1), dim3(kTh), lds, s, p, HM, b, st);
}
void launch_final_res(const SmallParams& p, const double* part, int nblk, SmallBufs b,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_final_res, dim3(1), dim3(256), 0, s, p, part, nblk, b);
}

size_t small_max_lds(int m, int kint) {
  size_t a = tharm_lds(m, kint);
  size_t o = ((size_t)m * m + m) * sizeof(double);
  return a > o ? a : o;
}

hipError_t small_set_attributes(int m, int kint) {
  hipError_t e = hipFuncSetAttribute((const void*)k_tharm_small,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)tharm_lds(m, kint));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_ortho_small,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(((size_t)m * m + m) * sizeof(double)));
}

}  // namespace plhr
