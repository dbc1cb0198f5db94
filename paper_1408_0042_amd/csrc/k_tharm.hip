// The projected eigenproblem of one PLHR iteration, eq. (3.5):
//
//     G_L y = xi G_R y,   G_L = Zhat^*(A - sigma B) T (A - sigma B) Zhat (HPD),
//                         G_R = Zhat^*(A - sigma B) T B Zhat,
//
// on the kept slots of Zhat, with selection of the kint eigenvectors of
// smallest |xi| (Definition 3.1) and, for these real problems, the real
// basis Y' = [Y0 YR ytilde_R YI] of Algorithm 3.
//
// With G_L = L L^T and tau = 1/xi the problem is the standard one
// C u = tau u, C = L^-1 G_R L^-T, y = L^-T u; the wanted pairs are those of
// largest |tau|.  Three kernels, the matrices passed through a small
// global work area (L2-resident):
//   k_tharm_reduce  (256 threads) Cholesky of G_L, C, Householder
//                   reduction of C to upper Hessenberg H = Q^T C Q
//   k_tharm_qr      (two wavefronts) Francis double-shift QR of H to real
//                   Schur form T, accumulating Q; 2x2 blocks with real
//                   eigenvalues are split by a rotation
//   k_tharm_vectors (256 threads) eigenvalues and their ordering by
//                   (|xi|, Re xi, -Im xi) with conjugate pairs kept
//                   together, selection, eigenvectors of T by back
//                   substitution (16 lanes per eigenvector), y = L^-T Q x,
//                   normalisation and scatter into Y'.
#include <cmath>

#include "common.cuh"

namespace plhr {

namespace {

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

constexpr int kNT = 256;  // threads of the parallel phases
constexpr int kQR = 128;  // the QR workgroup (two wavefronts)

// 1/d from the hardware reciprocal estimate and two Newton steps (the
// Householder coefficients need a few-ulp reciprocal, not an IEEE
// division; this saves most of the latency of the division sequence).
__device__ __forceinline__ double fast_rcp(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return r;
}

// Frobenius norm of the n x n matrix X (row stride ld), by every thread
// of the block in a fixed order; `red` is LDS scratch of blockDim/64
// doubles.  Must be called by all threads.
__device__ double block_fro(const double* X, int n, int ld, double* red) {
  const int t = threadIdx.x, nt = blockDim.x;
  double a = 0.0;
  for (int e = t; e < n * n; e += nt) {
    const int i = e / n, j = e - i * n;
    a += X[i * ld + j] * X[i * ld + j];
  }
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
  if ((t & 63) == 0) red[t >> 6] = a;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nt / 64; ++w) s += red[w];
  __syncthreads();
  return sqrt(s);
}

// Compact list of kept slots (shared by all three kernels).
__device__ int kept_slots(const int* keep, int m, int* idx) {
  __shared__ int cnt;
  if (threadIdx.x == 0) {
    int c = 0;
    for (int s = 0; s < m; ++s)
      if (keep[s]) idx[c++] = s;
    cnt = c;
  }
  __syncthreads();
  return cnt;
}

}  // namespace

// ------------------------------------------------------------ reduction
// LDS: H n*n | L n*n (L is written out once C is formed and the region
// then holds Q) | u n | w n | red 256
__device__ void k_tharm_reduce_body(SmallParams p, SmallBufs b, DevStatus* st) {
  if (halted(st)) return;
  if (threadIdx.x == 0) st->tphase[0] = clock64();
  extern __shared__ double sm[];
  __shared__ int idx[256];
  const int m = p.m, t = threadIdx.x;
  const int n = kept_slots(b.keep, m, idx);
  if (n < p.kint) {  // fewer independent basis vectors than wanted columns
    if (t == 0) {
      st->error = PLHR_ERR_BREAKDOWN;
      st->reason = kReasonVVanished;
    }
    return;
  }
  const int tx = t & 15, ty = t >> 4;
  const int ld = n | 1;  // odd row stride: column sweeps spread over the LDS banks
  double* H = sm;
  double* L = H + n * ld;
  double* Q = L;  // after L has been written out
  double* u = L + n * ld;
  double* w = u + n;
  double* red = w + n;
  const int ld2 = 2 * m;
  for (int i = ty; i < n; i += 16)
    for (int c = tx; c < n; c += 16) {
      const int ia = idx[i], ic = idx[c];
      L[i * ld + c] = 0.5 * (b.GLR[(size_t)ia * ld2 + ic] + b.GLR[(size_t)ic * ld2 + ia]);
      H[i * ld + c] = b.GLR[(size_t)ia * ld2 + m + ic];
    }
  __syncthreads();
  // Cholesky G_L = L L^T (right-looking).  A pivot in [-1e-10, 1e-15] max
  // diag (G_L singular to rounding: sigma an eigenvalue whose vector lies
  // in span Z, xi = 0) is raised to 1e-15 max diag.  A pivot below
  // -1e-10 max diag cannot come from an HPD G_L: the stored products of
  // that slot no longer agree (T(A - sigma B)Z carried by linear
  // combination has drifted from T applied to (A - sigma B)Z), and the
  // slot is left out: its row and column of L become e_j and those of G_R
  // zero, so that it contributes only tau = 0 (xi = infinity), never
  // selected, and the remaining slots form the projected problem on
  // their own span.
  __shared__ int dead[256];
  __shared__ int ndead;
  double maxd = 0.0;
  for (int j = 0; j < n; ++j) maxd = fmax(maxd, L[j * ld + j]);
  const double floor_ = fmax(1e-15 * maxd, 1e-300);
  for (int j = t; j < n; j += kNT) dead[j] = 0;
  if (t == 0) ndead = 0;
  for (int j = 0; j < n; ++j) {
    const double p0 = L[j * ld + j];
    __syncthreads();
    if (p0 < -1e-10 * maxd) {  // uniform
      for (int i = j + 1 + t; i < n; i += kNT) L[i * ld + j] = 0.0;
      for (int c = t; c < j; c += kNT) L[j * ld + c] = 0.0;
      if (t == 0) {
        L[j * ld + j] = 1.0;
        dead[j] = 1;
        ++ndead;
      }
      __syncthreads();
      continue;
    }
    const double djj = sqrt(fmax(p0, floor_));
    for (int i = j + 1 + t; i < n; i += kNT) L[i * ld + j] /= djj;
    if (t == 0) L[j * ld + j] = djj;
    __syncthreads();
    for (int i = j + 1 + ty; i < n; i += 16) {
      const double lij = L[i * ld + j];
      for (int c = j + 1 + tx; c <= i; c += 16) L[i * ld + c] -= lij * L[c * ld + j];
    }
    __syncthreads();
  }
  if (ndead) {  // uniform
    for (int i = ty; i < n; i += 16)
      for (int c = tx; c < n; c += 16)
        if (dead[i] || dead[c]) H[i * ld + c] = 0.0;
    if (t == 0) st->n_excluded += ndead;
    __syncthreads();
    if (n - ndead < p.kint) {
      if (t == 0) {
        st->error = PLHR_ERR_BREAKDOWN;
        st->reason = kReasonVVanished;
      }
      return;
    }
  }
  for (int i = ty; i < n; i += 16)
    for (int c = tx; c < n; c += 16)
      if (c > i) L[i * ld + c] = 0.0;
  if (t == 0) st->tphase[1] = clock64();
  __syncthreads();
  // H <- L^-1 H (rows, right-looking forward substitution)
  for (int i = 0; i < n; ++i) {
    const double inv = 1.0 / L[i * ld + i];
    for (int c = t; c < n; c += kNT) H[i * ld + c] *= inv;
    __syncthreads();
    for (int r = i + 1 + ty; r < n; r += 16) {
      const double lri = L[r * ld + i];
      for (int c = tx; c < n; c += 16) H[r * ld + c] -= lri * H[i * ld + c];
    }
    __syncthreads();
  }
  // H <- H L^-T (columns)
  for (int i = 0; i < n; ++i) {
    const double inv = 1.0 / L[i * ld + i];
    for (int r = t; r < n; r += kNT) H[r * ld + i] *= inv;
    __syncthreads();
    for (int c = i + 1 + ty; c < n; c += 16) {
      const double lci = L[c * ld + i];
      for (int r = tx; r < n; r += 16) H[r * ld + c] -= lci * H[r * ld + i];
    }
    __syncthreads();
  }
  // L (compact n x n) to the work area; its LDS region becomes Q = I
  double* gw = b.work;
  for (int e = t; e < n * n; e += kNT) {
    const int i = e / n, j = e - i * n;
    gw[e] = L[i * ld + j];
  }
  __syncthreads();
  for (int i = ty; i < n; i += 16)
    for (int c = tx; c < n; c += 16) Q[i * ld + c] = (i == c) ? 1.0 : 0.0;
  __syncthreads();
  if (t == 0) st->tphase[2] = clock64();
  // Householder reduction to upper Hessenberg form, Q accumulated
  for (int k = 0; k + 2 < n; ++k) {
    double part = 0.0;
    for (int i = k + 2 + t; i < n; i += kNT) part += H[i * ld + k] * H[i * ld + k];
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if ((t & 63) == 0) red[t >> 6] = part;
    __syncthreads();
    const double ss = (red[0] + red[1]) + (red[2] + red[3]);
    const double x0 = H[(k + 1) * ld + k];
    __syncthreads();
    if (ss == 0.0) continue;  // column already reduced (uniform)
    const double nrm = sqrt(x0 * x0 + ss);
    const double alpha = (x0 >= 0.0) ? -nrm : nrm;
    const double beta = 1.0 / (nrm * (nrm + fabs(x0)));  // 2 / (u.u)
    for (int i = k + 1 + t; i < n; i += kNT) u[i] = (i == k + 1) ? x0 - alpha : H[i * ld + k];
    __syncthreads();
    // left: w_j = beta * sum_i u_i H_ij, j >= k; H -= u w^T
    for (int j = k + t; j < n; j += kNT) {
      double s = 0.0;
      for (int i = k + 1; i < n; ++i) s += u[i] * H[i * ld + j];
      w[j] = beta * s;
    }
    __syncthreads();
    for (int i = k + 1 + ty; i < n; i += 16) {
      const double ui = u[i];
      for (int j = k + tx; j < n; j += 16) H[i * ld + j] -= ui * w[j];
    }
    __syncthreads();
    // right: rows of H and Q: z_i = beta * sum_q X_iq u_q ; X -= z u^T
    for (int r = t; r < 2 * n; r += kNT) {
      const double* X = (r < n) ? H + r * ld : Q + (r - n) * ld;
      double s = 0.0;
      for (int q = k + 1; q < n; ++q) s += X[q] * u[q];
      red[r] = beta * s;  // 2n <= 200 < 256
    }
    __syncthreads();
    for (int r = ty; r < 2 * n; r += 16) {
      double* X = (r < n) ? H + r * ld : Q + (r - n) * ld;
      const double z = red[r];
      for (int q = k + 1 + tx; q < n; q += 16) X[q] -= z * u[q];
    }
    __syncthreads();
    if (t == 0) H[(k + 1) * ld + k] = alpha;
    for (int i = k + 2 + t; i < n; i += kNT) H[i * ld + k] = 0.0;
    __syncthreads();
  }
  // H and Q (n x n each, compact) to the work area after L
  for (int e = t; e < n * n; e += kNT) {
    const int i = e / n, j = e - i * n;
    gw[n * n + e] = H[i * ld + j];
    gw[2 * n * n + e] = Q[i * ld + j];
  }
  if (t == 0) st->tphase[3] = clock64();
}

__global__ __launch_bounds__(kNT) void k_tharm_reduce(SmallParams p, SmallBufs b, DevStatus* st) {
  k_tharm_reduce_body(p, b, st);
}
// batched: workgroup b runs problem b
__global__ __launch_bounds__(kNT) void k_tharm_reduce_b(const BatchSmall* __restrict__ bs) {
  const BatchSmall& q = bs[blockIdx.x];
  k_tharm_reduce_body(q.p, q.b, q.st);
}


// ------------------------------------------------------------ Francis QR
// Double-shift QR on the upper Hessenberg H (n x n) with Schur vectors
// accumulated into Q.  Deflation: the usual relative test, a normwise one
// (a subdiagonal below ulp*||H|| is a backward-stable perturbation), and
// a threshold that widens by 10x every 10 sweeps without deflation, up to
// 1e8*ulp: degenerate eigenvalues of the pencil (symmetric grids) make
// clusters of three or more equal tau, on which double-shift sweeps make
// no progress, and the widened test accepts the tiny coupling inside such
// a cluster, whose eigenvalues are equal to that accuracy.  Exceptional
// shifts every 10 sweeps without deflation.
//
// Layout: row stride ld >= n + 1 and n + 1 rows for each of H and Q
// (Q = H + (n + 1) ld); row n and column n are padding.  A bulge step
// k applies P = I - tau v v^T (v = (1, v1, v2) on indices k..k+2) as
// H <- P H P, Q <- Q P in a single pass over disjoint groups of three
// entries: the left update of each column outside the 3 x 3 block, the
// right update of each row outside it, the right update of each row of
// Q, and both updates of the block (one lane).  Every lane issues all of
// its loads before the reflector is formed; groups that do not exist
// (past n, or inside the block) point at the padding, so no lane
// branches, and for the last step of a sweep (two rows) v2 = 0 makes the
// third entry of each group a no-op.  One barrier per bulge step.
__device__ bool francis_qr(double* H, double* Q, int n, int ld, double hnorm, int* sweeps,
                           int* steps) {
  constexpr int NT = kQR;
  constexpr int U = (kMaxM + NT) / NT;  // groups of each kind per lane
  const int t = threadIdx.x, lane = t & 63;
  const double ulp = 2.220446049250313e-16;
  const double small = 1e-300;
  int hi = n - 1;
  int its = 0, total = 0, nsteps = 0;
  while (hi >= 0) {
    const double mult = (its >= 10) ? pow(10.0, (double)min(its / 10, 8)) : 1.0;
    int l = 0;
    for (int base = hi; base >= 1; base -= 64) {
      const int lc = base - lane;
      bool ok = false;
      if (lc >= 1) {
        const double h = fabs(H[lc * ld + lc - 1]);
        double tst = fabs(H[(lc - 1) * ld + lc - 1]) + fabs(H[lc * ld + lc]);
        if (tst == 0.0) tst = hnorm;
        ok = (h <= mult * ulp * tst || h <= ulp * hnorm || h <= small);
      }
      const unsigned long long bal = __ballot64(ok);
      if (bal) {
        l = base - (__ffsll(bal) - 1);
        break;
      }
    }
    __syncthreads();
    if (l > 0) {
      if (t == 0) H[l * ld + l - 1] = 0.0;
      __syncthreads();
    }
    if (l == hi) {
      --hi;
      its = 0;
      continue;
    }
    if (l == hi - 1) {
      const int q = hi - 1;
      const double a = H[q * ld + q], bb = H[q * ld + q + 1], c = H[(q + 1) * ld + q],
                   dd = H[(q + 1) * ld + q + 1];
      const double pq = 0.5 * (a - dd);
      const double disc = pq * pq + bb * c;
      if (c != 0.0 && disc >= 0.0) {
        const double sq = sqrt(disc);
        const double lam = dd + (pq >= 0.0 ? pq + sq : pq - sq);
        const double e1 = lam - dd, e2 = c;
        const double r = hypot(e1, e2);
        const double cs = e1 / r, sn = e2 / r;
        __syncthreads();
        for (int j = q + t; j < n; j += NT) {
          const double h0 = H[q * ld + j], h1 = H[(q + 1) * ld + j];
          H[q * ld + j] = cs * h0 + sn * h1;
          H[(q + 1) * ld + j] = -sn * h0 + cs * h1;
        }
        __syncthreads();
        for (int i = t; i <= q + 1; i += NT) {
          const double h0 = H[i * ld + q], h1 = H[i * ld + q + 1];
          H[i * ld + q] = cs * h0 + sn * h1;
          H[i * ld + q + 1] = -sn * h0 + cs * h1;
        }
        for (int i = t; i < n; i += NT) {
          const double z0 = Q[i * ld + q], z1 = Q[i * ld + q + 1];
          Q[i * ld + q] = cs * z0 + sn * z1;
          Q[i * ld + q + 1] = -sn * z0 + cs * z1;
        }
        __syncthreads();
        if (t == 0) H[(q + 1) * ld + q] = 0.0;
        __syncthreads();
      }
      hi -= 2;
      its = 0;
      continue;
    }
    if (total >= 60 * n) return false;
    ++its;
    ++total;
    nsteps += hi - l;
    double h11, h12, h21, h22;
    if (its % 10 == 0) {
      const double s = fabs(H[hi * ld + hi - 1]) + fabs(H[(hi - 1) * ld + hi - 2]);
      h11 = 0.75 * s + H[hi * ld + hi];
      h12 = -0.4375 * s;
      h21 = s;
      h22 = h11;
    } else {
      h11 = H[(hi - 1) * ld + hi - 1];
      h12 = H[(hi - 1) * ld + hi];
      h21 = H[hi * ld + hi - 1];
      h22 = H[hi * ld + hi];
    }
    const double tr = h11 + h22, det = h11 * h22 - h12 * h21;
    double x = H[l * ld + l] * H[l * ld + l] + H[l * ld + l + 1] * H[(l + 1) * ld + l] -
               tr * H[l * ld + l] + det;
    double y = H[(l + 1) * ld + l] * (H[l * ld + l] + H[(l + 1) * ld + l + 1] - tr);
    double z = H[(l + 1) * ld + l] * H[(l + 2) * ld + l + 1];
    const int dummyR = n * ld;  // row n: padding
    for (int k = l; k <= hi - 1; ++k) {
      const bool three = (k < hi - 1);
      const int nr = three ? 3 : 2;
      const int jlo = (k > l) ? k - 1 : l;
      const int ihi = (k + 3 < hi) ? k + 3 : hi;
      if (k > l) {
        x = H[k * ld + k - 1];
        y = H[(k + 1) * ld + k - 1];
        const double zz = H[(k + 2) * ld + k - 1];
        z = three ? zz : 0.0;
      }
      // groups: three entries each, at offset o, o + s, o + 2s; invalid
      // groups point at padding
      double aL[U][3], aR[U][3], aQ[U][3];
      int oL[U], oR[U], oQ[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = jlo + t + NT * u;
        const bool vl = (j < n) && (j < k || j >= k + nr);
        oL[u] = k * ld + (vl ? j : n);
        aL[u][0] = H[oL[u]];
        aL[u][1] = H[oL[u] + ld];
        aL[u][2] = H[oL[u] + 2 * ld];
        const int i = t + NT * u;
        const bool vr = (i <= ihi) && (i < k || i >= k + nr);
        oR[u] = (vr ? i * ld : dummyR) + k;
        aR[u][0] = H[oR[u]];
        aR[u][1] = H[oR[u] + 1];
        aR[u][2] = H[oR[u] + 2];
        oQ[u] = ((i < n) ? i * ld : dummyR) + k;
        aQ[u][0] = Q[oQ[u]];
        aQ[u][1] = Q[oQ[u] + 1];
        aQ[u][2] = Q[oQ[u] + 2];
      }
      double blk[3][3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) blk[r][c] = H[(k + r) * ld + k + c];
      const double s = fabs(x) + fabs(y) + fabs(z);
      if (s == 0.0) continue;  // uniform
      const double ss = fma(z, z, fma(y, y, x * x));
      double r = __builtin_amdgcn_rsq(ss);
      double e = fma(-ss * r, r, 1.0);
      r = fma(0.5 * r, e, r);
      e = fma(-ss * r, r, 1.0);
      r = fma(0.5 * r, e, r);
      const double nrm = ss * r;
      const double sg = (x >= 0.0) ? 1.0 : -1.0;
      const double beta = -sg * nrm;
      const double tau = (beta - x) * (-sg * r);
      const double iv = fast_rcp(x - beta);
      const double v1 = y * iv, v2 = three ? z * iv : 0.0;
      const int sub = (k > l) ? k * ld + k - 1 : -1;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double sl = tau * (aL[u][0] + v1 * aL[u][1] + v2 * aL[u][2]);
        const bool zs = (oL[u] == sub);
        H[oL[u]] = aL[u][0] - sl;
        H[oL[u] + ld] = zs ? 0.0 : aL[u][1] - sl * v1;
        H[oL[u] + 2 * ld] = zs ? 0.0 : aL[u][2] - sl * v2;
        const double sr = tau * (aR[u][0] + v1 * aR[u][1] + v2 * aR[u][2]);
        H[oR[u]] = aR[u][0] - sr;
        H[oR[u] + 1] = aR[u][1] - sr * v1;
        H[oR[u] + 2] = aR[u][2] - sr * v2;
        const double sq = tau * (aQ[u][0] + v1 * aQ[u][1] + v2 * aQ[u][2]);
        Q[oQ[u]] = aQ[u][0] - sq;
        Q[oQ[u] + 1] = aQ[u][1] - sq * v1;
        Q[oQ[u] + 2] = aQ[u][2] - sq * v2;
      }
      if (t == NT - 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double sm = tau * (blk[0][c] + v1 * blk[1][c] + v2 * blk[2][c]);
          blk[0][c] -= sm;
          blk[1][c] -= sm * v1;
          blk[2][c] -= sm * v2;
        }
#pragma unroll
        for (int rr = 0; rr < 3; ++rr) {
          const double sm = tau * (blk[rr][0] + v1 * blk[rr][1] + v2 * blk[rr][2]);
          blk[rr][0] -= sm;
          blk[rr][1] -= sm * v1;
          blk[rr][2] -= sm * v2;
        }
#pragma unroll
        for (int rr = 0; rr < 3; ++rr)
#pragma unroll
          for (int c = 0; c < 3; ++c)
            if (rr < nr && c < nr) H[(k + rr) * ld + k + c] = blk[rr][c];
      }
      __syncthreads();
    }
  }
  __syncthreads();
  *sweeps = total;
  *steps = nsteps;
  return true;
}


// LDS: H (n + 1) x ld | Q (n + 1) x ld, ld = (n + 1) | 1
__device__ void k_tharm_qr_body(SmallParams p, SmallBufs b, DevStatus* st) {
  if (halted(st)) return;
  extern __shared__ double sm[];
  __shared__ int idx[256];
  const int t = threadIdx.x;
  const int n = kept_slots(b.keep, p.m, idx);
  // odd row stride (in doubles) so that column sweeps spread over the LDS
  // banks, and at least n + 1 for the padding column
  const int ld = (n + 1) | 1;
  double* H = sm;
  double* Q = H + (n + 1) * ld;
  const double* gH = b.work + n * n;
  const double* gQ = b.work + 2 * n * n;
  for (int e = t; e < 2 * (n + 1) * ld; e += kQR) sm[e] = 0.0;
  __syncthreads();
  for (int e = t; e < n * n; e += kQR) {
    const int i = e / n, j = e - i * n;
    H[i * ld + j] = gH[e];
    Q[i * ld + j] = gQ[e];
  }
  __syncthreads();
  __shared__ double red[kQR / 64];
  const double hn = block_fro(H, n, ld, red);
  if (t == 0) st->tphase[4] = clock64();
  int sweeps = 0, steps = 0;
  const bool ok = francis_qr(H, Q, n, ld, hn > 0.0 ? hn : 1.0, &sweeps, &steps);
  if (t == 0) {
    st->tphase[10] = steps;
    st->tphase[11] = sweeps;
  }
  if (!ok) {
    if (t == 0) {
      st->error = PLHR_ERR_BREAKDOWN;
      st->reason = kReasonQR;
    }
    return;
  }
  double* oH = b.work + n * n;
  double* oQ = b.work + 2 * n * n;
  for (int e = t; e < n * n; e += kQR) {
    const int i = e / n, j = e - i * n;
    oH[e] = H[i * ld + j];
    oQ[e] = Q[i * ld + j];
  }
  if (t == 0) st->tphase[5] = clock64();
}

__global__ __launch_bounds__(kQR) void k_tharm_qr(SmallParams p, SmallBufs b, DevStatus* st) {
  k_tharm_qr_body(p, b, st);
}
// batched: workgroup b runs problem b
__global__ __launch_bounds__(kQR) void k_tharm_qr_b(const BatchSmall* __restrict__ bs) {
  const BatchSmall& q = bs[blockIdx.x];
  k_tharm_qr_body(q.p, q.b, q.st);
}


// ---------------------------------------------------------- eigenvectors
// LDS: T n*n | Q n*n | Xre n*ks | Xim n*ks | 5n doubles | 5n ints.  L is
// read from the work area; once the eigenvectors of T are known, the T
// region holds the real parts of Y and the Xre region the imaginary parts.
__device__ void k_tharm_vectors_body(SmallParams p, SmallBufs b, DevStatus* st) {
  if (halted(st)) return;
  extern __shared__ double sm[];
  __shared__ int idx[256];
  const int m = p.m, kint = p.kint, t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  const int n = kept_slots(b.keep, m, idx);
  const int ks = kint;
  const int ld = n | 1;  // odd row stride (LDS banks)
  const double* L = b.work;  // compact, row stride n
  double* T = sm;
  double* Q = T + n * ld;
  double* Xre = Q + n * ld;
  double* Xim = Xre + n * ks;
  double* tre = Xim + n * ks;
  double* tim = tre + n;
  double* kya = tim + n;
  double* kyb = kya + n;
  double* kyc = kyb + n;
  int* unitsz = (int*)(kyc + n);
  int* rnk = unitsz + n;
  int* selcol = rnk + n;
  int* selkind = selcol + n;
  int* order = selkind + n;
  for (int e = t; e < n * n; e += kNT) {
    const int i = e / n, j = e - i * n;
    T[i * ld + j] = b.work[n * n + e];
    Q[i * ld + j] = b.work[2 * n * n + e];
  }
  __syncthreads();
  __shared__ double red[kNT / 64];
  const double hn = block_fro(T, n, ld, red);
  if (t == 0) {
    st->tphase[6] = clock64();
    // eigenvalues tau from the 1x1 and 2x2 blocks; a complex block's
    // leader is the member with Im tau < 0 (its xi has Im > 0)
    int q = 0;
    while (q < n) {
      if (q + 1 < n && T[(q + 1) * ld + q] != 0.0) {
        const double a = T[q * ld + q], bb = T[q * ld + q + 1], c = T[(q + 1) * ld + q],
                     dd = T[(q + 1) * ld + q + 1];
        const double pq = 0.5 * (a - dd);
        const double disc = pq * pq + bb * c;
        const double mu = 0.5 * (a + dd);
        const double nu = sqrt(fmax(-disc, 0.0));
        tre[q] = mu;
        tim[q] = -nu;
        tre[q + 1] = mu;
        tim[q + 1] = nu;
        unitsz[q] = 2;
        unitsz[q + 1] = 0;
        q += 2;
      } else {
        tre[q] = T[q * ld + q];
        tim[q] = 0.0;
        unitsz[q] = 1;
        q += 1;
      }
    }
  }
  __syncthreads();
  for (int q = t; q < n; q += kNT) {
    const double a2 = tre[q] * tre[q] + tim[q] * tim[q];
    if (a2 == 0.0) {
      kya[q] = INFINITY;
      kyb[q] = INFINITY;
      kyc[q] = 0.0;
    } else {
      const double xr = tre[q] / a2, xi_ = -tim[q] / a2;  // xi = 1 / tau
      kya[q] = sqrt(xr * xr + xi_ * xi_);
      kyb[q] = xr;
      kyc[q] = -xi_;
    }
    selcol[q] = -1;
  }
  __syncthreads();
  for (int q = t; q < n; q += kNT) {
    if (unitsz[q] == 0) {
      rnk[q] = -1;
      continue;
    }
    int r = 0;
    for (int o = 0; o < n; ++o) {
      if (unitsz[o] == 0 || o == q) continue;
      const bool less =
          kya[o] < kya[q] ||
          (kya[o] == kya[q] &&
           (kyb[o] < kyb[q] ||
            (kyb[o] == kyb[q] && (kyc[o] < kyc[q] || (kyc[o] == kyc[q] && o < q)))));
      r += less ? 1 : 0;
    }
    rnk[q] = r;
  }
  __syncthreads();
  __shared__ int nsel_s;
  if (t == 0) {
    int nu = 0;
    for (int q = 0; q < n; ++q)
      if (unitsz[q]) order[rnk[q]] = q, ++nu;
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
      selcol[q] = r;
    }
    // output columns [Y0 | YR | ytilde | YI]; Xre/Xim column = output column
    // of the unit's first vector
    int cr = 0, cp = 0, ns = 0;
    for (int r = 0; r < nu; ++r) {
      const int q = order[r];
      if (selcol[q] < 0) continue;
      if (selkind[q] == 0)
        selcol[q] = cr++;
      else if (selkind[q] == 1)
        selcol[q] = nreal + cp++;
      else
        selcol[q] = nreal + npair;
      order[ns++] = q;  // selected leaders, reusing `order`
    }
    nsel_s = ns;
    for (int c = 0; c < kint; ++c) {
      b.kinds[c] = 0;
      b.pair[c] = -1;
    }
    for (int i = 0; i < ns; ++i) {
      const int q = order[i];
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
    for (int r = 0; r < m; ++r) {
      b.xi[r] = 0.0;
      b.xi[m + r] = 0.0;
    }
    int r2 = 0;
    for (int q = 0; q < n; ++q) {
      if (!unitsz[q]) continue;
      const int rk = rnk[q];
      if (rk < m) {
        b.xi[rk] = (kya[q] < INFINITY) ? kyb[q] : INFINITY;
        b.xi[m + rk] = -kyc[q];
      }
      ++r2;
    }
    st->tphase[7] = clock64();
  }
  __syncthreads();
  const int nsel = nsel_s;
  // Q <- L^-T Q (solve L^T Y = Q, right-looking from the last row)
  for (int i = n - 1; i >= 0; --i) {
    const double inv = 1.0 / L[i * n + i];
    for (int c = t; c < n; c += kNT) Q[i * ld + c] *= inv;
    __syncthreads();
    for (int r = ty; r < i; r += 16) {
      const double lir = L[i * n + r];
      for (int c = tx; c < n; c += 16) Q[r * ld + c] -= lir * Q[i * ld + c];
    }
    __syncthreads();
  }
  if (t == 0) st->tphase[8] = clock64();
  // eigenvectors of T: 16 lanes per selected unit; lane l owns the
  // entries j with j % 16 == l (it alone writes and reads them), so the
  // 16 partial sums meet only through shuffles.
  const double smin = fmax(2.220446049250313e-16 * hn, 1e-290);
  const int grp = t >> 4, ln = t & 15;
  for (int base = 0; base < nsel; base += kNT / 16) {
    const int si = base + grp;
    if (si < nsel) {
      const int q = order[si];
      const int u = selcol[q];
      const cplx tau = {tre[q], tim[q]};
      const int sz = unitsz[q];
      for (int j = ln; j < n; j += 16) {
        Xre[j * ks + u] = 0.0;
        Xim[j * ks + u] = 0.0;
      }
      int pend, i;
      if (sz == 1) {
        if ((q & 15) == ln) Xre[q * ks + u] = 1.0;
        pend = q;
      } else {
        const double a = T[q * ld + q], bb = T[q * ld + q + 1];
        if ((q & 15) == ln) {
          Xre[q * ks + u] = bb;
          Xim[q * ks + u] = 0.0;
        }
        if (((q + 1) & 15) == ln) {
          Xre[(q + 1) * ks + u] = tau.re - a;
          Xim[(q + 1) * ks + u] = tau.im;
        }
        pend = q + 1;
      }
      i = q - 1;
      int steps = 0;
      while (i >= 0) {
        const bool two = (i > 0 && T[i * ld + i - 1] != 0.0);
        // partial sums over owned j in (i, pend]
        double r1r = 0.0, r1i = 0.0, r2r = 0.0, r2i = 0.0;
        for (int j = i + 1 + ((ln - (i + 1)) & 15); j <= pend; j += 16) {
          const double xr = Xre[j * ks + u], xim = Xim[j * ks + u];
          r2r -= T[i * ld + j] * xr;
          r2i -= T[i * ld + j] * xim;
          if (two) {
            r1r -= T[(i - 1) * ld + j] * xr;
            r1i -= T[(i - 1) * ld + j] * xim;
          }
        }
        for (int off = 8; off > 0; off >>= 1) {
          r2r += __shfl_xor(r2r, off, 16);
          r2i += __shfl_xor(r2i, off, 16);
          if (two) {
            r1r += __shfl_xor(r1r, off, 16);
            r1i += __shfl_xor(r1i, off, 16);
          }
        }
        if (two) {
          const cplx r1 = {r1r, r1i}, r2 = {r2r, r2i};
          const cplx a11 = {T[(i - 1) * ld + i - 1] - tau.re, -tau.im};
          const cplx a12 = {T[(i - 1) * ld + i], 0.0};
          const cplx a21 = {T[i * ld + i - 1], 0.0};
          const cplx a22 = {T[i * ld + i] - tau.re, -tau.im};
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
          if (((i - 1) & 15) == ln) {
            Xre[(i - 1) * ks + u] = x1.re;
            Xim[(i - 1) * ks + u] = x1.im;
          }
          if ((i & 15) == ln) {
            Xre[i * ks + u] = x2.re;
            Xim[i * ks + u] = x2.im;
          }
          i -= 2;
        } else {
          cplx den = {T[i * ld + i] - tau.re, -tau.im};
          if (cabs2(den) < smin * smin) den = {smin, 0.0};
          const cplx x = cdiv({r2r, r2i}, den);
          if ((i & 15) == ln) {
            Xre[i * ks + u] = x.re;
            Xim[i * ks + u] = x.im;
          }
          i -= 1;
        }
        if (((++steps) & 7) == 0) {
          // rescale on growth (each lane checks its own entries)
          double big = 0.0;
          for (int j = (i + 1) + ((ln - (i + 1)) & 15); j <= pend; j += 16)
            big = fmax(big, fabs(Xre[j * ks + u]) + fabs(Xim[j * ks + u]));
          for (int off = 8; off > 0; off >>= 1) big = fmax(big, __shfl_xor(big, off, 16));
          if (big > 1e100)
            for (int j = ln; j <= pend; j += 16) {
              Xre[j * ks + u] *= 1e-100;
              Xim[j * ks + u] *= 1e-100;
            }
        }
      }
    }
  }
  __syncthreads();
  if (t == 0) st->tphase[9] = clock64();
  // y = (L^-T Q) x: real parts into the T region (free after the back
  // substitution), then imaginary parts into the Xre region (free once the
  // real parts are formed)
  double* Yre = T;
  double* Yim = Xre;
  for (int e = t; e < n * nsel; e += kNT) {
    const int i = e / nsel, si = e - i * nsel;
    const int u = selcol[order[si]];
    double sr = 0.0;
    for (int q = 0; q < n; ++q) sr += Q[i * ld + q] * Xre[q * ks + u];
    Yre[i * ks + u] = sr;
  }
  __syncthreads();
  for (int e = t; e < n * nsel; e += kNT) {
    const int i = e / nsel, si = e - i * nsel;
    const int u = selcol[order[si]];
    double sim = 0.0;
    for (int q = 0; q < n; ++q) sim += Q[i * ld + q] * Xim[q * ks + u];
    Yim[i * ks + u] = sim;
  }
  for (int e = t; e < m * kint; e += kNT) b.Y[e] = 0.0;
  __syncthreads();
  // normalise and scatter into Y' (16 lanes per unit)
  for (int base = 0; base < nsel; base += kNT / 16) {
    const int si = base + grp;
    if (si >= nsel) continue;
    const int q = order[si];
    const int u = selcol[q];
    double nr2 = 0.0, big = -1.0;
    int im = 0;
    for (int i = ln; i < n; i += 16) {
      nr2 += Yre[i * ks + u] * Yre[i * ks + u] + Yim[i * ks + u] * Yim[i * ks + u];
      if (fabs(Yre[i * ks + u]) > big) big = fabs(Yre[i * ks + u]), im = i;
    }
    for (int off = 8; off > 0; off >>= 1) {
      nr2 += __shfl_xor(nr2, off, 16);
      const double ob = __shfl_xor(big, off, 16);
      const int oi = __shfl_xor(im, off, 16);
      if (ob > big || (ob == big && oi < im)) big = ob, im = oi;
    }
    double sc = (nr2 > 0.0) ? 1.0 / sqrt(nr2) : 0.0;
    const int kind = (unitsz[q] == 1) ? 0 : selkind[q];
    if (kind == 0 && Yre[im * ks + u] < 0.0) sc = -sc;  // largest entry positive
    const int ci = (kind == 1) ? b.pair[u] : -1;
    for (int i = ln; i < n; i += 16) {
      b.Y[(size_t)idx[i] * kint + u] = Yre[i * ks + u] * sc;
      if (kind == 1) b.Y[(size_t)idx[i] * kint + ci] = Yim[i * ks + u] * sc;
    }
  }
}

__global__ __launch_bounds__(kNT) void k_tharm_vectors(SmallParams p, SmallBufs b, DevStatus* st) {
  k_tharm_vectors_body(p, b, st);
}
// batched: workgroup b runs problem b
__global__ __launch_bounds__(kNT) void k_tharm_vectors_b(const BatchSmall* __restrict__ bs) {
  const BatchSmall& q = bs[blockIdx.x];
  k_tharm_vectors_body(q.p, q.b, q.st);
}


static size_t reduce_lds(int m) { return ((size_t)2 * m * (m | 1) + 2 * m + kNT) * sizeof(double); }
static size_t qr_lds(int m) { return (size_t)2 * (m + 1) * ((m + 1) | 1) * sizeof(double); }
static size_t vectors_lds(int m, int kint) {
  return ((size_t)2 * m * (m | 1) + 2 * (size_t)m * kint + 5 * m) * sizeof(double) +
         5 * m * sizeof(int);
}

hipError_t tharm_set_attributes(int m, int kint) {
  const void* fr[2] = {(const void*)k_tharm_reduce, (const void*)k_tharm_reduce_b};
  const void* fq[2] = {(const void*)k_tharm_qr, (const void*)k_tharm_qr_b};
  const void* fv[2] = {(const void*)k_tharm_vectors, (const void*)k_tharm_vectors_b};
  for (int i = 0; i < 2; ++i) {
    hipError_t e = hipFuncSetAttribute(fr[i], hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)reduce_lds(m));
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(fq[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)qr_lds(m));
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(fv[i], hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)vectors_lds(m, kint));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void launch_tharm_small(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s) {
  // model operation counts at the full width m (the kept width is known
  // only on the device): Cholesky m^3/3, C = L^-1 G_R L^-T 2m^3,
  // Hessenberg reduction with Q 14m^3/3; Francis QR to the real Schur
  // form with Schur vectors about 20m^3 (two double-shift sweeps per
  // eigenvalue pair); L^-T Q m^3 and Y = (L^-T Q) X 2 m^2 kint
  const double m3 = (double)p.m * p.m * p.m, mm = (double)p.m * p.m;
  prof_begin(KC_THARM_REDUCE, 2.0 * mm * 8.0 + 3.0 * mm * 8.0, (1.0 / 3.0 + 2.0 + 14.0 / 3.0) * m3, s);
  hipLaunchKernelGGL(k_tharm_reduce, dim3(1), dim3(kNT), reduce_lds(p.m), s, p, b, st);
  prof_end(KC_THARM_REDUCE, s);
  prof_begin(KC_THARM_QR, 4.0 * mm * 8.0, 20.0 * m3, s);
  hipLaunchKernelGGL(k_tharm_qr, dim3(1), dim3(kQR), qr_lds(p.m), s, p, b, st);
  prof_end(KC_THARM_QR, s);
  prof_begin(KC_THARM_VECTORS, 3.0 * mm * 8.0 + mm * 8.0, m3 + 2.0 * mm * p.kint, s);
  hipLaunchKernelGGL(k_tharm_vectors, dim3(1), dim3(kNT), vectors_lds(p.m, p.kint), s, p, b, st);
  prof_end(KC_THARM_VECTORS, s);
}

void launch_tharm_small_b(const BatchSmall* bs, int nb, int m, int kint, hipStream_t s) {
  const double m3 = (double)m * m * m, mm = (double)m * m;
  prof_begin(KC_THARM_REDUCE, nb * 5.0 * mm * 8.0, nb * (1.0 / 3.0 + 2.0 + 14.0 / 3.0) * m3, s);
  hipLaunchKernelGGL(k_tharm_reduce_b, dim3(nb), dim3(kNT), reduce_lds(m), s, bs);
  prof_end(KC_THARM_REDUCE, s);
  prof_begin(KC_THARM_QR, nb * 4.0 * mm * 8.0, nb * 20.0 * m3, s);
  hipLaunchKernelGGL(k_tharm_qr_b, dim3(nb), dim3(kQR), qr_lds(m), s, bs);
  prof_end(KC_THARM_QR, s);
  prof_begin(KC_THARM_VECTORS, nb * 4.0 * mm * 8.0, nb * (m3 + 2.0 * mm * kint), s);
  hipLaunchKernelGGL(k_tharm_vectors_b, dim3(nb), dim3(kNT), vectors_lds(m, kint), s, bs);
  prof_end(KC_THARM_VECTORS, s);
}

}  // namespace plhr
