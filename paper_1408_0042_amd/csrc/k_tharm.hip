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
//   k_tharm_qr      (four wavefronts) Francis double-shift QR of H to real
//                   Schur form T, accumulating Q; 2x2 blocks with real
//                   eigenvalues are split by a rotation
//   k_tharm_vectors (256 threads) eigenvalues and their ordering by
//                   (|xi|, Re xi, -Im xi) with conjugate pairs kept
//                   together, selection, eigenvectors of T by back
//                   substitution (16 lanes per eigenvector), y = L^-T Q x,
//                   normalisation and scatter into Y'.
#include <algorithm>
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
constexpr int kQR = 256;  // the QR workgroup (four wavefronts)

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
// then holds Q) | u n | bv n | red 256
//
// Cholesky: right-looking on unscaled columns (the trailing update of
// column j divides by the pivot, the scaling 1/sqrt(pivot) of column j is
// applied once at the end), one barrier per column.  C = L^-1 G_R L^-T:
// forward substitutions, one thread per column of G_R, then one thread per
// row.  Householder reduction to Hessenberg form: each step reads the
// column norm from per-wave partial sums left by the previous step, forms
// Hu, u^T H and Qu in one pass (one thread per row of H, of Q and per
// column of H) and applies H <- (I - beta u u^T) H (I - beta u u^T) as one
// rank-2 update with the coefficient gamma = u^T H u, Q <- Q (I - beta u
// u^T); two barriers per step.
__device__ __forceinline__ double wave_sum(double a) {
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
  return a;
}

__device__ void k_tharm_reduce_body(SmallParams p, SmallBufs b, DevStatus* st) {
  static_assert(kNT >= 3 * kMaxM, "one thread per row of H, of Q and per column of H");
  static_assert(8 + 88 + kMaxM <= kNT && kMaxM <= 88, "column buffers inside red");
  if (halted(st)) return;
  if (threadIdx.x == 0) st->tphase[0] = clock64();
  extern __shared__ __attribute__((aligned(16))) double sm[];
  __shared__ int idx[256];
  const int m = p.m, t = threadIdx.x, wv = t >> 6;
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
  double* bv = u + n;
  double* red = bv + n;
  const int ld2 = 2 * m;
  // fixed-trip (predicated) loops: every global load of a lane is issued
  // before the first is used
  static_assert(kMaxM <= 6 * 16, "six rows and columns per lane");
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    const int i = ty + 16 * a;
    if (i < n) {
      const int ia = idx[i];
      double g1[6], g2[6], g3[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const int c = tx + 16 * q;
        if (c < n) {
          const int ic = idx[c];
          g1[q] = b.GLR[(size_t)ia * ld2 + ic];
          g2[q] = b.GLR[(size_t)ic * ld2 + ia];
          g3[q] = b.GLR[(size_t)ia * ld2 + m + ic];
        }
      }
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const int c = tx + 16 * q;
        if (c < n) {
          L[i * ld + c] = 0.5 * (g1[q] + g2[q]);
          H[i * ld + c] = g3[q];
        }
      }
    }
  }
  // Cholesky G_L = L L^T.  A pivot in [-1e-10, 1e-15] max diag (G_L
  // singular to rounding: sigma an eigenvalue whose vector lies in span Z,
  // xi = 0) is raised to 1e-15 max diag.  A pivot below -1e-10 max diag
  // cannot come from an HPD G_L: the stored products of that slot no
  // longer agree (T(A - sigma B)Z carried by linear combination has
  // drifted from T applied to (A - sigma B)Z), and the slot is left out:
  // its row and column of L become e_j and those of G_R zero, so that it
  // contributes only tau = 0 (xi = infinity), never selected, and the
  // remaining slots form the projected problem on their own span.
  __shared__ int dead[256];
  __shared__ int ndead;
  double* dsc = bv;   // 1/sqrt(pivot) per column
  double* djj = red;  // sqrt(pivot): the diagonal of L
  for (int j = t; j < n; j += kNT) dead[j] = 0;
  if (t == 0) ndead = 0;
  __syncthreads();
  double maxd = 0.0;
  for (int j = 0; j < n; ++j) maxd = fmax(maxd, L[j * ld + j]);
  const double floor_ = fmax(1e-15 * maxd, 1e-300);
  for (int j = 0; j < n; ++j) {
    const double p0 = L[j * ld + j];
    if (p0 < -1e-10 * maxd) {  // uniform; no update, so no barrier
      if (t == 0) {
        dead[j] = 1;
        ++ndead;
        dsc[j] = 0.0;
      }
      continue;
    }
    const double pp = fmax(p0, floor_);
    const double inv = 1.0 / pp;
    if (t == 0) djj[j] = pp;  // its square root after the loop, by all lanes
    for (int i = j + 1 + ty; i < n; i += 16) {
      const double lij = L[i * ld + j] * inv;
      for (int c = j + 1 + tx; c <= i; c += 16) L[i * ld + c] -= lij * L[c * ld + j];
    }
    __syncthreads();
  }
  __syncthreads();
  for (int j = t; j < n; j += kNT)
    if (!dead[j]) {
      djj[j] = sqrt(djj[j]);
      dsc[j] = 1.0 / djj[j];
    }
  __syncthreads();
  for (int i = ty; i < n; i += 16)
    for (int c = tx; c < n; c += 16) {
      double v = 0.0;
      if (dead[i] || dead[c])
        v = (i == c) ? 1.0 : 0.0;
      else if (c == i)  // the raised pivot, where it was raised
        v = djj[c];
      else if (c < i)
        v = L[i * ld + c] * dsc[c];
      L[i * ld + c] = v;
      if (dead[i] || dead[c]) H[i * ld + c] = 0.0;
    }
  if (t == 0 && ndead) st->n_excluded += ndead;
  if (ndead && n - ndead < p.kint) {  // uniform
    if (t == 0) {
      st->error = PLHR_ERR_BREAKDOWN;
      st->reason = kReasonVVanished;
    }
    return;
  }
  if (t == 0) st->tphase[1] = clock64();
  __syncthreads();
  // H <- L^-1 H and then H <- H L^-T, blocked by 16: the diagonal block
  // is solved by one thread per column (per row), then the rows (columns)
  // below it are updated by the whole workgroup, 16 x 16 threads.
  constexpr int NB = 16;
  for (int kb = 0; kb < n; kb += NB) {
    const int ke = (kb + NB < n) ? kb + NB : n, nb = ke - kb;
    if (t < n) {
      for (int i = kb; i < ke; ++i) {
        const double* Li = L + i * ld;
        double s0 = H[i * ld + t], s1 = 0.0;
        int r = kb;
        for (; r + 1 < i; r += 2) {
          s0 -= Li[r] * H[r * ld + t];
          s1 -= Li[r + 1] * H[(r + 1) * ld + t];
        }
        if (r < i) s0 -= Li[r] * H[r * ld + t];
        H[i * ld + t] = (s0 + s1) / Li[i];
      }
    }
    __syncthreads();
    for (int i = ke + ty; i < n; i += 16) {
      double lr[NB];
#pragma unroll
      for (int r = 0; r < NB; ++r) lr[r] = (r < nb) ? L[i * ld + kb + r] : 0.0;
      for (int c = tx; c < n; c += 16) {
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int r = 0; r < NB; r += 2) {
          a0 += lr[r] * H[((kb + r < n) ? kb + r : n - 1) * ld + c];
          a1 += lr[r + 1] * H[((kb + r + 1 < n) ? kb + r + 1 : n - 1) * ld + c];
        }
        H[i * ld + c] -= a0 + a1;
      }
    }
    __syncthreads();
  }
  for (int kb = 0; kb < n; kb += NB) {
    const int ke = (kb + NB < n) ? kb + NB : n, nb = ke - kb;
    if (t < n) {  // x L^T = h for row t
      double* Hr = H + t * ld;
      for (int i = kb; i < ke; ++i) {
        const double* Li = L + i * ld;
        double s0 = Hr[i], s1 = 0.0;
        int c = kb;
        for (; c + 1 < i; c += 2) {
          s0 -= Li[c] * Hr[c];
          s1 -= Li[c + 1] * Hr[c + 1];
        }
        if (c < i) s0 -= Li[c] * Hr[c];
        Hr[i] = (s0 + s1) / Li[i];
      }
    }
    __syncthreads();
    for (int r = ty; r < n; r += 16) {
      double hr[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) hr[c] = (c < nb) ? H[r * ld + kb + c] : 0.0;
      for (int i = ke + tx; i < n; i += 16) {
        const double* Li = L + i * ld + kb;
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int c = 0; c < NB; c += 2) {
          a0 += hr[c] * Li[(c < nb) ? c : 0];
          a1 += hr[c + 1] * Li[(c + 1 < nb) ? c + 1 : 0];
        }
        H[r * ld + i] -= a0 + a1;
      }
    }
    __syncthreads();
  }
  // L (compact n x n) to the work area; its LDS region becomes Q = I
  double* gw = b.work;
  store_square(L, gw, n, ld);
  __syncthreads();
  for (int i = ty; i < n; i += 16)
    for (int c = tx; c < n; c += 16) Q[i * ld + c] = (i == c) ? 1.0 : 0.0;
  if (t == 0) st->tphase[2] = clock64();
  // Householder reduction to upper Hessenberg form, Q accumulated.  Step
  // k forms, with the same strided dot-product code in every thread,
  // (Hu)_i for the rows of H (threads [0, n)), (Qu)_i for the rows of Q
  // ([n, 2n)) and (u^T H)_j for the columns j >= k ([2n, 3n - k)); after
  // a barrier every row of H and Q is updated by the same two-vector code,
  //   H[i][j] -= beta u_i (u^T H)_j + (beta (Hu)_i - beta^2 gamma u_i) u_j,
  //   Q[i][j] -= 0 + beta (Qu)_i u_j,   gamma = u^T H u,
  // so no wavefront runs two code paths.  Column k is kept contiguous in
  // ucol (written by the row owners during the previous step); u differs
  // from it only in entry k + 1.  red[0..3]: per-wave partial sums of the
  // squared column below the subdiagonal, red[4..7] of gamma.
  double* ucb[2] = {red + 8, red + 8 + 88};
  {
    const double h = (t < n) ? H[t * ld] : 0.0;
    if (t < n) ucb[0][t] = h;
    const double s = wave_sum((t >= 2 && t < n) ? h * h : 0.0);
    if ((t & 63) == 0) red[wv] = s;
  }
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    const double* ucol = ucb[k & 1];
    double* ucn = ucb[(k + 1) & 1];
    const double ss = ((red[0] + red[1]) + red[2]) + red[3];
    const double x0 = ucol[k + 1];
    if (ss == 0.0) {  // column already reduced (uniform): next column
      __syncthreads();
      const double h = (t < n) ? H[t * ld + k + 1] : 0.0;
      if (t < n) ucn[t] = h;
      const double s = wave_sum((t >= k + 3 && t < n) ? h * h : 0.0);
      if ((t & 63) == 0) red[wv] = s;
      __syncthreads();
      continue;
    }
    const double nrm = sqrt(x0 * x0 + ss);
    const double alpha = (x0 >= 0.0) ? -nrm : nrm;
    const double beta = 1.0 / (nrm * (nrm + fabs(x0)));  // 2 / (u.u)
    const double u1 = x0 - alpha;                        // u_{k+1}
    const double du = u1 - x0;                           // u - ucol at entry k + 1
    const bool isH = (t < n), isQ = (t >= n && t < 2 * n);
    const bool isC = (t >= 2 * n && t < 3 * n - k);
    const int len = n - k - 1;
    const double* base = isH ? H + t * ld + (k + 1)
                         : isQ ? Q + (t - n) * ld + (k + 1)
                         : isC ? H + (k + 1) * ld + (k + t - 2 * n)
                               : H;
    const int str = isC ? ld : 1;
    const double* uv = ucol + (k + 1);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int q = 0;
    for (; q + 3 < len; q += 4) {
      a0 += base[q * str] * uv[q];
      a1 += base[(q + 1) * str] * uv[q + 1];
      a2 += base[(q + 2) * str] * uv[q + 2];
      a3 += base[(q + 3) * str] * uv[q + 3];
    }
    for (; q < len; ++q) a0 += base[q * str] * uv[q];
    const double acc = ((a0 + a1) + (a2 + a3)) + base[0] * du;
    if (isC) bv[k + (t - 2 * n)] = acc;
    double ui = 0.0;
    if (t >= k + 1 && t < n) {
      ui = (t == k + 1) ? u1 : ucol[t];
      u[t] = ui;
    }
    {
      const double s = wave_sum(isH ? ui * acc : 0.0);
      if ((t & 63) == 0) red[4 + wv] = s;
    }
    __syncthreads();
    const double gamma = ((red[4] + red[5]) + red[6]) + red[7];
    double nxt = 0.0;
    if (t < 2 * n) {
      double* Xr = isH ? H + t * ld : Q + (t - n) * ld;
      const double s1 = isH ? beta * ui : 0.0;
      const double s2 = isH ? beta * acc - beta * beta * gamma * ui : beta * acc;
      if (isH && t >= k + 1) Xr[k] = (t == k + 1) ? alpha : 0.0;
      int j = k + 1;
      for (; j + 3 < n; j += 4) {
        const double x0_ = Xr[j], x1_ = Xr[j + 1], x2_ = Xr[j + 2], x3_ = Xr[j + 3];
        const double b0 = bv[j], b1 = bv[j + 1], b2 = bv[j + 2], b3 = bv[j + 3];
        const double c0 = u[j], c1 = u[j + 1], c2 = u[j + 2], c3 = u[j + 3];
        Xr[j] = x0_ - (s1 * b0 + s2 * c0);
        Xr[j + 1] = x1_ - (s1 * b1 + s2 * c1);
        Xr[j + 2] = x2_ - (s1 * b2 + s2 * c2);
        Xr[j + 3] = x3_ - (s1 * b3 + s2 * c3);
      }
      for (; j < n; ++j) Xr[j] -= s1 * bv[j] + s2 * u[j];
      if (isH) {
        const double h = Xr[k + 1];
        ucn[t] = h;
        if (t >= k + 3) nxt = h * h;
      }
    }
    {
      const double s = wave_sum(nxt);
      if ((t & 63) == 0) red[wv] = s;
    }
    __syncthreads();
  }
  // H and Q (n x n each, compact) to the work area after L
  store_square(H, gw + n * n, n, ld);
  store_square(Q, gw + 2 * n * n, n, ld);
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
// P = I - tau v v^T with v = (1, v1, v2) and P (x, y, z)^T = (beta, 0, 0)^T
// (Sec. 5.1 of Golub & Van Loan), beta = -sign(x) ||(x, y, z)||; the
// square root and reciprocal come from the hardware estimates refined by
// Newton steps.  A zero vector gives P = I.
__device__ __forceinline__ void householder3(double x, double y, double z, double& tau, double& v1,
                                             double& v2) {
  const double s = fabs(x) + fabs(y) + fabs(z);
  const double ss = fma(z, z, fma(y, y, x * x));
  double r = __builtin_amdgcn_rsq(ss);
  double e = fma(-ss * r, r, 1.0);
  r = fma(0.5 * r, e, r);
  e = fma(-ss * r, r, 1.0);
  r = fma(0.5 * r, e, r);
  const double nrm = ss * r;
  const double sg = (x >= 0.0) ? 1.0 : -1.0;
  const double beta = -sg * nrm;
  const double iv = fast_rcp(x - beta);
  const bool zero = (s == 0.0);
  tau = zero ? 0.0 : (beta - x) * (-sg * r);
  v1 = zero ? 0.0 : y * iv;
  v2 = zero ? 0.0 : z * iv;
}

// Francis double-shift QR of the upper Hessenberg H (n x n) to real Schur
// form, accumulating Q <- Q P for every reflector (Sec. 7.5 of Golub & Van
// Loan, standard deflation test on the subdiagonal, which is relaxed by a
// factor 10 per 10 sweeps without deflation so that the iteration also
// ends on a cluster, whose eigenvalues are equal to that accuracy).
// Exceptional shifts every 10 sweeps without deflation.  Real 2 x 2 blocks
// are split by a rotation.
//
// Layout: row stride ld >= n + 1 and n + 1 rows for each of H and Q
// (Q = H + (n + 1) ld); row n and column n are padding that stays zero.
//
// A bulge step k applies P = I - tau v v^T (v = (1, v1, v2) on indices
// k..k+2; v2 = 0 for the last step of a sweep) as H <- P H P, Q <- Q P.
// The four wavefronts of the workgroup have fixed roles:
//   waves 0, 1   the updates of disjoint 3-entry groups outside the 3 x 3
//                block at (k, k): group g < 96 is the right update of row
//                g of H when g <= min(k + 3, hi), otherwise the left update
//                of column g - 5 in rows k..k+2 (the columns left of k - 1
//                that this includes are exact zeros below the subdiagonal,
//                which the update keeps zero); group 96 + i is row i of Q.
//                Each lane runs groups t and t + 128.
//   wave 2       lanes 0..2: the columns of P B P for the block B.
//   wave 3       the reflector of step k + 1, computed during step k from B,
//                P_k and the row below the block, which before step k is
//                (0, 0, H[k+3][k+2]) with that entry read one step ahead
//                (no lane writes row k + 3 then).
// The reflectors pass through a double-buffered LDS slot.  Each step has
// two barriers: after the first, every read of the block region is done
// and wave 2 writes the new block; after the second, the step is complete.
// Groups that do not exist point at the padding.
__device__ bool francis_qr(double* H, double* Q, int n, int ld, double hnorm, int* sweeps,
                           int* steps, double* refl) {
  constexpr int NT = kQR;
  static_assert(NT == 256, "four wavefronts");
  static_assert(kMaxM + 5 <= 96 && 96 + kMaxM <= 2 * 128, "group index space");
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const double ulp = 2.220446049250313e-16;
  const double small = 1e-300;
  const int QOFF = (n + 1) * ld;  // Q follows H in the LDS array
  int tld[2], bQ[2], jL[2];
  bool lok[2], isH[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int g = t + 128 * u;
    isH[u] = (g < 96);
    tld[u] = g * ld;
    jL[u] = g - 5;
    lok[u] = isH[u] && (g >= 5) && (g - 5 < n);
    bQ[u] = (g >= 96 && g < 96 + n) ? QOFF + (g - 96) * ld : n * ld;
  }
  const int bc = t - 128;  // block column of the lanes of wave 2
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
    // first column of (H - s1)(H - s2) restricted to rows l..l+2
    const double x = H[l * ld + l] * H[l * ld + l] + H[l * ld + l + 1] * H[(l + 1) * ld + l] -
                     tr * H[l * ld + l] + det;
    const double y = H[(l + 1) * ld + l] * (H[l * ld + l] + H[(l + 1) * ld + l + 1] - tr);
    const double z = H[(l + 1) * ld + l] * H[(l + 2) * ld + l + 1];
    double tau = 0.0, v1 = 0.0, v2 = 0.0, s3 = 0.0;
    if (wv == 3) {
      householder3(x, y, z, tau, v1, v2);
      if (t == 192) {
        refl[(l & 1) * 4 + 0] = tau;
        refl[(l & 1) * 4 + 1] = v1;
        refl[(l & 1) * 4 + 2] = v2;
      }
      const int r = (l + 3 <= n) ? l + 3 : n, c = (l + 2 <= n) ? l + 2 : n;
      s3 = H[r * ld + c];
    }
    __syncthreads();
    for (int k = l; k <= hi - 1; ++k) {
      const bool three = (k < hi - 1);
      const int nr = three ? 3 : 2;
      double q0 = 0.0, q1 = 0.0, q2 = 0.0, sw = 0.0, w1 = 0.0, w2 = 0.0;
      if (wv < 2) {
        const int ihi = (k + 3 < hi) ? k + 3 : hi;
        const double* rf = refl + (k & 1) * 4;
        const double ta = rf[0], u1 = rf[1], u2 = rf[2];
        const int kld = k * ld;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int g = t + 128 * u;
          const bool isR = isH[u] && (g <= ihi);
          const bool vR = isR && ((unsigned)(g - k) >= (unsigned)nr);
          const bool vL = !isR && lok[u] && ((unsigned)(jL[u] - k) >= (unsigned)nr);
          const int base = vR ? tld[u] + k : vL ? kld + jL[u] : bQ[u] + k;
          const int str = vL ? ld : 1;
          const bool zs = vL && (jL[u] == k - 1);  // the bulge column: rows k+1, k+2 vanish
          const double a0 = H[base], a1 = H[base + str], a2 = H[base + 2 * str];
          const double sm = ta * (a0 + u1 * a1 + u2 * a2);
          H[base] = a0 - sm;
          H[base + str] = zs ? 0.0 : a1 - sm * u1;
          H[base + 2 * str] = zs ? 0.0 : a2 - sm * u2;
        }
      } else if (wv == 2) {
        if (bc < nr) {  // column bc of P B P = P (B p_bc)
          const double* rf = refl + (k & 1) * 4;
          const double ta = rf[0];
          w1 = rf[1];
          w2 = rf[2];
          const double* Bp = H + k * ld + k;
          const double bv0 = Bp[0] + w1 * Bp[1] + w2 * Bp[2];
          const double bv1 = Bp[ld] + w1 * Bp[ld + 1] + w2 * Bp[ld + 2];
          const double bv2 = Bp[2 * ld] + w1 * Bp[2 * ld + 1] + w2 * Bp[2 * ld + 2];
          const double vc = (bc == 0) ? 1.0 : (bc == 1) ? w1 : w2;
          const double tv = ta * vc;
          q0 = Bp[bc] - tv * bv0;
          q1 = Bp[ld + bc] - tv * bv1;
          q2 = Bp[2 * ld + bc] - tv * bv2;
          sw = ta * (q0 + w1 * q1 + w2 * q2);
        }
      } else {
        // column 0 of P B P below the diagonal and the right-updated row
        // below the block give the next step's x, y, z
        const double* Bp = H + k * ld + k;
        const double b00 = Bp[0], b01 = Bp[1], b02 = Bp[2];
        const double b10 = Bp[ld], b11 = Bp[ld + 1], b12 = Bp[ld + 2];
        const double b20 = Bp[2 * ld], b21 = Bp[2 * ld + 1], b22 = Bp[2 * ld + 2];
        double s3n;
        {
          const int r = (k + 4 <= n) ? k + 4 : n, c = (k + 3 <= n) ? k + 3 : n;
          s3n = H[r * ld + c];
        }
        const double bv0 = b00 + v1 * b01 + v2 * b02;
        const double bv1 = b10 + v1 * b11 + v2 * b12;
        const double bv2 = b20 + v1 * b21 + v2 * b22;
        const double d0 = b00 - tau * bv0, d1 = b10 - tau * bv1, d2 = b20 - tau * bv2;
        const double sd = tau * (d0 + v1 * d1 + v2 * d2);
        const double sm3 = tau * (v2 * s3);
        const bool th = (k + 1 < hi - 1);
        householder3(d1 - sd * v1, d2 - sd * v2, th ? -sm3 : 0.0, tau, v1, v2);
        if (t == 192) {
          refl[((k + 1) & 1) * 4 + 0] = tau;
          refl[((k + 1) & 1) * 4 + 1] = v1;
          refl[((k + 1) & 1) * 4 + 2] = v2;
        }
        s3 = s3n;
      }
      __syncthreads();  // every read of the block region is done
      if (wv == 2 && bc < nr) {
        double* Op = H + k * ld + k + bc;
        Op[0] = q0 - sw;
        Op[ld] = q1 - sw * w1;
        if (three) Op[2 * ld] = q2 - sw * w2;
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
  extern __shared__ __attribute__((aligned(16))) double sm[];
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
  load_square(gH, H, n, ld);
  load_square(gQ, Q, n, ld);
  __syncthreads();
  __shared__ double red[kQR / 64];
  const double hn = block_fro(H, n, ld, red);
  if (t == 0) st->tphase[4] = clock64();
  int sweeps = 0, steps = 0;
  __shared__ double refl[8];
  const bool ok = francis_qr(H, Q, n, ld, hn > 0.0 ? hn : 1.0, &sweeps, &steps, refl);
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
  store_square(H, oH, n, ld);
  store_square(Q, oQ, n, ld);
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
  extern __shared__ __attribute__((aligned(16))) double sm[];
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
  load_square(b.work + n * n, T, n, ld);
  load_square(b.work + 2 * n * n, Q, n, ld);
  __syncthreads();
  __shared__ double red[kNT / 64];
  const double hn = block_fro(T, n, ld, red);
  if (t == 0) st->tphase[6] = clock64();
  // eigenvalues tau from the 1x1 and 2x2 blocks; a complex block's leader
  // is the member with Im tau < 0 (its xi has Im > 0).  In the real Schur
  // form the QR returns no two consecutive subdiagonal entries are
  // nonzero, so every position classifies itself; the walk from the top
  // by one lane remains for a form that breaks this.
  __shared__ int nzsub[kMaxM + 1];
  for (int q = t; q < n; q += kNT) nzsub[q] = (q + 1 < n && T[(q + 1) * ld + q] != 0.0);
  __syncthreads();
  int bad = 0;
  for (int q = t; q + 1 < n; q += kNT) bad |= (nzsub[q] && nzsub[q + 1]);
  bad = __syncthreads_or(bad);
  if (!bad) {
    for (int q = t; q < n; q += kNT) {
      if (nzsub[q]) {
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
      } else if (!(q > 0 && nzsub[q - 1])) {
        tre[q] = T[q * ld + q];
        tim[q] = 0.0;
        unitsz[q] = 1;
      }
    }
  } else if (t == 0) {
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
  // units by rank, and xi by rank for the host (zero past the last unit)
  int isunit = 0;
  for (int q = t; q < n; q += kNT)
    if (unitsz[q]) {
      order[rnk[q]] = q;
      ++isunit;
      const int rk = rnk[q];
      if (rk < m) {
        b.xi[rk] = (kya[q] < INFINITY) ? kyb[q] : INFINITY;
        b.xi[m + rk] = -kyc[q];
      }
    }
  static_assert(kMaxM <= kNT, "one slot per lane");
  const int nu = __syncthreads_count(isunit);  // isunit is 0 or 1
  for (int r = nu + t; r < m; r += kNT) {
    b.xi[r] = 0.0;
    b.xi[m + r] = 0.0;
  }
  if (t == 0) {
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

    st->tphase[7] = clock64();
  }
  __syncthreads();
  const int nsel = nsel_s;
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
  // Q <- L^-T Q (solve L^T Y = Q), with L staged in the T region (free
  // after the back substitution); right-looking from the last row, the
  // rows unscaled until the end (step i subtracts L[i][r] / L[i][i] times
  // row i from the rows above it): one barrier per row
  double* Ls = T;
  load_square(L, Ls, n, ld);
  __syncthreads();
  for (int i = t; i < n; i += kNT) kyc[i] = 1.0 / Ls[i * ld + i];
  __syncthreads();
  for (int i = n - 1; i >= 0; --i) {
    const double inv = kyc[i];
    for (int r = ty; r < i; r += 16) {
      const double f = Ls[i * ld + r] * inv;
      for (int c = tx; c < n; c += 16) Q[r * ld + c] -= f * Q[i * ld + c];
    }
    __syncthreads();
  }
  for (int i = ty; i < n; i += 16) {
    const double inv = kyc[i];
    for (int c = tx; c < n; c += 16) Q[i * ld + c] *= inv;
  }
  __syncthreads();
  // y = (L^-T Q) x: real parts into the T region (L is no longer needed),
  // then imaginary parts into the Xre region (free once the real parts
  // are formed)
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
  (void)m;
  (void)kint;
  const void* f[6] = {(const void*)k_tharm_reduce,  (const void*)k_tharm_reduce_b,
                      (const void*)k_tharm_qr,      (const void*)k_tharm_qr_b,
                      (const void*)k_tharm_vectors, (const void*)k_tharm_vectors_b};
  for (const void* k : f) {
    const hipError_t e = set_lds_limit(k);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Largest dynamic LDS the three kernels ask for at (m, kint).
size_t tharm_lds_bytes(int m, int kint) {
  return std::max(reduce_lds(m), std::max(qr_lds(m), vectors_lds(m, kint)));
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
