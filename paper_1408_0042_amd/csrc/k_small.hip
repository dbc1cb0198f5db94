// Small dense kernels of the PLHR iteration, each one workgroup with all
// operands in LDS (m = 4 (k + k_extra) slots, m <= kMaxM = 84).
//
//   k_init_lam     Rayleigh quotients of the start block (Algorithm 3, step 2)
//   k_conv_check   relative residuals, soft locking, stopping test
//   k_ortho_small  Cholesky of the Gram matrix of Z = [V W S P] with column
//                  scaling and dropping of dependent W/S/P columns; returns
//                  M with Zhat = Z M B-orthonormal (Section 4: V, W, S, P
//                  are orthonormalised in this order, which is what a
//                  Cholesky factorisation of the Gram matrix in slot order
//                  computes); 256 threads, 1024 from m = 48
//   (the projected problem eq. (3.5) and the selection of Algorithm 3 are
//   in k_tharm.hip and k_tharm_sym.hip; the complex steps of Algorithms 1
//   and 2 in k_complex_small.hip, the PLMR refinement in k_single.hip)
//   k_rq_small     Rayleigh quotients of the new block, eq. (4.1) for pairs
//   k_final_rr     standard Rayleigh-Ritz on span(V) (the last step of
//                  Algorithms 2 and 3): Cholesky + cyclic Jacobi
//   k_final_res    relative residuals of the returned pairs
#include <cmath>

#include "common.cuh"

namespace plhr {

// rows (or columns) of an m x m matrix, m <= kMaxM, a lane of a 16 x 16
// thread tile visits with stride 16
constexpr int kOrthoSpan = (kMaxM + 15) / 16;

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
  if (s < per) {
    // eight loads in flight, added in the same order as one at a time
    int q = s;
    for (; q + 7 * per < nblk; q += 8 * per) {
      double w[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) w[u] = part[(size_t)(q + u * per) * nv + v];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += w[u];
    }
    for (; q < nblk; q += per) acc += part[(size_t)q * nv + v];
  }
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
__device__ void k_init_lam_body(SmallParams p, const double* __restrict__ part, int nblk,
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
    if (p.cplx) {  // complex vectors: columns 2j (re) and 2j + 1 (im)
      const int o = c ^ 1;
      b.lam[c] = p.sigma + (vq + sums[p.kint + o]) / (vv + sums[o]);
      b.kinds[c] = (c & 1) ? 3 : 1;
      b.pair[c] = o;
    }
  }
  if (c == 0) {
    st->done = 0;
    st->error = 0;
    st->iter = 0;
    st->have_p = 0;
    st->n_active = p.kint;
    st->m_kept = 0;
    st->n_dropped = 0;
    st->n_excluded = 0;
    st->max_rel_res = 0.0;
  }
}

__global__ __launch_bounds__(256) void k_init_lam(SmallParams p, const double* __restrict__ part, int nblk,
                           SmallBufs b, DevStatus* st) {
  k_init_lam_body(p, part, nblk, b, st);
}
// batched: workgroup b runs problem b
__global__ __launch_bounds__(256) void k_init_lam_b(const BatchSmall* __restrict__ bs) {
  const BatchSmall& q = bs[blockIdx.x];
  k_init_lam_body(q.p, q.part, q.nblk, q.b, q.st);
}


// Rank test of the start block: scaled Cholesky of G = V0^T B V0 (kint x
// kint, in b.G); a pivot below drop_tol means linearly dependent columns.
__device__ void k_start_check_body(SmallParams p, SmallBufs b, DevStatus* st) {
  if (threadIdx.x != 0) return;
  if (p.cplx) {  // no complex start vector may vanish (the complex
                 // orthonormalisation drops dependent ones later)
    for (int j = 0; 2 * j < p.kint; ++j) {
      const double g = b.G[(2 * j) * p.kint + 2 * j] + b.G[(2 * j + 1) * p.kint + 2 * j + 1];
      if (!(g > 0.0 && g < INFINITY)) {
        st->error = PLHR_ERR_BREAKDOWN;
        st->reason = kReasonStartRank;
      }
    }
    return;
  }
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

__global__ __launch_bounds__(64) void k_start_check(SmallParams p, SmallBufs b, DevStatus* st) {
  k_start_check_body(p, b, st);
}
// batched: workgroup b runs problem b
__global__ __launch_bounds__(64) void k_start_check_b(const BatchSmall* __restrict__ bs) {
  const BatchSmall& q = bs[blockIdx.x];
  k_start_check_body(q.p, q.b, q.st);
}


// ------------------------------------------------------- convergence test
__device__ void k_conv_check_body(SmallParams p, const double* __restrict__ part, int nblk,
                             SmallBufs b, DevStatus* st) {
  if (halted(st)) return;
  __shared__ double rel[128];
  __shared__ double red[256], sums[128];
  const int c = threadIdx.x;
  const int kint = p.kint;
  sum_partials(part, nblk, 2 * kint, sums, red);
  if (c < kint) {
    double rr = sums[c], vv = sums[kint + c];
    if (p.cplx) {  // residual and norm of the complex vector
      rr = sums[c] + sums[c ^ 1];
      vv = sums[kint + c] + sums[kint + (c ^ 1)];
    }
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
    rel[64 + c] = (rank < p.k || p.cplx == 1) ? 1.0 : 0.0;  // wanted flag
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

__global__ __launch_bounds__(256) void k_conv_check(SmallParams p, const double* __restrict__ part, int nblk,
                             SmallBufs b, DevStatus* st) {
  k_conv_check_body(p, part, nblk, b, st);
}
// batched: workgroup b runs problem b
__global__ __launch_bounds__(256) void k_conv_check_b(const BatchSmall* __restrict__ bs) {
  const BatchSmall& q = bs[blockIdx.x];
  k_conv_check_body(q.p, q.part, q.nblk, q.b, q.st);
}


// --------------------------------------------- Cholesky-QR in slot order
// LDS: Gs (m x m, Cholesky factor R in the upper triangle) | X (m x m,
// R^-1) | d (m)
// smallest pivot of the column-scaled Gram (squared relative norm of a
// column's part orthogonal to the earlier ones) below which one pass loses
// more than ~eps / pivot of B-orthogonality and a second pass is run
constexpr double kOrthoRedo = 1e-4;

__device__ void k_ortho_small_body(SmallParams p, SmallBufs b, DevStatus* st) {
  if (halted(st)) {
    if (p.pass == 1 && b.gate && threadIdx.x == 0) b.gate->done = 1;
    return;
  }
  if (p.pass == 2 && b.gate && b.gate->done) return;
  extern __shared__ __attribute__((aligned(16))) double sm[];
  const int m = p.m, kint = p.kint;
  double* Gs = sm;
  double* X = Gs + m * m;
  double* d = X + m * m;
  __shared__ int valid[256];
  __shared__ int flag;
  const int t = threadIdx.x, nt = blockDim.x;
  const int tx = t & 15, ty = t >> 4, nty = nt >> 4;  // 16 columns x nty rows of threads
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
#pragma unroll
  for (int a = 0; a < kOrthoSpan; ++a) {
    const int i = ty + nty * a;
    if (i < m) {
      double g[kOrthoSpan];
#pragma unroll
      for (int q = 0; q < kOrthoSpan; ++q) {  // loads first, then the uses
        const int j = tx + 16 * q;
        g[q] = (j < m) ? b.G[i * m + j] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < kOrthoSpan; ++q) {
        const int j = tx + 16 * q;
        if (j < m) {
          const int e = i * m + j;
          Gs[e] = (valid[i] && valid[j]) ? g[q] * d[i] * d[j] : 0.0;
          X[e] = (i == j) ? 1.0 : 0.0;
        }
      }
    }
  }
  if (t < kint && valid[t]) flag = 1;
  __syncthreads();
  if (!flag) {  // every V column vanished
    if (t == 0) {
      st->error = PLHR_ERR_BREAKDOWN;
      st->reason = kReasonVVanished;
    }
    return;
  }
  // right-looking Cholesky in slot order; a numerically dependent column
  // (V included) adds nothing to span(Z) and is dropped.  Rows of R stay
  // unscaled during the elimination (the update of step j divides by the
  // pivot): it is Gaussian elimination E G = U = D L^T with E = L^-1 unit
  // lower triangular, R = D^1/2 L^T, so R^-1 = E^T D^-1/2.  The same row
  // operations applied to X = I build E alongside (row j of E is final at
  // step j): one barrier per kept column and no separate inversion.  A
  // dropped column takes no barrier: the decision is uniform, column j is
  // read by no later step, and column j of E stays e_j.
  __shared__ double rsc[256];  // 1/sqrt(pivot) of each kept slot
  double minpiv = INFINITY;    // (thread 0) smallest kept pivot
  for (int j = 0; j < m; ++j) {
    if (!valid[j]) continue;
    const double piv = Gs[j * m + j];
    if (!(piv > p.drop_tol)) {
      if (t == 0) valid[j] = 0;
      continue;
    }
    minpiv = fmin(minpiv, piv);
    const double ip = 1.0 / piv;
    if (t == 0) rsc[j] = piv;  // 1 / sqrt(pivot) after the loop, by all lanes
    // rows and columns of slots left out at the start are exact zeros and
    // stay zero under the update, and a column dropped at step j' is read
    // by no later step: no per-element test of `valid` is needed
    // (trip counts from the live sizes: an unrolled loop over the widest
    // span issues the predicated-off combinations too, which at small m
    // cost more than the updates)
    const double* gj = Gs + j * m;
    const double* ej = X + j * m;
    for (int i = j + 1 + ty; i < m; i += nty) {
      const double gji = gj[i] * ip;
      double* gi = Gs + i * m;
      double* ei = X + i * m;
      for (int l = i + tx; l < m; l += 16) gi[l] -= gji * gj[l];
      for (int cc = tx; cc <= j; cc += 16) ei[cc] -= gji * ej[cc];
    }
    __syncthreads();
  }
  for (int j = t; j < m; j += nt)
    if (valid[j]) rsc[j] = 1.0 / sqrt(rsc[j]);
  __syncthreads();
  // M = D R^-1 = D E^T D_piv^-1/2 on the kept slots, zero elsewhere
  for (int i = ty; i < m; i += nty)
    for (int c = tx; c < m; c += 16)
      b.M[(size_t)i * m + c] =
          (valid[i] && valid[c] && c >= i) ? d[i] * X[c * m + i] * rsc[c] : 0.0;
  for (int s = t; s < m; s += nt) b.keep[s] = valid[s];
  if (t == 0) {
    int nk = 0, nd = 0;
    for (int s = 0; s < m; ++s) {
      nk += valid[s];
      if (!valid[s] && slot_valid(s, kint, b.active, have_p)) ++nd;
    }
    st->m_kept = nk;
    st->n_dropped = nd;
    if (p.pass == 1 && b.gate) {
      b.gate->error = 0;
      b.gate->done = (minpiv < kOrthoRedo) ? 0 : 1;
    }
  }
}

__global__ __launch_bounds__(1024) void k_ortho_small(SmallParams p, SmallBufs b, DevStatus* st) {
  k_ortho_small_body(p, b, st);
}
// batched: workgroup b runs problem b
__global__ __launch_bounds__(256) void k_ortho_small_b(const BatchSmall* __restrict__ bs) {
  const BatchSmall& q = bs[blockIdx.x];
  k_ortho_small_body(q.p, q.b, q.st);
}


// --------------------------------------------------- Rayleigh quotients
// part: nblk x 2kint, [v.v | v.(A - sigma B) v]
__device__ void k_rq_small_body(SmallParams p, const double* __restrict__ part, int nblk,
                           SmallBufs b, DevStatus* st, int end_of_iteration) {
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
  if (c == 0 && end_of_iteration) {
    st->iter += 1;
    st->have_p = 1;
  }
}

__global__ __launch_bounds__(256) void k_rq_small(SmallParams p, const double* __restrict__ part, int nblk,
                           SmallBufs b, DevStatus* st, int end_of_iteration) {
  k_rq_small_body(p, part, nblk, b, st, end_of_iteration);
}
// batched: workgroup b runs problem b
__global__ __launch_bounds__(256) void k_rq_small_b(const BatchSmall* __restrict__ bs, int end_of_iteration) {
  const BatchSmall& q = bs[blockIdx.x];
  k_rq_small_body(q.p, q.part, q.nblk, q.b, q.st, end_of_iteration);
}


static constexpr int kTh = 64;  // one wavefront

// ------------------------------------------------- final Rayleigh-Ritz
// HM: kint x 2kint = [V^T (A - sigma B) V | V^T B V]
__device__ void k_final_rr_body(SmallParams p, const double* __restrict__ HM,
                                                  SmallBufs b, DevStatus* st) {
  extern __shared__ __attribute__((aligned(16))) double sm[];
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
  // M and C scaled to unit diagonal of M; Cholesky of M in column order
  // with the trial-space dropping rule: a column of V that is numerically
  // dependent on the earlier ones (two columns converged to the same
  // eigenvector) is left out: its row and column of L become e_j and those
  // of C zero, so it yields an eigenvalue that the ordering skips and no
  // component in the other eigenvectors.  Fewer than k independent columns
  // is a breakdown.
  __shared__ int drop[128];
  __shared__ double dsc[128];
  // When at least k columns met the tolerance, the columns that did not
  // (guard columns still converging) are left out as well: a guard column
  // that shares a multiple eigenvalue with wanted pairs would otherwise be
  // mixed into the returned vectors by the rotation within that cluster.
  __shared__ int excl[128];
  __shared__ int nconv_s;
  if (t == 0) {
    int cnv = 0;
    for (int j = 0; j < n; ++j) cnv += (b.relres[j] <= p.tol) ? 1 : 0;
    nconv_s = cnv;
  }
  __syncthreads();
  for (int j = t; j < n; j += kTh) {
    const double g = L[j * n + j];
    dsc[j] = (g > 0.0 && g < INFINITY) ? 1.0 / sqrt(g) : 0.0;
    excl[j] = (nconv_s >= k && !(b.relres[j] <= p.tol)) ? 1 : 0;
  }
  __syncthreads();
  for (int e = t; e < n * n; e += kTh) {
    const int i = e / n, j = e - i * n;
    const double f = dsc[i] * dsc[j];
    L[e] *= f;
    C[e] *= f;
  }
  __syncthreads();
  int nkept = 0;
  for (int j = 0; j < n; ++j) {
    const double piv = L[j * n + j];
    __syncthreads();
    if (!(piv > p.drop_tol) || excl[j]) {  // uniform
      for (int i = t; i < n; i += kTh) {
        if (i > j) L[i * n + j] = 0.0;
        if (i < j) L[j * n + i] = 0.0;
        C[i * n + j] = 0.0;
        C[j * n + i] = 0.0;
      }
      if (t == 0) {
        L[j * n + j] = 1.0;
        drop[j] = 1;
      }
      __syncthreads();
      continue;
    }
    ++nkept;
    if (t == 0) drop[j] = 0;
    const double d = sqrt(piv);
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
  if (nkept < k) {  // uniform
    if (t == 0) {
      st->error = PLHR_ERR_NOT_HPD;
      st->reason = kReasonFinalGram;
    }
    return;
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
  for (int i = t; i < n; i += kTh) ev[i] = drop[i] ? INFINITY : C[i * n + i];
  __syncthreads();
  // X = D L^-T U (in U): back substitution per column, then the scaling
  for (int c = t; c < n; c += kTh)
    for (int i = n - 1; i >= 0; --i) {
      double s = U[i * n + c];
      for (int q = i + 1; q < n; ++q) s -= L[q * n + i] * U[q * n + c];
      U[i * n + c] = s / L[i * n + i];
    }
  __syncthreads();
  for (int e = t; e < n * n; e += kTh) U[e] *= dsc[e / n];
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

__global__ __launch_bounds__(kTh) void k_final_rr(SmallParams p, const double* __restrict__ HM,
                                                  SmallBufs b, DevStatus* st) {
  k_final_rr_body(p, HM, b, st);
}
// batched: workgroup b runs problem b
__global__ __launch_bounds__(kTh) void k_final_rr_b(const BatchSmall* __restrict__ bs) {
  const BatchSmall& q = bs[blockIdx.x];
  k_final_rr_body(q.p, q.HM, q.b, q.st);
}


// relative residuals of the returned pairs from column sums
__device__ void k_final_res_body(SmallParams p, const double* __restrict__ part, int nblk,
                            SmallBufs b) {
  __shared__ double red[256], sums[128];
  const int c = threadIdx.x, k = p.k;
  sum_partials(part, nblk, 2 * k, sums, red);
  if (c < k) {
    double rr = sums[c], vv = sums[k + c];
    if (p.cplx == 2) {  // complex Ritz vectors: columns 2j, 2j + 1
      rr += sums[c ^ 1];
      vv += sums[k + (c ^ 1)];
    }
    const double lam = b.final_theta[c];
    b.relres[c] = sqrt(rr) / ((p.normA1 + fabs(lam) * p.normB1) * sqrt(vv));
    b.vbv[c] = vv;
  }
}

__global__ __launch_bounds__(256) void k_final_res(SmallParams p, const double* __restrict__ part, int nblk,
                            SmallBufs b) {
  k_final_res_body(p, part, nblk, b);
}
// batched: workgroup b runs problem b
__global__ __launch_bounds__(256) void k_final_res_b(const BatchSmall* __restrict__ bs) {
  const BatchSmall& q = bs[blockIdx.x];
  k_final_res_body(q.p, q.part, q.nblk, q.b);
}


// ------------------------------------------ fused residual step (small n)
// One workgroup for a small problem with B = I: the column sums v.v and
// v.(A - sigma)v, the Rayleigh quotients, the residual block
// R = (A - sigma)V - V (Lam - sigma) with its column sums r.r and v.v, and
// the convergence test, in one launch instead of four.  Each column's sums
// are formed by a fixed group of threads in a fixed order and passed to the
// quotient and test bodies as a single partial block.
__global__ __launch_bounds__(256) void k_vstep_small(SmallParams p, size_t n,
                                                     const double* __restrict__ V, int ldv,
                                                     const double* __restrict__ QV, int ldq,
                                                     double* R, int ldr, double* part, SmallBufs b,
                                                     DevStatus* st) {
  if (halted(st)) return;
  __shared__ double red2[2][256];
  const int kint = p.kint, t = threadIdx.x;
  const int per = 256 / kint, c = t % kint, g = t / kint;
  auto column_sums = [&](double a0, double a1) {
    red2[0][t] = a0;
    red2[1][t] = a1;
    __syncthreads();
    if (t < kint) {
      double s0 = 0.0, s1 = 0.0;
      for (int q = 0; q < per; ++q) {
        s0 += red2[0][q * kint + t];
        s1 += red2[1][q * kint + t];
      }
      part[t] = s0;
      part[kint + t] = s1;
    }
    __threadfence_block();
    __syncthreads();
  };
  // eight rows of a thread in flight at a time, added in row order
  double a0 = 0.0, a1 = 0.0;
  if (g < per) {
    size_t r = g;
    for (; r + 7 * (size_t)per < n; r += 8 * (size_t)per) {
      double v[8], q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        v[u] = V[(r + u * per) * ldv + c];
        q[u] = QV[(r + u * per) * ldq + c];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a0 += v[u] * v[u];
        a1 += v[u] * q[u];
      }
    }
    for (; r < n; r += per) {
      const double v = V[r * ldv + c], q = QV[r * ldq + c];
      a0 += v * v;
      a1 += v * q;
    }
  }
  column_sums(a0, a1);
  k_rq_small_body(p, part, 1, b, st, 0);
  __threadfence_block();
  __syncthreads();
  const double sh = b.lam[c] - p.sigma;
  a0 = 0.0;
  a1 = 0.0;
  if (g < per) {
    size_t r = g;
    for (; r + 7 * (size_t)per < n; r += 8 * (size_t)per) {
      double v[8], q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        v[u] = V[(r + u * per) * ldv + c];
        q[u] = QV[(r + u * per) * ldq + c];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double rr = q[u] - v[u] * sh;
        R[(r + u * per) * ldr + c] = rr;
        a0 += rr * rr;
        a1 += v[u] * v[u];
      }
    }
    for (; r < n; r += per) {
      const double v = V[r * ldv + c];
      const double rr = QV[r * ldq + c] - v * sh;
      R[r * ldr + c] = rr;
      a0 += rr * rr;
      a1 += v * v;
    }
  }
  column_sums(a0, a1);
  k_conv_check_body(p, part, 1, b, st);
}

bool vstep_small_ok(size_t n, int kint) { return kint <= 64 && n * (size_t)kint <= 32768; }

void launch_vstep_small(const SmallParams& p, size_t n, const double* V, int ldv,
                        const double* QV, int ldq, double* R, int ldr, double* part,
                        SmallBufs b, DevStatus* st, hipStream_t s) {
  prof_begin(KC_SMALL, (double)n * p.kint * 8.0 * 5.0, 0.0, s);
  hipLaunchKernelGGL(k_vstep_small, dim3(1), dim3(256), 0, s, p, n, V, ldv, QV, ldq, R, ldr, part,
                     b, st);
  prof_end(KC_SMALL, s);
}

// ------------------------------------------------------------ launchers
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
static int ortho_threads(int m) { return (m >= 48) ? 1024 : 256; }

void launch_ortho_small(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s) {
  const size_t lds = ((size_t)2 * p.m * p.m + p.m) * sizeof(double);
  // model count: Cholesky m^3/3, inverse of the factor m^3/3, scaling
  const double m3 = (double)p.m * p.m * p.m;
  prof_begin(KC_ORTHO, 2.0 * p.m * p.m * 8.0, 2.0 * m3 / 3.0, s);
  // wider bases take more rows of threads: the elimination's work per
  // step grows as m^2, its chain of steps as m
  hipLaunchKernelGGL(k_ortho_small, dim3(1), dim3(ortho_threads(p.m)), lds, s, p, b, st);
  prof_end(KC_ORTHO, s);
}
void launch_rq_small(const SmallParams& p, const double* part, int nblk, SmallBufs b,
                     DevStatus* st, int end_of_iteration, hipStream_t s) {
  prof_begin(KC_SMALL, 0.0, 0.0, s);
  hipLaunchKernelGGL(k_rq_small, dim3(1), dim3(256), 0, s, p, part, nblk, b, st,
                     end_of_iteration);
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

// out[c] = the first of the two column sums of launch_xdots, c < k
// (k <= 64): u^* u of the returned vectors in the variables where B = I.
__global__ __launch_bounds__(256) void k_colsum_first(const double* __restrict__ part, int nblk,
                                                      int k, double* __restrict__ out) {
  __shared__ double red[256], sums[128];
  sum_partials(part, nblk, 2 * k, sums, red);
  if ((int)threadIdx.x < k) out[threadIdx.x] = sums[threadIdx.x];
}

void launch_colsum_first(const double* part, int nblk, int k, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum_first, dim3(1), dim3(256), 0, s, part, nblk, k, out);
}

// ---------------------------------------------------------------- batched
void launch_init_lam_b(const BatchSmall* bs, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_init_lam_b, dim3(nb), dim3(256), 0, s, bs);
}
void launch_start_check_b(const BatchSmall* bs, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_start_check_b, dim3(nb), dim3(64), 0, s, bs);
}
void launch_conv_check_b(const BatchSmall* bs, int nb, hipStream_t s) {
  prof_begin(KC_SMALL, 0.0, 0.0, s);
  hipLaunchKernelGGL(k_conv_check_b, dim3(nb), dim3(256), 0, s, bs);
  prof_end(KC_SMALL, s);
}
void launch_ortho_small_b(const BatchSmall* bs, int nb, int m, hipStream_t s) {
  const size_t lds = ((size_t)2 * m * m + m) * sizeof(double);
  const double m3 = (double)m * m * m;
  prof_begin(KC_ORTHO, nb * 2.0 * m * m * 8.0, nb * 2.0 * m3 / 3.0, s);
  hipLaunchKernelGGL(k_ortho_small_b, dim3(nb), dim3(256), lds, s, bs);
  prof_end(KC_ORTHO, s);
}
void launch_rq_small_b(const BatchSmall* bs, int nb, int end_of_iteration, hipStream_t s) {
  prof_begin(KC_SMALL, 0.0, 0.0, s);
  hipLaunchKernelGGL(k_rq_small_b, dim3(nb), dim3(256), 0, s, bs, end_of_iteration);
  prof_end(KC_SMALL, s);
}
void launch_final_rr_b(const BatchSmall* bs, int nb, int kint, hipStream_t s) {
  const size_t lds = (3 * (size_t)kint * kint + kint) * sizeof(double);
  hipLaunchKernelGGL(k_final_rr_b, dim3(nb), dim3(kTh), lds, s, bs);
}
void launch_final_res_b(const BatchSmall* bs, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_final_res_b, dim3(nb), dim3(256), 0, s, bs);
}

hipError_t small_set_attributes(int m, int kint) {
  hipError_t e = tharm_set_attributes(m, kint);
  if (e != hipSuccess) return e;
  e = set_lds_limit((const void*)k_ortho_small_b);
  if (e != hipSuccess) return e;
  return set_lds_limit((const void*)k_ortho_small);
}

}  // namespace plhr
