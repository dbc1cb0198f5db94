// Batched kernels: many independent 2-D problems (5-point Dirichlet
// stencil with a potential, one V-cycle per problem) advanced by the same
// launches.  Every launch covers all problems; a workgroup finds its
// problem through a table built on the host:
//   * row kernels (stencil, V-cycle levels): one workgroup per grid row,
//     RowMap[blockIdx] = (problem, row);
//   * point-range kernels (column sums, Grams, row products, copies):
//     Chunk[blockIdx] = (problem, first point, end point), chunks never
//     straddle two problems, and the partial sums of chunk c go to slot c
//     so that problem b reduces the contiguous slots of its own chunks.
// Problems are packed point-major one after another; problem b's points
// start at BProb::off (level 0) and BLev::off (coarser levels).  A
// workgroup of a converged or failed problem returns at once.
#include <cstdint>

#include "mfma.cuh"

namespace plhr {

// -------------------------------------------------------------- stencil
// out = (A_b - shift_b I) X on the problem's grid; optional epilogues as
// in the single-problem kernel: outr = out - X (lam_b - sigma_b), outc = out.
__global__ __launch_bounds__(256) void k_fd_b(const RowMap* __restrict__ rm,
                                              const BProb* __restrict__ pr, double diag,
                                              double off, int use_sigma,
                                              const double* __restrict__ X, int ldx,
                                              double* __restrict__ out, int ldo,
                                              double* __restrict__ outr, int ldr,
                                              double* __restrict__ outc, int ldc, int ncols) {
  const RowMap q = rm[blockIdx.x];
  const BProb& P = pr[q.b];
  if (halted(P.st)) return;
  const int nx = P.nx, ny = P.ny, j = q.j;
  const double shift = use_sigma ? P.sigma : 0.0;
  const size_t rowp = P.off + (size_t)j * nx;
  const ptrdiff_t sy = (ptrdiff_t)nx * ldx;
  const int P_ = blockDim.x / ncols, c = threadIdx.x % ncols, i0 = threadIdx.x / ncols;
  if (i0 >= P_) return;
  const double cs = outr ? P.lam[c] - P.sigma : 0.0;
  for (int i = i0; i < nx; i += P_) {
    const size_t p = rowp + i;
    const double* xp = X + p * ldx + c;
    const double xc = xp[0];
    double nb = 0.0;
    if (i > 0) nb += xp[-ldx];
    if (i < nx - 1) nb += xp[ldx];
    if (j > 0) nb += xp[-sy];
    if (j < ny - 1) nb += xp[sy];
    double d = diag - shift;
    if (P.pot) d += P.pot[p - P.off];
    const double y = d * xc + off * nb;
    out[p * ldo + c] = y;
    if (outr) outr[p * ldr + c] = y - xc * cs;
    if (outc) outc[p * ldc + c] = y;
  }
}

// ------------------------------------------------------------- V-cycle
// Level l of every problem: grid lv[b].nx x lv[b].ny at point offset
// lv[b].off of the packed level arrays (ld ncols).  The level-0 input and
// outputs are packed with the problems' level-0 offsets and their own
// leading dimensions.
__global__ __launch_bounds__(256) void k_jacobi_b(const RowMap* __restrict__ rm,
                                                  const BLev* __restrict__ lv,
                                                  const BProb* __restrict__ pr, double diag,
                                                  double off, double omega,
                                                  const double* __restrict__ xin,
                                                  const double* __restrict__ r, int ldr,
                                                  double* __restrict__ o0, int ld0,
                                                  double* __restrict__ o1, int ld1, int split,
                                                  int ncols) {
  const RowMap q = rm[blockIdx.x];
  if (halted(pr[q.b].st)) return;
  const BLev L = lv[q.b];
  const int nx = L.nx, ny = L.ny, j = q.j;
  const size_t rowp = L.off + (size_t)j * nx;
  const ptrdiff_t sy = (ptrdiff_t)nx * ncols;
  const int P_ = blockDim.x / ncols, c = threadIdx.x % ncols, i0 = threadIdx.x / ncols;
  if (i0 >= P_) return;
  const double w = omega / diag;
  double* const ob = (c < split) ? o0 + c : o1 + (c - split);
  const int ldo = (c < split) ? ld0 : ld1;
  for (int i = i0; i < nx; i += P_) {
    const size_t p = rowp + i;
    const double rv = r[p * ldr + c];
    double v;
    if (xin) {
      const double* xp = xin + p * ncols + c;
      const double xc = xp[0];
      double nb = 0.0;
      if (i > 0) nb += xp[-ncols];
      if (i < nx - 1) nb += xp[ncols];
      if (j > 0) nb += xp[-sy];
      if (j < ny - 1) nb += xp[sy];
      v = xc + w * (rv - (diag * xc + off * nb));
    } else {
      v = w * rv;
    }
    ob[p * ldo] = v;
  }
}

__global__ __launch_bounds__(256) void k_residual_b(const RowMap* __restrict__ rm,
                                                    const BLev* __restrict__ lv,
                                                    const BProb* __restrict__ pr, double diag,
                                                    double off, const double* __restrict__ x,
                                                    const double* __restrict__ r, int ldr,
                                                    double* __restrict__ res, int ncols) {
  const RowMap q = rm[blockIdx.x];
  if (halted(pr[q.b].st)) return;
  const BLev L = lv[q.b];
  const int nx = L.nx, ny = L.ny, j = q.j;
  const size_t rowp = L.off + (size_t)j * nx;
  const ptrdiff_t sy = (ptrdiff_t)nx * ncols;
  const int P_ = blockDim.x / ncols, c = threadIdx.x % ncols, i0 = threadIdx.x / ncols;
  if (i0 >= P_) return;
  for (int i = i0; i < nx; i += P_) {
    const size_t p = rowp + i;
    const double* xp = x + p * ncols + c;
    double nb = 0.0;
    if (i > 0) nb += xp[-ncols];
    if (i < nx - 1) nb += xp[ncols];
    if (j > 0) nb += xp[-sy];
    if (j < ny - 1) nb += xp[sy];
    res[p * ncols + c] = r[p * ldr + c] - (diag * xp[0] + off * nb);
  }
}

// coarse r = P^T res / 4 (one workgroup per coarse row of a problem)
__global__ __launch_bounds__(256) void k_restrict_b(const RowMap* __restrict__ rm,
                                                    const BLev* __restrict__ lf,
                                                    const BLev* __restrict__ lc,
                                                    const BProb* __restrict__ pr,
                                                    const double* __restrict__ res,
                                                    double* __restrict__ rc, int ncols) {
  const RowMap q = rm[blockIdx.x];
  if (halted(pr[q.b].st)) return;
  const BLev F = lf[q.b], Cc = lc[q.b];
  const int cnx = Cc.nx, cj = q.j, fnx = F.nx, fny = F.ny;
  const int P_ = blockDim.x / ncols, c = threadIdx.x % ncols, i0 = threadIdx.x / ncols;
  if (i0 >= P_) return;
  for (int ci = i0; ci < cnx; ci += P_) {
    double acc = 0.0;
    for (int dy = 0; dy < 4; ++dy) {
      const int fj = 2 * cj - 1 + dy;
      if (fj < 0 || fj >= fny) continue;
      const double wy = (dy == 0 || dy == 3) ? 0.25 : 0.75;
      const double* rp = res + (F.off + (size_t)fj * fnx) * ncols + c;
      const int f0 = 2 * ci - 1;
      double a = 0.75 * (rp[(size_t)(f0 + 1) * ncols] + rp[(size_t)(f0 + 2) * ncols]);
      if (f0 >= 0) a += 0.25 * rp[(size_t)f0 * ncols];
      if (f0 + 3 < fnx) a += 0.25 * rp[(size_t)(f0 + 3) * ncols];
      acc += wy * a;
    }
    rc[(Cc.off + (size_t)cj * cnx + ci) * ncols + c] = 0.25 * acc;
  }
}

// x += P e (one workgroup per fine row of a problem)
__global__ __launch_bounds__(256) void k_prolong_b(const RowMap* __restrict__ rm,
                                                   const BLev* __restrict__ lf,
                                                   const BLev* __restrict__ lc,
                                                   const BProb* __restrict__ pr,
                                                   const double* __restrict__ ec,
                                                   double* __restrict__ x, int ncols) {
  const RowMap q = rm[blockIdx.x];
  if (halted(pr[q.b].st)) return;
  const BLev F = lf[q.b], Cc = lc[q.b];
  const int nx = F.nx, j = q.j, cnx = Cc.nx, cny = Cc.ny;
  const int P_ = blockDim.x / ncols, c = threadIdx.x % ncols, i0 = threadIdx.x / ncols;
  if (i0 >= P_) return;
  const int pj = j >> 1, qj = (j & 1) ? pj + 1 : pj - 1;
  for (int i = i0; i < nx; i += P_) {
    const int pi = i >> 1, qi = (i & 1) ? pi + 1 : pi - 1;
    double acc = 0.0;
    for (int ay = 0; ay < 2; ++ay) {
      const int cj = ay ? qj : pj;
      if (cj < 0 || cj >= cny) continue;
      const double wy = ay ? 0.25 : 0.75;
      const double* ep = ec + (Cc.off + (size_t)cj * cnx) * ncols + c;
      acc += wy * 0.75 * ep[(size_t)pi * ncols];
      if (qi >= 0 && qi < cnx) acc += wy * 0.25 * ep[(size_t)qi * ncols];
    }
    x[(F.off + (size_t)j * nx + i) * ncols + c] += acc;
  }
}

// coarsest level: x = Ainv_b r, one workgroup per problem
__global__ __launch_bounds__(256) void k_dense_b(const BLev* __restrict__ lv,
                                                 const BProb* __restrict__ pr,
                                                 const double* const* __restrict__ inv,
                                                 const double* __restrict__ r,
                                                 double* __restrict__ x, int ncols) {
  const int b = blockIdx.x;
  if (halted(pr[b].st)) return;
  const BLev L = lv[b];
  const int nc = L.nx * L.ny;
  const double* A = inv[b];
  const double* rb = r + L.off * ncols;
  double* xb = x + L.off * ncols;
  for (int e = threadIdx.x; e < nc * ncols; e += blockDim.x) {
    const int i = e / ncols, c = e - i * ncols;
    const double* a = A + (size_t)i * nc;
    double acc = 0.0;
    for (int q = 0; q < nc; ++q) acc += a[q] * rb[(size_t)q * ncols + c];
    xb[e] = acc;
  }
}

// ---------------------------------------------------------- column sums
// Block-level sums of `acc` over the threads of one column; the result of
// chunk `slot` goes to part[slot * nv*ncols + v*ncols + c].
template <int NV>
__device__ __forceinline__ void chunk_colsum(double (&acc)[NV], int ncols, double* part,
                                             size_t slot) {
  __shared__ double red[NV][256];
  const int t = threadIdx.x;
  for (int v = 0; v < NV; ++v) red[v][t] = acc[v];
  __syncthreads();
  const int rpi = blockDim.x / ncols;
  if (t < ncols)
    for (int v = 0; v < NV; ++v) {
      double s = 0.0;
      for (int q = 0; q < rpi; ++q) s += red[v][q * ncols + t];
      part[slot * NV * ncols + v * ncols + t] = s;
    }
}

// part: |x|^2 and x.y per column over the chunk
__global__ __launch_bounds__(256) void k_xdots_b(const Chunk* __restrict__ ch,
                                                 const BProb* __restrict__ pr,
                                                 const double* __restrict__ X, int ldx,
                                                 const double* __restrict__ Y, int ldy, int ncols,
                                                 double* __restrict__ part) {
  const Chunk q = ch[blockIdx.x];
  const BProb& P = pr[q.b];
  const int rpi = blockDim.x / ncols, t = threadIdx.x, c = t % ncols, r0 = t / ncols;
  double acc[2] = {0.0, 0.0};
  if (r0 < rpi && !halted(P.st))
    for (size_t p = P.off + q.p0 + r0; p < P.off + q.p1; p += rpi) {
      const double x = X[p * ldx + c];
      acc[0] += x * x;
      acc[1] += x * Y[p * ldy + c];
    }
  chunk_colsum<2>(acc, ncols, part, blockIdx.x);
}

// R = QV - V (lam - sigma) (if R), part: |R|^2 and |V|^2 per column
__global__ __launch_bounds__(256) void k_resid_b(const Chunk* __restrict__ ch,
                                                 const BProb* __restrict__ pr,
                                                 const double* __restrict__ V, int ldv,
                                                 const double* __restrict__ QV, int ldq,
                                                 double* __restrict__ R, int ldr, int ncols,
                                                 double* __restrict__ part) {
  const Chunk q = ch[blockIdx.x];
  const BProb& P = pr[q.b];
  const int rpi = blockDim.x / ncols, t = threadIdx.x, c = t % ncols, r0 = t / ncols;
  double acc[2] = {0.0, 0.0};
  if (r0 < rpi && !halted(P.st)) {
    const double sh = P.lam[c] - P.sigma;
    for (size_t p = P.off + q.p0 + r0; p < P.off + q.p1; p += rpi) {
      const double v = V[p * ldv + c];
      const double rv = QV[p * ldq + c] - v * sh;
      if (R) R[p * ldr + c] = rv;
      acc[0] += rv * rv;
      acc[1] += v * v;
    }
  }
  chunk_colsum<2>(acc, ncols, part, blockIdx.x);
}

// ---------------------------------------------------------------- Grams
// chunk c: partial (mx x my) Gram of its rows into gpart[c]
__global__ __launch_bounds__(768) void k_gram_b(const Chunk* __restrict__ ch,
                                                const BProb* __restrict__ pr,
                                                const double* __restrict__ X, int ldx, int mx,
                                                const double* __restrict__ Y1, int ldy1, int my1,
                                                const double* __restrict__ Y2, int ldy2, int my,
                                                int nw, double* __restrict__ gpart) {
  const Chunk q = ch[blockIdx.x];
  const BProb& P = pr[q.b];
  if (halted(P.st)) return;
  gram_body(P.off + q.p0, P.off + q.p1, X, ldx, mx, Y1, ldy1, my1, Y2, ldy2, my, nw,
            gpart + (size_t)blockIdx.x * mx * my);
}

// out_b = sum of the chunk partials of problem b (in chunk order); one
// workgroup per (problem, 256 entries)
__global__ __launch_bounds__(256) void k_gram_reduce_b(const BProb* __restrict__ pr,
                                                       const double* __restrict__ gpart,
                                                       int total, double* __restrict__ out,
                                                       size_t ostride, int eblocks) {
  const int b = blockIdx.x / eblocks, eb = blockIdx.x - b * eblocks;
  const BProb& P = pr[b];
  if (halted(P.st)) return;
  const int e = eb * 256 + threadIdx.x;
  if (e >= total) return;
  double s = 0.0;
  for (int c = 0; c < P.nch; ++c) s += gpart[(size_t)(P.ch0 + c) * total + e];
  out[(size_t)b * ostride + e] = s;
}

// --------------------------------------------------------- row products
template <int TJ>
__global__ __launch_bounds__(256, 2) void k_rowmul_b(const Chunk* __restrict__ ch,
                                                     const BProb* __restrict__ pr, ArrPtrs arrs,
                                                     int narr, int ld, int m,
                                                     const double* __restrict__ Mall,
                                                     size_t mstride, int kout, int mode, int kv,
                                                     int kc, int pcol, double* __restrict__ part) {
  const Chunk q = ch[blockIdx.x];
  const BProb& P = pr[q.b];
  if (halted(P.st)) return;
  rowmul_body<TJ>(P.off + q.p0, P.off + q.p1, 0, 4, arrs, narr, ld, m, Mall + q.b * mstride,
                  kout, mode, kv, kc, pcol, part ? part + (size_t)blockIdx.x * 2 * kc : nullptr);
}

// Y[p, :kout] = X[p, :kin] C_b (small dense C per problem)
__global__ __launch_bounds__(256) void k_small_gemm_b(const Chunk* __restrict__ ch,
                                                      const BProb* __restrict__ pr,
                                                      const double* __restrict__ X, int ldx,
                                                      int kin, const double* __restrict__ Call,
                                                      size_t cstride, int kout,
                                                      double* __restrict__ Y, int ldy) {
  const Chunk q = ch[blockIdx.x];
  const BProb& P = pr[q.b];
  const double* C = Call + q.b * cstride;
  const size_t p0 = P.off + q.p0, p1 = P.off + q.p1;
  for (size_t e = threadIdx.x; e < (p1 - p0) * kout; e += blockDim.x) {
    const size_t p = p0 + e / kout;
    const int c = (int)(e % kout);
    double acc = 0.0;
    for (int i = 0; i < kin; ++i) acc += X[p * ldx + i] * C[i * kout + c];
    Y[p * ldy + c] = acc;
  }
}

// ------------------------------------------------------- copies and HF
// packed Z[:, :c] <- V0_b (n_b x c, leading dimension c) for every problem
__global__ __launch_bounds__(256) void k_copy_in_b(const Chunk* __restrict__ ch,
                                                   const BProb* __restrict__ pr,
                                                   const double* const* __restrict__ src, int c,
                                                   double* __restrict__ Z, int ldz) {
  const Chunk q = ch[blockIdx.x];
  const BProb& P = pr[q.b];
  const double* s = src[q.b];
  for (size_t e = threadIdx.x; e < (size_t)(q.p1 - q.p0) * c; e += blockDim.x) {
    const size_t p = q.p0 + e / c;
    const int j = (int)(e % c);
    Z[(P.off + p) * ldz + j] = s[p * c + j];
  }
}

// dst_b (n_b x c) <- packed X[:, :c]
__global__ __launch_bounds__(256) void k_copy_out_b(const Chunk* __restrict__ ch,
                                                    const BProb* __restrict__ pr,
                                                    const double* __restrict__ X, int ldx, int c,
                                                    double* const* __restrict__ dst) {
  const Chunk q = ch[blockIdx.x];
  const BProb& P = pr[q.b];
  double* d = dst[q.b];
  if (!d) return;
  for (size_t e = threadIdx.x; e < (size_t)(q.p1 - q.p0) * c; e += blockDim.x) {
    const size_t p = q.p0 + e / c;
    const int j = (int)(e % c);
    d[p * c + j] = X[(P.off + p) * ldx + j];
  }
}

// g_b(x) (+)= sum_j dl_bj v_j(x)^2 / (v_j . v_j)   (Hellmann-Feynman)
__global__ __launch_bounds__(256) void k_hf_b(const Chunk* __restrict__ ch,
                                              const BProb* __restrict__ pr,
                                              const double* __restrict__ V, int ldv, int k,
                                              const double* __restrict__ dl,
                                              const double* const* __restrict__ vbv,
                                              double* const* __restrict__ g, int accumulate) {
  const Chunk q = ch[blockIdx.x];
  const BProb& P = pr[q.b];
  double* gb = g[q.b];
  const double* w = vbv[q.b];
  for (int p = q.p0 + threadIdx.x; p < q.p1; p += blockDim.x) {
    const double* v = V + (P.off + p) * ldv;
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += dl[(size_t)q.b * k + j] * v[j] * v[j] / w[j];
    gb[p] = accumulate ? gb[p] + s : s;
  }
}

// ---------------------------------------------------------------- host
void launch_fd_b(const RowMap* rm, int nrows, const BProb* pr, double diag, double off,
                 int use_sigma, const double* X, int ldx, Blk out, Blk outr, Blk outc, int ncols,
                 int threads, hipStream_t s) {
  prof_begin(KC_STENCIL, 0.0, 0.0, s);
  hipLaunchKernelGGL(k_fd_b, dim3(nrows), dim3(threads), 0, s, rm, pr, diag, off, use_sigma, X,
                     ldx, out.ptr, out.ld, outr.ptr, outr.ld, outc.ptr, outc.ld, ncols);
  prof_end(KC_STENCIL, s);
}
void launch_jacobi_b(const RowMap* rm, int nrows, const BLev* lv, const BProb* pr, double diag,
                     double off, double omega, const double* xin, const double* r, int ldr,
                     Blk o0, Blk o1, int split, int ncols, int threads, hipStream_t s) {
  prof_begin(KC_JACOBI, 0.0, 0.0, s);
  hipLaunchKernelGGL(k_jacobi_b, dim3(nrows), dim3(threads), 0, s, rm, lv, pr, diag, off, omega,
                     xin, r, ldr, o0.ptr, o0.ld, o1.ptr, o1.ld, split, ncols);
  prof_end(KC_JACOBI, s);
}
void launch_residual_b(const RowMap* rm, int nrows, const BLev* lv, const BProb* pr,
                       double diag, double off, const double* x, const double* r, int ldr,
                       double* res, int ncols, int threads, hipStream_t s) {
  prof_begin(KC_RESIDUAL, 0.0, 0.0, s);
  hipLaunchKernelGGL(k_residual_b, dim3(nrows), dim3(threads), 0, s, rm, lv, pr, diag, off, x, r,
                     ldr, res, ncols);
  prof_end(KC_RESIDUAL, s);
}
void launch_restrict_b(const RowMap* rmc, int ncrows, const BLev* lf, const BLev* lc,
                       const BProb* pr, const double* res, double* rc, int ncols, int threads,
                       hipStream_t s) {
  prof_begin(KC_RESTRICT, 0.0, 0.0, s);
  hipLaunchKernelGGL(k_restrict_b, dim3(ncrows), dim3(threads), 0, s, rmc, lf, lc, pr, res, rc,
                     ncols);
  prof_end(KC_RESTRICT, s);
}
void launch_prolong_b(const RowMap* rm, int nrows, const BLev* lf, const BLev* lc,
                      const BProb* pr, const double* ec, double* x, int ncols, int threads,
                      hipStream_t s) {
  prof_begin(KC_PROLONG, 0.0, 0.0, s);
  hipLaunchKernelGGL(k_prolong_b, dim3(nrows), dim3(threads), 0, s, rm, lf, lc, pr, ec, x, ncols);
  prof_end(KC_PROLONG, s);
}
void launch_dense_b(int nb, const BLev* lv, const BProb* pr, const double* const* inv,
                    const double* r, double* x, int ncols, hipStream_t s) {
  prof_begin(KC_COARSE, 0.0, 0.0, s);
  hipLaunchKernelGGL(k_dense_b, dim3(nb), dim3(256), 0, s, lv, pr, inv, r, x, ncols);
  prof_end(KC_COARSE, s);
}
void launch_xdots_b(const Chunk* ch, int nch, const BProb* pr, const double* X, int ldx,
                    const double* Y, int ldy, int ncols, double* part, hipStream_t s) {
  prof_begin(KC_VEC, 0.0, 0.0, s);
  hipLaunchKernelGGL(k_xdots_b, dim3(nch), dim3(256), 0, s, ch, pr, X, ldx, Y, ldy, ncols, part);
  prof_end(KC_VEC, s);
}
void launch_resid_b(const Chunk* ch, int nch, const BProb* pr, const double* V, int ldv,
                    const double* QV, int ldq, double* R, int ldr, int ncols, double* part,
                    hipStream_t s) {
  prof_begin(KC_VEC, 0.0, 0.0, s);
  hipLaunchKernelGGL(k_resid_b, dim3(nch), dim3(256), 0, s, ch, pr, V, ldv, QV, ldq, R, ldr,
                     ncols, part);
  prof_end(KC_VEC, s);
}
void launch_gram_b(const Chunk* ch, int nch, int nb, const BProb* pr, const double* X, int ldx,
                   int mx, const double* Y1, int ldy1, int my1, const double* Y2, int ldy2,
                   int my, double* gpart, double* out, size_t ostride, size_t ntot,
                   hipStream_t s) {
  const int NW = (mx + 31) / 32, NJH = ((my + 31) / 32 + kJPW - 1) / kJPW;
  prof_begin(KC_GRAM, (double)ntot * (mx + my) * 8.0, 2.0 * ntot * mx * my, s);
  hipLaunchKernelGGL(k_gram_b, dim3(nch), dim3(64 * NW * NJH), 0, s, ch, pr, X, ldx, mx, Y1, ldy1,
                     my1, Y2, ldy2, my, NW, gpart);
  prof_end(KC_GRAM, s);
  const int total = mx * my, eb = (total + 255) / 256;
  prof_begin(KC_GRAM_REDUCE, (double)nch * total * 8.0, (double)nch * total, s);
  hipLaunchKernelGGL(k_gram_reduce_b, dim3(nb * eb), dim3(256), 0, s, pr, gpart, total, out,
                     ostride, eb);
  prof_end(KC_GRAM_REDUCE, s);
}
void launch_rowmul_b(const Chunk* ch, int nch, const BProb* pr, double* const* X, int narr,
                     int ld, int m, const double* Mall, size_t mstride, int kout, int mode,
                     int kv, int kc, int pcol, double* part, size_t ntot, hipStream_t s) {
  ArrPtrs a{};
  for (int i = 0; i < narr; ++i) a.a[i] = X[i];
  const int TJ = (kout + 15) / 16;
  const size_t shm = (size_t)m * (TJ * 16 + 4) * sizeof(double);
  const double bytes = (mode == 0) ? 2.0 * narr * ntot * m * 8.0
                                   : (double)narr * ntot * (m + kout) * 8.0;
  const int cat = (mode == 0) ? KC_TRANSFORM : KC_UPDATE;
  prof_begin(cat, bytes, 2.0 * narr * ntot * (double)m * kout, s);
#define ROWB_CASE(T)                                                                            \
  case T:                                                                                       \
    hipLaunchKernelGGL(k_rowmul_b<T>, dim3(nch), dim3(256), shm, s, ch, pr, a, narr, ld, m,     \
                       Mall, mstride, kout, mode, kv, kc, pcol, part);                          \
    break;
  switch (TJ) {
    ROWB_CASE(1) ROWB_CASE(2) ROWB_CASE(3) ROWB_CASE(4) ROWB_CASE(5) ROWB_CASE(6)
    default: break;
  }
#undef ROWB_CASE
  prof_end(cat, s);
}
void launch_small_gemm_b(const Chunk* ch, int nch, const BProb* pr, const double* X, int ldx,
                         int kin, const double* Call, size_t cstride, int kout, double* Y,
                         int ldy, hipStream_t s) {
  hipLaunchKernelGGL(k_small_gemm_b, dim3(nch), dim3(256), 0, s, ch, pr, X, ldx, kin, Call,
                     cstride, kout, Y, ldy);
}
void launch_copy_in_b(const Chunk* ch, int nch, const BProb* pr, const double* const* src,
                      int c, double* Z, int ldz, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_in_b, dim3(nch), dim3(256), 0, s, ch, pr, src, c, Z, ldz);
}
void launch_copy_out_b(const Chunk* ch, int nch, const BProb* pr, const double* X, int ldx,
                       int c, double* const* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_out_b, dim3(nch), dim3(256), 0, s, ch, pr, X, ldx, c, dst);
}
void launch_hf_b(const Chunk* ch, int nch, const BProb* pr, const double* V, int ldv, int k,
                 const double* dl, const double* const* vbv, double* const* g, int accumulate,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_hf_b, dim3(nch), dim3(256), 0, s, ch, pr, V, ldv, k, dl, vbv, g,
                     accumulate);
}
hipError_t batch_set_attributes(int m) {
  (void)m;
  hipError_t e = hipSuccess;
#define SETB(T)                                  \
  e = set_lds_limit((const void*)k_rowmul_b<T>); \
  if (e != hipSuccess) return e;
  SETB(1) SETB(2) SETB(3) SETB(4) SETB(5) SETB(6)
#undef SETB
  return e;
}

}  // namespace plhr
