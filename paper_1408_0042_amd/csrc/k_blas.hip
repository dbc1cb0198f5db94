// Tall-skinny block kernels on point-major blocks (n rows, few columns):
// residual formation, split-K Gram products, in-place right
// multiplication by a small matrix (B-orthonormalisation transform and the
// Ritz-vector update), copies and column reductions.
//
// All reductions are two-stage and deterministic: each workgroup writes
// its partial sums, a second pass (here or in a small kernel) adds them in
// a fixed order.
#include "common.cuh"

namespace plhr {

static constexpr int kRedBlocks = 512;  // workgroups of the column reductions

int resid_prep_blocks(size_t) { return kRedBlocks; }
int update_blocks(size_t) { return kRedBlocks; }

// Partial column sums of a thread-strided loop, reduced inside the
// workgroup: thread t owns column t % ncols and rows t / ncols + q*rpi.
// `vals` holds nv values per thread; the block result goes to
// part[blockIdx.x * nv*ncols + v*ncols + c].
template <int NV>
__device__ __forceinline__ void block_colsum(double (&acc)[NV], int ncols, double* part) {
  __shared__ double red[NV][256];
  const int t = threadIdx.x;
  for (int v = 0; v < NV; ++v) red[v][t] = acc[v];
  __syncthreads();
  const int rpi = blockDim.x / ncols;
  if (t < ncols) {
    for (int v = 0; v < NV; ++v) {
      double s = 0.0;
      for (int q = 0; q < rpi; ++q) s += red[v][q * ncols + t];
      part[(size_t)blockIdx.x * NV * ncols + v * ncols + t] = s;
    }
  }
}

// R = QV - V * (lam - sigma); partial |R|^2, |V|^2 per column.  With row
// weights bw (a diagonal mass b, the blocks in the variables u = b^1/2 v)
// the sums are the norms of the residual and of the vector in the
// original variables: sum b R^2 and sum V^2 / b.
__global__ __launch_bounds__(256) void k_resid_prep(size_t n, const double* __restrict__ V,
                                                    int ldv, const double* __restrict__ QV, int ldq,
                                                    const double* __restrict__ lam, double sigma,
                                                    double* __restrict__ R, int ldr, int ncols,
                                                    const double* __restrict__ bw,
                                                    const double* __restrict__ BV, int ldb,
                                                    double* __restrict__ part,
                                                    const DevStatus* st) {
  if (halted(st)) return;
  const int rpi = blockDim.x / ncols;
  const int t = threadIdx.x;
  const int c = t % ncols;
  const int r0 = t / ncols;
  double acc[2] = {0.0, 0.0};
  if (r0 < rpi) {
    const size_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const size_t pb = (size_t)blockIdx.x * chunk;
    const size_t pe = (pb + chunk < n) ? pb + chunk : n;
    const double sh = lam[c] - sigma;
    for (size_t p = pb + r0; p < pe; p += rpi) {
      const double v = V[p * ldv + c];
      const double r = QV[p * ldq + c] - (BV ? BV[p * ldb + c] : v) * sh;
      if (R) R[p * ldr + c] = r;
      if (bw) {
        const double b = bw[p];
        acc[0] += b * (r * r);
        acc[1] += (v * v) / b;
      } else {
        acc[0] += r * r;
        acc[1] += v * v;
      }
    }
  }
  block_colsum<2>(acc, ncols, part);
}

int launch_resid_prep(size_t n, const double* V, int ldv, const double* QV, int ldq,
                      const double* lam, double sigma, double* R, int ldr, int ncols,
                      const double* bw, const double* BV, int ldb, double* part,
                      const DevStatus* st, hipStream_t s) {
  prof_begin(KC_VEC, (double)n * ncols * 8.0 * (R ? 3.0 : 2.0) + (bw ? n * 8.0 : 0.0),
             5.0 * n * ncols, s);
  hipLaunchKernelGGL(k_resid_prep, dim3(kRedBlocks), dim3(256), 0, s, n, V, ldv, QV, ldq, lam,
                     sigma, R, ldr, ncols, bw, BV, ldb, part, st);
  prof_end(KC_VEC, s);
  return kRedBlocks;
}

// Partial column sums of x.(Bx) and x.y (for Rayleigh quotients); BX
// null means B = I.
__global__ __launch_bounds__(256) void k_xdots(size_t n, const double* __restrict__ X, int ldx,
                                               const double* __restrict__ Y, int ldy,
                                               const double* __restrict__ BX, int ldb, int ncols,
                                               double* __restrict__ part) {
  const int rpi = blockDim.x / ncols;
  const int t = threadIdx.x;
  const int c = t % ncols;
  const int r0 = t / ncols;
  double acc[2] = {0.0, 0.0};
  if (r0 < rpi) {
    const size_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const size_t pb = (size_t)blockIdx.x * chunk;
    const size_t pe = (pb + chunk < n) ? pb + chunk : n;
    for (size_t p = pb + r0; p < pe; p += rpi) {
      const double x = X[p * ldx + c];
      acc[0] += x * (BX ? BX[p * ldb + c] : x);
      acc[1] += x * Y[p * ldy + c];
    }
  }
  block_colsum<2>(acc, ncols, part);
}

int launch_xdots(size_t n, const double* X, int ldx, const double* Y, int ldy, int ncols,
                 double* part, hipStream_t s, const double* BX, int ldb) {
  hipLaunchKernelGGL(k_xdots, dim3(kRedBlocks), dim3(256), 0, s, n, X, ldx, Y, ldy, BX, ldb,
                     ncols, part);
  return kRedBlocks;
}

// Column sums for the final residual check: |QX - X*(lam - sigma)|^2, |X|^2.
int launch_coldots(size_t n, const double* X, int ldx, const double* QX, int ldq, int c,
                   const double* lam, double sigma, const double* bw, const double* BX, int ldb,
                   double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_resid_prep, dim3(kRedBlocks), dim3(256), 0, s, n, X, ldx, QX, ldq, lam,
                     sigma, (double*)nullptr, 0, c, bw, BX, ldb, part, (const DevStatus*)nullptr);
  return kRedBlocks;
}

// ------------------------------------------------------------ Gram kernel
// part[split][i][j] = sum over the split's rows of X[p, i] * Y[p, j].
// Thread (ty, tx) owns the 4x4 micro-tile rows 4ty.., columns 4tx..;
// rows of X and Y are staged in LDS kTR at a time.
static constexpr int kTR = 16;

__global__ void k_gram(size_t n, const double* __restrict__ X, int ldx, int mx,
                       const double* __restrict__ Y1, int ldy1, int my1,
                       const double* __restrict__ Y2, int ldy2, int my,
                       double* __restrict__ part, const DevStatus* st) {
  if (halted(st)) return;
  extern __shared__ __attribute__((aligned(16))) double sh[];
  const int mxp = (mx + 3) & ~3, myp = (my + 3) & ~3;
  double* sx = sh;                 // kTR x mxp
  double* sy = sh + kTR * mxp;     // kTR x myp
  const int tx = threadIdx.x % (myp / 4);
  const int ty = threadIdx.x / (myp / 4);
  const int nthr = blockDim.x;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  const size_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const size_t pb = (size_t)blockIdx.x * chunk;
  const size_t pe = (pb + chunk < n) ? pb + chunk : n;
  for (size_t p0 = pb; p0 < pe; p0 += kTR) {
    const int nr = (pe - p0 < (size_t)kTR) ? (int)(pe - p0) : kTR;
    for (int e = threadIdx.x; e < kTR * mxp; e += nthr) {
      const int r = e / mxp, c = e - r * mxp;
      sx[e] = (r < nr && c < mx) ? X[(p0 + r) * ldx + c] : 0.0;
    }
    for (int e = threadIdx.x; e < kTR * myp; e += nthr) {
      const int r = e / myp, c = e - r * myp;
      double v = 0.0;
      if (r < nr && c < my) v = (c < my1) ? Y1[(p0 + r) * ldy1 + c] : Y2[(p0 + r) * ldy2 + (c - my1)];
      sy[e] = v;
    }
    __syncthreads();
    if (ty * 4 < mxp) {
#pragma unroll 4
      for (int r = 0; r < kTR; ++r) {
        double xa[4], yb[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) xa[a] = sx[r * mxp + ty * 4 + a];
#pragma unroll
        for (int b = 0; b < 4; ++b) yb[b] = sy[r * myp + tx * 4 + b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] += xa[a] * yb[b];
      }
    }
    __syncthreads();
  }
  if (ty * 4 < mxp) {
    double* out = part + (size_t)blockIdx.x * mx * my;
    for (int a = 0; a < 4; ++a) {
      const int i = ty * 4 + a;
      if (i >= mx) continue;
      for (int b = 0; b < 4; ++b) {
        const int j = tx * 4 + b;
        if (j < my) out[(size_t)i * my + j] = acc[a][b];
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ part, int nblk,
                                                     int total, double* __restrict__ out,
                                                     const DevStatus* st) {
  if (halted(st)) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * total + e];
  out[e] = s;
}

hipError_t set_lds_limit(const void* kernel) {
  int dev = 0, lim = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  int optin = 0;
  if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) ==
          hipSuccess &&
      optin > lim)
    lim = optin;
  // the limit covers the kernel's static LDS as well
  hipFuncAttributes fa{};
  e = hipFuncGetAttributes(&fa, kernel);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             lim - (int)fa.sharedSizeBytes);
}

// Split-K blocks of the Gram products: 64 rows per block at least, at
// most 512 blocks (two per compute unit), so that a small basis still
// spreads over many compute units instead of walking its rows in a few.
int gram_blocks(size_t n) {
  size_t nb = (n + 63) / 64;
  if (nb > 512) nb = 512;
  if (nb < 1) nb = 1;
  return (int)nb;
}

void launch_gram(size_t n, const double* X, int ldx, int mx, const double* Y1, int ldy1, int my1,
                 const double* Y2, int ldy2, int my, double* part, int nblk, double* out,
                 const DevStatus* st, hipStream_t s) {
  const int mxp = (mx + 3) & ~3, myp = (my + 3) & ~3;
  const int threads = (mxp / 4) * (myp / 4);
  const size_t shm = (size_t)kTR * (mxp + myp) * sizeof(double);
  prof_begin(KC_GRAM, (double)n * (mx + my) * 8.0, 2.0 * n * mx * my, s);
  hipLaunchKernelGGL(k_gram, dim3(nblk), dim3(threads), shm, s, n, X, ldx, mx, Y1, ldy1, my1, Y2,
                     ldy2, my, part, st);
  prof_end(KC_GRAM, s);
  const int total = mx * my;
  prof_begin(KC_GRAM_REDUCE, (double)nblk * total * 8.0, (double)nblk * total, s);
  hipLaunchKernelGGL(k_gram_reduce, dim3((total + 255) / 256), dim3(256), 0, s, part, nblk, total,
                     out, st);
  prof_end(KC_GRAM_REDUCE, s);
}

// ----------------------------------------------- row-block right multiply
// For each array a: Out[p, :kout] = X_a[p, :kin] * M, in place (the whole
// row tile is read into LDS before any write).  Output columns [0, kv) of
// M-products go to columns [0, kv) ... see the two modes below.
//
// mode 0 (transform): X_a[p, 0:m] <- X_a[p, 0:m] * M   (M is m x m)
// mode 1 (update):    with Y (m x kc):
//                       V = X[p, 0:m] * Y,   P = X[p, kv:m] * Y[kv:m, :]
//                     X_a[p, 0:kc] <- V,  X_a[p, pcol:pcol+kc] <- P
// In mode 1, array 0's V rows are kept in LDS and array 1's V rows are
// dotted with them: partial sums of v.v and v.(Qv) per column.
static constexpr int kRB = 64;  // rows per workgroup tile

__global__ void k_rowmul(size_t n, ArrPtrs arrs, int narr, int ld, int m, const double* __restrict__ M,
                         int kout, int mode, int kv, int kc, int pcol, double* __restrict__ part,
                         const DevStatus* st) {
  if (halted(st)) return;
  extern __shared__ __attribute__((aligned(16))) double sh[];
  double* sM = sh;                    // m x kout
  double* sX = sM + m * kout;         // kRB x m
  double* sV = sX + kRB * m;          // kRB x kc (mode 1)
  const int nthr = blockDim.x;
  // mode 0: sM = M (m x m).  mode 1: sM = [Y | Y with the V rows zeroed]
  for (int e = threadIdx.x; e < m * kout; e += nthr) {
    if (mode == 0) {
      sM[e] = M[e];
    } else {
      const int q = e / kout, col = e - q * kout;
      const int c0 = (col < kc) ? col : col - kc;
      sM[e] = (col >= kc && q < kv) ? 0.0 : M[q * kc + c0];
    }
  }
  const int ncg = (kout + 3) / 4;     // column groups of 4
  const int tcol = threadIdx.x % ncg;
  const int trow = threadIdx.x / ncg; // row group of 4 (kRB/4 groups)
  double dacc[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
  const size_t ntiles = (n + kRB - 1) / kRB;
  for (size_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const size_t p0 = tile * kRB;
    const int nr = (n - p0 < (size_t)kRB) ? (int)(n - p0) : kRB;
    for (int a = 0; a < narr; ++a) {
      double* X = arrs.at(a);
      __syncthreads();
      for (int e = threadIdx.x; e < kRB * m; e += nthr) {
        const int r = e / m, c = e - r * m;
        sX[e] = (r < nr) ? X[(p0 + r) * ld + c] : 0.0;
      }
      __syncthreads();
      if (trow < kRB / 4) {
        double acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
        // mode 1 columns: [0,kc) = V (all rows of Y), [kc, 2kc) = P (rows >= kv)
        for (int q = 0; q < m; ++q) {
          double xr[4], mc[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) xr[i] = sX[(trow * 4 + i) * m + q];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int col = tcol * 4 + j;
            mc[j] = (col < kout) ? sM[q * kout + col] : 0.0;
          }
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] += xr[i] * mc[j];
        }
        // write
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = trow * 4 + i;
          if (r >= nr) continue;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int col = tcol * 4 + j;
            if (col >= kout) continue;
            const double v = acc[i][j];
            if (mode == 0) {
              X[(p0 + r) * ld + col] = v;
            } else {
              if (col < kc) {
                X[(p0 + r) * ld + col] = v;
                if (a == 0) sV[r * kc + col] = v;
                if (a == 1) {
                  const double vv = sV[r * kc + col];
                  if (narr < 4) dacc[0][j] += vv * vv;
                  dacc[1][j] += vv * v;
                }
                if (a == 3) dacc[0][j] += sV[r * kc + col] * v;  // v.(Bv)
              } else {
                X[(p0 + r) * ld + pcol + (col - kc)] = v;
              }
            }
          }
        }
      }
    }
  }
  if (mode == 1 && part) {
    // reduce dacc over row groups: thread (trow, tcol) holds columns tcol*4+j
    __syncthreads();
    // per column c < kc: sum over trow of dacc for (tcol = c/4, j = c%4)
    double* rbuf = sX;  // reuse LDS: (kRB/4) x ncg x 4 x 2
    const int ngr = kRB / 4;
    if (trow < ngr) {
      for (int j = 0; j < 4; ++j) {
        rbuf[((trow * ncg + tcol) * 4 + j) * 2 + 0] = dacc[0][j];
        rbuf[((trow * ncg + tcol) * 4 + j) * 2 + 1] = dacc[1][j];
      }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < kc; c += nthr) {
      double s0 = 0.0, s1 = 0.0;
      const int tc = c / 4, j = c % 4;
      for (int g = 0; g < ngr; ++g) {
        s0 += rbuf[((g * ncg + tc) * 4 + j) * 2 + 0];
        s1 += rbuf[((g * ncg + tc) * 4 + j) * 2 + 1];
      }
      part[(size_t)blockIdx.x * 2 * kc + c] = s0;
      part[(size_t)blockIdx.x * 2 * kc + kc + c] = s1;
    }
  }
}

static size_t rowmul_shm(int m, int kout, int kc) {
  size_t words = (size_t)m * kout + (size_t)kRB * m + (size_t)kRB * kc;
  // the final reduction reuses sX: needs kRB/4 * ncg * 8 words
  const size_t need = (size_t)(kRB / 4) * ((kout + 3) / 4) * 8;
  if (need > (size_t)kRB * m) words += need - (size_t)kRB * m;
  return words * sizeof(double);
}

void launch_transform(size_t n, double* const* X, int nx, int ld, int m, const double* M,
                      const DevStatus* st, hipStream_t s) {
  ArrPtrs a{};
  for (int i = 0; i < nx; ++i) a.a[i] = X[i];
  const int threads = (kRB / 4) * ((m + 3) / 4);
  const size_t ntiles = (n + kRB - 1) / kRB;
  const int nb = (int)(ntiles < 2048 ? ntiles : 2048);
  prof_begin(KC_TRANSFORM, 2.0 * nx * n * m * 8.0, 2.0 * nx * n * (double)m * m, s);
  hipLaunchKernelGGL(k_rowmul, dim3(nb), dim3(threads), rowmul_shm(m, m, 0), s, n, a, nx, ld, m,
                     M, m, 0, 0, 0, 0, (double*)nullptr, st);
  prof_end(KC_TRANSFORM, s);
}

int launch_update(size_t n, double* const* X, int nx, int ld, int m, int kv, const double* Y,
                  int kc, int pcol, double* part, const DevStatus* st, hipStream_t s) {
  ArrPtrs a{};
  for (int i = 0; i < nx; ++i) a.a[i] = X[i];
  const int kout = 2 * kc;
  const int threads = (kRB / 4) * ((kout + 3) / 4);
  prof_begin(KC_UPDATE, (double)nx * n * (m + kout) * 8.0, 2.0 * nx * n * (double)m * kout, s);
  hipLaunchKernelGGL(k_rowmul, dim3(kRedBlocks), dim3(threads), rowmul_shm(m, kout, kc), s, n, a,
                     nx, ld, m, Y, kout, 1, kv, kc, pcol, part, st);
  prof_end(KC_UPDATE, s);
  return kRedBlocks;
}

// Y[p, :kout] = X[p, :kin] * M  (out of place, small dense M)
__global__ __launch_bounds__(256) void k_small_gemm(size_t n, const double* __restrict__ X,
                                                    int ldx, int kin,
                                                    const double* __restrict__ M, int kout,
                                                    double* __restrict__ Y, int ldy) {
  const size_t tot = n * kout;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t p = e / kout;
    const int c = (int)(e - p * kout);
    double acc = 0.0;
    for (int q = 0; q < kin; ++q) acc += X[p * ldx + q] * M[q * kout + c];
    Y[p * ldy + c] = acc;
  }
}

void launch_small_gemm(size_t n, const double* X, int ldx, int kin, const double* M, int kout,
                       double* Y, int ldy, hipStream_t s) {
  hipLaunchKernelGGL(k_small_gemm, dim3(2048), dim3(256), 0, s, n, X, ldx, kin, M, kout, Y, ldy);
}

__global__ __launch_bounds__(256) void k_copy(size_t n, const double* __restrict__ X, int ldx,
                                              double* __restrict__ Y, int ldy, int c,
                                              const DevStatus* st) {
  if (halted(st)) return;
  const size_t tot = n * c;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t p = e / c;
    const int j = (int)(e - p * c);
    Y[p * ldy + j] = X[p * ldx + j];
  }
}

void launch_copy(size_t n, const double* X, int ldx, double* Y, int ldy, int c, hipStream_t s,
                 const DevStatus* st) {
  size_t tot = n * c;
  size_t nb = (tot + 255) / 256;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)nb), dim3(256), 0, s, n, X, ldx, Y, ldy, c, st);
}

// Y = diag(w) X (rows scaled; Y may be X with the same leading dimension).
__global__ __launch_bounds__(256) void k_rowscale(size_t n, const double* __restrict__ w,
                                                  const double* X, int ldx, double* Y, int ldy,
                                                  int c, const DevStatus* st) {
  if (halted(st)) return;
  const size_t tot = n * (size_t)c;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t p = e / c;
    const int j = (int)(e - p * c);
    Y[p * ldy + j] = w[p] * X[p * ldx + j];
  }
}

void launch_rowscale(size_t n, const double* w, const double* X, int ldx, double* Y, int ldy,
                     int c, hipStream_t s, const DevStatus* st) {
  if (c <= 0 || n == 0) return;
  const size_t tot = n * (size_t)c;
  const size_t want = (tot + 255) / 256;
  const int nb = (int)(want < 4096 ? want : 4096);
  prof_begin(KC_VEC, (double)n * c * 16.0 + n * 8.0, (double)n * c, s);
  hipLaunchKernelGGL(k_rowscale, dim3(nb), dim3(256), 0, s, n, w, X, ldx, Y, ldy, c, st);
  prof_end(KC_VEC, s);
}

// Hellmann-Feynman: g[x] (+)= sum_j dl[j] * V[x, j]^2 / vbv[j]
__global__ __launch_bounds__(256) void k_hf(size_t n, const double* __restrict__ V, int ldv, int k,
                                            const double* __restrict__ dl,
                                            const double* __restrict__ vbv,
                                            double* __restrict__ g, int accumulate) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (size_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) {
      const double v = V[p * ldv + j];
      s += dl[j] * v * v / vbv[j];
    }
    g[p] = accumulate ? g[p] + s : s;
  }
}

void launch_hf(size_t n, const double* V, int ldv, int k, const double* dl, const double* vbv,
               double* g, int accumulate, hipStream_t s) {
  size_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_hf, dim3((unsigned)nb), dim3(256), 0, s, n, V, ldv, k, dl, vbv, g,
                     accumulate);
}

}  // namespace plhr
