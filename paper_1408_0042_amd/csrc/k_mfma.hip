// FP64 matrix-core (MFMA) versions of the two dense tall-skinny products of
// the iteration:
//
//   k_gram_mfma    out(i, j) = sum_p X[p, i] Y[p, j]    (split over rows)
//   k_rowmul_mfma  X_a[p, :kout] = X_a[p, :m] M         (in place, per row)
//
// Both use v_mfma_f64_16x16x4f64, D(16x16) += A(16x4) B(4x16), with the
// operand layout of that instruction: lane l holds A[l%16][l/16] and
// B[l/16][l%16]; accumulator register r of lane l is D[4r + l/16][l%16].
//
// For the Gram the reduction dimension K is the grid-point index p: A is a
// 4-row slice of X read transposed, B the matching slice of Y.  For the
// row product K is the column index of X: A is a 16-row by 4-column tile
// of X, B a 4 x 16 tile of M.
#include "common.cuh"

namespace plhr {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- Gram
// Block = TI wavefronts (TI = ceil(mx/16)); wave w owns output rows
// 16w..16w+15 and all TJ = ceil(my/16) column tiles.  Rows of X and Y are
// staged in LDS kCH at a time.
static constexpr int kCH = 16;

template <int TJ>
__global__ __launch_bounds__(512) void k_gram_mfma(size_t n, const double* __restrict__ X, int ldx,
                                                   int mx, const double* __restrict__ Y1, int ldy1,
                                                   int my1, const double* __restrict__ Y2, int ldy2,
                                                   int my, double* __restrict__ part,
                                                   const DevStatus* st) {
  if (halted(st)) return;
  extern __shared__ double sh[];
  const int TI = blockDim.x / 64;
  const int mxp = TI * 16, myp = TJ * 16;
  double* sx = sh;               // kCH x mxp
  double* sy = sh + kCH * mxp;   // kCH x myp
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int w = tid >> 6, l = tid & 63;
  const int li = l & 15, lk = l >> 4;
  d4 acc[TJ];
#pragma unroll
  for (int t = 0; t < TJ; ++t) acc[t] = (d4){0.0, 0.0, 0.0, 0.0};
  const size_t chunk = ((n + gridDim.x - 1) / gridDim.x + kCH - 1) / kCH * kCH;
  const size_t pb = (size_t)blockIdx.x * chunk;
  const size_t pe = (pb + chunk < n) ? pb + chunk : n;
  for (size_t p0 = pb; p0 < pe; p0 += kCH) {
    const int nr = (pe - p0 < (size_t)kCH) ? (int)(pe - p0) : kCH;
    // stage the chunk: flattened so that each thread has several loads in
    // flight before its LDS stores
    {
      const int tx_ = kCH * mxp;
#pragma unroll 8
      for (int e = tid; e < tx_; e += nthr) {
        const int r = e / mxp, c = e - r * mxp;
        sx[e] = (r < nr && c < mx) ? X[(p0 + r) * ldx + c] : 0.0;
      }
      const int ty_ = kCH * myp;
#pragma unroll 8
      for (int e = tid; e < ty_; e += nthr) {
        const int r = e / myp, c = e - r * myp;
        double v = 0.0;
        if (r < nr && c < my)
          v = (c < my1) ? Y1[(p0 + r) * ldy1 + c] : Y2[(p0 + r) * ldy2 + (c - my1)];
        sy[e] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kCH / 4; ++kk) {
      const double a = sx[(4 * kk + lk) * mxp + w * 16 + li];
#pragma unroll
      for (int t = 0; t < TJ; ++t) acc[t] = mfma(a, sy[(4 * kk + lk) * myp + t * 16 + li], acc[t]);
    }
    __syncthreads();
  }
  double* out = part + (size_t)blockIdx.x * mx * my;
#pragma unroll
  for (int t = 0; t < TJ; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = w * 16 + 4 * r + lk, j = t * 16 + li;
      if (i < mx && j < my) out[(size_t)i * my + j] = acc[t][r];
    }
}

// Deterministic reduction of the per-block partials: 256 threads handle 32
// outputs, 8 threads per output each summing every 8th block, then LDS.
__global__ __launch_bounds__(256) void k_gram_reduce8(const double* __restrict__ part, int nblk,
                                                      int total, double* __restrict__ out,
                                                      const DevStatus* st) {
  if (halted(st)) return;
  __shared__ double red[8][32];
  const int t = threadIdx.x;
  const int e = blockIdx.x * 32 + (t & 31), g = t >> 5;
  double s = 0.0;
  if (e < total)
    for (int q = g; q < nblk; q += 8) s += part[(size_t)q * total + e];
  red[g][t & 31] = s;
  __syncthreads();
  if (t < 32 && e < total) {
    double a = 0.0;
    for (int q = 0; q < 8; ++q) a += red[q][t];
    out[e] = a;
  }
}

int gram_mfma_ok(int mx, int my) { return mx <= 128 && my <= 11 * 16; }

void launch_gram_mfma(size_t n, const double* X, int ldx, int mx, const double* Y1, int ldy1,
                      int my1, const double* Y2, int ldy2, int my, double* part, int nblk,
                      double* out, const DevStatus* st, hipStream_t s) {
  const int TI = (mx + 15) / 16, TJ = (my + 15) / 16;
  const size_t shm = (size_t)kCH * 16 * (TI + TJ) * sizeof(double);
  dim3 grid(nblk), block(64 * TI);
  prof_begin(KC_GRAM, (double)n * (mx + my) * 8.0, 2.0 * n * mx * my, s);
#define GRAM_CASE(T)                                                                             \
  case T:                                                                                        \
    hipLaunchKernelGGL(k_gram_mfma<T>, grid, block, shm, s, n, X, ldx, mx, Y1, ldy1, my1, Y2,  \
                       ldy2, my, part, st);                                                      \
    break;
  switch (TJ) {
    GRAM_CASE(1) GRAM_CASE(2) GRAM_CASE(3) GRAM_CASE(4) GRAM_CASE(5) GRAM_CASE(6) GRAM_CASE(7)
    GRAM_CASE(8) GRAM_CASE(9) GRAM_CASE(10) GRAM_CASE(11)
    default: break;
  }
#undef GRAM_CASE
  prof_end(KC_GRAM, s);
  const int total = mx * my;
  prof_begin(KC_GRAM_REDUCE, (double)nblk * total * 8.0, (double)nblk * total, s);
  hipLaunchKernelGGL(k_gram_reduce8, dim3((total + 31) / 32), dim3(256), 0, s, part, nblk, total,
                     out, st);
  prof_end(KC_GRAM_REDUCE, s);
}

// ------------------------------------------------------------ row product
// Block = 4 wavefronts on a tile of 64 rows; wave w owns rows 16w..16w+15
// and all TJ = ceil(kout/16) column tiles.  M (m x kout) stays in LDS for
// the whole kernel; the tile of X is staged per array.
//
// mode 0 (B-orthonormalising transform): X_a[p, 0:m] <- X_a[p, 0:m] M.
// mode 1 (Ritz-vector update) with Y (m x kc): the product uses
//   [Y | Y with rows < kv zeroed]  (kout = 2 kc),
// columns [0, kc) (new V) go to slots [0, kc), columns [kc, 2kc) (new P)
// to slots [pcol, pcol + kc); for arrays 0 and 1 the column sums of v*v
// and v*(Qv) are accumulated into part (nblk x 2kc).
static constexpr int kRT = 64;  // rows per tile

template <int TJ>
__global__ __launch_bounds__(256) void k_rowmul_mfma(size_t n, ArrPtrs arrs, int narr, int ld,
                                                     int m, const double* __restrict__ M,
                                                     int kout, int mode, int kv, int kc, int pcol,
                                                     double* __restrict__ part,
                                                     const DevStatus* st) {
  if (halted(st)) return;
  extern __shared__ double sh[];
  const int mp = (m + 3) & ~3;
  const int xs = mp + 1;        // padded row stride of the X tile
  const int koutp = TJ * 16;
  double* sM = sh;                      // mp x koutp
  double* sX = sM + mp * koutp;         // kRT x xs
  double* sV = sX + kRT * xs;           // kRT x kc (mode 1)
  __shared__ double dred[4][2][TJ * 16];
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63;
  const int li = l & 15, lk = l >> 4;
  for (int e = tid; e < mp * koutp; e += 256) {
    const int q = e / koutp, col = e - q * koutp;
    double v = 0.0;
    if (q < m && col < kout) {
      if (mode == 0) {
        v = M[q * kout + col];
      } else {
        const int c0 = (col < kc) ? col : col - kc;
        v = (col >= kc && q < kv) ? 0.0 : M[q * kc + c0];
      }
    }
    sM[e] = v;
  }
  double dsum[TJ][2];
#pragma unroll
  for (int t = 0; t < TJ; ++t) dsum[t][0] = dsum[t][1] = 0.0;
  const size_t ntiles = (n + kRT - 1) / kRT;
  for (size_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const size_t p0 = tile * kRT;
    const int nr = (n - p0 < (size_t)kRT) ? (int)(n - p0) : kRT;
    for (int a = 0; a < narr; ++a) {
      double* Xa = arrs.a[a];
      __syncthreads();
      {
        const int tot = kRT * mp;
#pragma unroll 8
        for (int e = tid; e < tot; e += 256) {
          const int r = e / mp, c = e - r * mp;
          sX[r * xs + c] = (r < nr && c < m) ? Xa[(p0 + r) * ld + c] : 0.0;
        }
      }
      __syncthreads();
      d4 acc[TJ];
#pragma unroll
      for (int t = 0; t < TJ; ++t) acc[t] = (d4){0.0, 0.0, 0.0, 0.0};
      for (int kk = 0; kk < mp / 4; ++kk) {
        const double av = sX[(w * 16 + li) * xs + 4 * kk + lk];
#pragma unroll
        for (int t = 0; t < TJ; ++t)
          acc[t] = mfma(av, sM[(4 * kk + lk) * koutp + t * 16 + li], acc[t]);
      }
#pragma unroll
      for (int t = 0; t < TJ; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = w * 16 + 4 * r + lk, col = t * 16 + li;
          if (row >= nr || col >= kout) continue;
          const double v = acc[t][r];
          double* dst = Xa + (p0 + row) * ld;
          if (mode == 0) {
            dst[col] = v;
          } else if (col < kc) {
            dst[col] = v;
            if (a == 0) sV[row * kc + col] = v;
            if (a == 1) {
              const double vv = sV[row * kc + col];
              dsum[t][0] += vv * vv;
              dsum[t][1] += vv * v;
            }
          } else {
            dst[pcol + col - kc] = v;
          }
        }
    }
  }
  if (mode == 1 && part) {
    // lanes with the same li (and t) hold the same column: sum over lk by
    // shuffles, then over the 4 wavefronts in LDS
#pragma unroll
    for (int t = 0; t < TJ; ++t)
      for (int v = 0; v < 2; ++v) {
        double x = dsum[t][v];
        x += __shfl_xor(x, 16);
        x += __shfl_xor(x, 32);
        if (lk == 0) dred[w][v][t * 16 + li] = x;
      }
    __syncthreads();
    for (int c = tid; c < kc; c += 256) {
      double s0 = 0.0, s1 = 0.0;
      for (int q = 0; q < 4; ++q) s0 += dred[q][0][c], s1 += dred[q][1][c];
      part[(size_t)blockIdx.x * 2 * kc + c] = s0;
      part[(size_t)blockIdx.x * 2 * kc + kc + c] = s1;
    }
  }
}

size_t rowmul_mfma_shm(int m, int kout, int kc) {
  const int mp = (m + 3) & ~3;
  const int koutp = ((kout + 15) / 16) * 16;
  return ((size_t)mp * koutp + (size_t)kRT * (mp + 1) + (size_t)kRT * kc) * sizeof(double);
}

int rowmul_mfma_ok(int m, int kout) { return kout <= 9 * 16 && m <= 144; }

void launch_rowmul_mfma(size_t n, double* const* X, int narr, int ld, int m, const double* M,
                        int kout, int mode, int kv, int kc, int pcol, double* part, int nblk,
                        const DevStatus* st, hipStream_t s) {
  ArrPtrs a{};
  for (int i = 0; i < narr; ++i) a.a[i] = X[i];
  const int TJ = (kout + 15) / 16;
  const size_t shm = rowmul_mfma_shm(m, kout, mode == 1 ? kc : 0);
  const double bytes = (mode == 0) ? 2.0 * narr * n * m * 8.0 : (double)narr * n * (m + kout) * 8.0;
  const int cat = (mode == 0) ? KC_TRANSFORM : KC_UPDATE;
  prof_begin(cat, bytes, 2.0 * narr * n * (double)m * kout, s);
#define ROW_CASE(T)                                                                             \
  case T:                                                                                       \
    hipLaunchKernelGGL(k_rowmul_mfma<T>, dim3(nblk), dim3(256), shm, s, n, a, narr, ld, m, M,  \
                       kout, mode, kv, kc, pcol, part, st);                                     \
    break;
  switch (TJ) {
    ROW_CASE(1) ROW_CASE(2) ROW_CASE(3) ROW_CASE(4) ROW_CASE(5) ROW_CASE(6) ROW_CASE(7)
    ROW_CASE(8) ROW_CASE(9)
    default: break;
  }
#undef ROW_CASE
  prof_end(cat, s);
}

hipError_t mfma_set_attributes(int m, int kint) {
  // largest dynamic LDS each kernel can ask for at these sizes
  const int kouts[2] = {m, 2 * kint};
  hipError_t e = hipSuccess;
#define SET_ROW(T)                                                                        \
  e = hipFuncSetAttribute((const void*)k_rowmul_mfma<T>,                                  \
                          hipFuncAttributeMaxDynamicSharedMemorySize,                     \
                          (int)rowmul_mfma_shm(m, 144, kint));                            \
  if (e != hipSuccess) return e;
  SET_ROW(1) SET_ROW(2) SET_ROW(3) SET_ROW(4) SET_ROW(5) SET_ROW(6) SET_ROW(7) SET_ROW(8)
  SET_ROW(9)
#undef SET_ROW
  (void)kouts;
  return e;
}

}  // namespace plhr
