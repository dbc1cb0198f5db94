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
#include <cstdint>

#include "common.cuh"

namespace plhr {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- Gram
// out(i, j) = sum_p X[p, i] Ycat[p, j] over the block's chunk of rows,
// Ycat = [Y1 | Y2] (my1 + (my - my1) columns).  The reduction index of the
// instruction is the row p: lane (li, lk) supplies A = X[p + lk, i(li)]
// and B = Ycat[p + lk, j(li)], so every load is a row segment.  Each lane
// loads two adjacent columns at once (16 bytes), which feed two MFMA
// tiles (even and odd columns).  Wavefront (wi, wj) of the block owns the
// output rows 32 wi .. 32 wi + 31 and the kJPW column pairs (32 columns
// each) starting at pair kJPW wj.  Operands come straight from global
// memory (no LDS); the accumulators stay small enough for several
// wavefronts per SIMD.
static constexpr int kJPW = 2;

__global__ __launch_bounds__(768) void k_gram_mfma(size_t n, const double* __restrict__ X, int ldx,
                                                   int mx, const double* __restrict__ Y1, int ldy1,
                                                   int my1, const double* __restrict__ Y2, int ldy2,
                                                   int my, int nw, double* __restrict__ part,
                                                   const DevStatus* st) {
  if (halted(st)) return;
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63;
  const int wi = w % nw, wj = w / nw;
  const int li = l & 15, lk = l >> 4;
  const int ci = 32 * wi + 2 * li;  // this lane's X column pair
  d4 acc[2][2 * kJPW];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int t = 0; t < 2 * kJPW; ++t) acc[a][t] = (d4){0.0, 0.0, 0.0, 0.0};
  const size_t chunk = ((n + gridDim.x - 1) / gridDim.x + 3) / 4 * 4;
  const size_t pb = (size_t)blockIdx.x * chunk;
  const size_t pe = (pb + chunk < n) ? pb + chunk : n;
  const bool xok = ci < mx;  // mx even: the pair is whole or absent
  // operands of one step (4 rows); the next step's loads are issued
  // before the current step's MFMAs
  auto load = [&](size_t p0, double2& av, double2* bv) {
    const size_t p = p0 + lk;
    const bool rok = p < pe;
    av = {0.0, 0.0};
    if (rok && xok) av = *reinterpret_cast<const double2*>(X + p * ldx + ci);
#pragma unroll
    for (int q = 0; q < kJPW; ++q) {
      const int cj = 32 * (kJPW * wj + q) + 2 * li;
      bv[q] = {0.0, 0.0};
      if (rok && cj < my) {
        const double* src = (cj < my1) ? Y1 + p * ldy1 + cj : Y2 + p * ldy2 + (cj - my1);
        bv[q] = *reinterpret_cast<const double2*>(src);
      }
    }
  };
  double2 av, bv[kJPW];
  load(pb, av, bv);
  for (size_t p0 = pb; p0 < pe; p0 += 4) {
    double2 an, bn[kJPW];
    load(p0 + 4, an, bn);  // rows past pe load zeros
#pragma unroll
    for (int q = 0; q < kJPW; ++q) {
      acc[0][2 * q] = mfma(av.x, bv[q].x, acc[0][2 * q]);
      acc[0][2 * q + 1] = mfma(av.x, bv[q].y, acc[0][2 * q + 1]);
      acc[1][2 * q] = mfma(av.y, bv[q].x, acc[1][2 * q]);
      acc[1][2 * q + 1] = mfma(av.y, bv[q].y, acc[1][2 * q + 1]);
    }
    av = an;
#pragma unroll
    for (int q = 0; q < kJPW; ++q) bv[q] = bn[q];
  }
  // lane (li, lk) holds D[4r + lk][li] of each tile: output row
  // 32 wi + 2(4r + lk) + a, column 32 jp + 2 li + b
  double* out = part + (size_t)blockIdx.x * mx * my;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int q = 0; q < kJPW; ++q)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 32 * wi + 2 * (4 * r + lk) + a, j = 32 * (kJPW * wj + q) + 2 * li + b;
          if (i < mx && j < my) out[(size_t)i * my + j] = acc[a][2 * q + b][r];
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

// Shapes the kernel handles: up to 4 x 3 wavefronts (mx <= 128 rows,
// my <= 192 columns), even column counts (16-byte operand loads).
int gram_mfma_ok(int mx, int my) { return mx <= 128 && my <= 192 && mx % 2 == 0 && my % 2 == 0; }

void launch_gram_mfma(size_t n, const double* X, int ldx, int mx, const double* Y1, int ldy1,
                      int my1, const double* Y2, int ldy2, int my, double* part, int nblk,
                      double* out, const DevStatus* st, hipStream_t s) {
  const int NW = (mx + 31) / 32, NJH = ((my + 31) / 32 + kJPW - 1) / kJPW;
  dim3 grid(nblk), block(64 * NW * NJH);
  prof_begin(KC_GRAM, (double)n * (mx + my) * 8.0, 2.0 * n * mx * my, s);
  hipLaunchKernelGGL(k_gram_mfma, grid, block, 0, s, n, X, ldx, mx, Y1, ldy1, my1, Y2, ldy2, my,
                     NW, part, st);
  prof_end(KC_GRAM, s);
  const int total = mx * my;
  prof_begin(KC_GRAM_REDUCE, (double)nblk * total * 8.0, (double)nblk * total, s);
  hipLaunchKernelGGL(k_gram_reduce8, dim3((total + 31) / 32), dim3(256), 0, s, part, nblk, total,
                     out, st);
  prof_end(KC_GRAM_REDUCE, s);
}

// ------------------------------------------------------------ row product
// Each wavefront owns 16-row tiles (grid-stride over tiles); the block's 4
// wavefronts share B (m x kout) in LDS, loaded once per block.
//
// The contraction index k is permuted so that each lane's operands are
// contiguous: at step kk (0 <= kk < kq = m/4) lane (li, lk) supplies
// A = X[row li][lk kq + kk] and B = M[lk kq + kk][t 16 + li]; the four lk
// groups together cover k = lk kq + kk, so after kq steps every k in
// [0, m) has been summed exactly once.  A lane's kq values of X are one
// contiguous run of its row (16-byte loads), held in registers: the tile
// is read once and written in place after all of it has been read.
//
// mode 0 (B-orthonormalising transform): X_a[p, 0:m] <- X_a[p, 0:m] M.
// mode 1 (Ritz-vector update) with Y (m x kc): the product uses
//   [Y | Y with rows < kv zeroed]  (kout = 2 kc),
// columns [0, kc) (new V) go to slots [0, kc), columns [kc, 2kc) (new P)
// to slots [pcol, pcol + kc); for arrays 0 and 1 the column sums of v*v
// and v*(Qv) are accumulated into part (nblk x 2kc).
static constexpr int kMaxKq = (kMaxM + 3) / 4;

template <int TJ>
__global__ __launch_bounds__(256, 2) void k_rowmul_mfma(size_t n, ArrPtrs arrs, int narr, int ld,
                                                        int m, const double* __restrict__ M,
                                                        int kout, int mode, int kv, int kc,
                                                        int pcol, double* __restrict__ part,
                                                        const DevStatus* st) {
  if (halted(st)) return;
  extern __shared__ double sh[];
  const int kq = m / 4;               // m = 4 kint
  const int sms = TJ * 16 + 4;        // padded row stride of B in LDS
  double* sM = sh;                    // m x sms
  __shared__ double dred[4][2][TJ * 16];
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63;
  const int li = l & 15, lk = l >> 4;
  for (int e = tid; e < m * TJ * 16; e += 256) {
    const int q = e / (TJ * 16), col = e - q * (TJ * 16);
    double v = 0.0;
    if (col < kout) {
      if (mode == 0) {
        v = M[q * kout + col];
      } else {
        const int c0 = (col < kc) ? col : col - kc;
        v = (col >= kc && q < kv) ? 0.0 : M[q * kc + c0];
      }
    }
    sM[q * sms + col] = v;
  }
  __syncthreads();
  const bool vec2 = ((ld & 1) == 0) && ((kq & 1) == 0);
  double dsum[TJ][2];
#pragma unroll
  for (int t = 0; t < TJ; ++t) dsum[t][0] = dsum[t][1] = 0.0;
  const size_t ntiles = (n + 15) / 16;
  const double* sB = sM + (lk * kq) * sms + li;
  for (size_t tile = (size_t)blockIdx.x * 4 + w; tile < ntiles; tile += (size_t)gridDim.x * 4) {
    const size_t p0 = tile * 16;
    const bool rowok = (p0 + li < n);
    double vkeep[TJ][4];
    for (int a = 0; a < narr; ++a) {
      double* Xa = arrs.a[a];
      double A[kMaxKq];
      const double* src = Xa + (p0 + li) * ld + lk * kq;
      if (rowok && vec2 && ((((uintptr_t)Xa) & 15) == 0)) {
#pragma unroll
        for (int j = 0; j < kMaxKq; j += 2)
          if (j < kq) {
            const double2 v = *reinterpret_cast<const double2*>(src + j);
            A[j] = v.x;
            if (j + 1 < kMaxKq) A[j + 1] = v.y;
          }
      } else {
#pragma unroll
        for (int j = 0; j < kMaxKq; ++j) A[j] = (rowok && j < kq) ? src[j] : 0.0;
      }
      d4 acc[TJ];
#pragma unroll
      for (int t = 0; t < TJ; ++t) acc[t] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < kMaxKq; ++kk) {
        if (kk < kq) {
#pragma unroll
          for (int t = 0; t < TJ; ++t) acc[t] = mfma(A[kk], sB[kk * sms + t * 16], acc[t]);
        }
      }
      // lane (li, lk) holds D[4r + lk][t 16 + li]
#pragma unroll
      for (int t = 0; t < TJ; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 4 * r + lk, col = t * 16 + li;
          const double v = acc[t][r];
          if (p0 + row >= n || col >= kout) continue;
          double* dst = Xa + (p0 + row) * ld;
          if (mode == 0) {
            dst[col] = v;
          } else if (col < kc) {
            dst[col] = v;
            if (a == 0) vkeep[t][r] = v;
            if (a == 1) {
              const double vv = vkeep[t][r];
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

size_t rowmul_mfma_shm(int m, int kout, int) {
  const int koutp = ((kout + 15) / 16) * 16;
  return (size_t)m * (koutp + 4) * sizeof(double);
}

int rowmul_mfma_ok(int m, int kout) { return kout <= 6 * 16 && m <= kMaxM && (m % 4) == 0; }

void launch_rowmul_mfma(size_t n, double* const* X, int narr, int ld, int m, const double* M,
                        int kout, int mode, int kv, int kc, int pcol, double* part, int nblk,
                        const DevStatus* st, hipStream_t s) {
  ArrPtrs a{};
  for (int i = 0; i < narr; ++i) a.a[i] = X[i];
  const int TJ = (kout + 15) / 16;
  const size_t shm = rowmul_mfma_shm(m, kout, 0);
  const double bytes = (mode == 0) ? 2.0 * narr * n * m * 8.0 : (double)narr * n * (m + kout) * 8.0;
  const int cat = (mode == 0) ? KC_TRANSFORM : KC_UPDATE;
  prof_begin(cat, bytes, 2.0 * narr * n * (double)m * kout, s);
#define ROW_CASE(T)                                                                             \
  case T:                                                                                       \
    hipLaunchKernelGGL(k_rowmul_mfma<T>, dim3(nblk), dim3(256), shm, s, n, a, narr, ld, m, M,  \
                       kout, mode, kv, kc, pcol, part, st);                                     \
    break;
  switch (TJ) {
    ROW_CASE(1) ROW_CASE(2) ROW_CASE(3) ROW_CASE(4) ROW_CASE(5) ROW_CASE(6)
    default: break;
  }
#undef ROW_CASE
  prof_end(cat, s);
}

hipError_t mfma_set_attributes(int m, int kint) {
  // largest dynamic LDS each row-product instance can ask for
  (void)kint;
  hipError_t e = hipSuccess;
#define SET_ROW(T)                                                                         \
  e = hipFuncSetAttribute((const void*)k_rowmul_mfma<T>,                                   \
                          hipFuncAttributeMaxDynamicSharedMemorySize,                      \
                          (int)rowmul_mfma_shm(m, T * 16, 0));                             \
  if (e != hipSuccess) return e;
  SET_ROW(1) SET_ROW(2) SET_ROW(3) SET_ROW(4) SET_ROW(5) SET_ROW(6)
#undef SET_ROW
  return e;
}

}  // namespace plhr
