// Device bodies of the FP64 matrix-core (MFMA) Gram and row-product
// kernels, shared by the single-problem kernels (k_mfma.hip) and the
// batched ones (k_batch.hip).
//
// Both use v_mfma_f64_16x16x4f64, D(16x16) += A(16x4) B(4x16), with the
// operand layout of that instruction: lane l holds A[l%16][l/16] and
// B[l/16][l%16]; accumulator register r of lane l is D[4r + l/16][l%16].
#pragma once
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

// Rows [pb, pe) of X and Ycat; the partial (mx x my) goes to out.
__device__ __forceinline__ void gram_body(size_t pb, size_t pe, const double* __restrict__ X,
                                          int ldx, int mx, const double* __restrict__ Y1,
                                          int ldy1, int my1, const double* __restrict__ Y2,
                                          int ldy2, int my, int nw, double* __restrict__ out) {
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
  // 16-byte operand loads need even column counts and leading dimensions
  // and 16-byte aligned blocks (uniform); otherwise each element is loaded
  // on its own
  const bool vec = (((mx | my | my1 | ldx | ldy1 | ldy2) & 1) == 0) &&
                   ((((uintptr_t)X | (uintptr_t)Y1 | (uintptr_t)Y2) & 15) == 0);
  auto yel = [&](size_t p, int cj) -> double {
    if (cj >= my) return 0.0;
    return (cj < my1) ? Y1[p * ldy1 + cj] : Y2[p * ldy2 + (cj - my1)];
  };
  // operands of one step (4 rows); the next step's loads are issued
  // before the current step's MFMAs
  auto load = [&](size_t p0, double2& av, double2* bv) {
    const size_t p = p0 + lk;
    const bool rok = p < pe;
    av = {0.0, 0.0};
    if (rok && ci < mx) {
      if (vec) {
        av = *reinterpret_cast<const double2*>(X + p * ldx + ci);
      } else {
        av.x = X[p * ldx + ci];
        av.y = (ci + 1 < mx) ? X[p * ldx + ci + 1] : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < kJPW; ++q) {
      const int cj = 32 * (kJPW * wj + q) + 2 * li;
      bv[q] = {0.0, 0.0};
      if (rok && cj < my) {
        if (vec) {
          const double* src = (cj < my1) ? Y1 + p * ldy1 + cj : Y2 + p * ldy2 + (cj - my1);
          bv[q] = *reinterpret_cast<const double2*>(src);
        } else {
          bv[q].x = yel(p, cj);
          bv[q].y = yel(p, cj + 1);
        }
      }
    }
  };
  // a ring of kDepth steps of operands in registers: slot d is consumed
  // and refilled with the step kDepth steps ahead (rows past pe load
  // zeros), so kDepth x 4 rows of loads are in flight behind the MFMAs
  constexpr int kDepth = 4;
  double2 av[kDepth], bv[kDepth][kJPW];
#pragma unroll
  for (int d = 0; d < kDepth; ++d) load(pb + 4 * d, av[d], bv[d]);
  for (size_t p0 = pb; p0 < pe; p0 += 4 * kDepth) {
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
#pragma unroll
      for (int q = 0; q < kJPW; ++q) {
        acc[0][2 * q] = mfma(av[d].x, bv[d][q].x, acc[0][2 * q]);
        acc[0][2 * q + 1] = mfma(av[d].x, bv[d][q].y, acc[0][2 * q + 1]);
        acc[1][2 * q] = mfma(av[d].y, bv[d][q].x, acc[1][2 * q]);
        acc[1][2 * q + 1] = mfma(av[d].y, bv[d][q].y, acc[1][2 * q + 1]);
      }
      load(p0 + 4 * (kDepth + d), av[d], bv[d]);
    }
  }
  // lane (li, lk) holds D[4r + lk][li] of each tile: output row
  // 32 wi + 2(4r + lk) + a, column 32 jp + 2 li + b
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
// to slots [pcol, pcol + kc); the column sums of v*(Bv) and v*(Qv) are
// accumulated into part (nblk x 2kc): v from array 0, Qv from array 1,
// Bv from array 3 when there are four arrays (else B = I).
static constexpr int kMaxKq = (kMaxM + 3) / 4;

// Rows [pbeg, pend) of the arrays (pbeg a multiple of 16; tiles of 16
// rows taken by the block's wavefronts from tile `first` with stride
// `stride`); the column sums of mode 1 go to part[0 .. 2kc).
template <int TJ>
__device__ __forceinline__ void rowmul_body(size_t pbeg, size_t pend, size_t first,
                                            size_t stride, ArrPtrs arrs, int narr, int ld, int m,
                                            const double* __restrict__ M, int kout, int mode,
                                            int kv, int kc, int pcol, double* __restrict__ part) {
  extern __shared__ __attribute__((aligned(16))) double sh[];
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
  const size_t ntiles = (pend - pbeg + 15) / 16;
  const size_t n = pend;
  const double* sB = sM + (lk * kq) * sms + li;
  // work items (tile, array) of this wavefront in order; the operands of
  // item it + 1 are loaded into registers while item it is multiplied
  const size_t nmine = (first + w < ntiles) ? (ntiles - first - w + stride - 1) / stride : 0;
  const size_t nitems = nmine * (size_t)narr;
  auto fetch = [&](size_t it, double* A) {
    const size_t tile = first + w + stride * (it / narr);
    const int a = (int)(it % narr);
    const size_t p0 = pbeg + tile * 16;
    const bool rowok = (it < nitems) && (p0 + li < n);
    const double* Xa = arrs.at(a);
    const double* src = Xa + (rowok ? (p0 + li) * ld + lk * kq : 0);
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
  };
  double vkeep[TJ][4];
  double Acur[kMaxKq], Anext[kMaxKq];
  if (nitems > 0) fetch(0, Acur);
  for (size_t it = 0; it < nitems; ++it) {
    fetch(it + 1, Anext);  // past the last item: zeros, no load
    const size_t tile = first + w + stride * (it / narr);
    const int a = (int)(it % narr);
    const size_t p0 = pbeg + tile * 16;
    double* Xa = arrs.at(a);
    d4 acc[TJ];
#pragma unroll
    for (int t = 0; t < TJ; ++t) acc[t] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < kMaxKq; ++kk) {
      if (kk < kq) {
#pragma unroll
        for (int t = 0; t < TJ; ++t) acc[t] = mfma(Acur[kk], sB[kk * sms + t * 16], acc[t]);
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
            if (narr < 4) dsum[t][0] += vv * vv;
            dsum[t][1] += vv * v;
          }
          if (a == 3) dsum[t][0] += vkeep[t][r] * v;  // v.(Bv) with B X as array 3
        } else {
          dst[pcol + col - kc] = v;
        }
      }
#pragma unroll
    for (int j = 0; j < kMaxKq; ++j) Acur[j] = Anext[j];
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
      part[c] = s0;
      part[kc + c] = s1;
    }
  }
}

}  // namespace plhr
