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
#include <algorithm>
#include <cstdint>

#include "mfma.cuh"

namespace plhr {

__global__ __launch_bounds__(768) void k_gram_mfma(size_t n, const double* __restrict__ X, int ldx,
                                                   int mx, const double* __restrict__ Y1, int ldy1,
                                                   int my1, const double* __restrict__ Y2, int ldy2,
                                                   int my, int nw, double* __restrict__ part,
                                                   const DevStatus* st) {
  if (halted(st)) return;
  const size_t chunk = ((n + gridDim.x - 1) / gridDim.x + 3) / 4 * 4;
  const size_t pb = (size_t)blockIdx.x * chunk;
  const size_t pe = (pb + chunk < n) ? pb + chunk : n;
  gram_body(pb, pe, X, ldx, mx, Y1, ldy1, my1, Y2, ldy2, my, nw,
            part + (size_t)blockIdx.x * mx * my);
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
  if (e < total) {
    // eight loads in flight, added in the same order as one at a time
    int q = g;
    for (; q + 56 < nblk; q += 64) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(q + 8 * u) * total + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; q < nblk; q += 8) s += part[(size_t)q * total + e];
  }
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

// Complex Hermitian Gram from the real Gram of the interleaved views:
// with X' and Y' the (re, im)-interleaved real blocks, G'(2a+s, 2b+t) =
// sum_p X'[p, 2a+s] Y'[p, 2b+t], and
//   (X^H Y)(a, b) = G'(2a, 2b) + G'(2a+1, 2b+1)
//                   + i (G'(2a, 2b+1) - G'(2a+1, 2b)).
// Gc is one mxc x myc chunk of G' (row-major, even sizes) whose first
// entry is G'(2 a0, 2 b0); G is mx x ldg complex, row-major.
__global__ __launch_bounds__(256) void k_cgram_combine(const double* __restrict__ Gc, int mxc,
                                                       int myc, int a0, int b0,
                                                       double2* __restrict__ G, int ldg) {
  const int ha = mxc / 2, hb = myc / 2;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ha * hb; t += gridDim.x * blockDim.x) {
    const int a = t / hb, b = t - a * hb;
    const double* r0 = Gc + (size_t)(2 * a) * myc + 2 * b;
    const double* r1 = r0 + myc;
    G[(size_t)(a0 + a) * ldg + b0 + b] = make_double2(r0[0] + r1[1], r0[1] - r1[0]);
  }
}

size_t cgram_workspace_bytes(size_t n, int mx, int my) {
  const int nblk = gram_blocks(n);
  const int cx = std::min(2 * mx, 128), cy = std::min(2 * my, 192);
  return ((size_t)nblk * cx * cy * 8 + 255) / 256 * 256 + (size_t)cx * cy * 8;
}

// G = X^H Y (complex128, n x mx and n x my, point-major): the real Gram of
// the interleaved views in chunks of at most 128 x 192 real columns (the
// MFMA Gram's shape limits), each combined into its block of G.
void launch_cgram(size_t n, const double* X, int mx, const double* Y, int my, double* G,
                  double* ws, hipStream_t s) {
  const int nblk = gram_blocks(n);
  const int cx = std::min(2 * mx, 128), cy = std::min(2 * my, 192);
  double* part = ws;
  double* gc = ws + ((size_t)nblk * cx * cy * 8 + 255) / 256 * 256 / 8;
  for (int x0 = 0; x0 < 2 * mx; x0 += cx) {
    const int mxc = std::min(cx, 2 * mx - x0);
    for (int y0 = 0; y0 < 2 * my; y0 += cy) {
      const int myc = std::min(cy, 2 * my - y0);
      launch_gram_mfma(n, X + x0, 2 * mx, mxc, Y + y0, 2 * my, myc, nullptr, 0, myc, part, nblk,
                       gc, nullptr, s);
      const int tot = (mxc / 2) * (myc / 2);
      hipLaunchKernelGGL(k_cgram_combine, dim3((tot + 255) / 256), dim3(256), 0, s, gc, mxc,
                         myc, x0 / 2, y0 / 2, reinterpret_cast<double2*>(G), my);
    }
  }
}

template <int TJ>
__global__ __launch_bounds__(256, 2) void k_rowmul_mfma(size_t n, ArrPtrs arrs, int narr, int ld,
                                                        int m, const double* __restrict__ M,
                                                        int kout, int mode, int kv, int kc,
                                                        int pcol, double* __restrict__ part,
                                                        const DevStatus* st) {
  if (halted(st)) return;
  rowmul_body<TJ>(0, n, (size_t)blockIdx.x * 4, (size_t)gridDim.x * 4, arrs, narr, ld, m, M, kout,
                  mode, kv, kc, pcol, part ? part + (size_t)blockIdx.x * 2 * kc : nullptr);
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
  (void)m;
  (void)kint;
  hipError_t e = hipSuccess;
#define SET_ROW(T)                                          \
  e = set_lds_limit((const void*)k_rowmul_mfma<T>);         \
  if (e != hipSuccess) return e;
  SET_ROW(1) SET_ROW(2) SET_ROW(3) SET_ROW(4) SET_ROW(5) SET_ROW(6)
#undef SET_ROW
  return e;
}

}  // namespace plhr
