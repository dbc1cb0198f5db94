// Cholesky-QR orthonormalisation of a complex block (the orthonormalising
// step of the complex iteration, Section 4): with G = Z^H Z = R^H R (R
// upper triangular with a real positive diagonal), Q = Z R^-1.
//
//   k_cchol_inv  one workgroup: R and R^-1 from G, in LDS (m <= 64)
//   k_cright     Q = Z R^-1, tiles of rows spread over workgroups, R^-1
//                and the tile in LDS (the vector form, triangular or full)
//   k_crowmul_mfma  the general product Y = Z M of the block updates on
//                the FP64 matrix cores
#include <cmath>

#include "common.cuh"

namespace plhr {

namespace {
__device__ __forceinline__ double2 cmac(double2 acc, double2 a, double2 b) {
  return make_double2(acc.x + (a.x * b.x - a.y * b.y), acc.y + (a.x * b.y + a.y * b.x));
}
}  // namespace

__global__ __launch_bounds__(256) void k_cchol_inv(int m, const double2* __restrict__ G,
                                                   double2* __restrict__ R,
                                                   double2* __restrict__ Rinv,
                                                   int* __restrict__ fail) {
  extern __shared__ double2 sh[];
  double2* A = sh;          // m x m: G, then R in its upper triangle
  double2* X = sh + m * m;  // m x m: R^-1
  __shared__ int bad;
  const int t = threadIdx.x;
  for (int e = t; e < m * m; e += blockDim.x) A[e] = G[e];
  if (t == 0) bad = 0;
  __syncthreads();
  double maxd = 0.0;
  for (int j = 0; j < m; ++j) maxd = fmax(maxd, A[j * m + j].x);
  for (int j = 0; j < m; ++j) {
    const double d = A[j * m + j].x;  // the same value in every lane
    if (!(d > 1e-14 * maxd)) {        // uniform: not positive definite to rounding
      if (t == 0) bad = 1;
      break;
    }
    const double rd = sqrt(d), inv = 1.0 / rd;
    __syncthreads();
    for (int i = j + t; i < m; i += blockDim.x) {
      const double2 a = A[j * m + i];
      A[j * m + i] = (i == j) ? make_double2(rd, 0.0) : make_double2(a.x * inv, a.y * inv);
    }
    __syncthreads();
    // trailing update of the upper triangle: A[r][c] -= conj(R[j][r]) R[j][c]
    const int w = m - j - 1;
    for (int e = t; e < w * w; e += blockDim.x) {
      const int r = j + 1 + e / w, c = j + 1 + e % w;
      if (c < r) continue;
      const double2 u = A[j * m + r], v = A[j * m + c];
      const double2 a = A[r * m + c];
      A[r * m + c] = make_double2(a.x - (u.x * v.x + u.y * v.y), a.y - (u.x * v.y - u.y * v.x));
    }
    __syncthreads();
  }
  __syncthreads();
  const int failed = bad;
  if (!failed && t < m) {
    // column t of R^-1 by back substitution: R X = e_t
    const int c = t;
    for (int i = c; i >= 0; --i) {
      double2 s = make_double2(i == c ? 1.0 : 0.0, 0.0);
      for (int k = i + 1; k <= c; ++k) {
        const double2 r = A[i * m + k], x = X[k * m + c];
        s = make_double2(s.x - (r.x * x.x - r.y * x.y), s.y - (r.x * x.y + r.y * x.x));
      }
      const double rii = A[i * m + i].x;
      X[i * m + c] = make_double2(s.x / rii, s.y / rii);
    }
  }
  __syncthreads();
  for (int e = t; e < m * m; e += blockDim.x) {
    const int i = e / m, c = e - i * m;
    const bool up = (c >= i) && !failed;
    if (R) R[e] = up ? A[e] : make_double2(0.0, 0.0);
    Rinv[e] = up ? X[e] : make_double2(0.0, 0.0);
  }
  if (t == 0) *fail = failed;
}

// Y = Z M (Z n x m, M m x k, k <= 64) by tiles of 16 rows staged in LDS
// next to M: lane (b, g) (b = column, g = row group) accumulates the rows
// g, g + 4, g + 8, g + 12 of the tile; the row values are LDS broadcasts
// within a wavefront.  tri: M upper triangular (R^-1 of the Cholesky-QR),
// the sum for column b stops at a = b.
constexpr int kCrTile = 16;

__global__ __launch_bounds__(256) void k_cright(size_t n, int m, int k, int tri,
                                                const double2* __restrict__ Z,
                                                const double2* __restrict__ M,
                                                double2* __restrict__ Q) {
  extern __shared__ double2 ri[];
  double2* zt = ri + m * k;
  for (int e = threadIdx.x; e < m * k; e += blockDim.x) ri[e] = M[e];
  const int b = threadIdx.x & 63, g = threadIdx.x >> 6;
  const size_t ntiles = (n + kCrTile - 1) / kCrTile;
  for (size_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const size_t p0 = tile * kCrTile;
    const int rows = (n - p0 < (size_t)kCrTile) ? (int)(n - p0) : kCrTile;
    __syncthreads();  // M loaded; the previous tile's rows consumed
    for (int e = threadIdx.x; e < rows * m; e += blockDim.x) zt[e] = Z[p0 * m + e];
    __syncthreads();
    if (b < k) {
      double2 acc[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = make_double2(0.0, 0.0);
      const int amax = tri ? b : m - 1;
      for (int a = 0; a <= amax; ++a) {
        const double2 r = ri[a * k + b];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = cmac(acc[q], zt[(g + 4 * q) * m + a], r);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = g + 4 * q;
        if (row < rows) Q[(p0 + row) * k + b] = acc[q];
      }
    }
  }
}

// Y = Z M on the FP64 matrix cores (v_mfma_f64_16x16x4f64; lane l holds
// A[l%16][l/16] and B[l/16][l%16], accumulator r of lane l is
// D[4r + l/16][l%16]).  With Z', Y' the interleaved real views (n x 2m,
// n x 2k), Y' = Z' M' where M' (2m x 2k) holds each complex entry of M as
// the real 2 x 2 block [[re, im], [-im, re]]; M' is built in LDS.  Each
// wavefront takes 16-row tiles of Z' and all 2k columns (up to 8 tiles of
// 16), stepping the contraction 4 at a time.
typedef double cd4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_crowmul_mfma(size_t n, int m, int k,
                                                      const double* __restrict__ Z,
                                                      const double2* __restrict__ M,
                                                      double* __restrict__ Y) {
  extern __shared__ double mp[];  // 2m x 2k, rows padded to an odd stride
  const int K2 = 2 * m, N2 = 2 * k, NP = N2 + 1;
  for (int e = threadIdx.x; e < m * k; e += blockDim.x) {
    const int a = e / k, b = e - a * k;
    const double2 v = M[e];
    mp[(2 * a) * NP + 2 * b] = v.x;
    mp[(2 * a) * NP + 2 * b + 1] = v.y;
    mp[(2 * a + 1) * NP + 2 * b] = -v.y;
    mp[(2 * a + 1) * NP + 2 * b + 1] = v.x;
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int li = l & 15, lk = l >> 4;
  const int nct = (N2 + 15) / 16;
  const size_t ntiles = (n + 15) / 16;
  for (size_t tile = (size_t)blockIdx.x * 4 + w; tile < ntiles; tile += (size_t)gridDim.x * 4) {
    const size_t row0 = tile * 16;
    const size_t ra = row0 + li;  // this lane's A row
    cd4 acc[8];
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) acc[ct] = (cd4){0.0, 0.0, 0.0, 0.0};
    for (int kk = 0; kk < K2; kk += 4) {
      const int kc = kk + lk;
      const double a = (ra < n && kc < K2) ? Z[ra * K2 + kc] : 0.0;
#pragma unroll
      for (int ct = 0; ct < 8; ++ct) {
        if (ct < nct) {
          const int col = ct * 16 + li;
          const double b = (kc < K2 && col < N2) ? mp[kc * NP + col] : 0.0;
          acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[ct], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) {
      if (ct >= nct) continue;
      const int col = ct * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const size_t row = row0 + 4 * r + lk;
        if (row < n && col < N2) Y[row * N2 + col] = acc[ct][r];
      }
    }
  }
}

static bool cchol_attr_done = false;

static hipError_t cplx_attrs() {
  if (cchol_attr_done) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)k_cchol_inv,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(2 * 64 * 64 * sizeof(double2)));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_cright, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)((64 * 64 + kCrTile * 64) * sizeof(double2)));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_crowmul_mfma, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(128 * 129 * sizeof(double)));
  if (e != hipSuccess) return e;
  cchol_attr_done = true;
  return hipSuccess;
}

static void launch_cright(size_t n, int m, int k, int tri, const double* Z, const double* M,
                          double* Y, hipStream_t s) {
  size_t nb = (n + kCrTile - 1) / kCrTile;
  if (nb > 2048) nb = 2048;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_cright, dim3((unsigned)nb), dim3(256),
                     (size_t)(m * k + kCrTile * m) * sizeof(double2), s, n, m, k, tri,
                     reinterpret_cast<const double2*>(Z), reinterpret_cast<const double2*>(M),
                     reinterpret_cast<double2*>(Y));
}

hipError_t launch_crowmul(size_t n, int m, int k, const double* Z, const double* M, double* Y,
                          hipStream_t s) {
  const hipError_t e = cplx_attrs();
  if (e != hipSuccess) return e;
  size_t nb = (n + 63) / 64;  // four 16-row tiles per workgroup
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_crowmul_mfma, dim3((unsigned)nb), dim3(256),
                     (size_t)2 * m * (2 * k + 1) * sizeof(double), s, n, m, k, Z,
                     reinterpret_cast<const double2*>(M), Y);
  return hipGetLastError();
}

hipError_t launch_cholqr_tail(size_t n, int m, const double* Z, const double* G, double* R,
                              double* Rinv, int* fail, double* Q, hipStream_t s) {
  const size_t lds = (size_t)2 * m * m * sizeof(double2);
  const hipError_t e = cplx_attrs();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cchol_inv, dim3(1), dim3(256), lds, s, m,
                     reinterpret_cast<const double2*>(G), reinterpret_cast<double2*>(R),
                     reinterpret_cast<double2*>(Rinv), fail);
  launch_cright(n, m, m, 1, Z, Rinv, Q, s);
  return hipGetLastError();
}

}  // namespace plhr
