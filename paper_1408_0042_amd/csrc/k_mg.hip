// Geometric multigrid V-cycle used as the HPD preconditioner T.
//
// The paper requires T = T^* > 0 (Section 5) and builds its Laplacian
// preconditioners as multigrid V-cycles (Appendix A, Algorithm 4 with
// B_l = L_l on the fine levels).  This is that plain V-cycle:
//   * level l has spacing 2^l h and every dimension halved (cell-centred
//     pairing of neighbouring points), re-discretised stencil, no potential;
//   * weighted Jacobi smoothing, nu_pre sweeps from a zero guess, the same
//     number after the coarse correction;
//   * prolongation P: 3/4 from the parent, 1/4 from the parent's neighbour
//     in each direction (zero outside the Dirichlet box); R = P^T / 2^d;
//   * the coarsest level is solved with a dense inverse formed at setup.
// With R proportional to P^T, equal sweep counts and a symmetric smoother,
// T is symmetric; omega = 2/3 makes the smoother convergent, so T is
// positive definite.
//
// Appendix A's AV-MG (Algorithm 4) and INV-MG (Algorithm 5) reuse the
// same hierarchy with other level operators B_l and Richardson smoothing
// w <- w + alpha_l (r - B_l w):
//   * B_l = L_l (the plain Laplacian; alpha_l = omega / diag makes this
//     weighted Jacobi) where sqrt(sigma / scale) h_l < delta,
//   * B_l = p_m(L_l - sigma I), the Jackson-damped Chebyshev series of |x|
//     of degree m on [-sigma, lambda_max(L_l) - sigma], applied by the
//     three-term recurrence (one stencil pass per degree), on the other
//     levels of AV-MG, alpha_l = 1 / max p_m,
//   * B_l = L_l - sigma I on every level of INV-MG (alpha_l = omega/diag),
// and the coarsest level solved with |L_0 - sigma I_0|^-1 (AV-MG) or
// (L_0 - sigma I_0)^-1 (INV-MG) from a host eigendecomposition.
// A level whose dimensions are all odd coarsens vertex-centred
// (N -> (N - 1)/2, linear interpolation, full weighting R = P^T / 2^d).
//
// Every level works on point-major blocks of ncols columns; kernels assign
// one workgroup per grid row so accesses stay contiguous.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "common.cuh"

namespace plhr {

// Vector access: each thread handles W consecutive columns of one grid
// point (W * sizeof(S) <= 16 bytes per load where the layout allows it).
template <typename T, int N>
using vec = T __attribute__((ext_vector_type(N)));

template <int W, typename S, typename T>
__device__ __forceinline__ vec<S, W> vload(const T* p) {
  if constexpr (sizeof(T) * W <= 16) {
    return __builtin_convertvector(*reinterpret_cast<const vec<T, W>*>(p), vec<S, W>);
  } else {  // four doubles: two 16-byte loads
    const vec<T, 2> a = *reinterpret_cast<const vec<T, 2>*>(p);
    const vec<T, 2> b = *reinterpret_cast<const vec<T, 2>*>(p + 2);
    return vec<S, W>{(S)a.x, (S)a.y, (S)b.x, (S)b.y};
  }
}
template <int W, typename S, typename T>
__device__ __forceinline__ void vstore(T* p, vec<S, W> v) {
  if constexpr (sizeof(T) * W <= 16) {
    *reinterpret_cast<vec<T, W>*>(p) = __builtin_convertvector(v, vec<T, W>);
  } else {
    *reinterpret_cast<vec<T, 2>*>(p) = vec<T, 2>{(T)v.x, (T)v.y};
    *reinterpret_cast<vec<T, 2>*>(p + 2) = vec<T, 2>{(T)v.z, (T)v.w};
  }
}

// Thread layout of the row kernels: ncols / W consecutive threads share
// one grid point (thread t: columns W (t % (ncols/W)) .., point
// t / (ncols/W)), P = blockDim / (ncols/W) points per pass; the remaining
// threads idle.  No division inside the loops.
struct RowLanes {
  int c, i0, P;
  bool on;
};
template <int W>
__device__ __forceinline__ RowLanes row_lanes(int ncols) {
  const int nl = ncols / W;
  RowLanes r;
  r.P = blockDim.x / nl;
  r.c = (threadIdx.x % nl) * W;
  r.i0 = threadIdx.x / nl;
  r.on = r.i0 < r.P;
  return r;
}

template <int DIM, int W, typename S, typename T>
__device__ __forceinline__ vec<S, W> nb_sum(const T* xp, int i, int j, int l, int nx, int ny,
                                            int nz, int ld) {
  const ptrdiff_t sy = (ptrdiff_t)nx * ld;
  const ptrdiff_t sz = (ptrdiff_t)nx * ny * ld;
  vec<S, W> nb = (S)0;
  if (i > 0) nb += vload<W, S>(xp - ld);
  if (i < nx - 1) nb += vload<W, S>(xp + ld);
  if (j > 0) nb += vload<W, S>(xp - sy);
  if (j < ny - 1) nb += vload<W, S>(xp + sy);
  if (DIM == 3) {
    if (l > 0) nb += vload<W, S>(xp - sz);
    if (l < nz - 1) nb += vload<W, S>(xp + sz);
  }
  return nb;
}

// x_out = x_in + w (r - A x_in), A = diag I + off (neighbour sum) (diag
// includes a shift of the level operator; w = omega / diag of the
// Laplacian is weighted Jacobi); x_in == nullptr means zero.
// Level storage and arithmetic in S; r is read as RT (the FP64 input block
// at level 0), the output written as OT; columns [0, split) go to o0, the
// rest to o1 (split is a multiple of W).
template <int DIM, int W, typename S, typename RT, typename OT>
__global__ __launch_bounds__(256) void k_jacobi(int nx, int ny, int nz, S diag, S off, S w,
                                                const S* __restrict__ xin,
                                                const RT* __restrict__ r, int ldr,
                                                OT* __restrict__ o0, int ld0,
                                                OT* __restrict__ o1, int ld1, int split,
                                                int ncols, const DevStatus* st) {
  if (halted(st)) return;
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = row % ny, l = row / ny;
  const RowLanes ln = row_lanes<W>(ncols);
  if (!ln.on) return;
  const size_t rowp = (size_t)row * nx;
  const int c = ln.c;
  OT* const ob = (c < split) ? o0 + c : o1 + (c - split);
  const int ldo = (c < split) ? ld0 : ld1;
  for (int i = ln.i0; i < nx; i += ln.P) {
    const size_t p = rowp + i;
    const vec<S, W> rv = vload<W, S>(r + p * ldr + c);
    vec<S, W> v;
    if (xin) {
      const S* xp = xin + p * ncols + c;
      const vec<S, W> xc = vload<W, S>(xp);
      const vec<S, W> ax = diag * xc + off * nb_sum<DIM, W, S>(xp, i, j, l, nx, ny, nz, ncols);
      v = xc + w * (rv - ax);
    } else {
      v = w * rv;
    }
    vstore<W, S>(ob + p * ldo, v);
  }
}

// The first two sweeps from a zero guess in one pass over r:
//   x1 = w r,  x2 = x1 + w (r - A x1) = w (2 r - w A r)
// (A x1 = w A r because w is a constant).
template <int DIM, int W, typename S, typename RT>
__global__ __launch_bounds__(256) void k_jacobi2z(int nx, int ny, int nz, S diag, S off, S w,
                                                  const RT* __restrict__ r, int ldr,
                                                  S* __restrict__ o, int ncols,
                                                  const DevStatus* st) {
  if (halted(st)) return;
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = row % ny, l = row / ny;
  const RowLanes ln = row_lanes<W>(ncols);
  if (!ln.on) return;
  const size_t rowp = (size_t)row * nx;
  const int c = ln.c;
  for (int i = ln.i0; i < nx; i += ln.P) {
    const size_t p = rowp + i;
    const RT* rp = r + p * ldr + c;
    const vec<S, W> rv = vload<W, S>(rp);
    const vec<S, W> ar = diag * rv + off * nb_sum<DIM, W, S>(rp, i, j, l, nx, ny, nz, ldr);
    vstore<W, S>(o + p * ncols + c, w * ((S)2 * rv - w * ar));
  }
}

// res = r - A x
template <int DIM, int W, typename S, typename RT>
__global__ __launch_bounds__(256) void k_residual(int nx, int ny, int nz, S diag, S off,
                                                  const S* __restrict__ x,
                                                  const RT* __restrict__ r, int ldr,
                                                  S* __restrict__ res, int ncols,
                                                  const DevStatus* st) {
  if (halted(st)) return;
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = row % ny, l = row / ny;
  const RowLanes ln = row_lanes<W>(ncols);
  if (!ln.on) return;
  const size_t rowp = (size_t)row * nx;
  const int c = ln.c;
  for (int i = ln.i0; i < nx; i += ln.P) {
    const size_t p = rowp + i;
    const S* xp = x + p * ncols + c;
    const vec<S, W> ax =
        diag * vload<W, S>(xp) + off * nb_sum<DIM, W, S>(xp, i, j, l, nx, ny, nz, ncols);
    vstore<W, S>(res + p * ncols + c, vload<W, S>(r + p * ldr + c) - ax);
  }
}

// Coarse r = P^T res / 2^d.  One workgroup per coarse row (cj, cl): the
// 4 (2-D) or 4 x 4 (3-D) fine rows under it are summed with their y/z
// weights into an LDS row s (fine nx points x ncols), which the x weights
// (1/4, 3/4, 3/4, 1/4) then reduce to the coarse row; every fine value is
// read once per coarse row that covers it.
template <int DIM, int W, typename S>
__global__ __launch_bounds__(256) void k_restrict(int cnx, int cny, int cnz,
                                                  const S* __restrict__ res,
                                                  S* __restrict__ rc, int ncols,
                                                  const DevStatus* st) {
  if (halted(st)) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_r[];
  S* srow = reinterpret_cast<S*>(smem_r);
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int cj = row % cny, cl = row / cny;
  const int fnx = 2 * cnx, fny = 2 * cny, fnz = 2 * cnz;
  const RowLanes ln = row_lanes<W>(ncols);
  const int c = ln.c;
  const S norm = (DIM == 3) ? (S)0.125 : (S)0.25;
  constexpr int NR = (DIM == 3) ? 16 : 4;
  size_t rb[NR];
  S rw[NR];
  int nrows = 0;
  for (int dz = 0; dz < ((DIM == 3) ? 4 : 1); ++dz) {
    int fl = 0;
    S wz = 1;
    if (DIM == 3) {
      fl = 2 * cl - 1 + dz;
      wz = (dz == 0 || dz == 3) ? (S)0.25 : (S)0.75;
      if (fl < 0 || fl >= fnz) wz = 0, fl = 0;
    }
    for (int dy = 0; dy < 4; ++dy) {
      int fj = 2 * cj - 1 + dy;
      S wy = wz * ((dy == 0 || dy == 3) ? (S)0.25 : (S)0.75);
      if (fj < 0 || fj >= fny) wy = 0, fj = 0;
      rb[nrows] = ((size_t)fl * fny + fj) * fnx;
      rw[nrows] = wy;
      ++nrows;
    }
  }
  if (ln.on) {
    for (int f = ln.i0; f < fnx; f += ln.P) {
      vec<S, W> acc = (S)0;
#pragma unroll
      for (int q = 0; q < NR; ++q) acc += rw[q] * vload<W, S>(res + (rb[q] + f) * ncols + c);
      vstore<W, S>(srow + (size_t)f * ncols + c, acc);
    }
  }
  __syncthreads();
  if (!ln.on) return;
  for (int ci = ln.i0; ci < cnx; ci += ln.P) {
    const int f0 = 2 * ci - 1;
    vec<S, W> a = (S)0.75 * (vload<W, S>(srow + (size_t)(f0 + 1) * ncols + c) +
                             vload<W, S>(srow + (size_t)(f0 + 2) * ncols + c));
    if (f0 >= 0) a += (S)0.25 * vload<W, S>(srow + (size_t)f0 * ncols + c);
    if (f0 + 3 < fnx) a += (S)0.25 * vload<W, S>(srow + (size_t)(f0 + 3) * ncols + c);
    const size_t cp = ((size_t)cl * cny + cj) * cnx + ci;
    vstore<W, S>(rc + cp * ncols + c, a * norm);
  }
}

// x += P e (fine grid dims nx, ny, nz; coarse dims half).
template <int DIM, int W, typename S>
__global__ __launch_bounds__(256) void k_prolong_add(int nx, int ny, int nz,
                                                     const S* __restrict__ ec,
                                                     S* __restrict__ x, int ncols,
                                                     const DevStatus* st) {
  if (halted(st)) return;
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = row % ny, l = row / ny;
  const int cnx = nx / 2, cny = ny / 2, cnz = (DIM == 3) ? nz / 2 : 1;
  const RowLanes ln = row_lanes<W>(ncols);
  if (!ln.on) return;
  const int c = ln.c;
  const size_t rowp = (size_t)row * nx;
  // parent and neighbour-parent coarse rows in y and z, with weights
  const int pj = j >> 1, qj = (j & 1) ? pj + 1 : pj - 1;
  const int pl = (DIM == 3) ? (l >> 1) : 0;
  const int ql = (DIM == 3) ? ((l & 1) ? pl + 1 : pl - 1) : 0;
  size_t cb[4];
  S cw[4];
  for (int az = 0; az < 2; ++az)
    for (int ay = 0; ay < 2; ++ay) {
      const int q = az * 2 + ay;
      int cl = (DIM == 3) ? (az ? ql : pl) : 0;
      int cj = ay ? qj : pj;
      S w = (ay ? (S)0.25 : (S)0.75) * ((DIM == 3) ? (az ? (S)0.25 : (S)0.75) : (az ? (S)0 : (S)1));
      if (cl < 0 || cl >= cnz || cj < 0 || cj >= cny) w = 0, cl = 0, cj = 0;
      cb[q] = ((size_t)cl * cny + cj) * cnx;
      cw[q] = w;
    }
  for (int i = ln.i0; i < nx; i += ln.P) {
    const int pi = i >> 1, qi = (i & 1) ? pi + 1 : pi - 1;
    const bool hq = (qi >= 0 && qi < cnx);
    vec<S, W> acc = (S)0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const S* ep = ec + cb[q] * ncols + c;
      vec<S, W> a = (S)0.75 * vload<W, S>(ep + (size_t)pi * ncols);
      if (hq) a += (S)0.25 * vload<W, S>(ep + (size_t)qi * ncols);
      acc += cw[q] * a;
    }
    S* xp = x + (rowp + i) * ncols + c;
    vstore<W, S>(xp, vload<W, S>(xp) + acc);
  }
}

// Vertex-centred transfers (all fine dimensions odd, coarse point c on
// fine point 2c + 1).  Restriction: coarse r = P^T res / 2^d, i.e. full
// weighting with the 1-D weights (1/4, 1/2, 1/4) on fine points 2c, 2c + 1,
// 2c + 2; one workgroup per coarse row, the 3^d fine values read directly.
template <int DIM, int W, typename S>
__global__ __launch_bounds__(256) void k_restrict_v(int cnx, int cny, int cnz,
                                                    const S* __restrict__ res,
                                                    S* __restrict__ rc, int ncols,
                                                    const DevStatus* st) {
  if (halted(st)) return;
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int cj = row % cny, cl = row / cny;
  const int fnx = 2 * cnx + 1, fny = 2 * cny + 1;
  const RowLanes ln = row_lanes<W>(ncols);
  if (!ln.on) return;
  const int c = ln.c;
  const S w1[3] = {(S)0.25, (S)0.5, (S)0.25};
  for (int ci = ln.i0; ci < cnx; ci += ln.P) {
    vec<S, W> acc = (S)0;
#pragma unroll
    for (int dz = 0; dz < ((DIM == 3) ? 3 : 1); ++dz) {
      const int fl = (DIM == 3) ? 2 * cl + dz : 0;
      const S wz = (DIM == 3) ? w1[dz] : (S)1;
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const int fj = 2 * cj + dy;
        const S wy = wz * w1[dy];
        const S* rp = res + (((size_t)fl * fny + fj) * fnx + 2 * ci) * ncols + c;
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) acc += (wy * w1[dx]) * vload<W, S>(rp + (size_t)dx * ncols);
      }
    }
    const size_t cp = ((size_t)cl * cny + cj) * cnx + ci;
    vstore<W, S>(rc + cp * ncols + c, acc);
  }
}

// x += P e, vertex-centred (fine dims nx, ny, nz odd; coarse (n - 1)/2):
// per direction an odd fine index i takes coarse (i - 1)/2, an even one
// the mean of coarse i/2 - 1 and i/2 (zero outside the box).
template <int DIM, int W, typename S>
__global__ __launch_bounds__(256) void k_prolong_add_v(int nx, int ny, int nz,
                                                       const S* __restrict__ ec,
                                                       S* __restrict__ x, int ncols,
                                                       const DevStatus* st) {
  if (halted(st)) return;
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = row % ny, l = row / ny;
  const int cnx = (nx - 1) / 2, cny = (ny - 1) / 2, cnz = (DIM == 3) ? (nz - 1) / 2 : 1;
  const RowLanes ln = row_lanes<W>(ncols);
  if (!ln.on) return;
  const int c = ln.c;
  // coarse rows (y, z) and their weights
  int cjs[2], cls[2];
  S wjs[2], wls[2];
  auto one = [](int f, int nc, int* cs, S* ws) {
    if (f & 1) {
      cs[0] = (f - 1) >> 1, ws[0] = (S)1;
      cs[1] = 0, ws[1] = (S)0;
    } else {
      const int a = (f >> 1) - 1, b = f >> 1;
      cs[0] = (a >= 0) ? a : 0, ws[0] = (a >= 0) ? (S)0.5 : (S)0;
      cs[1] = (b < nc) ? b : 0, ws[1] = (b < nc) ? (S)0.5 : (S)0;
    }
  };
  one(j, cny, cjs, wjs);
  if (DIM == 3) {
    one(l, cnz, cls, wls);
  } else {
    cls[0] = 0, wls[0] = (S)1, cls[1] = 0, wls[1] = (S)0;
  }
  const size_t rowp = (size_t)row * nx;
  for (int i = ln.i0; i < nx; i += ln.P) {
    int cis[2];
    S wis[2];
    one(i, cnx, cis, wis);
    vec<S, W> acc = (S)0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const S wzy = wls[a] * wjs[b];
        const S* ep = ec + ((size_t)cls[a] * cny + cjs[b]) * cnx * ncols + c;
#pragma unroll
        for (int q = 0; q < 2; ++q)
          acc += (wzy * wis[q]) * vload<W, S>(ep + (size_t)cis[q] * ncols);
      }
    S* xp = x + (rowp + i) * ncols + c;
    vstore<W, S>(xp, vload<W, S>(xp) + acc);
  }
}

// One step of the Chebyshev recurrence for y = p(L - sigma I) x, with
// X = ca (L - sigma I) + cb I (the interval mapped to [-1, 1]) and
// L - sigma I = adiag I + off (neighbour sum):
//   first step:  t_1 = X t_0,                y = c_0 t_0 + c_1 t_1
//   later steps: t_{j+1} = 2 X t_j - t_{j-1}, y = y + c_{j+1} t_{j+1}
// tc is t_j (read with its neighbours), tp is t_{j-1} (point-wise, may be
// the output buffer tn), tn receives t_{j+1} (null on the last step), yin
// may be yout.
template <int DIM, int W, typename S>
__global__ __launch_bounds__(256) void k_cheb_step(int nx, int ny, int nz, S adiag, S off, S ca,
                                                   S cb, const S* __restrict__ tc, const S* tp,
                                                   S* tn, const S* yin, S* yout, S c0, S cj,
                                                   int first, int ncols, const DevStatus* st) {
  if (halted(st)) return;
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = row % ny, l = row / ny;
  const RowLanes ln = row_lanes<W>(ncols);
  if (!ln.on) return;
  const size_t rowp = (size_t)row * nx;
  const int c = ln.c;
  for (int i = ln.i0; i < nx; i += ln.P) {
    const size_t e = (rowp + i) * ncols + c;
    const S* xp = tc + e;
    const vec<S, W> xv = vload<W, S>(xp);
    const vec<S, W> sx = adiag * xv + off * nb_sum<DIM, W, S>(xp, i, j, l, nx, ny, nz, ncols);
    const vec<S, W> xt = ca * sx + cb * xv;
    vec<S, W> t, y;
    if (first) {
      t = xt;
      y = c0 * xv + cj * xt;
    } else {
      t = (S)2 * xt - vload<W, S>(tp + e);
      y = vload<W, S>(yin + e) + cj * t;
    }
    if (tn) vstore<W, S>(tn + e, t);
    vstore<W, S>(yout + e, y);
  }
}

// out = x + w (r - y), x and y null meaning zero (the Richardson step of a
// polynomial level, or its residual with x = null and w = 1); r read as RT
// with leading dimension ldr, the output as OT split at `split` like the
// Jacobi sweep.
template <int W, typename S, typename RT, typename OT>
__global__ __launch_bounds__(256) void k_lincomb(int nx, const S* __restrict__ x,
                                                 const RT* __restrict__ r, int ldr,
                                                 const S* __restrict__ y, S w,
                                                 OT* __restrict__ o0, int ld0,
                                                 OT* __restrict__ o1, int ld1, int split,
                                                 int ncols, const DevStatus* st) {
  if (halted(st)) return;
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const RowLanes ln = row_lanes<W>(ncols);
  if (!ln.on) return;
  const size_t rowp = (size_t)row * nx;
  const int c = ln.c;
  OT* const ob = (c < split) ? o0 + c : o1 + (c - split);
  const int ldo = (c < split) ? ld0 : ld1;
  for (int i = ln.i0; i < nx; i += ln.P) {
    const size_t p = rowp + i;
    vec<S, W> v = vload<W, S>(r + p * ldr + c);
    if (y) v -= vload<W, S>(y + p * ncols + c);
    v = w * v;
    if (x) v += vload<W, S>(x + p * ncols + c);
    vstore<W, S>(ob + p * ldo, v);
  }
}

// x = Ainv r on the coarsest level (nc points).
template <typename S>
__global__ __launch_bounds__(256) void k_dense_apply(int nc, const S* __restrict__ Ainv,
                                                     const S* __restrict__ r,
                                                     S* __restrict__ x, int ncols,
                                                     const DevStatus* st) {
  if (halted(st)) return;
  const int tot = nc * ncols;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += gridDim.x * blockDim.x) {
    const int i = e / ncols;
    const int c = e - i * ncols;
    const S* a = Ainv + (size_t)i * nc;
    S acc = 0;
    for (int q = 0; q < nc; ++q) acc += a[q] * r[(size_t)q * ncols + c];
    x[(size_t)i * ncols + c] = acc;
  }
}

// ---------------------------------------- coarse levels, one launch, in LDS
// The levels whose grids hold at most kCoarseMaxPts points (and the dense
// coarsest solve) run as one V-cycle per launch: the columns are
// independent, so workgroup g takes the column chunk [g cc, (g + 1) cc),
// copies its right-hand side into LDS, runs the same sweeps, residual,
// restriction, dense solve and prolongation as the row kernels on LDS
// arrays (stride cc), one phase after another with a barrier between
// phases, and writes the chunk of the first level's x buffer.  This
// replaces about fifteen launches of a few microseconds each by one.
constexpr int kCoarseNT = 512;
constexpr int kCoarseMaxPts = 4096;
constexpr size_t kCoarseMaxLds = 160 * 1024;
constexpr int kCoarseMaxLev = 4;

struct CoarseLev {
  int nx, ny, nz, n;
  float inx, inxy;  // 1/nx and 1/(nx ny) for the index arithmetic
  double diag, off;  // level operator (diag includes a shift)
  double w;          // Richardson weight of the sweeps
  int vtx;           // the transfer to the next level is vertex-centred
};
struct CoarseArgs {
  CoarseLev lv[kCoarseMaxLev];
  int nlev;  // levels handled; the last one is solved densely
  int nu_pre, nu_post;
  const void* Ainv;  // nc x nc
  int nc;
  int ncols, cc;
  const void* r0;  // first level: right-hand side (ld ncols)
  void* x0;        // first level: result (ld ncols)
};

// Element e of an LDS level array (n points x cc columns): point p, column
// c, grid indices i, j, l.  Float reciprocals are exact here: e and p stay
// below 2^14 and the fractional margins exceed 1/512.
struct CIdx {
  int p, c, i, j, l;
};
template <int DIM>
__device__ __forceinline__ CIdx cidx(int e, int cc, float icc, const CoarseLev& L) {
  CIdx x;
  x.p = (int)(((float)e + 0.5f) * icc);
  x.c = e - x.p * cc;
  x.l = (DIM == 3) ? (int)(((float)x.p + 0.5f) * L.inxy) : 0;
  const int rem = x.p - x.l * L.nx * L.ny;
  x.j = (int)(((float)rem + 0.5f) * L.inx);
  x.i = rem - x.j * L.nx;
  return x;
}
template <int DIM, typename S>
__device__ __forceinline__ S cc_nb(const S* xp, const CIdx& q, const CoarseLev& L, int cc) {
  const int sy = L.nx * cc, sz = L.nx * L.ny * cc;
  S nb = 0;
  if (q.i > 0) nb += xp[-cc];
  if (q.i < L.nx - 1) nb += xp[cc];
  if (q.j > 0) nb += xp[-sy];
  if (q.j < L.ny - 1) nb += xp[sy];
  if (DIM == 3) {
    if (q.l > 0) nb += xp[-sz];
    if (q.l < L.nz - 1) nb += xp[sz];
  }
  return nb;
}

// mode 0: out = xin + w (r - A xin), xin == nullptr meaning zero;
// mode 1: out = w (2 r - w A r) (two sweeps from zero); mode 2: out = r - A xin
template <int DIM, typename S>
__device__ void cc_sweep(const CoarseLev& L, const S* xin, const S* r, S* out, int mode, int cc,
                         float icc) {
  const S diag = (S)L.diag, off = (S)L.off, w = (S)L.w;
  for (int e = threadIdx.x; e < L.n * cc; e += kCoarseNT) {
    const CIdx q = cidx<DIM>(e, cc, icc, L);
    const S rv = r[e];
    S v;
    if (mode == 1) {
      v = w * ((S)2 * rv - w * (diag * rv + off * cc_nb<DIM, S>(r + e, q, L, cc)));
    } else if (xin == nullptr) {
      v = w * rv;
    } else {
      const S ax = diag * xin[e] + off * cc_nb<DIM, S>(xin + e, q, L, cc);
      v = (mode == 2) ? rv - ax : xin[e] + w * (rv - ax);
    }
    out[e] = v;
  }
}

// coarse r (level C) = P^T res (level F) / 2^d
template <int DIM, typename S>
__device__ void cc_restrict(const CoarseLev& F, const CoarseLev& C, const S* res, S* rc, int cc,
                            float icc) {
  const S norm = (DIM == 3) ? (S)0.125 : (S)0.25;
  if (F.vtx) {  // full weighting on fine points 2c, 2c + 1, 2c + 2
    for (int e = threadIdx.x; e < C.n * cc; e += kCoarseNT) {
      const CIdx q = cidx<DIM>(e, cc, icc, C);
      S acc = 0;
#pragma unroll
      for (int dz = 0; dz < ((DIM == 3) ? 3 : 1); ++dz) {
        const int fl = (DIM == 3) ? 2 * q.l + dz : 0;
        const S wz = (DIM == 3) ? ((dz == 1) ? (S)0.5 : (S)0.25) : (S)1;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          const int fj = 2 * q.j + dy;
          const S wy = wz * ((dy == 1) ? (S)0.5 : (S)0.25);
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) {
            const int fi = 2 * q.i + dx;
            const S wx = (dx == 1) ? (S)0.5 : (S)0.25;
            acc += (wy * wx) * res[(((size_t)fl * F.ny + fj) * F.nx + fi) * cc + q.c];
          }
        }
      }
      rc[e] = acc;
    }
    return;
  }
  for (int e = threadIdx.x; e < C.n * cc; e += kCoarseNT) {
    const CIdx q = cidx<DIM>(e, cc, icc, C);
    S acc = 0;
#pragma unroll
    for (int dz = 0; dz < ((DIM == 3) ? 4 : 1); ++dz) {
      int fl = (DIM == 3) ? 2 * q.l - 1 + dz : 0;
      S wz = (DIM == 3) ? ((dz == 0 || dz == 3) ? (S)0.25 : (S)0.75) : (S)1;
      if (fl < 0 || fl >= F.nz) wz = 0, fl = 0;
#pragma unroll
      for (int dy = 0; dy < 4; ++dy) {
        int fj = 2 * q.j - 1 + dy;
        S wy = wz * ((dy == 0 || dy == 3) ? (S)0.25 : (S)0.75);
        if (fj < 0 || fj >= F.ny) wy = 0, fj = 0;
#pragma unroll
        for (int dx = 0; dx < 4; ++dx) {
          int fi = 2 * q.i - 1 + dx;
          S wx = (dx == 0 || dx == 3) ? (S)0.25 : (S)0.75;
          if (fi < 0 || fi >= F.nx) wx = 0, fi = 0;
          acc += (wy * wx) * res[(((size_t)fl * F.ny + fj) * F.nx + fi) * cc + q.c];
        }
      }
    }
    rc[e] = acc * norm;
  }
}

// the coarse neighbours of fine index f (vertex-centred) and weights
__device__ __forceinline__ void vtx_parents(int f, int nc, int* cs, float* ws) {
  if (f & 1) {
    cs[0] = (f - 1) >> 1, ws[0] = 1.0f, cs[1] = 0, ws[1] = 0.0f;
  } else {
    const int a = (f >> 1) - 1, b = f >> 1;
    cs[0] = (a >= 0) ? a : 0, ws[0] = (a >= 0) ? 0.5f : 0.0f;
    cs[1] = (b < nc) ? b : 0, ws[1] = (b < nc) ? 0.5f : 0.0f;
  }
}

// x (level F) += P e (level C)
template <int DIM, typename S>
__device__ void cc_prolong(const CoarseLev& F, const CoarseLev& C, const S* ec, S* x, int cc,
                           float icc) {
  if (F.vtx) {
    for (int e = threadIdx.x; e < F.n * cc; e += kCoarseNT) {
      const CIdx q = cidx<DIM>(e, cc, icc, F);
      int ci[2], cj[2], cl[2];
      float wi[2], wj[2], wl[2];
      vtx_parents(q.i, C.nx, ci, wi);
      vtx_parents(q.j, C.ny, cj, wj);
      if (DIM == 3)
        vtx_parents(q.l, C.nz, cl, wl);
      else
        cl[0] = cl[1] = 0, wl[0] = 1.0f, wl[1] = 0.0f;
      S acc = 0;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int d = 0; d < 2; ++d)
            acc += (S)(wl[a] * wj[b] * wi[d]) *
                   ec[(((size_t)cl[a] * C.ny + cj[b]) * C.nx + ci[d]) * cc + q.c];
      x[e] += acc;
    }
    return;
  }
  for (int e = threadIdx.x; e < F.n * cc; e += kCoarseNT) {
    const CIdx q = cidx<DIM>(e, cc, icc, F);
    const int pi = q.i >> 1, qi = (q.i & 1) ? pi + 1 : pi - 1;
    const int pj = q.j >> 1, qj = (q.j & 1) ? pj + 1 : pj - 1;
    const int pl = q.l >> 1, ql = (q.l & 1) ? pl + 1 : pl - 1;
    S acc = 0;
#pragma unroll
    for (int az = 0; az < ((DIM == 3) ? 2 : 1); ++az) {
      int cl = (DIM == 3) ? (az ? ql : pl) : 0;
      S wz = (DIM == 3) ? (az ? (S)0.25 : (S)0.75) : (S)1;
      if (cl < 0 || cl >= C.nz) wz = 0, cl = 0;
#pragma unroll
      for (int ay = 0; ay < 2; ++ay) {
        int cj = ay ? qj : pj;
        S wy = wz * (ay ? (S)0.25 : (S)0.75);
        if (cj < 0 || cj >= C.ny) wy = 0, cj = 0;
#pragma unroll
        for (int ax = 0; ax < 2; ++ax) {
          int ci = ax ? qi : pi;
          S wx = ax ? (S)0.25 : (S)0.75;
          if (ci < 0 || ci >= C.nx) wx = 0, ci = 0;
          acc += (wy * wx) * ec[(((size_t)cl * C.ny + cj) * C.nx + ci) * cc + q.c];
        }
      }
    }
    x[e] += acc;
  }
}

// LDS: per level x, t, r (n_q x cc each), then Ainv (nc x nc)
template <int DIM, typename S>
__global__ __launch_bounds__(kCoarseNT) void k_coarse_cycle(CoarseArgs a, const DevStatus* st) {
  if (halted(st)) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_c[];
  S* lds = reinterpret_cast<S*>(smem_c);
  const int cc = a.cc, c0 = blockIdx.x * cc, ncols = a.ncols;
  const float icc = 1.0f / (float)cc;
  S* X[kCoarseMaxLev];
  S* T[kCoarseMaxLev];
  S* R[kCoarseMaxLev];
  S* Am;  // the coarsest inverse
  {
    S* q = lds;
#pragma unroll
    for (int l = 0; l < kCoarseMaxLev; ++l) {
      const int sz = (l < a.nlev) ? a.lv[l].n * cc : 0;
      X[l] = q;
      T[l] = q + sz;
      R[l] = q + 2 * sz;
      q += 3 * sz;
    }
    Am = q;
    const S* gA = reinterpret_cast<const S*>(a.Ainv);
    for (int e = threadIdx.x; e < a.nc * a.nc; e += kCoarseNT) Am[e] = gA[e];
    const S* r0 = reinterpret_cast<const S*>(a.r0);
    for (int e = threadIdx.x; e < a.lv[0].n * cc; e += kCoarseNT) {
      const int p = (int)(((float)e + 0.5f) * icc);
      R[0][e] = r0[(size_t)p * ncols + c0 + (e - p * cc)];
    }
  }
  __syncthreads();
  unsigned inx = 0;  // bit l: level l's iterate is in X[l] (else T[l])
#pragma unroll
  for (int l = 0; l + 1 < kCoarseMaxLev; ++l) {
    if (l + 1 >= a.nlev) break;
    const CoarseLev& L = a.lv[l];
    S* cur = X[l];
    S* oth = T[l];
    int it;
    if (a.nu_pre >= 2) {
      cc_sweep<DIM, S>(L, nullptr, R[l], cur, 1, cc, icc);
      it = 2;
    } else {
      cc_sweep<DIM, S>(L, nullptr, R[l], cur, 0, cc, icc);
      it = 1;
    }
    __syncthreads();
    for (; it < a.nu_pre; ++it) {
      cc_sweep<DIM, S>(L, cur, R[l], oth, 0, cc, icc);
      __syncthreads();
      S* tmp = cur;
      cur = oth;
      oth = tmp;
    }
    cc_sweep<DIM, S>(L, cur, R[l], oth, 2, cc, icc);  // residual
    __syncthreads();
    cc_restrict<DIM, S>(L, a.lv[l + 1], oth, R[l + 1], cc, icc);
    __syncthreads();
    if (cur == X[l]) inx |= 1u << l;
  }
  {  // coarsest: x = Ainv r
    const int lc = a.nlev - 1;
    S* x = X[0];
    const S* r = R[0];
#pragma unroll
    for (int l = 1; l < kCoarseMaxLev; ++l)
      if (l == lc) x = X[l], r = R[l];
    for (int e = threadIdx.x; e < a.nc * cc; e += kCoarseNT) {
      const int i = (int)(((float)e + 0.5f) * icc);
      const int c = e - i * cc;
      const S* arow = Am + (size_t)i * a.nc;
      S acc0 = 0, acc1 = 0;
      int q = 0;
      for (; q + 1 < a.nc; q += 2) {
        acc0 += arow[q] * r[q * cc + c];
        acc1 += arow[q + 1] * r[(q + 1) * cc + c];
      }
      if (q < a.nc) acc0 += arow[q] * r[q * cc + c];
      x[e] = acc0 + acc1;
    }
    __syncthreads();
    inx |= 1u << lc;
  }
#pragma unroll
  for (int l = kCoarseMaxLev - 2; l >= 0; --l) {
    if (l + 1 >= a.nlev) continue;
    const CoarseLev& L = a.lv[l];
    S* cur = (inx >> l & 1u) ? X[l] : T[l];
    S* oth = (inx >> l & 1u) ? T[l] : X[l];
    const S* ec = (inx >> (l + 1) & 1u) ? X[l + 1] : T[l + 1];
    cc_prolong<DIM, S>(L, a.lv[l + 1], ec, cur, cc, icc);
    __syncthreads();
    for (int it = 0; it < a.nu_post; ++it) {
      cc_sweep<DIM, S>(L, cur, R[l], oth, 0, cc, icc);
      __syncthreads();
      S* tmp = cur;
      cur = oth;
      oth = tmp;
    }
    if (cur == X[l])
      inx |= 1u << l;
    else
      inx &= ~(1u << l);
  }
  const S* res = (inx & 1u) ? X[0] : T[0];
  S* x0 = reinterpret_cast<S*>(a.x0);
  for (int e = threadIdx.x; e < a.lv[0].n * cc; e += kCoarseNT) {
    const int p = (int)(((float)e + 0.5f) * icc);
    x0[(size_t)p * ncols + c0 + (e - p * cc)] = res[e];
  }
}

static size_t coarse_lds(const MG& mg, int lev, int cc, size_t es) {
  size_t n = (size_t)mg.nc * mg.nc;
  for (int q = lev; q < (int)mg.lv.size(); ++q) n += 3 * mg.lv[q].g.n() * cc;
  return n * es;
}

// ---------------------------------------------------------------- host side
static void coarse_dense(const Grid& g, std::vector<double>& A) {
  const int n = (int)g.n();
  A.assign((size_t)n * n, 0.0);
  const double d = g.diag(), o = g.off();
  for (int l = 0; l < g.nz; ++l)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        const int p = i + g.nx * (j + g.ny * l);
        A[(size_t)p * n + p] = d;
        auto link = [&](int q) { A[(size_t)p * n + q] = o; };
        if (i > 0) link(p - 1);
        if (i < g.nx - 1) link(p + 1);
        if (j > 0) link(p - g.nx);
        if (j < g.ny - 1) link(p + g.nx);
        if (g.dim == 3) {
          if (l > 0) link(p - g.nx * g.ny);
          if (l < g.nz - 1) link(p + g.nx * g.ny);
        }
      }
}

// Inverse of an SPD matrix by Cholesky (host, FP64).  Returns false if a
// pivot is not positive.
static bool spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> L((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(s > 0.0)) return false;
    const double djj = std::sqrt(s);
    L[(size_t)j * n + j] = djj;
    for (int i = j + 1; i < n; ++i) {
      double t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = t / djj;
    }
  }
  // inverse = L^-T L^-1, column by column
  std::vector<double> col(n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * col[k];
      col[i] = t / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = col[i];
      for (int k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * col[k];
      col[i] = t / L[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) A[(size_t)i * n + c] = col[i];
  }
  return true;
}

bool coarse_inverse(const Grid& g, std::vector<double>& inv) {
  coarse_dense(g, inv);
  return spd_inverse(inv, (int)g.n());
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

bool mg_coarsen(Grid& g, int* vtx) {
  const int d[3] = {g.nx, g.ny, g.nz};
  const int nd = g.dim;
  bool even = true, odd = true;
  for (int q = 0; q < nd; ++q) {
    even = even && (d[q] % 2 == 0);
    odd = odd && (d[q] % 2 == 1 && d[q] >= 3);
  }
  if (!even && !odd) return false;
  *vtx = odd ? 1 : 0;
  g.nx = even ? g.nx / 2 : (g.nx - 1) / 2;
  g.ny = even ? g.ny / 2 : (g.ny - 1) / 2;
  if (nd == 3) g.nz = even ? g.nz / 2 : (g.nz - 1) / 2;
  g.h *= 2.0;
  return true;
}

size_t mg_workspace_bytes(const Grid& fine, int levels, int cmax, int mode) {
  size_t bytes = 0;
  Grid g = fine;
  for (int lv = 0; lv < levels; ++lv) {
    const size_t blk = align256(g.n() * cmax * sizeof(double));
    bytes += (lv == 0 ? 2 : 3) * blk + (mode ? 3 * blk : 0);
    if (lv == levels - 1)
      bytes += align256(g.n() * g.n() * sizeof(double)) + align256(g.n() * g.n() * sizeof(float));
    int vtx = 0;
    if (lv + 1 < levels && !mg_coarsen(g, &vtx)) break;
  }
  return bytes;
}

static hipError_t coarse_set_attributes() {
  const void* f[4] = {(const void*)k_coarse_cycle<3, double>, (const void*)k_coarse_cycle<3, float>,
                      (const void*)k_coarse_cycle<2, double>, (const void*)k_coarse_cycle<2, float>};
  for (const void* k : f) {
    const hipError_t e =
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCoarseMaxLds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Eigendecomposition of a symmetric n x n matrix (row-major, host, FP64):
// on return A holds the eigenvectors as columns and d the eigenvalues.
// Householder reduction to tridiagonal form with the transformations
// accumulated, then the implicit symmetric QR iteration with Wilkinson
// shifts on the tridiagonal matrix, the Givens rotations applied to the
// accumulated basis (Golub & Van Loan, Sec. 8.3).
static void sym_eig(std::vector<double>& A, int n, std::vector<double>& d) {
  std::vector<double> Q((size_t)n * n, 0.0), v(n), p(n), w(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  auto at = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  for (int k = 0; k + 2 < n; ++k) {
    double nrm = 0.0;
    for (int i = k + 1; i < n; ++i) nrm += at(i, k) * at(i, k);
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) continue;
    const double x0 = at(k + 1, k);
    const double alpha = (x0 >= 0.0) ? -nrm : nrm;  // new subdiagonal entry
    for (int i = 0; i < n; ++i) v[i] = 0.0;
    v[k + 1] = x0 - alpha;
    for (int i = k + 2; i < n; ++i) v[i] = at(i, k);
    double vv = 0.0;
    for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    // A <- H A H on rows/columns k.. with H = I - beta v v^T (v zero above k+1)
    for (int i = k; i < n; ++i) {
      double acc = 0.0;
      for (int j = k + 1; j < n; ++j) acc += at(i, j) * v[j];
      p[i] = beta * acc;
    }
    double kk = 0.0;
    for (int i = k + 1; i < n; ++i) kk += v[i] * p[i];
    kk *= 0.5 * beta;
    for (int i = k; i < n; ++i) w[i] = p[i] - kk * v[i];
    for (int i = k; i < n; ++i)
      for (int j = k; j < n; ++j) at(i, j) -= v[i] * w[j] + w[i] * v[j];
    // Q <- Q H
    for (int i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int j = k + 1; j < n; ++j) acc += Q[(size_t)i * n + j] * v[j];
      acc *= beta;
      for (int j = k + 1; j < n; ++j) Q[(size_t)i * n + j] -= acc * v[j];
    }
  }
  d.assign(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = at(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = at(i + 1, i);
  // implicit QR on the tridiagonal (d, e): deflate from the bottom
  int hi = n - 1;
  int guard = 0;
  while (hi > 0 && guard < 60 * n) {
    const double tiny = 1e-15 * (std::fabs(d[hi - 1]) + std::fabs(d[hi]));
    if (std::fabs(e[hi - 1]) <= tiny || std::fabs(e[hi - 1]) < 1e-300) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && std::fabs(e[lo - 1]) > 1e-15 * (std::fabs(d[lo - 1]) + std::fabs(d[lo])))
      --lo;
    ++guard;
    // Wilkinson shift from the trailing 2 x 2 block
    const double dd = 0.5 * (d[hi - 1] - d[hi]);
    const double ee = e[hi - 1];
    const double den = dd + ((dd >= 0.0) ? 1.0 : -1.0) * std::hypot(dd, ee);
    const double mu = d[hi] - ((den != 0.0) ? ee * ee / den : 0.0);
    double x = d[lo] - mu, z = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, z);
      const double c = (r == 0.0) ? 1.0 : x / r, sn = (r == 0.0) ? 0.0 : -z / r;
      // rotate rows/columns k, k+1 of the tridiagonal
      if (k > lo) e[k - 1] = r;
      const double a11 = d[k], a22 = d[k + 1], a12 = e[k];
      d[k] = c * c * a11 - 2.0 * c * sn * a12 + sn * sn * a22;
      d[k + 1] = sn * sn * a11 + 2.0 * c * sn * a12 + c * c * a22;
      e[k] = c * sn * (a11 - a22) + (c * c - sn * sn) * a12;
      if (k + 1 < hi) {
        x = e[k];
        z = -sn * e[k + 1];
        e[k + 1] *= c;
      }
      for (int i = 0; i < n; ++i) {
        const double qa = Q[(size_t)i * n + k], qb = Q[(size_t)i * n + k + 1];
        Q[(size_t)i * n + k] = c * qa - sn * qb;
        Q[(size_t)i * n + k + 1] = sn * qa + c * qb;
      }
    }
  }
  A.swap(Q);
}

// f(L_0 - sigma I) for the coarsest level from its eigendecomposition:
// f(x) = 1/|x| (AV-MG) or 1/x (INV-MG).  False when an eigenvalue of the
// shifted operator vanishes to rounding (sigma on a coarse eigenvalue).
static bool coarse_function(const Grid& g, double sigma, bool absval, std::vector<double>& out) {
  const int n = (int)g.n();
  std::vector<double> A, d;
  coarse_dense(g, A);
  for (int i = 0; i < n; ++i) A[(size_t)i * n + i] -= sigma;
  sym_eig(A, n, d);
  double big = 0.0;
  for (double x : d) big = std::max(big, std::fabs(x));
  std::vector<double> f(n);
  for (int i = 0; i < n; ++i) {
    if (!(std::fabs(d[i]) > 1e-13 * big)) return false;
    f[i] = absval ? 1.0 / std::fabs(d[i]) : 1.0 / d[i];
  }
  out.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int q = 0; q < n; ++q) acc += A[(size_t)i * n + q] * f[q] * A[(size_t)j * n + q];
      out[(size_t)i * n + j] = acc;
    }
  return true;
}

// Jackson-damped Chebyshev series of |x| of degree m on [a, b]: the
// coefficients of the series (discrete cosine sums over 8192 Chebyshev
// points) times the Jackson factors, which make the truncated series a
// convolution of |x| with a nonnegative kernel (so the polynomial stays
// positive on [a, b]).
static std::vector<double> abs_cheb(double a, double b, int m) {
  const int N = 8192;
  std::vector<double> f(N), c(m + 1, 0.0);
  for (int j = 0; j < N; ++j) {
    const double th = M_PI * (j + 0.5) / N;
    f[j] = std::fabs(0.5 * (b - a) * std::cos(th) + 0.5 * (a + b));
  }
  for (int i = 0; i <= m; ++i) {
    double acc = 0.0;
    for (int j = 0; j < N; ++j) acc += f[j] * std::cos(i * M_PI * (j + 0.5) / N);
    c[i] = 2.0 * acc / N;
  }
  c[0] *= 0.5;
  const int K = m + 1;
  const double q = M_PI / (K + 1);
  for (int i = 0; i <= m; ++i)
    c[i] *= ((K - i + 1) * std::cos(i * q) + std::sin(i * q) / std::tan(q)) / (K + 1);
  return c;
}

static double cheb_value(const std::vector<double>& c, double t) {
  double t0 = 1.0, t1 = t, y = c[0] + (c.size() > 1 ? c[1] * t : 0.0);
  for (size_t i = 2; i < c.size(); ++i) {
    const double t2 = 2.0 * t * t1 - t0;
    y += c[i] * t2;
    t0 = t1;
    t1 = t2;
  }
  return y;
}

plhr_status mg_setup(MG& mg, const Grid& fine, int levels, int nu_pre, int nu_post, double omega,
                     int cmax, char*& ws, hipStream_t s, const MGOpts& av) {
  PLHR_HIP_CHECK(coarse_set_attributes());
  {  // the cell-centred restriction stages one fine row of cmax FP64 columns in LDS
    Grid g = fine;
    for (int lv = 0; lv + 1 < levels; ++lv) {
      int vtx = 0;
      Grid f = g;
      if (!mg_coarsen(g, &vtx)) {
        set_error("multigrid: a level cannot be coarsened (dimensions must be all even or all "
                  "odd and >= 3)");
        return PLHR_ERR_ARG;
      }
      if (!vtx && (size_t)f.nx * cmax * sizeof(double) > 65536) {
        set_error("multigrid: a fine grid row of the block exceeds 64 KiB");
        return PLHR_ERR_UNSUPPORTED;
      }
    }
  }
  mg.levels = levels;
  mg.nu_pre = nu_pre;
  mg.nu_post = nu_post;
  mg.omega = omega;
  mg.cmax = cmax;
  mg.av = av;
  mg.lv.clear();
  Grid g = fine;
  for (int lv = 0; lv < levels; ++lv) {
    MGLevel L;
    L.g = g;
    const size_t blk = align256(g.n() * cmax * sizeof(double));
    L.x = (double*)ws;
    ws += blk;
    L.t = (double*)ws;
    ws += blk;
    if (lv > 0) {
      L.r = (double*)ws;
      ws += blk;
    }
    if (av.mode) {
      L.u0 = (double*)ws;
      ws += blk;
      L.u1 = (double*)ws;
      ws += blk;
      L.u2 = (double*)ws;
      ws += blk;
    }
    // the level operator and its smoother
    L.w = omega / g.diag();
    if (av.mode == 2) {
      L.kind = 1;
      L.shift = av.sigma;
    } else if (av.mode == 1 && !(std::sqrt(std::max(av.sigma, 0.0) / g.scale) * g.h < av.delta)) {
      L.kind = 2;
      L.shift = av.sigma;
      const double a = -av.sigma, b = 2.0 * g.diag() - av.sigma;  // Gershgorin bound
      L.cheb = abs_cheb(a, b, av.degree);
      double pmax = 0.0;
      for (int q = 0; q <= 20000; ++q) pmax = std::max(pmax, cheb_value(L.cheb, -1.0 + q / 1e4));
      L.w = 1.0 / pmax;
      L.ca = 2.0 / (b - a);
      L.cb = -(a + b) / (b - a);
    }
    if (lv == levels - 1) {
      mg.lv.push_back(L);
      break;
    }
    int vtx = 0;
    mg_coarsen(g, &vtx);
    L.vtx = vtx;
    mg.lv.push_back(L);
  }
  const Grid& gc = mg.lv.back().g;
  mg.nc = (int)gc.n();
  std::vector<double> A;
  if (av.mode == 0) {
    coarse_dense(gc, A);
    if (!spd_inverse(A, mg.nc)) {
      set_error("coarsest multigrid operator is not positive definite");
      return PLHR_ERR_NOT_HPD;
    }
  } else if (!coarse_function(gc, av.sigma, av.mode == 1, A)) {
    set_error("sigma is an eigenvalue of the coarsest multigrid operator (to rounding)");
    return PLHR_ERR_ARG;
  }
  mg.coarse_inv = (double*)ws;
  ws += align256((size_t)mg.nc * mg.nc * sizeof(double));
  PLHR_HIP_CHECK(hipMemcpyAsync(mg.coarse_inv, A.data(), A.size() * sizeof(double),
                                hipMemcpyHostToDevice, s));
  // FP32 copy for the mixed-precision cycle
  std::vector<float> A32(A.begin(), A.end());
  mg.coarse_inv32 = (float*)ws;
  ws += align256((size_t)mg.nc * mg.nc * sizeof(float));
  PLHR_HIP_CHECK(hipMemcpyAsync(mg.coarse_inv32, A32.data(), A32.size() * sizeof(float),
                                hipMemcpyHostToDevice, s));
  PLHR_HIP_CHECK(hipStreamSynchronize(s));
  return PLHR_OK;
}

#define PROF_LAUNCH(cat, bytes, flops, ...)  \
  do {                                        \
    prof_begin(cat, bytes, flops, s);         \
    hipLaunchKernelGGL(__VA_ARGS__);          \
    prof_end(cat, s);                         \
  } while (0)

// y = p(L_l - sigma I) x on a polynomial level, by the three-term
// recurrence (L.u0, L.u1 hold the terms, y is L.u2).
template <int DIM, int W, typename S>
static S* cheb_apply(MGLevel& L, const S* x, int ncols, const DevStatus* st, hipStream_t s) {
  const Grid& g = L.g;
  const int rows = g.ny * g.nz;
  const double nb = (double)g.n() * ncols * sizeof(S);
  const double fl = (double)g.n() * ncols;
  const S adiag = (S)(g.diag() - L.shift), off = (S)g.off(), ca = (S)L.ca, cb = (S)L.cb;
  S* tb[2] = {reinterpret_cast<S*>(L.u0), reinterpret_cast<S*>(L.u1)};
  S* y = reinterpret_cast<S*>(L.u2);
  const int m = (int)L.cheb.size() - 1;
  // t_1 = X x, y = c_0 x + c_1 t_1
  PROF_LAUNCH(KC_JACOBI, 3.0 * nb, (2.0 * DIM + 6.0) * fl, (k_cheb_step<DIM, W, S>), dim3(rows),
              dim3(256), 0, s, g.nx, g.ny, g.nz, adiag, off, ca, cb, x, (const S*)nullptr,
              m > 1 ? tb[0] : (S*)nullptr, (const S*)nullptr, y, (S)L.cheb[0], (S)L.cheb[1], 1,
              ncols, st);
  for (int j = 1; j < m; ++j) {
    // t_{j+1} = 2 X t_j - t_{j-1}, y += c_{j+1} t_{j+1}
    const S* tc = tb[(j - 1) & 1];
    const S* tp = (j == 1) ? x : tb[j & 1];
    S* tn = (j + 1 < m) ? tb[j & 1] : nullptr;
    PROF_LAUNCH(KC_JACOBI, 5.0 * nb, (2.0 * DIM + 8.0) * fl, (k_cheb_step<DIM, W, S>), dim3(rows),
                dim3(256), 0, s, g.nx, g.ny, g.nz, adiag, off, ca, cb, tc, tp, tn, (const S*)y, y,
                (S)0, (S)L.cheb[j + 1], 0, ncols, st);
  }
  return y;
}

// One V-cycle at level `lev` on input r (ld ldr, element type RT).  Level
// storage and arithmetic in S.  At level 0 the result goes to out0/out1
// (FP64, split by column); at coarser levels it is left in one of the
// level's work buffers, whose address is returned.
template <int DIM, int W, typename S, typename RT>
static S* cycle(MG& mg, int lev, const RT* r, int ldr, Blk out0, Blk out1, int split, int ncols,
                const DevStatus* st, hipStream_t s) {
  MGLevel& L = mg.lv[lev];
  const Grid& g = L.g;
  const int rows = g.ny * g.nz;
  const dim3 blk(256);
  const bool coarsest = (lev == (int)mg.lv.size() - 1);
  const double nb = (double)g.n() * ncols * sizeof(S);  // one pass over this level
  const double fl = (double)g.n() * ncols;
  S* Lx = reinterpret_cast<S*>(L.x);
  S* Lt = reinterpret_cast<S*>(L.t);
  const S* Ainv = (sizeof(S) == 4) ? reinterpret_cast<const S*>(mg.coarse_inv32)
                                   : reinterpret_cast<const S*>(mg.coarse_inv);
  // every level from here down is small (and none is a polynomial level):
  // one launch runs the rest of the cycle, one workgroup per column chunk,
  // in LDS
  {
    const int nl_tot = (int)mg.lv.size() - lev;
    bool small = lev > 0 && nl_tot >= 2 && nl_tot <= kCoarseMaxLev;
    for (int q = lev; small && q < (int)mg.lv.size(); ++q)
      small = mg.lv[q].g.n() <= (size_t)kCoarseMaxPts && mg.lv[q].kind != 2;
    // one column per workgroup: the blocks here have at most 2 k_int
    // columns, far fewer than the compute units, and each workgroup runs
    // the coarse cycle's levels one after another (its latency is the cost)
    int cc = 0;
    if (small && coarse_lds(mg, lev, 1, sizeof(S)) <= kCoarseMaxLds) cc = 1;
    if (small && cc > 0) {
      CoarseArgs a{};
      a.nlev = nl_tot;
      a.nu_pre = mg.nu_pre;
      a.nu_post = mg.nu_post;
      a.Ainv = Ainv;
      a.nc = mg.nc;
      a.ncols = ncols;
      a.cc = cc;
      a.r0 = r;
      a.x0 = Lx;
      double bytes = (double)mg.nc * mg.nc * sizeof(S) + 2.0 * g.n() * ncols * sizeof(S);
      double flops = 2.0 * mg.nc * (double)mg.nc * ncols;
      for (int q = 0; q < nl_tot; ++q) {
        const MGLevel& M = mg.lv[lev + q];
        CoarseLev& c = a.lv[q];
        c.nx = M.g.nx;
        c.ny = M.g.ny;
        c.nz = M.g.nz;
        c.n = (int)M.g.n();
        c.inx = 1.0f / (float)M.g.nx;
        c.inxy = 1.0f / (float)(M.g.nx * M.g.ny);
        c.diag = M.g.diag() - M.shift;
        c.off = M.g.off();
        c.w = M.w;
        c.vtx = M.vtx;
        flops += 40.0 * (double)M.g.n() * ncols;
      }
      PROF_LAUNCH(KC_COARSE, bytes, flops, (k_coarse_cycle<DIM, S>), dim3(ncols / cc),
                  dim3(kCoarseNT), coarse_lds(mg, lev, cc, sizeof(S)), s, a, st);
      return Lx;
    }
  }
  if (coarsest) {  // lev > 0 here (a single level runs dense_only)
    const int tot = mg.nc * ncols;
    const int nbk = (tot + 255) / 256;
    PROF_LAUNCH(KC_COARSE, (double)mg.nc * mg.nc * sizeof(S) + 2.0 * nb, 2.0 * mg.nc * fl,
                k_dense_apply<S>, dim3(nbk), blk, 0, s, mg.nc, Ainv,
                reinterpret_cast<const S*>(r), Lx, ncols, st);
    return Lx;
  }
  const S diag = (S)(g.diag() - L.shift), off = (S)g.off(), wr = (S)L.w;
  const double rb = sizeof(RT) / (double)sizeof(S);  // input pass relative to a level pass
  const bool poly = (L.kind == 2);
  S* cur = Lx;
  S* oth = Lt;
  // pre-smoothing from a zero guess (nu_pre >= 1)
  int it0 = 0;
  if (poly) {
    // w_1 = alpha r, then w <- w + alpha (r - B w)
    PROF_LAUNCH(KC_JACOBI, (1.0 + rb) * nb, fl, (k_lincomb<W, S, RT, S>), dim3(rows), blk, 0, s,
                g.nx, (const S*)nullptr, r, ldr, (const S*)nullptr, wr, cur, ncols, cur, ncols,
                ncols, ncols, st);
    for (int it = 1; it < mg.nu_pre; ++it) {
      const S* y = cheb_apply<DIM, W, S>(L, cur, ncols, st, s);
      PROF_LAUNCH(KC_JACOBI, (3.0 + rb) * nb, 3.0 * fl, (k_lincomb<W, S, RT, S>), dim3(rows), blk,
                  0, s, g.nx, (const S*)cur, r, ldr, y, wr, oth, ncols, oth, ncols, ncols, ncols,
                  st);
      std::swap(cur, oth);
    }
  } else {
    // the first two sweeps in one kernel
    if (mg.nu_pre >= 2) {
      PROF_LAUNCH(KC_JACOBI, (1.0 + rb) * nb, (2.0 * DIM + 6.0) * fl,
                  (k_jacobi2z<DIM, W, S, RT>), dim3(rows), blk, 0, s, g.nx, g.ny, g.nz, diag, off,
                  wr, r, ldr, oth, ncols, st);
      std::swap(cur, oth);
      it0 = 2;
    }
    for (int it = it0; it < mg.nu_pre; ++it) {
      PROF_LAUNCH(KC_JACOBI, (it == 0 ? 1.0 + rb : 2.0 + rb) * nb,
                  (it == 0 ? 1.0 : 2.0 * DIM + 5.0) * fl, (k_jacobi<DIM, W, S, RT, S>),
                  dim3(rows), blk, 0, s, g.nx, g.ny, g.nz, diag, off, wr,
                  it == 0 ? (const S*)nullptr : (const S*)cur, r, ldr, oth, ncols, oth, ncols,
                  ncols, ncols, st);
      std::swap(cur, oth);
    }
  }
  // residual -> oth, restrict -> coarse r, coarse cycle, prolongate into cur
  if (poly) {
    const S* y = cheb_apply<DIM, W, S>(L, cur, ncols, st, s);
    PROF_LAUNCH(KC_RESIDUAL, (2.0 + rb) * nb, 2.0 * fl, (k_lincomb<W, S, RT, S>), dim3(rows), blk,
                0, s, g.nx, (const S*)nullptr, r, ldr, y, (S)1, oth, ncols, oth, ncols, ncols,
                ncols, st);
  } else {
    PROF_LAUNCH(KC_RESIDUAL, (2.0 + rb) * nb, (2.0 * DIM + 3.0) * fl,
                (k_residual<DIM, W, S, RT>), dim3(rows), blk, 0, s, g.nx, g.ny, g.nz, diag, off,
                cur, r, ldr, oth, ncols, st);
  }
  MGLevel& C = mg.lv[lev + 1];
  const int crows = C.g.ny * C.g.nz;
  S* Cr = reinterpret_cast<S*>(C.r);
  if (L.vtx)
    PROF_LAUNCH(KC_RESTRICT, nb * (1.0 + 1.0 / (1 << DIM)), 2.0 * (1 << DIM) * fl,
                (k_restrict_v<DIM, W, S>), dim3(crows), blk, 0, s, C.g.nx, C.g.ny, C.g.nz, oth,
                Cr, ncols, st);
  else
    PROF_LAUNCH(KC_RESTRICT, nb * (1.0 + 1.0 / (1 << DIM)), 2.0 * (1 << DIM) * fl,
                (k_restrict<DIM, W, S>), dim3(crows), blk, (size_t)g.nx * ncols * sizeof(S), s,
                C.g.nx, C.g.ny, C.g.nz, oth, Cr, ncols, st);
  S* ec = cycle<DIM, W, S, S>(mg, lev + 1, Cr, ncols, Blk{nullptr, 0}, Blk{nullptr, 0}, ncols,
                           ncols, st, s);
  if (L.vtx)
    PROF_LAUNCH(KC_PROLONG, nb * (2.0 + 1.0 / (1 << DIM)), 2.0 * (1 << DIM) * fl,
                (k_prolong_add_v<DIM, W, S>), dim3(rows), blk, 0, s, g.nx, g.ny, g.nz, ec, cur,
                ncols, st);
  else
    PROF_LAUNCH(KC_PROLONG, nb * (2.0 + 1.0 / (1 << DIM)), 2.0 * (1 << DIM) * fl,
                (k_prolong_add<DIM, W, S>), dim3(rows), blk, 0, s, g.nx, g.ny, g.nz, ec, cur,
                ncols, st);
  // post-smoothing (nu_post >= 1); at level 0 the last sweep writes the
  // FP64 output
  for (int it = 0; it < mg.nu_post; ++it) {
    const bool last0 = (it == mg.nu_post - 1 && lev == 0);
    if (poly) {
      const S* y = cheb_apply<DIM, W, S>(L, cur, ncols, st, s);
      if (last0) {
        PROF_LAUNCH(KC_JACOBI, (2.0 + rb) * nb + fl * 8.0, 3.0 * fl,
                    (k_lincomb<W, S, RT, double>), dim3(rows), blk, 0, s, g.nx, (const S*)cur, r,
                    ldr, y, wr, out0.ptr, out0.ld, out1.ptr, out1.ld, split, ncols, st);
        return nullptr;
      }
      PROF_LAUNCH(KC_JACOBI, (3.0 + rb) * nb, 3.0 * fl, (k_lincomb<W, S, RT, S>), dim3(rows), blk,
                  0, s, g.nx, (const S*)cur, r, ldr, y, wr, oth, ncols, oth, ncols, ncols, ncols,
                  st);
      std::swap(cur, oth);
      continue;
    }
    if (last0) {
      PROF_LAUNCH(KC_JACOBI, (1.0 + rb) * nb + fl * 8.0, (2.0 * DIM + 5.0) * fl,
                  (k_jacobi<DIM, W, S, RT, double>), dim3(rows), blk, 0, s, g.nx, g.ny, g.nz, diag,
                  off, wr, cur, r, ldr, out0.ptr, out0.ld, out1.ptr, out1.ld, split, ncols, st);
      return nullptr;
    }
    PROF_LAUNCH(KC_JACOBI, (2.0 + rb) * nb, (2.0 * DIM + 5.0) * fl, (k_jacobi<DIM, W, S, RT, S>),
                dim3(rows), blk, 0, s, g.nx, g.ny, g.nz, diag, off, wr, cur, r, ldr, oth, ncols,
                oth, ncols, ncols, ncols, st);
    std::swap(cur, oth);
  }
  return cur;
}

// A single level: T is the dense inverse of the whole (small) operator.
static void dense_only(MG& mg, const double* R, int ldr, Blk out0, Blk out1, int split,
                       int ncols, const DevStatus* st, hipStream_t s) {
  MGLevel& L = mg.lv[0];
  const double nb = (double)L.g.n() * ncols * 8.0;
  launch_copy(L.g.n(), R, ldr, L.t, ncols, ncols, s);
  const int nbk = (mg.nc * ncols + 255) / 256;
  PROF_LAUNCH(KC_COARSE, (double)mg.nc * mg.nc * 8.0 + 2.0 * nb, 2.0 * mg.nc * L.g.n() * ncols,
              k_dense_apply<double>, dim3(nbk), dim3(256), 0, s, mg.nc, mg.coarse_inv, L.t, L.x,
              ncols, st);
  if (split > 0) launch_copy(L.g.n(), L.x, ncols, out0.ptr, out0.ld, split, s);
  if (split < ncols) launch_copy(L.g.n(), L.x + split, ncols, out1.ptr, out1.ld, ncols - split, s);
}

static bool fits(int w, const void* p) { return p == nullptr || ((uintptr_t)p % 16) == 0; }

// Vector width: 16 bytes of the level type per load when every column
// count, leading dimension and split is a multiple of it and the FP64
// input/output blocks are 16-byte aligned; otherwise one element.
static int pick_width(int w, const double* R, int ldr, Blk o0, Blk o1, int split, int ncols) {
  if (ncols % w || ldr % w || split % w) return 1;
  if ((o0.ptr && o0.ld % w) || (o1.ptr && o1.ld % w)) return 1;
  if (!fits(w, R) || !fits(w, o0.ptr) || !fits(w, o1.ptr)) return 1;
  return w;
}

template <int DIM>
static void cycle_top(MG& mg, const double* R, int ldr, Blk out0, Blk out1, int split, int ncols,
                      bool f32, const DevStatus* st, hipStream_t s) {
  if (f32) {
    if (pick_width(4, R, ldr, out0, out1, split, ncols) == 4)
      cycle<DIM, 4, float, double>(mg, 0, R, ldr, out0, out1, split, ncols, st, s);
    else
      cycle<DIM, 1, float, double>(mg, 0, R, ldr, out0, out1, split, ncols, st, s);
  } else {
    if (pick_width(2, R, ldr, out0, out1, split, ncols) == 2)
      cycle<DIM, 2, double, double>(mg, 0, R, ldr, out0, out1, split, ncols, st, s);
    else
      cycle<DIM, 1, double, double>(mg, 0, R, ldr, out0, out1, split, ncols, st, s);
  }
}

void mg_apply(MG& mg, const double* R, int ldr, Blk out0, Blk out1, int split, int ncols,
              bool f32, const DevStatus* st, hipStream_t s) {
  if (mg.lv.size() == 1) {
    dense_only(mg, R, ldr, out0, out1, split, ncols, st, s);
    return;
  }
  if (mg.lv[0].g.dim == 3)
    cycle_top<3>(mg, R, ldr, out0, out1, split, ncols, f32, st, s);
  else
    cycle_top<2>(mg, R, ldr, out0, out1, split, ncols, f32, st, s);
}

}  // namespace plhr
