// Bloch-periodic block product in complex arithmetic:
//
//   Y = (scale (-Laplacian_theta) + diag(V) - shift I) X
//
// on an nx x ny x nz periodic box of spacing h, 7-point stencil.  The
// Hamiltonian is Hermitian but complex (Algorithm 2 of Section 4, and the
// periodic Kohn-Sham operators of Section 6.3 at one quasi-momentum): a
// neighbour across the box face in direction d is the point at the other
// end of that direction, multiplied by exp(+i theta_d) going forward and
// by exp(-i theta_d) going backward.  With one point in a direction both
// neighbours are the point itself, which leaves 2 - 2 cos(theta_d) on the
// diagonal.
//
// Blocks are point-major complex128: row p holds ncols interleaved
// (re, im) pairs, 16 bytes each.  One workgroup owns one grid row (fixed
// y, z; all x) and every column, so the row is nx*ncols contiguous 16-byte
// elements: loads and stores coalesce, the x neighbours share cache lines
// and the y/z neighbour rows belong to nearby workgroups (XCD-aware
// numbering keeps them in one L2).
#include <algorithm>
#include <cmath>

#include "common.cuh"

namespace plhr {

__device__ __forceinline__ double2 cmul(double2 a, double2 f) {
  return make_double2(a.x * f.x - a.y * f.y, a.x * f.y + a.y * f.x);
}

__global__ __launch_bounds__(256) void k_bloch_apply(int nx, int ny, int nz, double cs,
                                                     const double* __restrict__ pot,
                                                     double shift, double2 fx, double2 fy,
                                                     double2 fz, const double2* __restrict__ X,
                                                     int ldx, double2* __restrict__ Y, int ldy,
                                                     int ncols, const DevStatus* st) {
  if (halted(st)) return;
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = row % ny;
  const int l = row / ny;
  const int nelem = nx * ncols;
  const size_t rowp = (size_t)row * nx;
  // element offsets of the y and z neighbours, and of the wrapped ones
  const ptrdiff_t sx = ldx;
  const ptrdiff_t sy = (ptrdiff_t)nx * ldx;
  const ptrdiff_t sz = (ptrdiff_t)nx * ny * ldx;
  const ptrdiff_t ym = (j > 0) ? -sy : (ptrdiff_t)(ny - 1) * sy;
  const ptrdiff_t yp = (j < ny - 1) ? sy : -(ptrdiff_t)(ny - 1) * sy;
  const ptrdiff_t zm = (l > 0) ? -sz : (ptrdiff_t)(nz - 1) * sz;
  const ptrdiff_t zp = (l < nz - 1) ? sz : -(ptrdiff_t)(nz - 1) * sz;
  // phase factors of the y/z neighbours of this row (1 unless wrapped)
  const double2 one = make_double2(1.0, 0.0);
  const double2 gym = (j > 0) ? one : make_double2(fy.x, -fy.y);
  const double2 gyp = (j < ny - 1) ? one : fy;
  const double2 gzm = (l > 0) ? one : make_double2(fz.x, -fz.y);
  const double2 gzp = (l < nz - 1) ? one : fz;
  const double2 gxm_w = make_double2(fx.x, -fx.y);
  // (i, c) of this thread's element, advanced incrementally by the stride
  int i = threadIdx.x / ncols;
  int c = threadIdx.x - i * ncols;
  const int di = blockDim.x / ncols, dc = blockDim.x - di * ncols;
  for (int e = threadIdx.x; e < nelem; e += blockDim.x) {
    const size_t p = rowp + i;
    const double2* xp = X + p * ldx + c;
    const ptrdiff_t xm = (i > 0) ? -sx : (ptrdiff_t)(nx - 1) * sx;
    const ptrdiff_t xq = (i < nx - 1) ? sx : -(ptrdiff_t)(nx - 1) * sx;
    const double2 x0 = xp[0];
    const double2 a = xp[xm], b = xp[xq], u = xp[ym], v = xp[yp], w = xp[zm], z = xp[zp];
    const double2 na = (i > 0) ? a : cmul(a, gxm_w);
    const double2 nb = (i < nx - 1) ? b : cmul(b, fx);
    const double2 nu = cmul(u, gym), nv = cmul(v, gyp), nw = cmul(w, gzm), nz2 = cmul(z, gzp);
    const double sre = ((na.x + nb.x) + (nu.x + nv.x)) + (nw.x + nz2.x);
    const double sim = ((na.y + nb.y) + (nu.y + nv.y)) + (nw.y + nz2.y);
    double d = 6.0 * cs - shift;
    if (pot) d += pot[p];
    Y[p * ldy + c] = make_double2(d * x0.x - cs * sre, d * x0.y - cs * sim);
    c += dc;
    i += di;
    if (c >= ncols) {
      c -= ncols;
      ++i;
    }
  }
}

void launch_bloch_apply(int nx, int ny, int nz, double h, double scale, const double* theta,
                        const double* pot, double shift, const double* X, double* Y, int ncols,
                        hipStream_t s, int ldx, int ldy, const DevStatus* st) {
  if (ldx <= 0) ldx = ncols;
  if (ldy <= 0) ldy = ncols;
  const double cs = scale / (h * h);
  const double2 fx = make_double2(std::cos(theta[0]), std::sin(theta[0]));
  const double2 fy = make_double2(std::cos(theta[1]), std::sin(theta[1]));
  const double2 fz = make_double2(std::cos(theta[2]), std::sin(theta[2]));
  hipLaunchKernelGGL(k_bloch_apply, dim3(ny * nz), dim3(256), 0, s, nx, ny, nz, cs, pot, shift,
                     fx, fy, fz, reinterpret_cast<const double2*>(X), ldx,
                     reinterpret_cast<double2*>(Y), ldy, ncols, st);
}

// ------------------------------------------------------------- V-cycle
// The multigrid preconditioner of the Bloch operator (the Laplacian part,
// no potential): the same stencil on every level with spacing 2^l h and
// the same phases, cell-centred d-linear transfer with the phases across
// the periodic faces, R = P^H / 8, weighted Jacobi, a dense coarsest
// solve.  All blocks are point-major complex128 (n_l x ncols).

// One level's fused update  out = alpha w + beta (r - A_l w): alpha = 1,
// beta = omega / diag is a weighted-Jacobi sweep; alpha = 0, beta = 1 the
// residual.  w = NULL stands for w = 0.  out must not overlap w.  Row
// strides (complex entries): ldw of w, ldr of r; columns c < split go to
// out (stride ldo), the others to out1 (stride ldo1) at column c - split.
// kStrided = false: every stride is ncols and every column goes to out
// (the contiguous level buffers, with the plain index arithmetic).
template <bool kStrided>
__global__ __launch_bounds__(256) void k_bloch_level(int nx, int ny, int nz, double cs,
                                                     double2 fx, double2 fy, double2 fz,
                                                     const double2* __restrict__ w, int ldw,
                                                     const double2* __restrict__ r, int ldr,
                                                     double alpha, double beta,
                                                     double2* __restrict__ out, int ldo,
                                                     double2* __restrict__ out1, int ldo1,
                                                     int split, int ncols) {
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = row % ny;
  const int l = row / ny;
  const int nelem = nx * ncols;
  const size_t rowp = (size_t)row * nx;
  if (!kStrided) {
    ldw = ncols;
    ldr = ncols;
    ldo = ncols;
  }
  const ptrdiff_t sx = ldw;
  const ptrdiff_t sy = (ptrdiff_t)nx * ldw;
  const ptrdiff_t sz = (ptrdiff_t)nx * ny * ldw;
  const ptrdiff_t ym = (j > 0) ? -sy : (ptrdiff_t)(ny - 1) * sy;
  const ptrdiff_t yp = (j < ny - 1) ? sy : -(ptrdiff_t)(ny - 1) * sy;
  const ptrdiff_t zm = (l > 0) ? -sz : (ptrdiff_t)(nz - 1) * sz;
  const ptrdiff_t zp = (l < nz - 1) ? sz : -(ptrdiff_t)(nz - 1) * sz;
  const double2 one = make_double2(1.0, 0.0);
  const double2 gym = (j > 0) ? one : make_double2(fy.x, -fy.y);
  const double2 gyp = (j < ny - 1) ? one : fy;
  const double2 gzm = (l > 0) ? one : make_double2(fz.x, -fz.y);
  const double2 gzp = (l < nz - 1) ? one : fz;
  const double2 gxm_w = make_double2(fx.x, -fx.y);
  int i = threadIdx.x / ncols;
  int c = threadIdx.x - i * ncols;
  const int di = blockDim.x / ncols, dc = blockDim.x - di * ncols;
  for (int e = threadIdx.x; e < nelem; e += blockDim.x) {
    const size_t p = rowp + i;
    const double2 r0 = r[p * ldr + c];
    double2 y;
    if (w) {
      const double2* xp = w + p * ldw + c;
      const ptrdiff_t xm = (i > 0) ? -sx : (ptrdiff_t)(nx - 1) * sx;
      const ptrdiff_t xq = (i < nx - 1) ? sx : -(ptrdiff_t)(nx - 1) * sx;
      const double2 x0 = xp[0];
      const double2 a = xp[xm], b = xp[xq], u = xp[ym], v = xp[yp], ww = xp[zm], z = xp[zp];
      const double2 na = (i > 0) ? a : cmul(a, gxm_w);
      const double2 nb = (i < nx - 1) ? b : cmul(b, fx);
      const double2 nu = cmul(u, gym), nv = cmul(v, gyp), nw = cmul(ww, gzm), nz2 = cmul(z, gzp);
      const double sre = ((na.x + nb.x) + (nu.x + nv.x)) + (nw.x + nz2.x);
      const double sim = ((na.y + nb.y) + (nu.y + nv.y)) + (nw.y + nz2.y);
      const double d = 6.0 * cs;
      const double2 aw = make_double2(d * x0.x - cs * sre, d * x0.y - cs * sim);
      y = make_double2(alpha * x0.x + beta * (r0.x - aw.x), alpha * x0.y + beta * (r0.y - aw.y));
    } else {
      y = make_double2(beta * r0.x, beta * r0.y);
    }
    if (!kStrided || c < split)
      out[p * ldo + c] = y;
    else
      out1[p * ldo1 + (c - split)] = y;
    c += dc;
    i += di;
    if (c >= ncols) {
      c -= ncols;
      ++i;
    }
  }
}

// The four fine points feeding coarse point cc of one direction under
// R = P^H (up to the 1/8): 2cc and 2cc+1 with weight 3/4, the outer
// neighbours 2cc-1 and 2cc+2 with 1/4, wrapped across the periodic face
// with the conjugate of the prolongation's phase.
struct BlochTaps {
  int f[4];
  double2 w[4];
};
__device__ __forceinline__ BlochTaps restrict_taps(int cc, int Nc, double2 ph) {
  BlochTaps t;
  const int Nf = 2 * Nc;
  t.f[0] = 2 * cc;
  t.w[0] = make_double2(0.75, 0.0);
  t.f[1] = 2 * cc + 1;
  t.w[1] = make_double2(0.75, 0.0);
  t.f[2] = (cc > 0) ? 2 * cc - 1 : Nf - 1;
  t.w[2] = (cc > 0) ? make_double2(0.25, 0.0) : make_double2(0.25 * ph.x, -0.25 * ph.y);
  t.f[3] = (cc < Nc - 1) ? 2 * cc + 2 : 0;
  t.w[3] = (cc < Nc - 1) ? make_double2(0.25, 0.0) : make_double2(0.25 * ph.x, 0.25 * ph.y);
  return t;
}

// rc = P^H res / 8 (coarse grid nxc x nyc x nzc, fine grid twice that).
__global__ __launch_bounds__(256) void k_bloch_restrict(int nxc, int nyc, int nzc, double2 fx,
                                                        double2 fy, double2 fz,
                                                        const double2* __restrict__ res,
                                                        double2* __restrict__ rc, int ncols) {
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int jc = row % nyc;
  const int lc = row / nyc;
  const int nxf = 2 * nxc, nyf = 2 * nyc;
  const BlochTaps ty = restrict_taps(jc, nyc, fy);
  const BlochTaps tz = restrict_taps(lc, nzc, fz);
  const int nelem = nxc * ncols;
  int i = threadIdx.x / ncols;
  int c = threadIdx.x - i * ncols;
  const int di = blockDim.x / ncols, dc = blockDim.x - di * ncols;
  for (int e = threadIdx.x; e < nelem; e += blockDim.x) {
    const BlochTaps tx = restrict_taps(i, nxc, fx);
    double2 acc = make_double2(0.0, 0.0);
    for (int a = 0; a < 4; ++a) {
      for (int b = 0; b < 4; ++b) {
        const double2 wyz = cmul(tz.w[a], ty.w[b]);
        const size_t rowf = ((size_t)tz.f[a] * nyf + ty.f[b]) * nxf;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double2 v = res[(rowf + tx.f[q]) * ncols + c];
          const double2 wq = cmul(wyz, tx.w[q]);
          acc = make_double2(acc.x + (wq.x * v.x - wq.y * v.y), acc.y + (wq.x * v.y + wq.y * v.x));
        }
      }
    }
    rc[((size_t)row * nxc + i) * ncols + c] = make_double2(0.125 * acc.x, 0.125 * acc.y);
    c += dc;
    i += di;
    if (c >= ncols) {
      c -= ncols;
      ++i;
    }
  }
}

// The same restriction with the fine rows staged: workgroup (jc, lc)
// first combines its 16 fine rows (4 taps in z times 4 in y) into one fine
// row in LDS, reading each fine row with coalesced loads, then applies the
// x taps from LDS.  A fine row is read by 4 workgroups instead of each
// fine value by 8 gathers.  Needs nxf * ncols * 16 bytes of LDS.
__global__ __launch_bounds__(256) void k_bloch_restrict_lds(int nxc, int nyc, int nzc,
                                                            double2 fx, double2 fy, double2 fz,
                                                            const double2* __restrict__ res,
                                                            double2* __restrict__ rc,
                                                            int ncols) {
  extern __shared__ double2 srow[];
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int jc = row % nyc;
  const int lc = row / nyc;
  const int nxf = 2 * nxc, nyf = 2 * nyc;
  const BlochTaps ty = restrict_taps(jc, nyc, fy);
  const BlochTaps tz = restrict_taps(lc, nzc, fz);
  double2 wyz[16];
  size_t rows[16];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      wyz[4 * a + b] = cmul(tz.w[a], ty.w[b]);
      rows[4 * a + b] = ((size_t)tz.f[a] * nyf + ty.f[b]) * nxf * ncols;
    }
  const int nf = nxf * ncols;
  for (int e = threadIdx.x; e < nf; e += blockDim.x) {
    double2 v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = res[rows[q] + e];
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < 16; ++q)
      acc = make_double2(acc.x + (wyz[q].x * v[q].x - wyz[q].y * v[q].y),
                         acc.y + (wyz[q].x * v[q].y + wyz[q].y * v[q].x));
    srow[e] = acc;
  }
  __syncthreads();
  const int nelem = nxc * ncols;
  int i = threadIdx.x / ncols;
  int c = threadIdx.x - i * ncols;
  const int di = blockDim.x / ncols, dc = blockDim.x - di * ncols;
  for (int e = threadIdx.x; e < nelem; e += blockDim.x) {
    const BlochTaps tx = restrict_taps(i, nxc, fx);
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 v = srow[tx.f[q] * ncols + c];
      acc = make_double2(acc.x + (tx.w[q].x * v.x - tx.w[q].y * v.y),
                         acc.y + (tx.w[q].x * v.y + tx.w[q].y * v.x));
    }
    rc[((size_t)row * nxc + i) * ncols + c] = make_double2(0.125 * acc.x, 0.125 * acc.y);
    c += dc;
    i += di;
    if (c >= ncols) {
      c -= ncols;
      ++i;
    }
  }
}

// The two coarse points feeding fine point f of one direction under P:
// its parent f/2 with 3/4 and the parent's neighbour on f's side with 1/4,
// wrapped across the periodic face with exp(-/+ i theta).
__device__ __forceinline__ void prolong_taps(int f, int Nc, double2 ph, int* cidx, double2* w) {
  const int cp = f >> 1;
  cidx[0] = cp;
  w[0] = make_double2(0.75, 0.0);
  if ((f & 1) == 0) {
    cidx[1] = (cp > 0) ? cp - 1 : Nc - 1;
    w[1] = (cp > 0) ? make_double2(0.25, 0.0) : make_double2(0.25 * ph.x, -0.25 * ph.y);
  } else {
    cidx[1] = (cp < Nc - 1) ? cp + 1 : 0;
    w[1] = (cp < Nc - 1) ? make_double2(0.25, 0.0) : make_double2(0.25 * ph.x, 0.25 * ph.y);
  }
}

// x += P ec (fine grid nx x ny x nz, coarse grid half that).
__global__ __launch_bounds__(256) void k_bloch_prolong_add(int nx, int ny, int nz, double2 fx,
                                                           double2 fy, double2 fz,
                                                           const double2* __restrict__ ec,
                                                           double2* __restrict__ x, int ncols) {
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = row % ny;
  const int l = row / ny;
  const int nxc = nx / 2, nyc = ny / 2, nzc = nz / 2;
  int cy[2], cz[2];
  double2 wy[2], wz[2];
  prolong_taps(j, nyc, fy, cy, wy);
  prolong_taps(l, nzc, fz, cz, wz);
  const int nelem = nx * ncols;
  int i = threadIdx.x / ncols;
  int c = threadIdx.x - i * ncols;
  const int di = blockDim.x / ncols, dc = blockDim.x - di * ncols;
  for (int e = threadIdx.x; e < nelem; e += blockDim.x) {
    int cx[2];
    double2 wx[2];
    prolong_taps(i, nxc, fx, cx, wx);
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const double2 wyz = cmul(wz[a], wy[b]);
        const size_t rowc = ((size_t)cz[a] * nyc + cy[b]) * nxc;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const double2 v = ec[(rowc + cx[q]) * ncols + c];
          const double2 wq = cmul(wyz, wx[q]);
          acc = make_double2(acc.x + (wq.x * v.x - wq.y * v.y), acc.y + (wq.x * v.y + wq.y * v.x));
        }
      }
    const size_t o = ((size_t)row * nx + i) * ncols + c;
    const double2 x0 = x[o];
    x[o] = make_double2(x0.x + acc.x, x0.y + acc.y);
    c += dc;
    i += di;
    if (c >= ncols) {
      c -= ncols;
      ++i;
    }
  }
}

// The same prolongation with the coarse rows staged: workgroup (j, l)
// first combines its 4 coarse rows (2 taps in z times 2 in y) into one
// coarse row in LDS, then interpolates in x from LDS.  Needs
// nxc * ncols * 16 bytes of LDS.
__global__ __launch_bounds__(256) void k_bloch_prolong_add_lds(int nx, int ny, int nz,
                                                               double2 fx, double2 fy,
                                                               double2 fz,
                                                               const double2* __restrict__ ec,
                                                               double2* __restrict__ x,
                                                               int ncols) {
  extern __shared__ double2 crow[];
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = row % ny;
  const int l = row / ny;
  const int nxc = nx / 2, nyc = ny / 2, nzc = nz / 2;
  int cy[2], cz[2];
  double2 wy[2], wz[2];
  prolong_taps(j, nyc, fy, cy, wy);
  prolong_taps(l, nzc, fz, cz, wz);
  double2 wyz[4];
  size_t rows[4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      wyz[2 * a + b] = cmul(wz[a], wy[b]);
      rows[2 * a + b] = ((size_t)cz[a] * nyc + cy[b]) * nxc * ncols;
    }
  const int ncr = nxc * ncols;
  for (int e = threadIdx.x; e < ncr; e += blockDim.x) {
    double2 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = ec[rows[q] + e];
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      acc = make_double2(acc.x + (wyz[q].x * v[q].x - wyz[q].y * v[q].y),
                         acc.y + (wyz[q].x * v[q].y + wyz[q].y * v[q].x));
    crow[e] = acc;
  }
  __syncthreads();
  const int nelem = nx * ncols;
  int i = threadIdx.x / ncols;
  int c = threadIdx.x - i * ncols;
  const int di = blockDim.x / ncols, dc = blockDim.x - di * ncols;
  for (int e = threadIdx.x; e < nelem; e += blockDim.x) {
    int cx[2];
    double2 wx[2];
    prolong_taps(i, nxc, fx, cx, wx);
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const double2 v = crow[cx[q] * ncols + c];
      acc = make_double2(acc.x + (wx[q].x * v.x - wx[q].y * v.y),
                         acc.y + (wx[q].x * v.y + wx[q].y * v.x));
    }
    const size_t o = ((size_t)row * nx + i) * ncols + c;
    const double2 x0 = x[o];
    x[o] = make_double2(x0.x + acc.x, x0.y + acc.y);
    c += dc;
    i += di;
    if (c >= ncols) {
      c -= ncols;
      ++i;
    }
  }
}

// x = Ainv r on the coarsest level (nc points, Ainv row-major complex).
// Workgroup (i, column chunk of 64): its 256 lanes are 64 columns by 4
// slices of the sum over q (q = slice mod 4), combined through LDS.
__global__ __launch_bounds__(256) void k_bloch_dense(int nc, const double2* __restrict__ Ainv,
                                                     const double2* __restrict__ r, int ldr,
                                                     double2* __restrict__ x, int ldx,
                                                     double2* __restrict__ x1, int ldx1,
                                                     int split, int ncols) {
  __shared__ double2 part[4][64];
  const int i = blockIdx.x;
  const int cl = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int c = blockIdx.y * 64 + cl;
  const double2* a = Ainv + (size_t)i * nc;
  double2 acc = make_double2(0.0, 0.0);
  if (c < ncols) {
    for (int q = sl; q < nc; q += 4) {
      const double2 m = a[q], v = r[(size_t)q * ldr + c];
      acc = make_double2(acc.x + (m.x * v.x - m.y * v.y), acc.y + (m.x * v.y + m.y * v.x));
    }
  }
  part[sl][cl] = acc;
  __syncthreads();
  if (sl == 0 && c < ncols) {
    const double2 p1 = part[1][cl], p2 = part[2][cl], p3 = part[3][cl];
    const double2 v =
        make_double2(((acc.x + p1.x) + p2.x) + p3.x, ((acc.y + p1.y) + p2.y) + p3.y);
    if (c < split)
      x[(size_t)i * ldx + c] = v;
    else
      x1[(size_t)i * ldx1 + (c - split)] = v;
  }
}

static double2 phase(double t) { return make_double2(std::cos(t), std::sin(t)); }

void launch_bloch_level(int nx, int ny, int nz, double cs, const double* theta, const double* w,
                        const double* r, double alpha, double beta, double* out, int ncols,
                        hipStream_t s, const BlochLd& ld) {
  const int ldw = ld.w > 0 ? ld.w : ncols, ldr = ld.r > 0 ? ld.r : ncols;
  const int ldo = ld.o > 0 ? ld.o : ncols;
  const int split = ld.out1 ? ld.split : ncols;
  const bool strided = ldw != ncols || ldr != ncols || ldo != ncols || split != ncols;
  auto kern = strided ? k_bloch_level<true> : k_bloch_level<false>;
  hipLaunchKernelGGL(kern, dim3(ny * nz), dim3(256), 0, s, nx, ny, nz, cs, phase(theta[0]),
                     phase(theta[1]), phase(theta[2]), reinterpret_cast<const double2*>(w), ldw,
                     reinterpret_cast<const double2*>(r), ldr, alpha, beta,
                     reinterpret_cast<double2*>(out), ldo, reinterpret_cast<double2*>(ld.out1),
                     ld.o1, split, ncols);
}

void launch_bloch_restrict(int nxc, int nyc, int nzc, const double* theta, const double* res,
                           double* rc, int ncols, hipStream_t s) {
  const size_t lds = (size_t)2 * nxc * ncols * sizeof(double2);
  if (lds <= 65536) {
    hipLaunchKernelGGL(k_bloch_restrict_lds, dim3(nyc * nzc), dim3(256), lds, s, nxc, nyc, nzc,
                       phase(theta[0]), phase(theta[1]), phase(theta[2]),
                       reinterpret_cast<const double2*>(res), reinterpret_cast<double2*>(rc),
                       ncols);
    return;
  }
  hipLaunchKernelGGL(k_bloch_restrict, dim3(nyc * nzc), dim3(256), 0, s, nxc, nyc, nzc,
                     phase(theta[0]), phase(theta[1]), phase(theta[2]),
                     reinterpret_cast<const double2*>(res), reinterpret_cast<double2*>(rc), ncols);
}

void launch_bloch_prolong_add(int nx, int ny, int nz, const double* theta, const double* ec,
                              double* x, int ncols, hipStream_t s) {
  const size_t lds = (size_t)(nx / 2) * ncols * sizeof(double2);
  if (lds <= 65536) {
    hipLaunchKernelGGL(k_bloch_prolong_add_lds, dim3(ny * nz), dim3(256), lds, s, nx, ny, nz,
                       phase(theta[0]), phase(theta[1]), phase(theta[2]),
                       reinterpret_cast<const double2*>(ec), reinterpret_cast<double2*>(x),
                       ncols);
    return;
  }
  hipLaunchKernelGGL(k_bloch_prolong_add, dim3(ny * nz), dim3(256), 0, s, nx, ny, nz,
                     phase(theta[0]), phase(theta[1]), phase(theta[2]),
                     reinterpret_cast<const double2*>(ec), reinterpret_cast<double2*>(x), ncols);
}

void launch_bloch_dense(int nc, const double* Ainv, const double* r, double* x, int ncols,
                        hipStream_t s, const BlochLd& ld) {
  const int ldr = ld.r > 0 ? ld.r : ncols, ldo = ld.o > 0 ? ld.o : ncols;
  const int split = ld.out1 ? ld.split : ncols;
  hipLaunchKernelGGL(k_bloch_dense, dim3(nc, (ncols + 63) / 64), dim3(256), 0, s, nc,
                     reinterpret_cast<const double2*>(Ainv), reinterpret_cast<const double2*>(r),
                     ldr, reinterpret_cast<double2*>(x), ldo,
                     reinterpret_cast<double2*>(ld.out1), ld.o1, split, ncols);
}

}  // namespace plhr
