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
                                                     double2* __restrict__ Y, int ncols) {
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = row % ny;
  const int l = row / ny;
  const int nelem = nx * ncols;
  const size_t rowp = (size_t)row * nx;
  // element offsets of the y and z neighbours, and of the wrapped ones
  const ptrdiff_t sx = ncols;
  const ptrdiff_t sy = (ptrdiff_t)nx * ncols;
  const ptrdiff_t sz = (ptrdiff_t)nx * ny * ncols;
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
    const double2* xp = X + p * ncols + c;
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
    Y[p * ncols + c] = make_double2(d * x0.x - cs * sre, d * x0.y - cs * sim);
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
                        hipStream_t s) {
  const double cs = scale / (h * h);
  const double2 fx = make_double2(std::cos(theta[0]), std::sin(theta[0]));
  const double2 fy = make_double2(std::cos(theta[1]), std::sin(theta[1]));
  const double2 fz = make_double2(std::cos(theta[2]), std::sin(theta[2]));
  hipLaunchKernelGGL(k_bloch_apply, dim3(ny * nz), dim3(256), 0, s, nx, ny, nz, cs, pot, shift,
                     fx, fy, fz, reinterpret_cast<const double2*>(X),
                     reinterpret_cast<double2*>(Y), ncols);
}

}  // namespace plhr
