// Finite-difference block products (A - shift I) X for the 5-point (2-D)
// and 7-point (3-D) Dirichlet stencils, point-major blocks.
//
// One workgroup owns one grid row (fixed y, z; all x) and all columns of
// the block, so a row of the block is nx*ncols contiguous scalars: loads
// and stores are fully coalesced and the x-neighbours come from the same
// cache lines.  The y/z neighbours are rows owned by nearby workgroups; the
// XCD-aware renumbering keeps those rows in the same L2.
#include "common.cuh"

namespace plhr {

template <int DIM>
__global__ __launch_bounds__(256) void k_fd_apply(
    int nx, int ny, int nz, double diag, double off, const double* __restrict__ pot,
    double shift, const double* __restrict__ X, int ldx, double* __restrict__ out, int ldo,
    double* __restrict__ outr, int ldr, const double* __restrict__ colshift, double csub,
    double* __restrict__ outc, int ldc, int ncols, const DevStatus* st) {
  if (halted(st)) return;
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = row % ny;
  const int l = row / ny;
  const int nelem = nx * ncols;
  const size_t rowp = (size_t)row * nx;  // first point of the row
  const ptrdiff_t sy = (ptrdiff_t)nx * ldx;
  const ptrdiff_t sz = (ptrdiff_t)nx * ny * ldx;
  for (int e = threadIdx.x; e < nelem; e += blockDim.x) {
    const int i = e / ncols;
    const int c = e - i * ncols;
    const size_t p = rowp + i;
    const double* xp = X + p * ldx + c;
    const double xc = xp[0];
    double nb = 0.0;
    if (i > 0) nb += xp[-ldx];
    if (i < nx - 1) nb += xp[ldx];
    if (j > 0) nb += xp[-sy];
    if (j < ny - 1) nb += xp[sy];
    if (DIM == 3) {
      if (l > 0) nb += xp[-sz];
      if (l < nz - 1) nb += xp[sz];
    }
    double d = diag - shift;
    if (pot) d += pot[p];
    const double y = d * xc + off * nb;
    out[p * ldo + c] = y;
    if (outr) outr[p * ldr + c] = y - xc * (colshift[c] - csub);
    if (outc) outc[p * ldc + c] = y;
  }
}

void launch_fd_apply(const Grid& g, const double* pot, double shift, const double* X, int ldx,
                     Blk out, Blk out_r, const double* colshift, double csub, Blk out_c,
                     int ncols, const DevStatus* st, hipStream_t s) {
  const int rows = g.ny * g.nz;
  dim3 grid(rows), block(256);
  const double nc = (double)g.n() * ncols * 8.0;
  prof_begin(KC_STENCIL, nc * (2 + (out_r.ptr ? 1 : 0) + (out_c.ptr ? 1 : 0)) + (pot ? g.n() * 8.0 : 0.0),
             (double)g.n() * ncols * (2.0 * g.dim + 3.0), s);
  if (g.dim == 3)
    hipLaunchKernelGGL(k_fd_apply<3>, grid, block, 0, s, g.nx, g.ny, g.nz, g.diag(), g.off(),
                       pot, shift, X, ldx, out.ptr, out.ld, out_r.ptr, out_r.ld, colshift, csub,
                       out_c.ptr, out_c.ld, ncols, st);
  else
    hipLaunchKernelGGL(k_fd_apply<2>, grid, block, 0, s, g.nx, g.ny, g.nz, g.diag(), g.off(),
                       pot, shift, X, ldx, out.ptr, out.ld, out_r.ptr, out_r.ld, colshift, csub,
                       out_c.ptr, out_c.ld, ncols, st);
  prof_end(KC_STENCIL, s);
}

}  // namespace plhr
