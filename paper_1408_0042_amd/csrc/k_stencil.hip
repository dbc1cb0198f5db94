// Finite-difference block products (A - shift I) X for the 5-point (2-D)
// and 7-point (3-D) Dirichlet stencils, point-major blocks.  With a row
// scaling sc (a diagonal mass B = diag(b), sc = b^-1/2) the product is
// (S A S - shift I) X, S = diag(sc): the operator of the pencil (A, B)
// in the variables u = B^1/2 v, where B becomes the identity.
//
// One workgroup owns one grid row (fixed y, z; all x) and all columns of
// the block, so a row of the block is nx*ncols contiguous scalars: loads
// and stores are fully coalesced and the x-neighbours come from the same
// cache lines.  The y/z neighbours are rows owned by nearby workgroups; the
// XCD-aware renumbering keeps those rows in the same L2.
#include "common.cuh"

namespace plhr {

template <int DIM, bool SC>
__global__ __launch_bounds__(256) void k_fd_apply(
    int nx, int ny, int nz, double diag, double off, const double* __restrict__ pot,
    const double* __restrict__ sc, double shift, const double* __restrict__ X, int ldx,
    double* __restrict__ out, int ldo,
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
    double y;
    if constexpr (SC) {
      const double* sp = sc + p;
      const ptrdiff_t py = nx, pz = (ptrdiff_t)nx * ny;
      if (i > 0) nb += sp[-1] * xp[-ldx];
      if (i < nx - 1) nb += sp[1] * xp[ldx];
      if (j > 0) nb += sp[-py] * xp[-sy];
      if (j < ny - 1) nb += sp[py] * xp[sy];
      if (DIM == 3) {
        if (l > 0) nb += sp[-pz] * xp[-sz];
        if (l < nz - 1) nb += sp[pz] * xp[sz];
      }
      double d = diag;
      if (pot) d += pot[p];
      const double s0 = sp[0];
      y = s0 * (d * (s0 * xc) + off * nb) - shift * xc;
    } else {
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
      y = d * xc + off * nb;
    }
    out[p * ldo + c] = y;
    if (outr) outr[p * ldr + c] = y - xc * (colshift[c] - csub);
    if (outc) outc[p * ldc + c] = y;
  }
}

void launch_fd_apply(const Grid& g, const double* pot, const double* sc, double shift,
                     const double* X, int ldx, Blk out, Blk out_r, const double* colshift,
                     double csub, Blk out_c, int ncols, const DevStatus* st, hipStream_t s) {
  const int rows = g.ny * g.nz;
  dim3 grid(rows), block(256);
  const double nc = (double)g.n() * ncols * 8.0;
  prof_begin(KC_STENCIL,
             nc * (2 + (out_r.ptr ? 1 : 0) + (out_c.ptr ? 1 : 0)) + (pot ? g.n() * 8.0 : 0.0) +
                 (sc ? g.n() * 8.0 : 0.0),
             (double)g.n() * ncols * (2.0 * g.dim + 3.0 + (sc ? 2.0 * g.dim + 3.0 : 0.0)), s);
#define PLHR_FD_LAUNCH(D, S)                                                                   \
  hipLaunchKernelGGL((k_fd_apply<D, S>), grid, block, 0, s, g.nx, g.ny, g.nz, g.diag(), g.off(), \
                     pot, sc, shift, X, ldx, out.ptr, out.ld, out_r.ptr, out_r.ld, colshift,     \
                     csub, out_c.ptr, out_c.ld, ncols, st)
  if (g.dim == 3) {
    if (sc)
      PLHR_FD_LAUNCH(3, true);
    else
      PLHR_FD_LAUNCH(3, false);
  } else {
    if (sc)
      PLHR_FD_LAUNCH(2, true);
    else
      PLHR_FD_LAUNCH(2, false);
  }
#undef PLHR_FD_LAUNCH
  prof_end(KC_STENCIL, s);
}

}  // namespace plhr
