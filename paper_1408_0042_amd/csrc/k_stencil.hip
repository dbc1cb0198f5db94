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

// The same product two columns per lane (16-byte loads and stores) for
// blocks whose column count, leading dimensions and column offsets are
// even; the arithmetic of each column is that of k_fd_apply.
template <int DIM>
__global__ __launch_bounds__(256) void k_fd_apply2(
    int nx, int ny, int nz, double diag, double off, const double* __restrict__ pot,
    double shift, const double* __restrict__ X, int ldx, double* __restrict__ out, int ldo,
    double* __restrict__ outr, int ldr, const double* __restrict__ colshift, double csub,
    double* __restrict__ outc, int ldc, int ncols, const DevStatus* st) {
  if (halted(st)) return;
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = row % ny;
  const int l = row / ny;
  const int nc2 = ncols / 2;
  const int nelem = nx * nc2;
  const size_t rowp = (size_t)row * nx;
  const ptrdiff_t sy = (ptrdiff_t)nx * ldx;
  const ptrdiff_t sz = (ptrdiff_t)nx * ny * ldx;
  for (int e = threadIdx.x; e < nelem; e += blockDim.x) {
    const int i = e / nc2;
    const int c = 2 * (e - i * nc2);
    const size_t p = rowp + i;
    const double* xp = X + p * ldx + c;
    const double2 xc = *reinterpret_cast<const double2*>(xp);
    double nbx = 0.0, nby = 0.0;
    auto add = [&](const double* q) {
      const double2 v = *reinterpret_cast<const double2*>(q);
      nbx += v.x;
      nby += v.y;
    };
    if (i > 0) add(xp - ldx);
    if (i < nx - 1) add(xp + ldx);
    if (j > 0) add(xp - sy);
    if (j < ny - 1) add(xp + sy);
    if (DIM == 3) {
      if (l > 0) add(xp - sz);
      if (l < nz - 1) add(xp + sz);
    }
    double d = diag - shift;
    if (pot) d += pot[p];
    const double yx = d * xc.x + off * nbx;
    const double yy = d * xc.y + off * nby;
    *reinterpret_cast<double2*>(out + p * ldo + c) = double2{yx, yy};
    if (outr)
      *reinterpret_cast<double2*>(outr + p * ldr + c) =
          double2{yx - xc.x * (colshift[c] - csub), yy - xc.y * (colshift[c + 1] - csub)};
    if (outc) *reinterpret_cast<double2*>(outc + p * ldc + c) = double2{yx, yy};
  }
}

static bool even16(const void* q, int ld) {
  return q == nullptr || ((((uintptr_t)q) & 15) == 0 && (ld & 1) == 0);
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
  if (!sc && (ncols & 1) == 0 && even16(X, ldx) && even16(out.ptr, out.ld) &&
      even16(out_r.ptr, out_r.ld) && even16(out_c.ptr, out_c.ld)) {
    if (g.dim == 3)
      hipLaunchKernelGGL(k_fd_apply2<3>, grid, block, 0, s, g.nx, g.ny, g.nz, g.diag(), g.off(),
                         pot, shift, X, ldx, out.ptr, out.ld, out_r.ptr, out_r.ld, colshift, csub,
                         out_c.ptr, out_c.ld, ncols, st);
    else
      hipLaunchKernelGGL(k_fd_apply2<2>, grid, block, 0, s, g.nx, g.ny, g.nz, g.diag(), g.off(),
                         pot, shift, X, ldx, out.ptr, out.ld, out_r.ptr, out_r.ld, colshift, csub,
                         out_c.ptr, out_c.ld, ncols, st);
    prof_end(KC_STENCIL, s);
    return;
  }
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


// Bilinear (2-D) / trilinear (3-D) finite elements on a uniform mesh with
// Dirichlet boundary, interior nodes only: the stiffness and the
// consistent mass are tensor products of the 1-D element matrices, so
// both are 9- / 27-point stencils whose weights depend only on the offset
// (the finite-element model problem of Section 6).  One pass gives
//   out  = (A - shift B) X,  A = scale K + diag(pot),  B = M (bmass) or I
//   outb = B X                                  (if outb.ptr)
//   outr = out - (B X) (colshift - csub)        (if out_r.ptr)
//   outc = out                                  (if out_c.ptr)
template <int DIM>
__global__ __launch_bounds__(256) void k_q1_apply(
    int nx, int ny, int nz, Q1Weights w, const double* __restrict__ pot, double shift, int bmass,
    const double* __restrict__ X, int ldx, double* __restrict__ out, int ldo,
    double* __restrict__ outr, int ldr, const double* __restrict__ colshift, double csub,
    double* __restrict__ outc, int ldc, double* __restrict__ outb, int ldb, int ncols,
    const DevStatus* st) {
  if (halted(st)) return;
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = row % ny;
  const int l = row / ny;
  const int nelem = nx * ncols;
  const size_t rowp = (size_t)row * nx;
  const ptrdiff_t sy = (ptrdiff_t)nx * ldx;
  const ptrdiff_t sz = (ptrdiff_t)nx * ny * ldx;
  const int zlo = (DIM == 3) ? -1 : 0, zhi = (DIM == 3) ? 1 : 0;
  for (int e = threadIdx.x; e < nelem; e += blockDim.x) {
    const int i = e / ncols;
    const int c = e - i * ncols;
    const size_t p = rowp + i;
    const double* xp = X + p * ldx + c;
    double ka = 0.0, mb = 0.0;
    for (int dz = zlo; dz <= zhi; ++dz) {
      if (l + dz < 0 || l + dz >= nz) continue;
      for (int dy = -1; dy <= 1; ++dy) {
        if (j + dy < 0 || j + dy >= ny) continue;
        for (int dx = -1; dx <= 1; ++dx) {
          if (i + dx < 0 || i + dx >= nx) continue;
          const int o = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
          const double xv = xp[dz * sz + dy * sy + dx * ldx];
          ka += w.a[o] * xv;
          mb += w.m[o] * xv;
        }
      }
    }
    const double xc = xp[0];
    if (pot) ka += pot[p] * xc;
    const double bx = bmass ? mb : xc;
    const double y = ka - shift * bx;
    out[p * ldo + c] = y;
    if (outb) outb[p * ldb + c] = bx;
    if (outr) outr[p * ldr + c] = y - bx * (colshift[c] - csub);
    if (outc) outc[p * ldc + c] = y;
  }
}

Q1Weights q1_weights(const Grid& g) {
  // 1-D element matrices on interior nodes: K1 = (1/h)[-1 2 -1],
  // M1 = (h/6)[1 4 1]; K = sum_a M1 x .. x K1(a) x .. x M1, M = M1 x .. x M1
  const double h = g.h;
  const double k1[3] = {-1.0 / h, 2.0 / h, -1.0 / h};
  const double m1[3] = {h / 6.0, 4.0 * h / 6.0, h / 6.0};
  Q1Weights w{};
  for (int dz = 0; dz < 3; ++dz)
    for (int dy = 0; dy < 3; ++dy)
      for (int dx = 0; dx < 3; ++dx) {
        const int o = dz * 9 + dy * 3 + dx;
        if (g.dim == 2) {
          if (dz != 1) continue;
          w.a[o] = g.scale * (k1[dx] * m1[dy] + m1[dx] * k1[dy]);
          w.m[o] = m1[dx] * m1[dy];
        } else {
          w.a[o] = g.scale * (k1[dx] * m1[dy] * m1[dz] + m1[dx] * k1[dy] * m1[dz] +
                              m1[dx] * m1[dy] * k1[dz]);
          w.m[o] = m1[dx] * m1[dy] * m1[dz];
        }
      }
  return w;
}

void launch_q1_apply(const Grid& g, const double* pot, double shift, bool bmass, const double* X,
                     int ldx, Blk out, Blk out_r, const double* colshift, double csub, Blk out_c,
                     Blk out_b, int ncols, const DevStatus* st, hipStream_t s) {
  const int rows = g.ny * g.nz;
  const double nc = (double)g.n() * ncols * 8.0;
  const int npt = (g.dim == 3) ? 27 : 9;
  prof_begin(KC_STENCIL,
             nc * (2 + (out_r.ptr ? 1 : 0) + (out_c.ptr ? 1 : 0) + (out_b.ptr ? 1 : 0)) +
                 (pot ? g.n() * 8.0 : 0.0),
             (double)g.n() * ncols * (4.0 * npt + 4.0), s);
  const Q1Weights w = q1_weights(g);
  if (g.dim == 3)
    hipLaunchKernelGGL(k_q1_apply<3>, dim3(rows), dim3(256), 0, s, g.nx, g.ny, g.nz, w, pot,
                       shift, (int)bmass, X, ldx, out.ptr, out.ld, out_r.ptr, out_r.ld, colshift,
                       csub, out_c.ptr, out_c.ld, out_b.ptr, out_b.ld, ncols, st);
  else
    hipLaunchKernelGGL(k_q1_apply<2>, dim3(rows), dim3(256), 0, s, g.nx, g.ny, g.nz, w, pot,
                       shift, (int)bmass, X, ldx, out.ptr, out.ld, out_r.ptr, out_r.ld, colshift,
                       csub, out_c.ptr, out_c.ld, out_b.ptr, out_b.ld, ncols, st);
  prof_end(KC_STENCIL, s);
}


// General sparse (CSR) block products on point-major blocks: one thread
// per (row, column) element; the lanes of one row share its index and
// value loads, and neighbouring columns of a gathered row of X are
// contiguous.  out = (A - shift B)X with B the CSR matrix Bm (or I when
// Bm.row_ptr is null); extra outputs as for the Q1 stencil.
__global__ __launch_bounds__(256) void k_csr_apply(
    int n, CsrMat Am, CsrMat Bm, const double* __restrict__ pot, double shift,
    const double* __restrict__ X, int ldx, double* __restrict__ out, int ldo,
    double* __restrict__ outr, int ldr, const double* __restrict__ colshift, double csub,
    double* __restrict__ outc, int ldc, double* __restrict__ outb, int ldb, int ncols,
    const DevStatus* st) {
  if (halted(st)) return;
  const size_t tot = (size_t)n * ncols;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / ncols);
    const int c = (int)(e - (size_t)i * ncols);
    double ka = 0.0;
    const int q0 = Am.row_ptr[i], q1 = Am.row_ptr[i + 1];
#pragma unroll 4
    for (int q = q0; q < q1; ++q) ka += Am.values[q] * X[(size_t)Am.col_idx[q] * ldx + c];
    const double xc = X[(size_t)i * ldx + c];
    if (pot) ka += pot[i] * xc;
    double bx = xc;
    if (Bm.row_ptr) {
      bx = 0.0;
      for (int q = Bm.row_ptr[i]; q < Bm.row_ptr[i + 1]; ++q)
        bx += Bm.values[q] * X[(size_t)Bm.col_idx[q] * ldx + c];
    }
    const double y = ka - shift * bx;
    out[(size_t)i * ldo + c] = y;
    if (outb) outb[(size_t)i * ldb + c] = bx;
    if (outr) outr[(size_t)i * ldr + c] = y - bx * (colshift[c] - csub);
    if (outc) outc[(size_t)i * ldc + c] = y;
  }
}

// Two columns per lane (16-byte gathers) when the column count, leading
// dimensions and column offsets are even; per column the arithmetic of
// k_csr_apply.
__global__ __launch_bounds__(256) void k_csr_apply2(
    int n, CsrMat Am, CsrMat Bm, const double* __restrict__ pot, double shift,
    const double* __restrict__ X, int ldx, double* __restrict__ out, int ldo,
    double* __restrict__ outr, int ldr, const double* __restrict__ colshift, double csub,
    double* __restrict__ outc, int ldc, double* __restrict__ outb, int ldb, int ncols,
    const DevStatus* st) {
  if (halted(st)) return;
  const int nc2 = ncols / 2;
  const size_t tot = (size_t)n * nc2;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / nc2);
    const int c = 2 * (int)(e - (size_t)i * nc2);
    double kx = 0.0, ky = 0.0;
    const int q0 = Am.row_ptr[i], q1 = Am.row_ptr[i + 1];
#pragma unroll 4
    for (int q = q0; q < q1; ++q) {
      const double a = Am.values[q];
      const double2 v = *reinterpret_cast<const double2*>(X + (size_t)Am.col_idx[q] * ldx + c);
      kx += a * v.x;
      ky += a * v.y;
    }
    const double2 xc = *reinterpret_cast<const double2*>(X + (size_t)i * ldx + c);
    if (pot) {
      kx += pot[i] * xc.x;
      ky += pot[i] * xc.y;
    }
    double bx = xc.x, by = xc.y;
    if (Bm.row_ptr) {
      bx = 0.0;
      by = 0.0;
      for (int q = Bm.row_ptr[i]; q < Bm.row_ptr[i + 1]; ++q) {
        const double b = Bm.values[q];
        const double2 v = *reinterpret_cast<const double2*>(X + (size_t)Bm.col_idx[q] * ldx + c);
        bx += b * v.x;
        by += b * v.y;
      }
    }
    const double yx = kx - shift * bx, yy = ky - shift * by;
    *reinterpret_cast<double2*>(out + (size_t)i * ldo + c) = double2{yx, yy};
    if (outb) *reinterpret_cast<double2*>(outb + (size_t)i * ldb + c) = double2{bx, by};
    if (outr)
      *reinterpret_cast<double2*>(outr + (size_t)i * ldr + c) =
          double2{yx - bx * (colshift[c] - csub), yy - by * (colshift[c + 1] - csub)};
    if (outc) *reinterpret_cast<double2*>(outc + (size_t)i * ldc + c) = double2{yx, yy};
  }
}

void launch_csr_apply(int n, const CsrMat& A, const CsrMat& B, const double* pot, double shift,
                      const double* X, int ldx, Blk out, Blk out_r, const double* colshift,
                      double csub, Blk out_c, Blk out_b, int ncols, const DevStatus* st,
                      hipStream_t s) {
  const double nc = (double)n * ncols * 8.0;
  const double nnz = (double)A.nnz + (B.row_ptr ? (double)B.nnz : 0.0);
  prof_begin(KC_STENCIL,
             nc * (2 + (out_r.ptr ? 1 : 0) + (out_c.ptr ? 1 : 0) + (out_b.ptr ? 1 : 0)) +
                 nnz * 12.0 + (n + 1.0) * 4.0 * (B.row_ptr ? 2.0 : 1.0) + (pot ? n * 8.0 : 0.0),
             2.0 * nnz * ncols + 4.0 * (double)n * ncols, s);
  if ((ncols & 1) == 0 && even16(X, ldx) && even16(out.ptr, out.ld) &&
      even16(out_r.ptr, out_r.ld) && even16(out_c.ptr, out_c.ld) &&
      even16(out_b.ptr, out_b.ld)) {
    const size_t tot2 = (size_t)n * (ncols / 2);
    const size_t want2 = (tot2 + 255) / 256;
    const int nb2 = (int)(want2 < (size_t)1 << 30 ? want2 : (size_t)1 << 30);
    hipLaunchKernelGGL(k_csr_apply2, dim3(nb2 > 0 ? nb2 : 1), dim3(256), 0, s, n, A, B, pot,
                       shift, X, ldx, out.ptr, out.ld, out_r.ptr, out_r.ld, colshift, csub,
                       out_c.ptr, out_c.ld, out_b.ptr, out_b.ld, ncols, st);
    prof_end(KC_STENCIL, s);
    return;
  }
  // one element per lane: the gathers of a lane's row are its only
  // dependent loads
  const size_t tot = (size_t)n * ncols;
  const size_t want = (tot + 255) / 256;
  const int nb = (int)(want < (size_t)1 << 30 ? want : (size_t)1 << 30);
  hipLaunchKernelGGL(k_csr_apply, dim3(nb > 0 ? nb : 1), dim3(256), 0, s, n, A, B, pot, shift, X,
                     ldx, out.ptr, out.ld, out_r.ptr, out_r.ld, colshift, csub, out_c.ptr,
                     out_c.ld, out_b.ptr, out_b.ld, ncols, st);
  prof_end(KC_STENCIL, s);
}

}  // namespace plhr
