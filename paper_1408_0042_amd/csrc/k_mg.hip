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
// Every level works on point-major blocks of ncols columns; kernels assign
// one workgroup per grid row so accesses stay contiguous.
#include <cmath>
#include <cstring>
#include <vector>

#include "common.cuh"

namespace plhr {

template <int DIM>
__device__ __forceinline__ double nb_sum(const double* xp, int i, int j, int l, int nx, int ny,
                                         int nz, int ld) {
  const ptrdiff_t sy = (ptrdiff_t)nx * ld;
  const ptrdiff_t sz = (ptrdiff_t)nx * ny * ld;
  double nb = 0.0;
  if (i > 0) nb += xp[-ld];
  if (i < nx - 1) nb += xp[ld];
  if (j > 0) nb += xp[-sy];
  if (j < ny - 1) nb += xp[sy];
  if (DIM == 3) {
    if (l > 0) nb += xp[-sz];
    if (l < nz - 1) nb += xp[sz];
  }
  return nb;
}

// x_out = x_in + omega * (r - A x_in) / diag; x_in == nullptr means zero.
// Output columns [0, split) go to o0, the rest to o1.
template <int DIM>
__global__ __launch_bounds__(256) void k_jacobi(int nx, int ny, int nz, double diag, double off,
                                                double omega, const double* __restrict__ xin,
                                                const double* __restrict__ r, int ldr,
                                                double* __restrict__ o0, int ld0,
                                                double* __restrict__ o1, int ld1, int split,
                                                int ncols, const DevStatus* st) {
  if (halted(st)) return;
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = row % ny, l = row / ny;
  const int nelem = nx * ncols;
  const size_t rowp = (size_t)row * nx;
  const double w = omega / diag;
  for (int e = threadIdx.x; e < nelem; e += blockDim.x) {
    const int i = e / ncols;
    const int c = e - i * ncols;
    const size_t p = rowp + i;
    const double rv = r[p * ldr + c];
    double v;
    if (xin) {
      const double* xp = xin + p * ncols + c;
      const double xc = xp[0];
      const double ax = diag * xc + off * nb_sum<DIM>(xp, i, j, l, nx, ny, nz, ncols);
      v = xc + w * (rv - ax);
    } else {
      v = w * rv;
    }
    if (c < split)
      o0[p * ld0 + c] = v;
    else
      o1[p * ld1 + (c - split)] = v;
  }
}

// res = r - A x
template <int DIM>
__global__ __launch_bounds__(256) void k_residual(int nx, int ny, int nz, double diag, double off,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ r, int ldr,
                                                  double* __restrict__ res, int ncols,
                                                  const DevStatus* st) {
  if (halted(st)) return;
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = row % ny, l = row / ny;
  const int nelem = nx * ncols;
  const size_t rowp = (size_t)row * nx;
  for (int e = threadIdx.x; e < nelem; e += blockDim.x) {
    const int i = e / ncols;
    const int c = e - i * ncols;
    const size_t p = rowp + i;
    const double* xp = x + p * ncols + c;
    const double ax = diag * xp[0] + off * nb_sum<DIM>(xp, i, j, l, nx, ny, nz, ncols);
    res[p * ncols + c] = r[p * ldr + c] - ax;
  }
}

// Coarse r = P^T res / 2^d.  One workgroup per coarse row.
template <int DIM>
__global__ __launch_bounds__(256) void k_restrict(int cnx, int cny, int cnz,
                                                  const double* __restrict__ res,
                                                  double* __restrict__ rc, int ncols,
                                                  const DevStatus* st) {
  if (halted(st)) return;
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int cj = row % cny, cl = row / cny;
  const int fnx = 2 * cnx, fny = 2 * cny, fnz = 2 * cnz;
  const int nelem = cnx * ncols;
  const double wt[4] = {0.25, 0.75, 0.75, 0.25};
  const double norm = (DIM == 3) ? 0.125 : 0.25;
  for (int e = threadIdx.x; e < nelem; e += blockDim.x) {
    const int ci = e / ncols;
    const int c = e - ci * ncols;
    double acc = 0.0;
    const int zlo = (DIM == 3) ? 0 : 1, zhi = (DIM == 3) ? 4 : 2;
    for (int dz = zlo; dz < zhi; ++dz) {
      int fl = 0;
      double wz = 1.0;
      if (DIM == 3) {
        fl = 2 * cl - 1 + dz;
        if (fl < 0 || fl >= fnz) continue;
        wz = wt[dz];
      }
      for (int dy = 0; dy < 4; ++dy) {
        const int fj = 2 * cj - 1 + dy;
        if (fj < 0 || fj >= fny) continue;
        const double wy = wz * wt[dy];
        const size_t base = ((size_t)fl * fny + fj) * fnx;
        for (int dx = 0; dx < 4; ++dx) {
          const int fi = 2 * ci - 1 + dx;
          if (fi < 0 || fi >= fnx) continue;
          acc += wy * wt[dx] * res[(base + fi) * ncols + c];
        }
      }
    }
    const size_t cp = ((size_t)cl * cny + cj) * cnx + ci;
    rc[cp * ncols + c] = acc * norm;
  }
}

// x += P e (fine grid dims nx, ny, nz; coarse dims half).
template <int DIM>
__global__ __launch_bounds__(256) void k_prolong_add(int nx, int ny, int nz,
                                                     const double* __restrict__ ec,
                                                     double* __restrict__ x, int ncols,
                                                     const DevStatus* st) {
  if (halted(st)) return;
  const int row = xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = row % ny, l = row / ny;
  const int cnx = nx / 2, cny = ny / 2, cnz = (DIM == 3) ? nz / 2 : 1;
  const int nelem = nx * ncols;
  const size_t rowp = (size_t)row * nx;
  // parent and neighbour-parent in y and z
  const int pj = j >> 1, qj = (j & 1) ? pj + 1 : pj - 1;
  const int pl = (DIM == 3) ? (l >> 1) : 0;
  const int ql = (DIM == 3) ? ((l & 1) ? pl + 1 : pl - 1) : 0;
  for (int e = threadIdx.x; e < nelem; e += blockDim.x) {
    const int i = e / ncols;
    const int c = e - i * ncols;
    const int pi = i >> 1, qi = (i & 1) ? pi + 1 : pi - 1;
    double acc = 0.0;
    const int nzz = (DIM == 3) ? 2 : 1;
    for (int az = 0; az < nzz; ++az) {
      int cl = pl;
      double wz = 1.0;
      if (DIM == 3) {
        cl = az ? ql : pl;
        if (cl < 0 || cl >= cnz) continue;
        wz = az ? 0.25 : 0.75;
      }
      for (int ay = 0; ay < 2; ++ay) {
        const int cj = ay ? qj : pj;
        if (cj < 0 || cj >= cny) continue;
        const double wy = wz * (ay ? 0.25 : 0.75);
        const size_t base = ((size_t)cl * cny + cj) * cnx;
        acc += wy * 0.75 * ec[(base + pi) * ncols + c];
        if (qi >= 0 && qi < cnx) acc += wy * 0.25 * ec[(base + qi) * ncols + c];
      }
    }
    x[(rowp + i) * ncols + c] += acc;
  }
}

// x = Ainv r on the coarsest level (nc points).
__global__ __launch_bounds__(256) void k_dense_apply(int nc, const double* __restrict__ Ainv,
                                                     const double* __restrict__ r,
                                                     double* __restrict__ x, int ncols,
                                                     const DevStatus* st) {
  if (halted(st)) return;
  const int tot = nc * ncols;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += gridDim.x * blockDim.x) {
    const int i = e / ncols;
    const int c = e - i * ncols;
    const double* a = Ainv + (size_t)i * nc;
    double acc = 0.0;
    for (int q = 0; q < nc; ++q) acc += a[q] * r[(size_t)q * ncols + c];
    x[(size_t)i * ncols + c] = acc;
  }
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

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t mg_workspace_bytes(const Grid& fine, int levels, int cmax) {
  size_t bytes = 0;
  Grid g = fine;
  for (int lv = 0; lv < levels; ++lv) {
    const size_t blk = align256(g.n() * cmax * sizeof(double));
    bytes += (lv == 0 ? 2 : 3) * blk;
    if (lv == levels - 1) bytes += align256(g.n() * g.n() * sizeof(double));
    g.nx /= 2;
    g.ny /= 2;
    if (g.dim == 3) g.nz /= 2;
    g.h *= 2.0;
  }
  return bytes;
}

plhr_status mg_setup(MG& mg, const Grid& fine, int levels, int nu_pre, int nu_post, double omega,
                     int cmax, char*& ws, hipStream_t s) {
  mg.levels = levels;
  mg.nu_pre = nu_pre;
  mg.nu_post = nu_post;
  mg.omega = omega;
  mg.cmax = cmax;
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
    mg.lv.push_back(L);
    if (lv == levels - 1) break;
    g.nx /= 2;
    g.ny /= 2;
    if (g.dim == 3) g.nz /= 2;
    g.h *= 2.0;
  }
  const Grid& gc = mg.lv.back().g;
  mg.nc = (int)gc.n();
  std::vector<double> A;
  coarse_dense(gc, A);
  if (!spd_inverse(A, mg.nc)) {
    set_error("coarsest multigrid operator is not positive definite");
    return PLHR_ERR_NOT_HPD;
  }
  mg.coarse_inv = (double*)ws;
  ws += align256((size_t)mg.nc * mg.nc * sizeof(double));
  PLHR_HIP_CHECK(hipMemcpyAsync(mg.coarse_inv, A.data(), A.size() * sizeof(double),
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

// One V-cycle at level `lev` on input r (ld ldr).  At level 0 the result
// goes to out0/out1 (split by column); at coarser levels it is left in one
// of the level's work buffers, whose address is returned.
template <int DIM>
static double* cycle(MG& mg, int lev, const double* r, int ldr, Blk out0, Blk out1, int split,
                     int ncols, const DevStatus* st, hipStream_t s) {
  MGLevel& L = mg.lv[lev];
  const Grid& g = L.g;
  const int rows = g.ny * g.nz;
  const dim3 blk(256);
  const bool coarsest = (lev == (int)mg.lv.size() - 1);
  const double nb = (double)g.n() * ncols * 8.0;        // one pass over this level
  const double fl = (double)g.n() * ncols;
  if (coarsest) {
    const int tot = mg.nc * ncols;
    const int nbk = (tot + 255) / 256;
    if (lev == 0) {
      // single-level "cycle": dense solve on the finest grid
      launch_copy(g.n(), r, ldr, L.t, ncols, ncols, s);
      PROF_LAUNCH(KC_COARSE, (double)mg.nc * mg.nc * 8.0 + 2.0 * nb, 2.0 * mg.nc * fl,
                  k_dense_apply, dim3(nbk), blk, 0, s, mg.nc, mg.coarse_inv, L.t, L.x, ncols, st);
      if (split > 0) launch_copy(g.n(), L.x, ncols, out0.ptr, out0.ld, split, s);
      if (split < ncols)
        launch_copy(g.n(), L.x + split, ncols, out1.ptr, out1.ld, ncols - split, s);
      return nullptr;
    }
    PROF_LAUNCH(KC_COARSE, (double)mg.nc * mg.nc * 8.0 + 2.0 * nb, 2.0 * mg.nc * fl,
                k_dense_apply, dim3(nbk), blk, 0, s, mg.nc, mg.coarse_inv, r, L.x, ncols, st);
    return L.x;
  }
  const double diag = g.diag(), off = g.off(), om = mg.omega;
  double* cur = L.x;
  double* oth = L.t;
  // pre-smoothing from a zero guess (nu_pre >= 1)
  for (int it = 0; it < mg.nu_pre; ++it) {
    PROF_LAUNCH(KC_JACOBI, (it == 0 ? 2.0 : 3.0) * nb, (it == 0 ? 1.0 : 2.0 * DIM + 5.0) * fl,
                k_jacobi<DIM>, dim3(rows), blk, 0, s, g.nx, g.ny, g.nz, diag, off, om,
                it == 0 ? (const double*)nullptr : (const double*)cur, r, ldr, oth, ncols, oth,
                ncols, ncols, ncols, st);
    std::swap(cur, oth);
  }
  // residual -> oth, restrict -> coarse r, coarse cycle, prolongate into cur
  PROF_LAUNCH(KC_RESIDUAL, 3.0 * nb, (2.0 * DIM + 3.0) * fl, k_residual<DIM>, dim3(rows), blk, 0,
              s, g.nx, g.ny, g.nz, diag, off, cur, r, ldr, oth, ncols, st);
  MGLevel& C = mg.lv[lev + 1];
  const int crows = C.g.ny * C.g.nz;
  PROF_LAUNCH(KC_RESTRICT, nb * (1.0 + 1.0 / (1 << DIM)), 2.0 * (1 << DIM) * fl,
              k_restrict<DIM>, dim3(crows), blk, 0, s, C.g.nx, C.g.ny, C.g.nz, oth, C.r, ncols, st);
  double* ec = cycle<DIM>(mg, lev + 1, C.r, ncols, Blk{nullptr, 0}, Blk{nullptr, 0}, ncols,
                          ncols, st, s);
  PROF_LAUNCH(KC_PROLONG, nb * (2.0 + 1.0 / (1 << DIM)), 2.0 * (1 << DIM) * fl,
              k_prolong_add<DIM>, dim3(rows), blk, 0, s, g.nx, g.ny, g.nz, ec, cur, ncols, st);
  // post-smoothing (nu_post >= 1); at level 0 the last sweep writes the output
  for (int it = 0; it < mg.nu_post; ++it) {
    if (it == mg.nu_post - 1 && lev == 0) {
      PROF_LAUNCH(KC_JACOBI, 3.0 * nb, (2.0 * DIM + 5.0) * fl, k_jacobi<DIM>, dim3(rows), blk, 0, s,
                  g.nx, g.ny, g.nz, diag, off, om, cur, r, ldr, out0.ptr, out0.ld, out1.ptr,
                  out1.ld, split, ncols, st);
      return nullptr;
    }
    PROF_LAUNCH(KC_JACOBI, 3.0 * nb, (2.0 * DIM + 5.0) * fl, k_jacobi<DIM>, dim3(rows), blk, 0, s,
                g.nx, g.ny, g.nz, diag, off, om, cur, r, ldr, oth, ncols, oth, ncols, ncols, ncols,
                st);
    std::swap(cur, oth);
  }
  return cur;
}

void mg_apply(MG& mg, const double* R, int ldr, Blk out0, Blk out1, int split, int ncols,
              const DevStatus* st, hipStream_t s) {
  if (mg.lv[0].g.dim == 3)
    cycle<3>(mg, 0, R, ldr, out0, out1, split, ncols, st, s);
  else
    cycle<2>(mg, 0, R, ldr, out0, out1, split, ncols, st, s);
}

}  // namespace plhr
