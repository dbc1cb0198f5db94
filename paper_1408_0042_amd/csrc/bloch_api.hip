// Host driver of the multigrid preconditioner of the complex Bloch
// operator (plhr_bloch_prec_*): the level hierarchy, the dense coarsest
// inverse (host Cholesky of the Hermitian coarse matrix at create) and the
// V-cycle recursion over the kernels of k_bloch.hip.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "internal.h"

using namespace plhr;

namespace {

// the dense coarse inverse is formed on the host at create (cubic cost)
constexpr int kBlochMaxCoarse = 1024;

struct BlochLevel {
  int nx, ny, nz;
  double cs;    // scale / h_l^2
  double diag;  // the stencil's diagonal (Jacobi)
  double* x = nullptr;
  double* t = nullptr;
  double* r = nullptr;  // right-hand side of the level (coarse levels)
  size_t n() const { return (size_t)nx * ny * nz; }
};

typedef std::complex<double> cd;

// Dense Bloch operator of a level (row-major), the same stencil as the
// product kernel: 6 cs on the diagonal, -cs times the phase factor for each
// of the six neighbours (a neighbour across a face picks up exp(+/- i theta),
// and with one point in a direction it is the point itself).
void bloch_dense(const BlochLevel& L, const double* theta, std::vector<cd>& A) {
  const int n = (int)L.n();
  A.assign((size_t)n * n, cd(0.0, 0.0));
  const int N[3] = {L.nx, L.ny, L.nz};
  for (int l = 0; l < L.nz; ++l)
    for (int j = 0; j < L.ny; ++j)
      for (int i = 0; i < L.nx; ++i) {
        const int p = i + L.nx * (j + L.ny * l);
        const int idx[3] = {i, j, l};
        A[(size_t)p * n + p] += 6.0 * L.cs;
        for (int d = 0; d < 3; ++d) {
          const cd ph = std::polar(1.0, theta[d]);
          for (int dir = -1; dir <= 1; dir += 2) {
            int q[3] = {idx[0], idx[1], idx[2]};
            int v = q[d] + dir;
            cd f(1.0, 0.0);
            if (v < 0) {
              v += N[d];
              f = std::conj(ph);
            } else if (v >= N[d]) {
              v -= N[d];
              f = ph;
            }
            q[d] = v;
            const int pq = q[0] + L.nx * (q[1] + L.ny * q[2]);
            A[(size_t)p * n + pq] -= L.cs * f;
          }
        }
      }
}

// In-place inverse of a Hermitian positive definite matrix, A = L L^H,
// A^-1 = L^-H L^-1.  False if a pivot is not clearly positive.
bool hpd_inverse(std::vector<cd>& A, int n) {
  std::vector<cd> L((size_t)n * n, cd(0.0, 0.0));
  double dmax = 0.0;
  for (int i = 0; i < n; ++i) dmax = std::max(dmax, std::abs(A[(size_t)i * n + i]));
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j].real();
    for (int k = 0; k < j; ++k) d -= std::norm(L[(size_t)j * n + k]);
    if (!(d > 1e-12 * dmax)) return false;
    const double djj = std::sqrt(d);
    L[(size_t)j * n + j] = djj;
    for (int i = j + 1; i < n; ++i) {
      cd t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * std::conj(L[(size_t)j * n + k]);
      L[(size_t)i * n + j] = t / djj;
    }
  }
  std::vector<cd> col(n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {  // L y = e_c
      cd t = (i == c) ? cd(1.0, 0.0) : cd(0.0, 0.0);
      for (int k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * col[k];
      col[i] = t / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {  // L^H x = y
      cd t = col[i];
      for (int k = i + 1; k < n; ++k) t -= std::conj(L[(size_t)k * n + i]) * col[k];
      col[i] = t / L[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) A[(size_t)i * n + c] = col[i];
  }
  return true;
}

}  // namespace

struct plhr_bloch_prec_s {
  std::vector<BlochLevel> lv;
  double theta[3] = {0.0, 0.0, 0.0};
  int nu = 1;
  double omega = 2.0 / 3.0;
  int max_cols = 0;
  int nc = 0;
  double* Ainv = nullptr;  // nc x nc complex, row-major
  std::vector<void*> allocs;
  hipStream_t stream = nullptr;

  // V-cycle on level lev for right-hand side r; returns the level's result
  // buffer, or the final output when `fin` is given (the last post-sweep,
  // or the coarsest solve of a one-level cycle, writes there).  At level 0
  // r may be strided (fin->r); the level buffers are contiguous.
  double* cycle(size_t lev, const double* r, int ncols, double* final_out,
                const BlochLd* fin = nullptr) {
    BlochLevel& L = lv[lev];
    BlochLd rin;  // r's stride at this level; everything else contiguous
    if (lev == 0 && fin) rin.r = fin->r;
    BlochLd rw = rin;  // w = r in the first fused pre-sweep
    rw.w = rin.r;
    BlochLd last = rin;  // the final write
    if (final_out && fin) {
      last.o = fin->o;
      last.out1 = fin->out1;
      last.o1 = fin->o1;
      last.split = fin->split;
    }
    if (lev + 1 == lv.size()) {
      double* out = final_out ? final_out : L.x;
      launch_bloch_dense(nc, Ainv, r, out, ncols, stream, final_out ? last : rin);
      return out;
    }
    const double bj = omega / L.diag;
    double* cur = L.x;
    double* oth = L.t;
    // pre-smoothing from w = 0; the first two sweeps in one pass over r:
    // w1 = bj r and w2 = w1 + bj (r - A w1) = (2 bj - bj^2) r + bj^2 (r - A r)
    int it0 = 1;
    if (nu >= 2) {
      launch_bloch_level(L.nx, L.ny, L.nz, L.cs, theta, r, r, 2.0 * bj - bj * bj, bj * bj, cur,
                         ncols, stream, rw);
      it0 = 2;
    } else {
      launch_bloch_level(L.nx, L.ny, L.nz, L.cs, theta, nullptr, r, 0.0, bj, cur, ncols, stream,
                         rin);
    }
    for (int it = it0; it < nu; ++it) {
      launch_bloch_level(L.nx, L.ny, L.nz, L.cs, theta, cur, r, 1.0, bj, oth, ncols, stream, rin);
      std::swap(cur, oth);
    }
    // residual, restriction, coarse correction
    launch_bloch_level(L.nx, L.ny, L.nz, L.cs, theta, cur, r, 0.0, 1.0, oth, ncols, stream, rin);
    BlochLevel& C = lv[lev + 1];
    launch_bloch_restrict(C.nx, C.ny, C.nz, theta, oth, C.r, ncols, stream);
    double* ec = cycle(lev + 1, C.r, ncols, nullptr);
    launch_bloch_prolong_add(L.nx, L.ny, L.nz, theta, ec, cur, ncols, stream);
    // post-smoothing
    for (int it = 0; it < nu; ++it) {
      const bool fl = final_out && it == nu - 1;
      double* dst = fl ? final_out : oth;
      launch_bloch_level(L.nx, L.ny, L.nz, L.cs, theta, cur, r, 1.0, bj, dst, ncols, stream,
                         fl ? last : rin);
      if (fl) return final_out;
      std::swap(cur, oth);
    }
    return cur;
  }

  ~plhr_bloch_prec_s() {
    for (void* p : allocs) (void)hipFree(p);
  }
};

namespace {

// Validation, hierarchy and buffers of a Bloch V-cycle.  With `size_only`
// it stops after the layout and stores the device bytes there (no device
// call); with a caller `workspace` (at least that many bytes, 256-byte
// aligned) the level buffers and the coarse inverse are carved from it and
// nothing is allocated on the device.
plhr_status bloch_prec_create_impl(const plhr_op_desc* A, const plhr_prec_desc* T,
                                   int32_t max_cols, void* stream, void* workspace,
                                   size_t ws_bytes, size_t* size_only, plhr_bloch_prec* out) {
  if (!A || !T || (!out && !size_only)) {
    set_error("plhr_bloch_prec_create: NULL argument");
    return PLHR_ERR_ARG;
  }
  if (out) *out = nullptr;
  if (A->kind != PLHR_OP_BLOCH7_3D || A->dtype != PLHR_C128) {
    set_error("plhr_bloch_prec_create: A must be PLHR_OP_BLOCH7_3D with PLHR_C128");
    return PLHR_ERR_UNSUPPORTED;
  }
  if (T->kind != PLHR_PREC_MG_VCYCLE) {
    set_error("plhr_bloch_prec_create: T must be PLHR_PREC_MG_VCYCLE");
    return PLHR_ERR_UNSUPPORTED;
  }
  if (A->nx < 1 || A->ny < 1 || A->nz < 1 || !(A->h > 0.0) || !(A->scale > 0.0) ||
      !std::isfinite(A->h) || !std::isfinite(A->scale) || !std::isfinite(A->theta[0]) ||
      !std::isfinite(A->theta[1]) || !std::isfinite(A->theta[2])) {
    set_error("plhr_bloch_prec_create: need nx, ny, nz >= 1, h and scale positive and finite, "
              "theta finite");
    return PLHR_ERR_ARG;
  }
  if (T->levels < 1 || T->nu_pre < 1 || T->nu_pre != T->nu_post || !(T->omega > 0.0) ||
      T->omega > 1.0) {
    set_error("plhr_bloch_prec_create: need levels >= 1, nu_pre == nu_post >= 1, "
              "0 < omega <= 1");
    return PLHR_ERR_ARG;
  }
  if (max_cols < 1 || max_cols > (1 << 22) || (int64_t)A->nx * max_cols >= (int64_t(1) << 31) ||
      (int64_t)A->ny * A->nz >= (int64_t(1) << 31)) {
    set_error("plhr_bloch_prec_create: need 1 <= max_cols <= 2^22, nx*max_cols and ny*nz below "
              "2^31");
    return PLHR_ERR_ARG;
  }
  if (T->levels > 16) {
    set_error("plhr_bloch_prec_create: at most 16 levels");
    return PLHR_ERR_ARG;
  }
  const int f = 1 << (T->levels - 1);
  if (A->nx % f || A->ny % f || A->nz % f) {
    set_error("plhr_bloch_prec_create: every grid dimension must be divisible by "
              "2^(levels - 1)");
    return PLHR_ERR_ARG;
  }
  const int64_t ncoarse = (int64_t)(A->nx / f) * (A->ny / f) * (A->nz / f);
  if (ncoarse > kBlochMaxCoarse) {
    set_error("plhr_bloch_prec_create: the coarsest grid exceeds 1024 points; add levels");
    return PLHR_ERR_UNSUPPORTED;
  }
  plhr_bloch_prec p = new plhr_bloch_prec_s();
  for (int d = 0; d < 3; ++d) p->theta[d] = A->theta[d];
  p->nu = T->nu_pre;
  p->omega = T->omega;
  p->max_cols = max_cols;
  p->stream = static_cast<hipStream_t>(stream);
  double h = A->h;
  int nx = A->nx, ny = A->ny, nz = A->nz;
  for (int lev = 0; lev < T->levels; ++lev) {
    BlochLevel L;
    L.nx = nx;
    L.ny = ny;
    L.nz = nz;
    L.cs = A->scale / (h * h);
    const int N[3] = {nx, ny, nz};
    double dg = 0.0;
    for (int d = 0; d < 3; ++d) dg += (N[d] == 1) ? 2.0 - 2.0 * std::cos(p->theta[d]) : 2.0;
    L.diag = L.cs * dg;
    p->lv.push_back(L);
    nx /= 2;
    ny /= 2;
    nz /= 2;
    h *= 2.0;
  }
  // device bytes: per level x, t (and r below the finest), the inverse
  p->nc = (int)p->lv.back().n();
  auto al256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
  size_t total = 0;
  for (size_t lev = 0; lev < p->lv.size(); ++lev)
    total += (lev == 0 ? 2 : 3) * al256(p->lv[lev].n() * (size_t)max_cols * 16);
  total += al256((size_t)p->nc * p->nc * sizeof(cd));
  if (size_only) {
    *size_only = total;
    delete p;
    return PLHR_OK;
  }
  if (workspace && (ws_bytes < total || ((uintptr_t)workspace & 255))) {
    delete p;
    set_error("plhr_bloch_prec_create: the workspace must hold "
              "plhr_bloch_prec_workspace_size bytes and be 256-byte aligned");
    return PLHR_ERR_ARG;
  }
  // the coarse inverse first (host only), then the device buffers
  std::vector<cd> M;
  bloch_dense(p->lv.back(), p->theta, M);
  if (!hpd_inverse(M, p->nc)) {
    delete p;
    set_error("plhr_bloch_prec_create: the coarsest Bloch operator is not positive definite "
              "(all phases 0 leaves the constant vector in its null space)");
    return PLHR_ERR_NOT_HPD;
  }
  char* wsp = static_cast<char*>(workspace);
  auto alloc = [&](size_t bytes) -> double* {
    if (wsp) {  // carve from the caller's workspace
      double* q = reinterpret_cast<double*>(wsp);
      wsp += al256(bytes);
      return q;
    }
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
      set_error(std::string("plhr_bloch_prec_create: hipMalloc: ") + hipGetErrorString(e));
      return nullptr;
    }
    p->allocs.push_back(q);
    return static_cast<double*>(q);
  };
  for (size_t lev = 0; lev < p->lv.size(); ++lev) {
    BlochLevel& L = p->lv[lev];
    const size_t bytes = L.n() * (size_t)max_cols * 16;
    L.x = alloc(bytes);
    L.t = L.x ? alloc(bytes) : nullptr;
    L.r = (lev == 0 || !L.t) ? nullptr : alloc(bytes);
    if (!L.x || !L.t || (lev > 0 && !L.r)) {
      delete p;
      return PLHR_ERR_HIP;
    }
  }
  p->Ainv = alloc(M.size() * sizeof(cd));
  if (!p->Ainv) {
    delete p;
    return PLHR_ERR_HIP;
  }
  const hipError_t e = hipMemcpy(p->Ainv, M.data(), M.size() * sizeof(cd), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    delete p;
    set_error(std::string("plhr_bloch_prec_create: hipMemcpy: ") + hipGetErrorString(e));
    return PLHR_ERR_HIP;
  }
  *out = p;
  return PLHR_OK;
}

}  // namespace

namespace plhr {

// One V-cycle of the handle on `s` (the solver context runs it on its own
// stream, or on the stream a graph is being recorded on).
void bloch_prec_cycle(plhr_bloch_prec p, const double* X, int ldx, double* Y0, int ld0,
                      double* Y1, int ld1, int split, int ncols, hipStream_t s) {
  p->stream = s;
  BlochLd fin;
  fin.r = ldx;
  fin.o = ld0;
  if (split < ncols) {
    fin.out1 = Y1;
    fin.o1 = ld1;
    fin.split = split;
  }
  p->cycle(0, X, ncols, Y0, &fin);
}

}  // namespace plhr

extern "C" {

plhr_status plhr_bloch_prec_workspace_size(const plhr_op_desc* A, const plhr_prec_desc* T,
                                           int32_t max_cols, size_t* ws_bytes) {
  if (!ws_bytes) {
    set_error("plhr_bloch_prec_workspace_size: ws_bytes is NULL");
    return PLHR_ERR_ARG;
  }
  return bloch_prec_create_impl(A, T, max_cols, nullptr, nullptr, 0, ws_bytes, nullptr);
}

plhr_status plhr_bloch_prec_create(const plhr_op_desc* A, const plhr_prec_desc* T,
                                   int32_t max_cols, void* stream, void* workspace,
                                   size_t ws_bytes, plhr_bloch_prec* out) {
  return bloch_prec_create_impl(A, T, max_cols, stream, workspace, ws_bytes, nullptr, out);
}

plhr_status plhr_bloch_prec_apply(plhr_bloch_prec p, const void* X, void* Y, int32_t ncols) {
  if (!p || (ncols > 0 && (!X || !Y))) {
    set_error("plhr_bloch_prec_apply: NULL argument");
    return PLHR_ERR_ARG;
  }
  if (ncols < 0 || ncols > p->max_cols) {
    set_error("plhr_bloch_prec_apply: need 0 <= ncols <= max_cols");
    return PLHR_ERR_ARG;
  }
  if (ncols == 0) return PLHR_OK;
  const size_t bytes = p->lv[0].n() * (size_t)ncols * 16;
  const char* xb = static_cast<const char*>(X);
  const char* yb = static_cast<const char*>(Y);
  if (xb < yb + bytes && yb < xb + bytes) {
    set_error("plhr_bloch_prec_apply: X and Y overlap");
    return PLHR_ERR_ARG;
  }
  p->cycle(0, static_cast<const double*>(X), ncols, static_cast<double*>(Y));
  PLHR_HIP_CHECK(hipGetLastError());
  return PLHR_OK;
}

void plhr_bloch_prec_destroy(plhr_bloch_prec p) { delete p; }

plhr_status plhr_gram_c128_workspace(int64_t n, int32_t mx, int32_t my, size_t* bytes) {
  if (!bytes || n < 0 || mx < 1 || my < 1 || mx > 1024 || my > 1024) {
    set_error("plhr_gram_c128_workspace: need bytes != NULL, n >= 0, 1 <= mx, my <= 1024");
    return PLHR_ERR_ARG;
  }
  *bytes = cgram_workspace_bytes((size_t)n, mx, my);
  return PLHR_OK;
}

plhr_status plhr_gram_c128(int64_t n, const void* X, int32_t mx, const void* Y, int32_t my,
                           void* G, void* workspace, size_t ws_bytes, void* stream) {
  size_t need = 0;
  const plhr_status st = plhr_gram_c128_workspace(n, mx, my, &need);
  if (st != PLHR_OK) return st;
  if (!G || !workspace || (n > 0 && (!X || !Y))) {
    set_error("plhr_gram_c128: NULL argument");
    return PLHR_ERR_ARG;
  }
  if (ws_bytes < need) {
    set_error("plhr_gram_c128: workspace smaller than plhr_gram_c128_workspace");
    return PLHR_ERR_ARG;
  }
  if (((uintptr_t)X | (uintptr_t)Y | (uintptr_t)G | (uintptr_t)workspace) & 15) {
    set_error("plhr_gram_c128: X, Y, G and the workspace must be 16-byte aligned");
    return PLHR_ERR_ARG;
  }
  launch_cgram((size_t)n, static_cast<const double*>(X), mx, static_cast<const double*>(Y), my,
               static_cast<double*>(G), static_cast<double*>(workspace),
               static_cast<hipStream_t>(stream));
  PLHR_HIP_CHECK(hipGetLastError());
  return PLHR_OK;
}

plhr_status plhr_rowmul_c128(int64_t n, const void* Z, int32_t m, const void* M, int32_t k,
                             void* Y, void* stream) {
  if (n < 0 || m < 1 || m > 64 || k < 1 || k > 64) {
    set_error("plhr_rowmul_c128: need n >= 0, 1 <= m, k <= 64");
    return PLHR_ERR_ARG;
  }
  if (n == 0) return PLHR_OK;
  if (!Z || !M || !Y) {
    set_error("plhr_rowmul_c128: NULL argument");
    return PLHR_ERR_ARG;
  }
  if (((uintptr_t)Z | (uintptr_t)M | (uintptr_t)Y) & 15) {
    set_error("plhr_rowmul_c128: Z, M and Y must be 16-byte aligned");
    return PLHR_ERR_ARG;
  }
  // every workgroup stages M while others already store Y: M must not
  // overlap Y either
  const size_t zb = (size_t)n * m * 16, yb = (size_t)n * k * 16, mb = (size_t)m * k * 16;
  const char* z = static_cast<const char*>(Z);
  const char* y = static_cast<const char*>(Y);
  const char* mm = static_cast<const char*>(M);
  if (z < y + yb && y < z + zb) {
    set_error("plhr_rowmul_c128: Z and Y overlap");
    return PLHR_ERR_ARG;
  }
  if (mm < y + yb && y < mm + mb) {
    set_error("plhr_rowmul_c128: M and Y overlap");
    return PLHR_ERR_ARG;
  }
  PLHR_HIP_CHECK(launch_crowmul((size_t)n, m, k, static_cast<const double*>(Z),
                                static_cast<const double*>(M), static_cast<double*>(Y),
                                static_cast<hipStream_t>(stream)));
  return PLHR_OK;
}

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

plhr_status plhr_cholqr_c128_workspace(int64_t n, int32_t m, size_t* bytes) {
  if (!bytes || n < 1 || m < 1 || m > 64 || n < m) {
    set_error("plhr_cholqr_c128_workspace: need bytes != NULL, 1 <= m <= 64, n >= m");
    return PLHR_ERR_ARG;
  }
  *bytes = al256(cgram_workspace_bytes((size_t)n, m, m)) + 2 * al256((size_t)m * m * 16) + 256;
  return PLHR_OK;
}

plhr_status plhr_cholqr_c128(int64_t n, const void* Z, int32_t m, void* Q, void* R,
                             void* workspace, size_t ws_bytes, void* stream) {
  size_t need = 0;
  const plhr_status st = plhr_cholqr_c128_workspace(n, m, &need);
  if (st != PLHR_OK) return st;
  if (!Z || !Q || !workspace) {
    set_error("plhr_cholqr_c128: NULL argument");
    return PLHR_ERR_ARG;
  }
  if (ws_bytes < need) {
    set_error("plhr_cholqr_c128: workspace smaller than plhr_cholqr_c128_workspace");
    return PLHR_ERR_ARG;
  }
  if (((uintptr_t)Z | (uintptr_t)Q | (uintptr_t)R | (uintptr_t)workspace) & 15) {
    set_error("plhr_cholqr_c128: Z, Q, R and the workspace must be 16-byte aligned");
    return PLHR_ERR_ARG;
  }
  const size_t bytes = (size_t)n * m * 16;
  const char* zb = static_cast<const char*>(Z);
  const char* qb = static_cast<const char*>(Q);
  if (zb < qb + bytes && qb < zb + bytes) {
    set_error("plhr_cholqr_c128: Z and Q overlap");
    return PLHR_ERR_ARG;
  }
  if (R) {  // R is written by the factor kernel while Z, Q and the workspace are in use
    const char* rb = static_cast<const char*>(R);
    const size_t rbytes = (size_t)m * m * 16;
    const char* wb = static_cast<const char*>(workspace);
    if ((rb < zb + bytes && zb < rb + rbytes) || (rb < qb + bytes && qb < rb + rbytes) ||
        (rb < wb + need && wb < rb + rbytes)) {
      set_error("plhr_cholqr_c128: R overlaps Z, Q or the workspace");
      return PLHR_ERR_ARG;
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(workspace);
  double* gws = reinterpret_cast<double*>(w);
  w += al256(cgram_workspace_bytes((size_t)n, m, m));
  double* G = reinterpret_cast<double*>(w);
  w += al256((size_t)m * m * 16);
  double* Rinv = reinterpret_cast<double*>(w);
  w += al256((size_t)m * m * 16);
  int* fail = reinterpret_cast<int*>(w);
  const double* Zd = static_cast<const double*>(Z);
  launch_cgram((size_t)n, Zd, m, Zd, m, G, gws, s);
  PLHR_HIP_CHECK(launch_cholqr_tail((size_t)n, m, Zd, G, static_cast<double*>(R), Rinv, fail,
                                    static_cast<double*>(Q), s));
  int hf = 0;
  PLHR_HIP_CHECK(hipMemcpyAsync(&hf, fail, sizeof(int), hipMemcpyDeviceToHost, s));
  PLHR_HIP_CHECK(hipStreamSynchronize(s));
  if (hf) {
    set_error("plhr_cholqr_c128: Z^H Z is not positive definite (dependent columns)");
    return PLHR_ERR_NOT_HPD;
  }
  return PLHR_OK;
}

}  // extern "C"
