// C ABI of libplhr and the host driver of the block PLHR iteration
// (Algorithm 3 of the paper for real symmetric A, B = I or a positive
// diagonal B, and an SPD T).
//
// A diagonal B = diag(b) is handled by running the iteration in the
// variables u = B^1/2 v, where the pencil becomes (S A S, I) with
// S = B^-1/2 and the preconditioner S^-1 T S^-1 = B^1/2 T B^1/2: every
// B-inner product of Algorithm 3 is then the Euclidean one of the u's,
// and the iterates are those of the original pencil mapped by B^1/2 (the
// Gram matrices, the projected problem and the Ritz values are identical).
// The stencil applies S A S directly, T gets the scaling on its input and
// output, residual norms are formed in the original variables, and the
// returned vectors are mapped back (v = S u).
//
// Device data layout (point-major, n rows):
//   Z, QZ, TQZ  n x m, m = 4 kint columns in slots V | W | S | P
//               Z = basis, QZ = (A - sigma B) Z, TQZ = T (A - sigma B) Z;
//               keeping the three blocks lets one iteration use two block
//               operator products and four block preconditioner
//               applications (Section 4, storage/cost paragraph).
//   R           n x 2 kint  preconditioner input staging
//   Vfin, QVfin n x k       returned Ritz vectors and their products
// All small matrices live in a separate region of the same workspace.
//
// One iteration, all on the caller's stream, no host round trip:
//   R = QV - V(Lam - sigma), column norms       (k_resid_prep)
//   relative residuals, soft locking, stop flag   (k_conv_check)
//   W = T R                                        (V-cycle)
//   QW = (A - sigma)W; [S | TQW] = T[QW - W(Lam - sigma) | QW]
//   QS = (A - sigma)S; TQS = T QS
//   G = Z^T Z, Cholesky with dropping, Z,QZ,TQZ <- (.)M   (B-orthonormalise)
//   [G_L | G_R] = TQZ^T [QZ | Z]                    (eq. 3.5)
//   T-harmonic eigensolve and real basis Y'         (Algorithm 3 steps 6-9)
//   V = Zhat Y', P = [What Shat Phat] Y'_{WSP}, same for QZ, TQZ
//   Rayleigh quotients, eq. (4.1) for pairs
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace plhr {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

static size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

static_assert(KC_COUNT == PLHR_KC_COUNT, "profile categories");
static constexpr int kRefreshT = 10;  // iterations between T(A - sigma B)V refreshes

static thread_local Prof* g_prof = nullptr;
void prof_attach(Prof* p) { g_prof = (p && p->cat != -2) ? p : nullptr; }

Grid make_grid(const plhr_op_desc* A) {
  Grid g;
  g.nx = A->nx;
  g.ny = A->ny;
  g.nz = A->nz;
  if (A->kind == PLHR_OP_CSR) {  // no grid: n = nx rows
    g.ny = g.nz = 1;
    return g;
  }
  g.dim = (A->kind == PLHR_OP_FD7_3D || A->kind == PLHR_OP_Q1_3D) ? 3 : 2;
  g.q1 = (A->kind == PLHR_OP_Q1_2D || A->kind == PLHR_OP_Q1_3D);
  g.h = A->h;
  g.scale = A->scale;
  return g;
}

// ||A||_1 and ||B||_1 (B = the consistent mass) of the finite-element
// pencil: largest absolute row sums of the stencils (A is symmetric).
void q1_norms(const Grid& g, const std::vector<double>& pot, double* nA, double* nB) {
  const Q1Weights w = q1_weights(g);
  double ba = 0.0, bb = 0.0;
  const int zl = (g.dim == 3) ? -1 : 0, zh = (g.dim == 3) ? 1 : 0;
  for (int l = 0; l < g.nz; ++l)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        const size_t p = (size_t)i + (size_t)g.nx * (j + (size_t)g.ny * l);
        double ra = 0.0, rb = 0.0;
        for (int dz = zl; dz <= zh; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              if (i + dx < 0 || i + dx >= g.nx || j + dy < 0 || j + dy >= g.ny || l + dz < 0 ||
                  l + dz >= g.nz)
                continue;
              const int o = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
              double a = w.a[o];
              if (o == 13 && !pot.empty()) a += pot[p];
              ra += fabs(a);
              rb += fabs(w.m[o]);
            }
        ba = std::max(ba, ra);
        bb = std::max(bb, rb);
      }
  *nA = ba;
  *nB = bb;
}

// Largest absolute row sum of a symmetric CSR matrix (its 1-norm), the
// potential added to the diagonal; the arrays are read from the device.
plhr_status csr_norm1(const plhr_op_desc* M, const std::vector<double>& pot, double* out) {
  const int n = M->nx;
  std::vector<int32_t> rp(n + 1);
  if (hipMemcpy(rp.data(), M->row_ptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return PLHR_ERR_HIP;
  const long long nnz = rp[n];
  if (rp[0] != 0 || nnz != M->nnz || nnz < 0) return PLHR_ERR_ARG;
  for (int i = 0; i < n; ++i)
    if (rp[i + 1] < rp[i]) return PLHR_ERR_ARG;
  std::vector<int32_t> ci(nnz > 0 ? nnz : 1);
  std::vector<double> v(nnz > 0 ? nnz : 1);
  if (nnz > 0 &&
      (hipMemcpy(ci.data(), M->col_idx, nnz * sizeof(int32_t), hipMemcpyDeviceToHost) !=
           hipSuccess ||
       hipMemcpy(v.data(), M->values, nnz * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess))
    return PLHR_ERR_HIP;
  double best = 0.0;
  for (int i = 0; i < n; ++i) {
    double r = 0.0, d = pot.empty() ? 0.0 : pot[i];
    for (long long q = rp[i]; q < rp[i + 1]; ++q) {
      if (ci[q] < 0 || ci[q] >= n || !std::isfinite(v[q])) return PLHR_ERR_ARG;
      if (ci[q] == i)
        d += v[q];
      else
        r += fabs(v[q]);
    }
    best = std::max(best, r + fabs(d));
  }
  *out = best;
  return PLHR_OK;
}

// ||A||_1 of the Bloch operator: per point |diagonal| plus the moduli of
// the off-diagonal entries.  A direction with one point folds both
// neighbours into the diagonal (-2 cs cos theta); with two points both
// neighbours are the same point, an entry of modulus 2 cs |cos(theta/2)|.
double bloch_norm1(const plhr_op_desc& A, const std::vector<double>& pot) {
  const double cs = A.scale / (A.h * A.h);
  const int N[3] = {A.nx, A.ny, A.nz};
  double dg = 6.0 * cs, off = 0.0;
  for (int d = 0; d < 3; ++d) {
    if (N[d] == 1)
      dg -= 2.0 * cs * std::cos(A.theta[d]);
    else if (N[d] == 2)
      off += 2.0 * cs * std::fabs(std::cos(0.5 * A.theta[d]));
    else
      off += 2.0 * cs;
  }
  const size_t n = (size_t)A.nx * A.ny * A.nz;
  double best = 0.0;
  for (size_t p = 0; p < n; ++p) best = std::max(best, std::fabs(dg + (pot.empty() ? 0.0 : pot[p])));
  return best + off;
}

double exact_norm1(const Grid& g, const std::vector<double>& pot) {
  // max over points of |diag + pot| + (#interior neighbours) * scale / h^2
  const double d = g.diag(), o = -g.off();
  double best = 0.0;
  for (int l = 0; l < g.nz; ++l)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        int nb = (i > 0) + (i < g.nx - 1) + (j > 0) + (j < g.ny - 1);
        if (g.dim == 3) nb += (l > 0) + (l < g.nz - 1);
        const size_t p = (size_t)i + (size_t)g.nx * (j + (size_t)g.ny * l);
        const double v = fabs(d + (pot.empty() ? 0.0 : pot[p])) + nb * o;
        if (v > best) best = v;
      }
  return best;
}


void prof_begin(int cat, double bytes, double flops, hipStream_t s) {
  Prof* p = g_prof;
  if (!p || (p->cat != -1 && p->cat != cat)) return;
  if (p->used + 2 > p->ev.size()) {
    p->skip_end = true;
    return;
  }
  p->skip_end = false;
  (void)hipEventRecord(p->ev[p->used], s);
  p->evcat[p->used / 2] = cat;
  p->bytes[cat] += bytes;
  p->flops[cat] += flops;
  p->launches[cat] += 1;
}

void prof_end(int cat, hipStream_t s) {
  Prof* p = g_prof;
  if (!p || (p->cat != -1 && p->cat != cat)) return;
  if (p->skip_end) return;
  (void)hipEventRecord(p->ev[p->used + 1], s);
  p->used += 2;
}


plhr_status prof_start(Prof& p, int category, int max_launches) {
  if (category < -1 || category >= KC_COUNT || max_launches < 1) {
    set_error("profile start: bad argument");
    return PLHR_ERR_ARG;
  }
  const size_t need = 2 * (size_t)max_launches;
  while (p.ev.size() < need) {
    hipEvent_t e;
    PLHR_HIP_CHECK(hipEventCreate(&e));
    p.ev.push_back(e);
  }
  p.evcat.assign(p.ev.size() / 2 + 1, 0);
  p.used = 0;
  for (int i = 0; i < KC_COUNT; ++i) p.bytes[i] = p.flops[i] = 0.0, p.launches[i] = 0;
  p.cat = category;
  return PLHR_OK;
}

plhr_status prof_stop(Prof& p, hipStream_t stream, plhr_profile* out) {
  PLHR_HIP_CHECK(hipStreamSynchronize(stream));
  std::memset(out, 0, sizeof(*out));
  for (size_t i = 0; i < p.used; i += 2) {
    float ms = 0.f;
    PLHR_HIP_CHECK(hipEventElapsedTime(&ms, p.ev[i], p.ev[i + 1]));
    out->total_ms[p.evcat[i / 2]] += ms;
  }
  long total = 0;
  for (int i = 0; i < KC_COUNT; ++i) {
    out->launches[i] = (int32_t)p.launches[i];
    out->bytes[i] = p.bytes[i];
    out->flops[i] = p.flops[i];
    total += p.launches[i];
  }
  out->truncated = (p.used / 2 < (size_t)total) ? 1 : 0;
  p.cat = -2;
  return PLHR_OK;
}

void prof_release(Prof& p) {
  for (hipEvent_t e : p.ev) (void)hipEventDestroy(e);
  p.ev.clear();
}

}  // namespace plhr

using namespace plhr;

struct plhr_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  Grid grid;
  const double* pot = nullptr;
  // diagonal B (caller's b, n doubles) and the workspace copies of b^1/2,
  // b^-1/2; Rs stages the scaled preconditioner input (n x 2 kint)
  const double* bdiag = nullptr;
  double *bsq = nullptr, *bisq = nullptr, *Rs = nullptr;
  // B = the consistent Q1 mass (a stencil): B Z carried with Z, QZ, TQZ
  // through the transform and the updates, fresh B V and B V_final
  bool bst = false;
  double *BZ = nullptr, *BVf = nullptr, *BVfin = nullptr;
  // general sparse operators (A, and B when it is CSR)
  bool csr = false;
  CsrMat Acsr{}, Bcsr{};
  int prec_kind = PLHR_PREC_IDENTITY;
  MG mg;
  const double* Tdense = nullptr;  // PLHR_PREC_DENSE: caller's n x n matrix
  double sigma = 0.0;
  int k = 0, kint = 0, m = 0;
  plhr_options opt{};
  double normA1 = 1.0, normB1 = 1.0;
  size_t n = 0;
  bool own_ws = false;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  double *Z = nullptr, *QZ = nullptr, *TQZ = nullptr, *R = nullptr;
  double *Vfin = nullptr, *QVfin = nullptr;
  double* QVf = nullptr;  // fresh (A - sigma B)V for residuals and RQs
  double *part = nullptr, *gpart = nullptr, *HM = nullptr;
  int gram_nblk = 1;
  SmallBufs sb{};
  SmallParams sp{};
  DevStatus* st = nullptr;
  DevStatus* gate = nullptr;  // the automatic second Cholesky-QR pass
  DevStatus* st_host = nullptr;
  bool started = false, finished = false;
  long host_iter = 0;  // iterations enqueued since plhr_start
  bool use_mfma = true;
  Prof prof;
  // use_graph: the captured iteration (index 1: with the refresh of the
  // carried products) and the stream it was recorded on
  hipStream_t cap = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  // the complex Bloch operator (Algorithm 2): each complex column is an
  // interleaved pair of real columns (re, im) of the basis blocks; its
  // product and its V-cycle take contiguous complex blocks, staged through
  // Xs and Ys (n x 2 kint real each).  k counts real columns (twice the
  // pairs returned).
  bool bloch = false;
  plhr_op_desc bop{};
  plhr_bloch_prec bprec = nullptr;
  double *Xs = nullptr, *Ys = nullptr;
};

namespace {
// Points the launch profiler at this context while an entry point runs.
struct ProfScope {
  explicit ProfScope(plhr_ctx_s* c) { g_prof = (c && c->prof.cat != -2) ? &c->prof : nullptr; }
  ~ProfScope() { g_prof = nullptr; }
};
}  // namespace

namespace {

struct Layout {
  size_t bytes = 0;
  size_t take(size_t b) {
    size_t off = bytes;
    bytes += al(b);
    return off;
  }
};

// 0 the plain V-cycle (or none), 1 AV-MG, 2 INV-MG
int mg_mode(const plhr_prec_desc* T) {
  if (!T) return 0;
  return T->kind == PLHR_PREC_AV_MG ? 1 : (T->kind == PLHR_PREC_INV_MG ? 2 : 0);
}

// T is one of the multigrid preconditioners (needs a hierarchy)
bool uses_mg(const plhr_prec_desc* T) {
  return T && (T->kind == PLHR_PREC_MG_VCYCLE || T->kind == PLHR_PREC_AV_MG ||
               T->kind == PLHR_PREC_INV_MG);
}

// block columns: k + k_extra, the two real columns of the complex vector
// of the single-vector iteration, PLMR's one real column, or the real
// column pairs of k + k_extra complex columns (the Bloch operator)
int block_cols(const plhr_op_desc* A, int32_t k, const plhr_options& o) {
  if (A->kind == PLHR_OP_BLOCH7_3D) return 2 * (k + o.k_extra);
  if (o.algorithm == PLHR_ALG_SINGLE) return 2;
  if (o.algorithm == PLHR_ALG_PLMR) return 1;
  return k + o.k_extra;
}

plhr_status check_options(const plhr_options* opt) {
  if (opt) {
    if (!(opt->tol > 0.0) || opt->max_iters < 0 || opt->check_every < 1 ||
        !(opt->drop_tol > 0.0) || opt->ortho_passes < 0 || opt->ortho_passes > 2 ||
        (opt->precision != PLHR_PREC_FP64 && opt->precision != PLHR_PREC_MIXED) ||
        (opt->extraction != PLHR_EXTRACT_T_HARMONIC &&
         opt->extraction != PLHR_EXTRACT_HARMONIC) ||
        (opt->use_graph != 0 && opt->use_graph != 1)) {
      set_error(
          "invalid options (tol > 0, max_iters >= 0, check_every >= 1, drop_tol > 0, "
          "ortho_passes 0..2, precision FP64 or MIXED, extraction T_HARMONIC or HARMONIC, "
          "use_graph 0 or 1)");
      return PLHR_ERR_ARG;
    }
  }
  return PLHR_OK;
}

// The complex Bloch operator runs the block iteration in complex
// arithmetic (Algorithm 2) with B = I and T the identity or its V-cycle.
plhr_status validate_bloch(const plhr_op_desc* A, const plhr_op_desc* B, const plhr_prec_desc* T,
                           double sigma, int32_t k, const plhr_options* opt) {
  if (A->dtype != PLHR_C128) {
    set_error("A: PLHR_OP_BLOCH7_3D needs PLHR_C128");
    return PLHR_ERR_UNSUPPORTED;
  }
  if (A->nx < 1 || A->ny < 1 || A->nz < 1 || !(A->h > 0.0) || !(A->scale > 0.0) ||
      !std::isfinite(A->h) || !std::isfinite(A->scale) || !std::isfinite(A->theta[0]) ||
      !std::isfinite(A->theta[1]) || !std::isfinite(A->theta[2])) {
    set_error("A: need nx, ny, nz >= 1, h and scale positive and finite, theta finite");
    return PLHR_ERR_ARG;
  }
  if (B && B->kind != PLHR_OP_IDENTITY) {
    set_error("B: the Bloch operator is solved with B = I");
    return PLHR_ERR_UNSUPPORTED;
  }
  if (!std::isfinite(sigma)) {
    set_error("sigma must be finite");
    return PLHR_ERR_ARG;
  }
  const int kextra = opt ? opt->k_extra : 1;
  if (k < 1 || kextra < 0) {
    set_error("k must be >= 1 and k_extra >= 0");
    return PLHR_ERR_ARG;
  }
  if (opt && opt->algorithm != PLHR_ALG_BLOCK) {
    set_error("the Bloch operator runs the block iteration (PLHR_ALG_BLOCK)");
    return PLHR_ERR_UNSUPPORTED;
  }
  const int kc = k + kextra;
  const size_t n = (size_t)A->nx * A->ny * A->nz;
  if ((size_t)4 * kc > n) {
    set_error("4*(k + k_extra) must not exceed n");
    return PLHR_ERR_ARG;
  }
  if (8 * kc > kMaxM) {
    set_error("8*(k + k_extra) > 84 (complex columns count twice) exceeds the on-chip "
              "projected-problem limit");
    return PLHR_ERR_UNSUPPORTED;
  }
  if ((int64_t)A->nx * 4 * kc >= (int64_t(1) << 31) ||
      (int64_t)A->ny * A->nz >= (int64_t(1) << 31)) {
    set_error("A: nx*4*(k + k_extra) and ny*nz must be below 2^31");
    return PLHR_ERR_ARG;
  }
  plhr_status st = check_options(opt);
  if (st != PLHR_OK) return st;
  if (opt && opt->precision != PLHR_PREC_FP64) {
    set_error("the Bloch operator runs in FP64 only");
    return PLHR_ERR_UNSUPPORTED;
  }
  if (T && T->kind != PLHR_PREC_IDENTITY) {
    if (T->kind != PLHR_PREC_MG_VCYCLE) {
      set_error("T: the Bloch operator takes the identity or PLHR_PREC_MG_VCYCLE");
      return PLHR_ERR_UNSUPPORTED;
    }
    size_t b = 0;
    st = plhr_bloch_prec_workspace_size(A, T, 2 * kc, &b);
    if (st != PLHR_OK) return st;
  }
  return PLHR_OK;
}

plhr_status validate(const plhr_op_desc* A, const plhr_op_desc* B, const plhr_prec_desc* T,
                     double sigma, int32_t k, const plhr_options* opt) {
  if (!A) {
    set_error("A descriptor is NULL");
    return PLHR_ERR_ARG;
  }
  if (A->kind == PLHR_OP_BLOCH7_3D) return validate_bloch(A, B, T, sigma, k, opt);
  if (A->kind != PLHR_OP_FD5_2D && A->kind != PLHR_OP_FD7_3D && A->kind != PLHR_OP_Q1_2D &&
      A->kind != PLHR_OP_Q1_3D && A->kind != PLHR_OP_CSR) {
    set_error("A: only PLHR_OP_FD5_2D, PLHR_OP_FD7_3D, PLHR_OP_Q1_2D, PLHR_OP_Q1_3D, "
              "PLHR_OP_CSR and PLHR_OP_BLOCH7_3D are supported");
    return PLHR_ERR_UNSUPPORTED;
  }
  const bool acsr = (A->kind == PLHR_OP_CSR);
  if (acsr && (!A->row_ptr || !A->col_idx || !A->values || A->nnz < 0 || A->nx < 1 ||
               A->ny != 1 || A->nz != 1)) {
    set_error("A: PLHR_OP_CSR needs row_ptr, col_idx, values, nnz >= 0 and n = nx (ny = nz = 1)");
    return PLHR_ERR_ARG;
  }
  if (A->dtype != PLHR_F64) {
    set_error("A: only PLHR_F64 is supported");
    return PLHR_ERR_UNSUPPORTED;
  }
  const bool a2d = (A->kind == PLHR_OP_FD5_2D || A->kind == PLHR_OP_Q1_2D);
  if (A->nx < 1 || A->ny < 1 || A->nz < 1 || (a2d && A->nz != 1)) {
    set_error("A: grid dimensions must be >= 1 (nz = 1 in 2-D)");
    return PLHR_ERR_ARG;
  }
  if (!acsr && (!(A->h > 0.0) || !std::isfinite(A->h) || !(A->scale > 0.0) ||
                !std::isfinite(A->scale))) {
    set_error("A: h and scale must be positive and finite");
    return PLHR_ERR_ARG;
  }
  if (B && B->kind != PLHR_OP_IDENTITY) {
    if (B->kind != PLHR_OP_DIAG && B->kind != PLHR_OP_Q1_MASS && B->kind != PLHR_OP_CSR) {
      set_error("B: only the identity, PLHR_OP_DIAG, PLHR_OP_Q1_MASS and PLHR_OP_CSR are supported");
      return PLHR_ERR_UNSUPPORTED;
    }
    if (B->kind == PLHR_OP_CSR &&
        (!acsr || !B->row_ptr || !B->col_idx || !B->values || B->nnz < 0 || B->nx != A->nx)) {
      set_error("B: PLHR_OP_CSR needs a CSR A of the same n and its row_ptr, col_idx, values");
      return PLHR_ERR_ARG;
    }
    if (acsr && B->kind != PLHR_OP_CSR) {
      set_error("B: with a CSR A, B must be the identity or CSR");
      return PLHR_ERR_UNSUPPORTED;
    }
    const bool aq1 = (A->kind == PLHR_OP_Q1_2D || A->kind == PLHR_OP_Q1_3D);
    if (B->kind == PLHR_OP_Q1_MASS && !aq1) {
      set_error("B: PLHR_OP_Q1_MASS needs a finite-element A (PLHR_OP_Q1_2D/3D)");
      return PLHR_ERR_ARG;
    }
    if (B->kind == PLHR_OP_DIAG && aq1) {
      set_error("B: PLHR_OP_DIAG is supported with a finite-difference A only");
      return PLHR_ERR_UNSUPPORTED;
    }
    if (B->dtype != PLHR_F64) {
      set_error("B: only PLHR_F64 is supported");
      return PLHR_ERR_UNSUPPORTED;
    }
    if (B->kind == PLHR_OP_DIAG && !B->potential) {
      set_error("B: PLHR_OP_DIAG carries its diagonal in `potential`, which is NULL");
      return PLHR_ERR_ARG;
    }
    if (B->kind == PLHR_OP_DIAG && (B->nx != A->nx || B->ny != A->ny || B->nz != A->nz)) {
      set_error("B: the grid dimensions must be those of A");
      return PLHR_ERR_ARG;
    }
  }
  if (!std::isfinite(sigma)) {
    set_error("sigma must be finite");
    return PLHR_ERR_ARG;
  }
  const int kextra = opt ? opt->k_extra : 1;
  if (k < 1 || kextra < 0) {
    set_error("k must be >= 1 and k_extra >= 0");
    return PLHR_ERR_ARG;
  }
  const bool single = opt && opt->algorithm == PLHR_ALG_SINGLE;
  const bool plmr = opt && opt->algorithm == PLHR_ALG_PLMR;
  if (opt && opt->algorithm != PLHR_ALG_BLOCK && !single && !plmr) {
    set_error("invalid options (algorithm PLHR_ALG_BLOCK, PLHR_ALG_SINGLE or PLHR_ALG_PLMR)");
    return PLHR_ERR_ARG;
  }
  if ((single || plmr) && k != 1) {
    set_error("PLHR_ALG_SINGLE and PLHR_ALG_PLMR compute one pair: k must be 1");
    return PLHR_ERR_ARG;
  }
  const size_t n = (size_t)A->nx * A->ny * A->nz;
  const int kint = single ? 2 : (plmr ? 1 : k + kextra);
  if ((size_t)4 * kint > n) {
    set_error("4*(k + k_extra) must not exceed n");
    return PLHR_ERR_ARG;
  }
  if (4 * kint > kMaxM) {
    set_error("4*(k + k_extra) > 84 exceeds the on-chip projected-problem limit");
    return PLHR_ERR_UNSUPPORTED;
  }
  {
    const plhr_status so = check_options(opt);
    if (so != PLHR_OK) return so;
  }
  if (T && T->kind == PLHR_PREC_DENSE) {
    if (!T->matrix || ((uintptr_t)T->matrix & 7)) {
      set_error("T: PLHR_PREC_DENSE needs `matrix`, an 8-byte aligned n x n device array");
      return PLHR_ERR_ARG;
    }
    if (n > ((size_t)1 << 31)) {
      set_error("T: PLHR_PREC_DENSE needs n <= 2^31");
      return PLHR_ERR_ARG;
    }
  } else if (T && T->kind != PLHR_PREC_IDENTITY) {
    if (T->kind != PLHR_PREC_MG_VCYCLE && T->kind != PLHR_PREC_AV_MG &&
        T->kind != PLHR_PREC_INV_MG) {
      set_error("T: unknown preconditioner kind");
      return PLHR_ERR_ARG;
    }
    if (acsr) {
      set_error("T: the multigrid V-cycle needs a grid operator; use the identity with CSR");
      return PLHR_ERR_UNSUPPORTED;
    }
    if (T->levels < 1 || T->nu_pre < 1 || T->nu_pre != T->nu_post || !(T->omega > 0.0) ||
        T->omega > 1.0) {
      set_error("T: need levels >= 1, nu_pre == nu_post >= 1, 0 < omega <= 1");
      return PLHR_ERR_ARG;
    }
    if (T->kind == PLHR_PREC_AV_MG &&
        (!(T->delta > 0.0) || !std::isfinite(T->delta) || T->degree < 1 || T->degree > 64)) {
      set_error("T: AV-MG needs delta > 0 and 1 <= degree <= 64");
      return PLHR_ERR_ARG;
    }
    Grid g = make_grid(A);
    for (int lv = 0; lv + 1 < T->levels; ++lv) {
      int vtx = 0;
      if (!mg_coarsen(g, &vtx)) {
        set_error("T: level " + std::to_string(lv) +
                  " cannot be coarsened (its dimensions must be all even, or all odd and >= 3)");
        return PLHR_ERR_ARG;
      }
    }
    if (g.n() > 1024) {
      set_error("T: coarsest level has more than 1024 points; add levels");
      return PLHR_ERR_ARG;
    }
  }
  return PLHR_OK;
}


// bloch: the staging blocks Xs, Ys and `bprec_bytes` for the Bloch V-cycle
// (carved last, 256-byte aligned)
Layout layout(const Grid& g, int k, int kint, bool mgpre, int levels, bool bdiag, bool bst,
              plhr_ctx_s* c, int mgmode = 0, bool bloch = false, size_t bprec_bytes = 0) {
  Layout L;
  const size_t n = g.n();
  const int m = 4 * kint;
  const int gnb = gram_blocks(n);
  size_t oZ = L.take(n * m * 8), oQZ = L.take(n * m * 8), oTQZ = L.take(n * m * 8);
  size_t oR = L.take(n * 2 * kint * 8);
  size_t oVf = L.take(n * k * 8), oQVf = L.take(n * k * 8);
  size_t oQVr = L.take(n * kint * 8);
  size_t opart = L.take((size_t)512 * 2 * kint * 8);
  size_t ogp = L.take((size_t)gnb * m * 2 * m * 8);
  size_t oHM = L.take((size_t)kint * 2 * kint * 8);
  size_t oG = L.take((size_t)m * m * 8), oM = L.take((size_t)m * m * 8);
  size_t oGLR = L.take((size_t)m * 2 * m * 8), oY = L.take((size_t)m * kint * 8);
  size_t olam = L.take(kint * 8), orel = L.take(kint * 8), oxi = L.take(2 * m * 8);
  size_t okeep = L.take(m * 4), oact = L.take(kint * 4), okind = L.take(kint * 4),
         opair = L.take(kint * 4);
  size_t ofc = L.take((size_t)kint * kint * 8), oft = L.take(kint * 8), ovbv = L.take(kint * 8);
  size_t owork = L.take((size_t)4 * m * m * 8);
  size_t ost = L.take(sizeof(DevStatus));
  size_t ogate = L.take(sizeof(DevStatus));
  size_t obsq = 0, obisq = 0, oRs = 0;
  if (bdiag) {
    obsq = L.take(n * 8);
    obisq = L.take(n * 8);
    oRs = L.take(n * 2 * kint * 8);
  }
  size_t oBZ = 0, oBVf = 0, oBVfin = 0;
  if (bst) {
    oBZ = L.take(n * m * 8);
    oBVf = L.take(n * kint * 8);
    oBVfin = L.take(n * k * 8);
  }
  size_t oXs = 0, oYs = 0;
  if (bloch) {
    oXs = L.take(n * 2 * kint * 8);
    oYs = L.take(n * 2 * kint * 8);
  }
  size_t omg = L.bytes;
  if (mgpre) L.bytes += mg_workspace_bytes(g, levels, 2 * kint, mgmode);
  if (bloch) L.bytes += al(bprec_bytes);
  if (c) {
    char* b = c->ws;
    c->Z = (double*)(b + oZ);
    c->QZ = (double*)(b + oQZ);
    c->TQZ = (double*)(b + oTQZ);
    c->R = (double*)(b + oR);
    c->Vfin = (double*)(b + oVf);
    c->QVfin = (double*)(b + oQVf);
    c->QVf = (double*)(b + oQVr);
    c->part = (double*)(b + opart);
    c->gpart = (double*)(b + ogp);
    c->gram_nblk = gnb;
    c->HM = (double*)(b + oHM);
    c->sb.G = (double*)(b + oG);
    c->sb.M = (double*)(b + oM);
    c->sb.GLR = (double*)(b + oGLR);
    c->sb.Y = (double*)(b + oY);
    c->sb.lam = (double*)(b + olam);
    c->sb.relres = (double*)(b + orel);
    c->sb.xi = (double*)(b + oxi);
    c->sb.keep = (int*)(b + okeep);
    c->sb.active = (int*)(b + oact);
    c->sb.kinds = (int*)(b + okind);
    c->sb.pair = (int*)(b + opair);
    c->sb.final_C = (double*)(b + ofc);
    c->sb.final_theta = (double*)(b + oft);
    c->sb.vbv = (double*)(b + ovbv);
    c->sb.work = (double*)(b + owork);
    c->sb.scratch = nullptr;
    c->st = (DevStatus*)(b + ost);
    c->gate = (DevStatus*)(b + ogate);
    if (bdiag) {
      c->bsq = (double*)(b + obsq);
      c->bisq = (double*)(b + obisq);
      c->Rs = (double*)(b + oRs);
    }
    if (bst) {
      c->BZ = (double*)(b + oBZ);
      c->BVf = (double*)(b + oBVf);
      c->BVfin = (double*)(b + oBVfin);
    }
    if (bloch) {
      c->Xs = (double*)(b + oXs);
      c->Ys = (double*)(b + oYs);
    }
    (void)omg;
  }
  return L;
}



// (A - shift B)X and its fused outputs; outb (B X) exists only when B is
// a stencil (the finite-element mass).
// The Bloch product on interleaved real column pairs: read from and
// written to the strided slots directly (a slot of 2 k_int real columns is
// k_int complex columns at a 16-byte aligned offset, row stride ld / 2
// complex entries), then the shifted residual form as launch_resid_prep
// writes it and the copy output.
void bloch_stencil(plhr_ctx_s* c, const double* X, int ldx, Blk out, Blk outr,
                   const double* colshift, Blk outc, int ncols, double shift,
                   const DevStatus* st) {
  const size_t n = c->n;
  hipStream_t s = c->stream;
  const plhr_op_desc& A = c->bop;
  launch_bloch_apply(A.nx, A.ny, A.nz, A.h, A.scale, A.theta, c->pot, shift, X, out.ptr,
                     ncols / 2, s, ldx / 2, out.ld / 2, st);
  if (outr.ptr)
    launch_resid_prep(n, X, ldx, out.ptr, out.ld, colshift, c->sigma, outr.ptr, outr.ld, ncols,
                      nullptr, nullptr, 0, c->part, st, s);
  if (outc.ptr) launch_copy(n, out.ptr, out.ld, outc.ptr, outc.ld, ncols, s, st);
}

void stencil(plhr_ctx_s* c, const double* X, int ldx, Blk out, Blk outr, const double* colshift,
             Blk outc, int ncols, double shift, const DevStatus* st, Blk outb = Blk{nullptr, 0}) {
  if (c->bloch)
    bloch_stencil(c, X, ldx, out, outr, colshift, outc, ncols, shift, st);
  else if (c->csr)
    launch_csr_apply((int)c->n, c->Acsr, c->Bcsr, c->pot, shift, X, ldx, out, outr, colshift,
                     c->sigma, outc, outb, ncols, st, c->stream);
  else if (c->grid.q1)
    launch_q1_apply(c->grid, c->pot, shift, c->bst, X, ldx, out, outr, colshift, c->sigma, outc,
                    outb, ncols, st, c->stream);
  else
    launch_fd_apply(c->grid, c->pot, c->bisq, shift, X, ldx, out, outr, colshift, c->sigma, outc,
                    ncols, st, c->stream);
}

// T applied to ncols columns of R (ld ldr); output split at `split`.
// `direction`: the result only spans search directions (W, S), so the
// mixed mode may compute it with the FP32 V-cycle; products that enter the
// T-harmonic Grams (T(A - sigma B)Z) always use the FP64 V-cycle.
void precond_raw(plhr_ctx_s* c, const double* Rin, int ldr, Blk o0, Blk o1, int split,
                 int ncols, const DevStatus* st, bool direction) {
  if (c->bprec && st != c->gate) {
    // the Bloch V-cycle reads the strided slot and writes the (split)
    // outputs directly (its kernels do not read the status: after
    // convergence they rewrite W, S and T(A - sigma)Z slots that are no
    // longer used)
    bloch_prec_cycle(c->bprec, Rin, ldr / 2, o0.ptr, o0.ld / 2, o1.ptr, o1.ld / 2, split / 2,
                     ncols / 2, c->stream);
  } else if (c->bprec) {
    // gated (the recomputation after a second Cholesky-QR pass): through
    // the staging blocks, whose copies honour the gate
    launch_copy(c->n, Rin, ldr, c->Xs, ncols, ncols, c->stream, st);
    bloch_prec_cycle(c->bprec, c->Xs, ncols / 2, c->Ys, ncols / 2, nullptr, 0, ncols / 2,
                     ncols / 2, c->stream);
    if (split > 0) launch_copy(c->n, c->Ys, ncols, o0.ptr, o0.ld, split, c->stream, st);
    if (split < ncols)
      launch_copy(c->n, c->Ys + split, ncols, o1.ptr, o1.ld, ncols - split, c->stream, st);
  } else if (c->prec_kind == PLHR_PREC_MG_VCYCLE) {
    const bool f32 = direction && c->opt.precision == PLHR_PREC_MIXED;
    mg_apply(c->mg, Rin, ldr, o0, o1, split, ncols, f32, st, c->stream);
  } else if (c->prec_kind == PLHR_PREC_DENSE) {
    launch_dense_prec(c->n, c->Tdense, Rin, ldr, o0, o1, split, ncols, st, c->stream);
  } else {
    if (split > 0) launch_copy(c->n, Rin, ldr, o0.ptr, o0.ld, split, c->stream, st);
    if (split < ncols)
      launch_copy(c->n, Rin + split, ldr, o1.ptr, o1.ld, ncols - split, c->stream, st);
  }
}

// With a diagonal B the iteration's preconditioner is B^1/2 T B^1/2.
void precond(plhr_ctx_s* c, const double* Rin, int ldr, Blk o0, Blk o1, int split, int ncols,
             const DevStatus* st, bool direction = false) {
  if (!c->bdiag) {
    precond_raw(c, Rin, ldr, o0, o1, split, ncols, st, direction);
    return;
  }
  launch_rowscale(c->n, c->bsq, Rin, ldr, c->Rs, ncols, ncols, c->stream, st);
  precond_raw(c, c->Rs, ncols, o0, o1, split, ncols, st, direction);
  if (split > 0)
    launch_rowscale(c->n, c->bsq, o0.ptr, o0.ld, o0.ptr, o0.ld, split, c->stream, st);
  if (split < ncols)
    launch_rowscale(c->n, c->bsq, o1.ptr, o1.ld, o1.ptr, o1.ld, ncols - split, c->stream, st);
}

// Gram product on the matrix cores when the shape fits.
void gram(plhr_ctx_s* c, const double* X, int ldx, int mx, const double* Y1, int ldy1, int my1,
          const double* Y2, int ldy2, int my, double* out, const DevStatus* st) {
  auto a16 = [](const void* q) { return q == nullptr || ((uintptr_t)q & 15) == 0; };
  const bool layout_ok = ((ldx | ldy1 | ldy2 | my1) & 1) == 0 && a16(X) && a16(Y1) && a16(Y2);
  if (c->use_mfma && layout_ok && gram_mfma_ok(mx, my))
    launch_gram_mfma(c->n, X, ldx, mx, Y1, ldy1, my1, Y2, ldy2, my, c->gpart, c->gram_nblk, out,
                     st, c->stream);
  else
    launch_gram(c->n, X, ldx, mx, Y1, ldy1, my1, Y2, ldy2, my, c->gpart, c->gram_nblk, out, st,
                c->stream);
}

void transform(plhr_ctx_s* c, double* const* arrs, int narr, const DevStatus* st) {
  const int m = c->m;
  if (c->use_mfma && rowmul_mfma_ok(m, m)) {
    // four 16-row tiles per block and pass; two blocks per compute unit
    const size_t ntiles = (c->n + 63) / 64;
    const int nb = (int)(ntiles < 512 ? ntiles : 512);
    launch_rowmul_mfma(c->n, arrs, narr, m, m, c->sb.M, m, 0, 0, 0, 0, nullptr, nb, st, c->stream);
  } else {
    launch_transform(c->n, arrs, narr, m, m, c->sb.M, st, c->stream);
  }
}

int update(plhr_ctx_s* c, double* const* arrs, int narr, const DevStatus* st) {
  const int m = c->m, kint = c->kint;
  if (c->use_mfma && rowmul_mfma_ok(m, 2 * kint)) {
    const int nb = update_blocks(c->n);
    launch_rowmul_mfma(c->n, arrs, narr, m, m, c->sb.Y, 2 * kint, 1, kint, kint, 3 * kint, c->part,
                       nb, st, c->stream);
    return nb;
  }
  return launch_update(c->n, arrs, narr, m, m, kint, c->sb.Y, kint, 3 * kint, c->part, st,
                       c->stream);
}

// B-orthonormalise Z = [V W S P] and the arrays carried with it (Cholesky-QR
// in slot order).  The first pass also decides (on the device, in the gate)
// whether the basis met a small pivot: then the B-orthogonality needs a
// second pass (ortho_passes 0: automatic; 2: always) and the carried
// products of the V and P slots, which the transform mixes with weights up
// to pivot^-1/2, are recomputed from the new basis (T(A - sigma B)Z too
// when `recompute_tq`).
void orthonormalise(plhr_ctx_s* c, double* const* arrs, int narr, bool recompute_tq) {
  const int kint = c->kint, m = c->m;
  hipStream_t s = c->stream;
  DevStatus* st = c->st;
  double *Z = c->Z, *QZ = c->QZ, *TQZ = c->TQZ, *BZ = c->BZ;
  const bool bst = c->bst;
  const Blk none{nullptr, 0};
  SmallParams p1 = c->sp, p2 = c->sp;
  SmallBufs b1 = c->sb;
  b1.gate = c->gate;
  p1.pass = 1;
  p2.pass = 2;
  // the complex iterations orthonormalise in the complex inner product of
  // their interleaved columns
  auto ortho = c->sp.cplx ? launch_cplx_ortho : launch_ortho_small;
  gram(c, Z, m, m, bst ? BZ : Z, m, m, nullptr, 0, m, c->sb.G, st);
  ortho(p1, b1, st, s);
  transform(c, arrs, narr, st);
  if (c->opt.ortho_passes == 0) {
    gram(c, Z, m, m, bst ? BZ : Z, m, m, nullptr, 0, m, c->sb.G, c->gate);
    ortho(p2, b1, st, s);
    transform(c, arrs, narr, c->gate);
  } else if (c->opt.ortho_passes == 2) {
    gram(c, Z, m, m, bst ? BZ : Z, m, m, nullptr, 0, m, c->sb.G, st);
    ortho(c->sp, c->sb, st, s);
    transform(c, arrs, narr, st);
  }
  // gated recomputation of (A - sigma B)Z and T(A - sigma B)Z for V and P
  for (int slot : {0, 3}) {
    stencil(c, Z + slot * kint, m, Blk{QZ + slot * kint, m}, none, nullptr, none, kint, c->sigma,
            c->gate, bst ? Blk{BZ + slot * kint, m} : none);
    if (recompute_tq)
      precond(c, QZ + slot * kint, m, Blk{TQZ + slot * kint, m}, none, kint, kint, c->gate);
  }
}

void enqueue_plmr_body(plhr_ctx_s* c, bool refresh);

// One pass through the loop of Algorithm 3; `refresh` recomputes the
// carried (A - sigma B)V and T(A - sigma B)V slots from V.  With the
// harmonic extraction the products with T that only enter the projection
// (T(A - sigma B)Z) are not formed.
void enqueue_iteration_body(plhr_ctx_s* c, bool refresh) {
  if (c->sp.plmr) {
    enqueue_plmr_body(c, refresh);
    return;
  }
  const int kint = c->kint, m = c->m;
  const size_t n = c->n;
  hipStream_t s = c->stream;
  DevStatus* st = c->st;
  double *Z = c->Z, *QZ = c->QZ, *TQZ = c->TQZ, *R = c->R;
  const Blk none{nullptr, 0};
  // T = I (with B = I or a stencil B): T(A - sigma B)Z is (A - sigma B)Z
  // itself, so the T-harmonic extraction is the harmonic one and no
  // T-products are formed; W = R and S = (A - lam B)W are written straight
  // into their slots.
  const bool tid = (c->prec_kind == PLHR_PREC_IDENTITY && !c->bdiag);
  const bool tharm = (c->opt.extraction == PLHR_EXTRACT_T_HARMONIC) && !tid;
  // (A - sigma B)V afresh from V, and the Rayleigh quotients from it: the
  // copy carried by the block updates drifts from the true product by
  // rounding (about 1e-11 relative after a thousand iterations), which
  // would let the convergence test and the soft locking act on residuals
  // that are not the true ones.  T(A - sigma B)V is refreshed every
  // kRefreshT iterations for the same reason.
  // The fresh product goes to its own buffer: the V slots of QZ and TQZ
  // must stay consistent with each other (the orthonormalising transform
  // divides by small pivots and would amplify any mismatch into P), so
  // they are refreshed together, every kRefreshT iterations.
  double* BZ = c->BZ;  // null unless B is a stencil
  const bool bst = c->bst;
  if (refresh) {
    stencil(c, Z, m, Blk{QZ, m}, none, nullptr, none, kint, c->sigma, st,
            bst ? Blk{BZ, m} : none);
    if (tharm) precond(c, QZ, m, Blk{TQZ, m}, none, kint, kint, st);
  }
  stencil(c, Z, m, Blk{c->QVf, kint}, none, nullptr, none, kint, c->sigma, st,
          bst ? Blk{c->BVf, kint} : none);
  int nb = 0;
  if (!bst && !c->bdiag && vstep_small_ok(n, kint)) {
    // small problem: quotients, residuals and the test in one workgroup
    launch_vstep_small(c->sp, n, Z, m, c->QVf, kint, tid ? Z + kint : R, tid ? m : kint,
                       c->part, c->sb, st, s);
  } else {
    nb = launch_xdots(n, Z, m, c->QVf, kint, kint, c->part, s, bst ? c->BVf : nullptr, kint);
    launch_rq_small(c->sp, c->part, nb, c->sb, st, 0, s);
    // residuals of the current block, convergence and locking
    nb = launch_resid_prep(n, Z, m, c->QVf, kint, c->sb.lam, c->sigma, tid ? Z + kint : R,
                           tid ? m : kint, kint, c->bdiag, bst ? c->BVf : nullptr, kint, c->part,
                           st, s);
    launch_conv_check(c->sp, c->part, nb, c->sb, st, c->opt.max_iters, s);
  }
  // W = T (A V - B V Lam)
  if (!tid) precond(c, R, kint, Blk{Z + kint, m}, none, kint, kint, st, true);
  // QW = (A - sigma) W;  R = [QW - W (Lam - sigma) | QW]
  stencil(c, Z + kint, m, Blk{QZ + kint, m}, tid ? Blk{Z + 2 * kint, m} : Blk{R, 2 * kint},
          c->sb.lam, tharm ? Blk{R + kint, 2 * kint} : none, kint, c->sigma, st,
          bst ? Blk{BZ + kint, m} : none);
  // S = T (A W - B W Lam), TQW = T (A - sigma) W
  if (tid) {
  } else if (!tharm) {
    precond(c, R, 2 * kint, Blk{Z + 2 * kint, m}, none, kint, kint, st, true);
  } else if (c->opt.precision == PLHR_PREC_MIXED) {
    precond(c, R, 2 * kint, Blk{Z + 2 * kint, m}, none, kint, kint, st, true);
    precond(c, R + kint, 2 * kint, Blk{TQZ + kint, m}, none, kint, kint, st);
  } else {
    precond(c, R, 2 * kint, Blk{Z + 2 * kint, m}, Blk{TQZ + kint, m}, kint, 2 * kint, st);
  }
  // QS = (A - sigma) S ; TQS = T QS
  stencil(c, Z + 2 * kint, m, Blk{QZ + 2 * kint, m}, none, nullptr, none, kint, c->sigma, st,
          bst ? Blk{BZ + 2 * kint, m} : none);
  if (tharm) precond(c, QZ + 2 * kint, m, Blk{TQZ + 2 * kint, m}, none, kint, kint, st);
  // B-orthonormalise Z = [V W S P] (Cholesky-QR in slot order)
  double* arrs[4];
  int narr = 0;
  arrs[narr++] = Z;
  arrs[narr++] = QZ;
  if (tharm) arrs[narr++] = TQZ;
  if (bst) arrs[narr++] = BZ;
  orthonormalise(c, arrs, narr, tharm);
  // [G_L | G_R] = (T Q Zhat)^T [Q Zhat | B Zhat]  (Q Zhat for the harmonic
  // extraction)
  gram(c, tharm ? TQZ : QZ, m, m, QZ, m, m, bst ? BZ : Z, m, 2 * m, c->sb.GLR, st);
  if (c->sp.cplx)
    launch_cplx_tharm(c->sp, c->sb, st, s);
  else if (c->sp.sym)
    launch_tharm_sym(c->sp, c->sb, st, s);
  else
    launch_tharm_small(c->sp, c->sb, st, s);
  // V <- Zhat Y', P <- [W S P]hat Y'_WSP  (and the same for QZ, TQZ)
  nb = update(c, arrs, narr, st);
  launch_rq_small(c->sp, c->part, nb, c->sb, st, 1, s);
}

// One iteration of PLMR (Section 3.3), one real column per slot: the
// trial subspace span{v, w, s, p} of Algorithm 1 and the refinement
// extraction at the current Rayleigh quotient lam.  The T slot carries
// T(A - lam B) of each basis column: of v it is w = T(A v - lam B v), of w
// it is s = T(A w - lam B w), and of s and p it is formed here, so an
// iteration applies T four times, as the T-harmonic one does.
void enqueue_plmr_body(plhr_ctx_s* c, bool refresh) {
  const int m = c->m;  // 4
  const size_t n = c->n;
  hipStream_t s = c->stream;
  DevStatus* st = c->st;
  double *Z = c->Z, *QZ = c->QZ, *TL = c->TQZ, *R = c->R, *BZ = c->BZ;
  const bool bst = c->bst;
  const Blk none{nullptr, 0};
  if (refresh)
    stencil(c, Z, m, Blk{QZ, m}, none, nullptr, none, 1, c->sigma, st, bst ? Blk{BZ, m} : none);
  stencil(c, Z, m, Blk{c->QVf, 1}, none, nullptr, none, 1, c->sigma, st,
          bst ? Blk{c->BVf, 1} : none);
  int nb = launch_xdots(n, Z, m, c->QVf, 1, 1, c->part, s, bst ? c->BVf : nullptr, 1);
  launch_rq_small(c->sp, c->part, nb, c->sb, st, 0, s);
  nb = launch_resid_prep(n, Z, m, c->QVf, 1, c->sb.lam, c->sigma, R, 1, 1, c->bdiag,
                         bst ? c->BVf : nullptr, 1, c->part, st, s);
  launch_conv_check(c->sp, c->part, nb, c->sb, st, c->opt.max_iters, s);
  // w = T(A v - lam B v)
  precond(c, R, 1, Blk{Z + 1, m}, none, 1, 1, st);
  // (A - sigma B) w, and R = (A - lam B) w; s = T R
  stencil(c, Z + 1, m, Blk{QZ + 1, m}, Blk{R, 1}, c->sb.lam, none, 1, c->sigma, st,
          bst ? Blk{BZ + 1, m} : none);
  precond(c, R, 1, Blk{Z + 2, m}, none, 1, 1, st);
  // (A - sigma B) s, and T(A - lam B) s
  stencil(c, Z + 2, m, Blk{QZ + 2, m}, Blk{R, 1}, c->sb.lam, none, 1, c->sigma, st,
          bst ? Blk{BZ + 2, m} : none);
  precond(c, R, 1, Blk{TL + 2, m}, none, 1, 1, st);
  // T(A - lam B) p from the carried (A - sigma B) p (zero before the first
  // update, when the P slot is empty)
  launch_resid_prep(n, Z + 3, m, QZ + 3, m, c->sb.lam, c->sigma, R, 1, 1, c->bdiag,
                    bst ? BZ + 3 : nullptr, m, c->part, st, s);
  precond(c, R, 1, Blk{TL + 3, m}, none, 1, 1, st);
  launch_copy(n, Z + 1, m, TL, m, 1, s, st);
  launch_copy(n, Z + 2, m, TL + 1, m, 1, s, st);
  double* arrs[4];
  int narr = 0;
  arrs[narr++] = Z;
  arrs[narr++] = QZ;
  arrs[narr++] = TL;
  if (bst) arrs[narr++] = BZ;
  orthonormalise(c, arrs, narr, false);
  // [G_1 | G_2] = (T(A - lam B)Zhat)^T [(A - sigma B)Zhat | B Zhat]
  gram(c, TL, m, m, QZ, m, m, bst ? BZ : Z, m, 2 * m, c->sb.GLR, st);
  launch_plmr_small(c->sp, c->sb, st, s);
  nb = update(c, arrs, narr, st);
  launch_rq_small(c->sp, c->part, nb, c->sb, st, 1, s);
}

void destroy_graphs(plhr_ctx_s* c) {
  for (int i = 0; i < 2; ++i) {
    if (c->gexec[i]) (void)hipGraphExecDestroy(c->gexec[i]);
    if (c->graph[i]) (void)hipGraphDestroy(c->graph[i]);
    c->gexec[i] = nullptr;
    c->graph[i] = nullptr;
  }
}

// Record one iteration (and one with the refresh) into HIP graphs, on a
// stream of the library's own (capture is not allowed on the null
// stream); they are replayed on the context's stream.  Every captured
// node is a kernel launch.
plhr_status capture_graphs(plhr_ctx_s* c) {
  destroy_graphs(c);
  if (!c->cap) PLHR_HIP_CHECK(hipStreamCreate(&c->cap));
  PLHR_HIP_CHECK(hipStreamSynchronize(c->stream));
  hipStream_t user = c->stream;
  c->stream = c->cap;
  hipError_t e = hipSuccess;
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) break;
    enqueue_iteration_body(c, i == 1);
    e = hipStreamEndCapture(c->cap, &c->graph[i]);
    if (e == hipSuccess) e = hipGraphInstantiate(&c->gexec[i], c->graph[i], nullptr, nullptr, 0);
  }
  c->stream = user;
  if (e != hipSuccess) {
    set_error(std::string("graph capture: ") + hipGetErrorString(e));
    destroy_graphs(c);
    return PLHR_ERR_HIP;
  }
  return PLHR_OK;
}

plhr_status enqueue_iteration(plhr_ctx_s* c) {
  const bool refresh = (c->host_iter % kRefreshT == kRefreshT - 1);
  if (c->opt.use_graph && c->prof.cat == -2) {
    if (!c->gexec[0]) {
      const plhr_status s = capture_graphs(c);
      if (s != PLHR_OK) return s;
    }
    PLHR_HIP_CHECK(hipGraphLaunch(c->gexec[refresh ? 1 : 0], c->stream));
  } else {
    enqueue_iteration_body(c, refresh);
  }
  ++c->host_iter;
  return PLHR_OK;
}

plhr_status read_status(plhr_ctx_s* c) {
  PLHR_HIP_CHECK(hipMemcpyAsync(c->st_host, c->st, sizeof(DevStatus), hipMemcpyDeviceToHost,
                                c->stream));
  PLHR_HIP_CHECK(hipStreamSynchronize(c->stream));
  return PLHR_OK;
}

plhr_status device_error(plhr_ctx_s* c) {
  const int e = c->st_host->error;
  if (e == 0) return PLHR_OK;
  set_error(std::string("device check failed: ") + reason_text(c->st_host->reason) +
            " (iteration " + std::to_string(c->st_host->iter) + ")");
  return (plhr_status)e;
}

}  // namespace

const char* plhr::reason_text(int r) {
  static const char* why[] = {"unspecified",
                              "the start block is rank deficient",
                              "the projected eigensolver did not converge",
                              "a wanted residual is not finite",
                              "V^T B V of the final Rayleigh-Ritz step is not positive definite",
                              "every column of V became linearly dependent"};
  return why[(r >= 0 && r <= 5) ? r : 0];
}

extern "C" {

const char* plhr_version(void) { return "plhr-mi355x 0.1 (gfx950, FP64)"; }

const char* plhr_last_error(void) { return g_last_error.c_str(); }

plhr_status plhr_options_default(plhr_options* opt) {
  if (!opt) {
    set_error("opt is NULL");
    return PLHR_ERR_ARG;
  }
  std::memset(opt, 0, sizeof(*opt));
  opt->tol = 1e-8;
  opt->max_iters = 10000;
  opt->k_extra = 1;
  opt->precision = PLHR_PREC_FP64;
  opt->lock = 1;
  opt->check_every = 1;
  opt->drop_tol = 1e-10;
  return PLHR_OK;
}

plhr_status plhr_workspace_size(const plhr_op_desc* A, const plhr_op_desc* B,
                                const plhr_prec_desc* T, double sigma, int32_t k,
                                const plhr_options* opt, size_t* ws_bytes) {
  plhr_options o;
  plhr_options_default(&o);
  if (opt) o = *opt;
  plhr_status s = validate(A, B, T, sigma, k, &o);
  if (s != PLHR_OK) return s;
  if (!ws_bytes) {
    set_error("ws_bytes is NULL");
    return PLHR_ERR_ARG;
  }
  const bool bloch = (A->kind == PLHR_OP_BLOCH7_3D);
  const bool mgp = !bloch && uses_mg(T);
  const bool bd = B && B->kind == PLHR_OP_DIAG;
  const bool bs = B && (B->kind == PLHR_OP_Q1_MASS || B->kind == PLHR_OP_CSR);
  const int kint = block_cols(A, k, o);
  size_t bpb = 0;
  if (bloch && T && T->kind == PLHR_PREC_MG_VCYCLE) {
    s = plhr_bloch_prec_workspace_size(A, T, kint, &bpb);
    if (s != PLHR_OK) return s;
  }
  Layout L = layout(make_grid(A), bloch ? 2 * k : k, kint, mgp, mgp ? T->levels : 0, bd, bs,
                    nullptr, mg_mode(T), bloch, bpb);
  *ws_bytes = L.bytes;
  return PLHR_OK;
}

plhr_status plhr_create(const plhr_op_desc* A, const plhr_op_desc* B, const plhr_prec_desc* T,
                        double sigma, int32_t k, const plhr_options* opt, void* stream,
                        void* workspace, size_t ws_bytes, plhr_ctx* out) {
  if (!out) {
    set_error("out is NULL");
    return PLHR_ERR_ARG;
  }
  *out = nullptr;
  plhr_options o;
  plhr_options_default(&o);
  if (opt) o = *opt;
  plhr_status s = validate(A, B, T, sigma, k, &o);
  if (s != PLHR_OK) return s;
  plhr_ctx_s* c = new plhr_ctx_s();
  PLHR_HIP_CHECK(hipGetDevice(&c->device));
  c->stream = (hipStream_t)stream;
  c->grid = make_grid(A);
  c->pot = A->potential;
  c->sigma = sigma;
  c->bloch = (A->kind == PLHR_OP_BLOCH7_3D);
  c->bop = *A;
  c->k = c->bloch ? 2 * k : k;
  c->kint = block_cols(A, k, o);
  c->m = 4 * c->kint;
  c->opt = o;
  c->n = c->grid.n();
  const bool mgp = !c->bloch && uses_mg(T);
  const bool bmg = c->bloch && T && T->kind == PLHR_PREC_MG_VCYCLE;
  c->prec_kind = (mgp || bmg) ? PLHR_PREC_MG_VCYCLE : PLHR_PREC_IDENTITY;
  size_t bpb = 0;
  if (bmg) {
    const plhr_status sb = plhr_bloch_prec_workspace_size(A, T, c->kint, &bpb);
    if (sb != PLHR_OK) {
      delete c;
      return sb;
    }
  }
  if (T && T->kind == PLHR_PREC_DENSE) {
    c->prec_kind = PLHR_PREC_DENSE;
    c->Tdense = T->matrix;
  }
  const bool bd = B && B->kind == PLHR_OP_DIAG;
  if (bd) c->bdiag = B->potential;
  c->bst = B && (B->kind == PLHR_OP_Q1_MASS || B->kind == PLHR_OP_CSR);
  c->csr = (A->kind == PLHR_OP_CSR);
  if (c->csr) c->Acsr = CsrMat{A->row_ptr, A->col_idx, A->values, (long long)A->nnz};
  if (B && B->kind == PLHR_OP_CSR)
    c->Bcsr = CsrMat{B->row_ptr, B->col_idx, B->values, (long long)B->nnz};
  Layout L = layout(c->grid, c->k, c->kint, mgp, mgp ? T->levels : 0, bd, c->bst, nullptr,
                    mg_mode(T), c->bloch, bpb);
  if (workspace) {
    if (ws_bytes < L.bytes) {
      set_error("workspace smaller than plhr_workspace_size");
      delete c;
      return PLHR_ERR_ARG;
    }
    if (((uintptr_t)workspace) & 255) {
      set_error("workspace must be 256-byte aligned");
      delete c;
      return PLHR_ERR_ARG;
    }
    c->ws = (char*)workspace;
    c->own_ws = false;
  } else {
    hipError_t e = hipMalloc((void**)&c->ws, L.bytes);
    if (e != hipSuccess) {
      set_error(std::string("workspace allocation failed: ") + hipGetErrorString(e));
      delete c;
      return PLHR_ERR_HIP;
    }
    c->own_ws = true;
  }
  c->ws_bytes = L.bytes;
  layout(c->grid, c->k, c->kint, mgp, mgp ? T->levels : 0, bd, c->bst, c, mg_mode(T), c->bloch,
         bpb);
  if (bmg) {
    // the V-cycle's levels and coarse inverse are carved from the end of
    // the workspace
    const plhr_status sb = plhr_bloch_prec_create(A, T, c->kint, c->stream,
                                                  c->ws + L.bytes - al(bpb), al(bpb), &c->bprec);
    if (sb != PLHR_OK) {
      plhr_destroy(c);
      return sb;
    }
  }
  // norms for the relative residual
  std::vector<double> pot;
  if (c->pot) {
    pot.resize(c->n);
    hipError_t e = hipMemcpy(pot.data(), c->pot, c->n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      set_error(std::string("reading the potential failed: ") + hipGetErrorString(e));
      plhr_destroy(c);
      return PLHR_ERR_HIP;
    }
  }
  c->normA1 = c->csr ? 0.0 : (c->bloch ? bloch_norm1(*A, pot) : exact_norm1(c->grid, pot));
  c->normB1 = 1.0;
  if (c->csr) {
    plhr_status e1 = csr_norm1(A, pot, &c->normA1);
    if (e1 == PLHR_OK && B && B->kind == PLHR_OP_CSR) e1 = csr_norm1(B, {}, &c->normB1);
    if (e1 != PLHR_OK) {
      set_error(e1 == PLHR_ERR_HIP ? "reading the CSR arrays failed"
                                   : "CSR: row_ptr must start at 0, be nondecreasing and end at "
                                     "nnz; columns in [0, n); finite values");
      plhr_destroy(c);
      return e1;
    }
  }
  if (c->grid.q1) {
    double nb1 = 1.0;
    q1_norms(c->grid, pot, &c->normA1, &nb1);
    if (c->bst) c->normB1 = nb1;
  }
  if (bd) {
    // B = diag(b): b > 0 and finite, ||B||_1 = max b, and the scalings
    std::vector<double> bh(c->n), sq(c->n), isq(c->n);
    hipError_t e = hipMemcpy(bh.data(), c->bdiag, c->n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      set_error(std::string("reading the diagonal of B failed: ") + hipGetErrorString(e));
      plhr_destroy(c);
      return PLHR_ERR_HIP;
    }
    double bmax = 0.0;
    for (size_t p = 0; p < c->n; ++p) {
      if (!(bh[p] > 0.0) || !std::isfinite(bh[p])) {
        set_error("B: every diagonal entry must be positive and finite (entry " +
                  std::to_string(p) + ")");
        plhr_destroy(c);
        return PLHR_ERR_ARG;
      }
      bmax = std::max(bmax, bh[p]);
      sq[p] = std::sqrt(bh[p]);
      isq[p] = 1.0 / sq[p];
    }
    c->normB1 = bmax;
    e = hipMemcpy(c->bsq, sq.data(), c->n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(c->bisq, isq.data(), c->n * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      set_error(std::string("uploading the scalings of B failed: ") + hipGetErrorString(e));
      plhr_destroy(c);
      return PLHR_ERR_HIP;
    }
  }
  if (mgp) {
    char* wp = c->ws + L.bytes - mg_workspace_bytes(c->grid, T->levels, 2 * c->kint, mg_mode(T));
    MGOpts av;
    av.mode = mg_mode(T);
    av.sigma = sigma;
    av.delta = T->delta;
    av.degree = T->degree;
    s = mg_setup(c->mg, c->grid, T->levels, T->nu_pre, T->nu_post, T->omega, 2 * c->kint, wp,
                 c->stream, av);
    if (s != PLHR_OK) {
      plhr_destroy(c);
      return s;
    }
  }
  c->sp.kint = c->kint;
  c->sp.k = c->k;
  c->sp.m = c->m;
  c->sp.sigma = sigma;
  c->sp.tol = o.tol;
  c->sp.normA1 = c->normA1;
  c->sp.normB1 = c->normB1;
  c->sp.drop_tol = o.drop_tol;
  c->sp.cplx = c->bloch ? 2 : ((o.algorithm == PLHR_ALG_SINGLE) ? 1 : 0);
  c->sp.plmr = (o.algorithm == PLHR_ALG_PLMR) ? 1 : 0;
  // soft locking in the block iterations, real and complex (a complex
  // column locks both of its real columns); not in the single-vector ones
  c->sp.lock = (c->sp.cplx == 1 || c->sp.plmr) ? 0 : o.lock;
  // G_R of eq. (3.5) is symmetric when T does not enter the projection
  // (T = I, or the harmonic extraction) and B = I: the projected problem
  // is then Hermitian-definite
  c->sp.sym = (!c->bst && (o.extraction == PLHR_EXTRACT_HARMONIC ||
                           (c->prec_kind == PLHR_PREC_IDENTITY && !c->bdiag)))
                  ? 1
                  : 0;
  if (getenv("PLHR_NO_SYM") || c->sp.cplx || c->sp.plmr) c->sp.sym = 0;
  c->use_mfma = (getenv("PLHR_NO_MFMA") == nullptr);
  hipError_t e = small_set_attributes(c->m, c->kint);
  if (e == hipSuccess) e = tharm_sym_set_attributes();
  if (e == hipSuccess) e = cplx_set_attributes();
  if (e == hipSuccess) e = mfma_set_attributes(c->m, c->kint);
  if (e != hipSuccess) {
    set_error(std::string("LDS attribute: ") + hipGetErrorString(e));
    plhr_destroy(c);
    return PLHR_ERR_HIP;
  }
  e = hipHostMalloc((void**)&c->st_host, sizeof(DevStatus), hipHostMallocDefault);
  if (e != hipSuccess) {
    set_error(std::string("pinned status allocation failed: ") + hipGetErrorString(e));
    plhr_destroy(c);
    return PLHR_ERR_HIP;
  }
  std::memset(c->st_host, 0, sizeof(DevStatus));
  *out = c;
  return PLHR_OK;
}

plhr_status plhr_start(plhr_ctx c, const double* V0) {
  ProfScope prof_scope(c);
  if (!c || !V0) {
    set_error("plhr_start: NULL argument");
    return PLHR_ERR_ARG;
  }
  const int kint = c->kint, m = c->m;
  const size_t n = c->n;
  hipStream_t s = c->stream;
  // clear the basis blocks: unused slots must hold finite values
  PLHR_HIP_CHECK(hipMemsetAsync(c->Z, 0, n * m * sizeof(double), s));
  PLHR_HIP_CHECK(hipMemsetAsync(c->QZ, 0, n * m * sizeof(double), s));
  PLHR_HIP_CHECK(hipMemsetAsync(c->TQZ, 0, n * m * sizeof(double), s));
  if (c->bst) PLHR_HIP_CHECK(hipMemsetAsync(c->BZ, 0, n * m * sizeof(double), s));
  PLHR_HIP_CHECK(hipMemsetAsync(c->st, 0, sizeof(DevStatus), s));
  PLHR_HIP_CHECK(hipMemsetAsync(c->gate, 0, sizeof(DevStatus), s));
  if (c->bdiag)
    launch_rowscale(n, c->bsq, V0, kint, c->Z, m, kint, s);  // u = B^1/2 v
  else
    launch_copy(n, V0, kint, c->Z, m, kint, s);
  const Blk none{nullptr, 0};
  stencil(c, c->Z, m, Blk{c->QZ, m}, none, nullptr, none, kint, c->sigma, nullptr,
          c->bst ? Blk{c->BZ, m} : none);
  if (c->opt.extraction == PLHR_EXTRACT_T_HARMONIC && !c->sp.plmr)
    precond(c, c->QZ, m, Blk{c->TQZ, m}, none, kint, kint, nullptr);
  const int nb = launch_xdots(n, c->Z, m, c->QZ, m, kint, c->part, s, c->bst ? c->BZ : nullptr, m);
  launch_init_lam(c->sp, c->part, nb, c->sb, c->st, s);
  gram(c, c->Z, m, kint, c->bst ? c->BZ : c->Z, m, kint, nullptr, 0, kint, c->sb.G, nullptr);
  launch_start_check(c->sp, c->sb, c->st, s);
  PLHR_HIP_CHECK(hipGetLastError());
  c->started = true;
  c->finished = false;
  c->host_iter = 0;
  plhr_status st = read_status(c);
  if (st != PLHR_OK) return st;
  return device_error(c);
}

plhr_status plhr_iterate(plhr_ctx c, int32_t n_steps, plhr_iter_info* info) {
  ProfScope prof_scope(c);
  if (!c) {
    set_error("plhr_iterate: NULL context");
    return PLHR_ERR_ARG;
  }
  if (!c->started) {
    set_error("plhr_iterate before plhr_start");
    return PLHR_ERR_STATE;
  }
  if (n_steps < 0) {
    set_error("n_steps must be >= 0");
    return PLHR_ERR_ARG;
  }
  int done_steps = 0;
  while (done_steps < n_steps) {
    const int chunk = std::min(c->opt.check_every, n_steps - done_steps);
    for (int i = 0; i < chunk; ++i) {
      const plhr_status e = enqueue_iteration(c);
      if (e != PLHR_OK) return e;
    }
    PLHR_HIP_CHECK(hipGetLastError());
    done_steps += chunk;
    plhr_status s = read_status(c);
    if (s != PLHR_OK) return s;
    if (c->st_host->error || c->st_host->done) break;
  }
  if (info) {
    info->iters = c->st_host->iter;
    info->converged = c->st_host->done;
    info->n_active = c->st_host->n_active;
    info->status = c->st_host->error;
    info->max_rel_res = c->st_host->max_rel_res;
    info->n_excluded = c->st_host->n_excluded;
    info->reserved0 = 0;
  }
  return device_error(c);
}

plhr_status plhr_finish(plhr_ctx c, double* eigvals, double* V, double* rel_res) {
  ProfScope prof_scope(c);
  if (!c) {
    set_error("plhr_finish: NULL context");
    return PLHR_ERR_ARG;
  }
  if (!c->started) {
    set_error("plhr_finish before plhr_start");
    return PLHR_ERR_STATE;
  }
  const int kint = c->kint, k = c->k, m = c->m;
  const size_t n = c->n;
  hipStream_t s = c->stream;
  // H = V^T (A - sigma) V, M = V^T V, from a fresh (A - sigma)V
  const Blk none0{nullptr, 0};
  stencil(c, c->Z, m, Blk{c->QZ, m}, none0, nullptr, none0, kint, c->sigma, nullptr,
          c->bst ? Blk{c->BZ, m} : none0);
  const int gnb = c->gram_nblk;
  gram(c, c->Z, m, kint, c->QZ, m, kint, c->bst ? c->BZ : c->Z, m, 2 * kint, c->HM, nullptr);
  (void)gnb;
  if (c->sp.cplx == 2)
    launch_cplx_final(c->sp, c->HM, c->sb, c->st, s);
  else
    launch_final_rr(c->sp, c->HM, c->sb, c->st, s);
  launch_small_gemm(n, c->Z, m, kint, c->sb.final_C, k, c->Vfin, k, s);
  const Blk none{nullptr, 0};
  stencil(c, c->Vfin, k, Blk{c->QVfin, k}, none, nullptr, none, k, c->sigma, nullptr,
          c->bst ? Blk{c->BVfin, k} : none);
  const int nb = launch_coldots(n, c->Vfin, k, c->QVfin, k, k, c->sb.final_theta, c->sigma,
                                c->bdiag, c->bst ? c->BVfin : nullptr, k, c->part, s);
  SmallParams fp = c->sp;
  launch_final_res(fp, c->part, nb, c->sb, s);
  if (c->bst) {
    // v^* B v for the gradient
    const int nx = launch_xdots(n, c->Vfin, k, c->QVfin, k, k, c->part, s, c->BVfin, k);
    launch_colsum_first(c->part, nx, k, c->sb.vbv, s);
  }
  if (c->bdiag) {
    // v^* B v = u^* u for the gradient, then v = B^-1/2 u
    const int nx = launch_xdots(n, c->Vfin, k, c->QVfin, k, k, c->part, s);
    launch_colsum_first(c->part, nx, k, c->sb.vbv, s);
    launch_rowscale(n, c->bisq, c->Vfin, k, c->Vfin, k, k, s);
  }
  // the Bloch operator returns k/2 complex pairs: each value twice in
  // final_theta and relres, the vectors as interleaved columns (complex128)
  const int kout = c->bloch ? k / 2 : k, es = c->bloch ? 2 : 1;
  if (eigvals)
    PLHR_HIP_CHECK(hipMemcpy2DAsync(eigvals, sizeof(double), c->sb.final_theta,
                                    es * sizeof(double), sizeof(double), kout,
                                    hipMemcpyDeviceToDevice, s));
  if (V)
    PLHR_HIP_CHECK(hipMemcpyAsync(V, c->Vfin, n * k * sizeof(double), hipMemcpyDeviceToDevice, s));
  std::vector<double> rr(k);
  PLHR_HIP_CHECK(hipMemcpyAsync(rr.data(), c->sb.relres, k * sizeof(double),
                                hipMemcpyDeviceToHost, s));
  PLHR_HIP_CHECK(hipGetLastError());
  plhr_status st = read_status(c);
  if (st != PLHR_OK) return st;
  if (rel_res)
    for (int j = 0; j < kout; ++j) rel_res[j] = rr[(size_t)j * es];
  c->finished = true;
  return device_error(c);
}

plhr_status plhr_solve(plhr_ctx c, const double* V0, double* eigvals, double* V, double* rel_res,
                       int32_t* iters) {
  plhr_status s = plhr_start(c, V0);
  if (s != PLHR_OK) return s;
  plhr_iter_info info{};
  s = plhr_iterate(c, c->opt.max_iters, &info);
  if (s != PLHR_OK) return s;
  if (iters) *iters = info.iters;
  s = plhr_finish(c, eigvals, V, rel_res);
  if (s != PLHR_OK) return s;
  if (!info.converged) {
    set_error("max_iters reached before convergence");
    return PLHR_ERR_NOT_CONVERGED;
  }
  return PLHR_OK;
}

plhr_status plhr_eigvals_backward(plhr_ctx c, const double* dL_dlambda, double* dL_dpot,
                                  int32_t accumulate) {
  if (!c || !dL_dlambda || !dL_dpot) {
    set_error("plhr_eigvals_backward: NULL argument");
    return PLHR_ERR_ARG;
  }
  if (!c->finished) {
    set_error("plhr_eigvals_backward before plhr_finish");
    return PLHR_ERR_STATE;
  }
  if (c->bloch) {
    set_error("plhr_eigvals_backward: not available for the Bloch operator");
    return PLHR_ERR_UNSUPPORTED;
  }
  launch_hf(c->n, c->Vfin, c->k, c->k, dL_dlambda, c->sb.vbv, dL_dpot, accumulate, c->stream);
  PLHR_HIP_CHECK(hipGetLastError());
  return PLHR_OK;
}

plhr_status plhr_apply(plhr_ctx c, int32_t which, const double* X, double* Y, int32_t ncols) {
  ProfScope prof_scope(c);
  if (!c || !X || !Y) {
    set_error("plhr_apply: NULL argument");
    return PLHR_ERR_ARG;
  }
  if (ncols < 1 || ncols > 2 * c->kint) {
    set_error("plhr_apply: need 1 <= ncols <= 2*(k + k_extra)");
    return PLHR_ERR_ARG;
  }
  if (c->bloch && (ncols & 1)) {
    set_error("plhr_apply: the Bloch operator takes whole complex columns (even ncols)");
    return PLHR_ERR_ARG;
  }
  const Blk none{nullptr, 0};
  if (which == 0 || which == 1) {
    // with a diagonal B: A X = B^1/2 (S A S)(B^1/2 X), and the same with the shift
    const double* Xin = X;
    if (c->bdiag) {
      launch_rowscale(c->n, c->bsq, X, ncols, c->Rs, ncols, ncols, c->stream);
      Xin = c->Rs;
    }
    stencil(c, Xin, ncols, Blk{Y, ncols}, none, nullptr, none, ncols,
            which == 1 ? c->sigma : 0.0, nullptr);
    if (c->bdiag) launch_rowscale(c->n, c->bsq, Y, ncols, Y, ncols, ncols, c->stream);
  } else if (which == 2) {
    precond_raw(c, X, ncols, Blk{Y, ncols}, none, ncols, ncols, nullptr, true);
  } else {
    set_error("plhr_apply: which must be 0, 1 or 2");
    return PLHR_ERR_ARG;
  }
  PLHR_HIP_CHECK(hipGetLastError());
  PLHR_HIP_CHECK(hipStreamSynchronize(c->stream));
  return PLHR_OK;
}

plhr_status plhr_get_state(plhr_ctx c, double* lam, double* V) {
  if (!c || !lam) {
    set_error("plhr_get_state: NULL argument");
    return PLHR_ERR_ARG;
  }
  if (!c->started) {
    set_error("plhr_get_state before plhr_start");
    return PLHR_ERR_STATE;
  }
  PLHR_HIP_CHECK(hipMemcpyAsync(lam, c->sb.lam, c->kint * sizeof(double), hipMemcpyDeviceToHost,
                                c->stream));
  if (V) {
    if (c->bdiag)
      launch_rowscale(c->n, c->bisq, c->Z, c->m, V, c->kint, c->kint, c->stream);
    else
      launch_copy(c->n, c->Z, c->m, V, c->kint, c->kint, c->stream);
  }
  PLHR_HIP_CHECK(hipGetLastError());
  PLHR_HIP_CHECK(hipStreamSynchronize(c->stream));
  return PLHR_OK;
}

plhr_status plhr_debug_read(plhr_ctx c, int32_t which, double* dst, size_t count) {
  if (!c || !dst) {
    set_error("plhr_debug_read: NULL argument");
    return PLHR_ERR_ARG;
  }
  const size_t m = c->m, kint = c->kint, n = c->n;
  const double* src = nullptr;
  size_t cap = 0;
  std::vector<double> tmp;
  switch (which) {
    case 0: src = c->sb.G; cap = m * m; break;
    case 1: src = c->sb.M; cap = m * m; break;
    case 2: src = c->sb.GLR; cap = 2 * m * m; break;
    case 3: src = c->sb.Y; cap = m * kint; break;
    case 4: src = c->sb.xi; cap = 2 * m; break;
    case 5: src = c->sb.lam; cap = kint; break;
    case 6: src = c->sb.relres; cap = kint; break;
    case 7: src = c->Z; cap = n * m; break;
    case 8: src = c->QZ; cap = n * m; break;
    case 9: src = c->TQZ; cap = n * m; break;
    case 10: case 11: break;
    case 12: {
      PLHR_HIP_CHECK(hipStreamSynchronize(c->stream));
      DevStatus hs;
      PLHR_HIP_CHECK(hipMemcpy(&hs, c->st, sizeof(DevStatus), hipMemcpyDeviceToHost));
      if (count > 12) {
        set_error("plhr_debug_read: count exceeds the buffer");
        return PLHR_ERR_ARG;
      }
      for (size_t i = 0; i < count; ++i) dst[i] = (double)hs.tphase[i];
      return PLHR_OK;
    }
    default:
      set_error("plhr_debug_read: unknown buffer");
      return PLHR_ERR_ARG;
  }
  PLHR_HIP_CHECK(hipStreamSynchronize(c->stream));
  if (which == 10 || which == 11) {
    const size_t cnt = (which == 10) ? m : 2 * kint;
    if (count > cnt) {
      set_error("plhr_debug_read: count exceeds the buffer");
      return PLHR_ERR_ARG;
    }
    std::vector<int> iv(cnt);
    if (which == 10) {
      PLHR_HIP_CHECK(hipMemcpy(iv.data(), c->sb.keep, m * sizeof(int), hipMemcpyDeviceToHost));
    } else {
      PLHR_HIP_CHECK(hipMemcpy(iv.data(), c->sb.kinds, kint * sizeof(int), hipMemcpyDeviceToHost));
      PLHR_HIP_CHECK(hipMemcpy(iv.data() + kint, c->sb.pair, kint * sizeof(int),
                               hipMemcpyDeviceToHost));
    }
    for (size_t i = 0; i < count; ++i) dst[i] = iv[i];
    return PLHR_OK;
  }
  if (count > cap) {
    set_error("plhr_debug_read: count exceeds the buffer");
    return PLHR_ERR_ARG;
  }
  PLHR_HIP_CHECK(hipMemcpy(dst, src, count * sizeof(double), hipMemcpyDeviceToHost));
  return PLHR_OK;
}

plhr_status plhr_profile_start(plhr_ctx c, int32_t category, int32_t max_launches) {
  if (!c) {
    set_error("plhr_profile_start: bad argument");
    return PLHR_ERR_ARG;
  }
  return prof_start(c->prof, category, max_launches);
}

plhr_status plhr_profile_stop(plhr_ctx c, plhr_profile* out) {
  if (!c || !out) {
    set_error("plhr_profile_stop: NULL argument");
    return PLHR_ERR_ARG;
  }
  return prof_stop(c->prof, c->stream, out);
}

plhr_status plhr_op_apply(const plhr_op_desc* A, double shift, const void* X, void* Y,
                          int32_t ncols, void* stream) {
  if (!A || (ncols > 0 && (!X || !Y))) {
    set_error("plhr_op_apply: NULL argument");
    return PLHR_ERR_ARG;
  }
  if (A->kind != PLHR_OP_BLOCH7_3D || A->dtype != PLHR_C128) {
    set_error("plhr_op_apply: only PLHR_OP_BLOCH7_3D with PLHR_C128 is supported (the real "
              "operators are applied through a context, plhr_apply)");
    return PLHR_ERR_UNSUPPORTED;
  }
  if (A->nx < 1 || A->ny < 1 || A->nz < 1 || ncols < 0) {
    set_error("plhr_op_apply: need nx, ny, nz >= 1 and ncols >= 0");
    return PLHR_ERR_ARG;
  }
  if (!(A->h > 0.0) || !(A->scale > 0.0) || !std::isfinite(A->h) || !std::isfinite(A->scale) ||
      !std::isfinite(shift) || !std::isfinite(A->theta[0]) || !std::isfinite(A->theta[1]) ||
      !std::isfinite(A->theta[2])) {
    set_error("plhr_op_apply: h and scale must be positive and finite, theta and shift finite");
    return PLHR_ERR_ARG;
  }
  if ((int64_t)A->nx * ncols >= (int64_t(1) << 31) ||
      (int64_t)A->ny * A->nz >= (int64_t(1) << 31)) {
    set_error("plhr_op_apply: nx*ncols and ny*nz must be below 2^31");
    return PLHR_ERR_ARG;
  }
  if (ncols == 0) return PLHR_OK;
  const size_t bytes = (size_t)A->nx * A->ny * A->nz * ncols * 16;
  const char* xb = static_cast<const char*>(X);
  const char* yb = static_cast<const char*>(Y);
  if (xb < yb + bytes && yb < xb + bytes) {
    set_error("plhr_op_apply: X and Y overlap");
    return PLHR_ERR_ARG;
  }
  launch_bloch_apply(A->nx, A->ny, A->nz, A->h, A->scale, A->theta, A->potential, shift,
                     static_cast<const double*>(X), static_cast<double*>(Y), ncols,
                     static_cast<hipStream_t>(stream));
  PLHR_HIP_CHECK(hipGetLastError());
  return PLHR_OK;
}

void plhr_destroy(plhr_ctx c) {
  if (!c) return;
  prof_release(c->prof);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  destroy_graphs(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  if (c->bprec) plhr_bloch_prec_destroy(c->bprec);
  if (c->own_ws && c->ws) (void)hipFree(c->ws);
  if (c->st_host) (void)hipHostFree(c->st_host);
  delete c;
}

}  // extern "C"
