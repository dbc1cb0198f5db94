// Batched driver: Algorithm 3 advanced for many independent 2-D problems
// by the same launches (the kernels are in k_batch.hip and the batched
// wrappers of the single-workgroup kernels), with the per-iteration
// sequence captured in a HIP graph and the chunking tuned by timing.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"

using namespace plhr;

namespace {
constexpr int kRefreshB = 10;  // iterations between refreshes of the V slots of QZ, TQZ
const int kChunkCand[4] = {512, 1024, 2048, 4096};
const int kRowCand[3] = {64, 128, 256};
size_t al(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

struct plhr_batch_s {
  int nb = 0, k = 0, kint = 0, m = 0;
  int levels = 0, nu = 2;
  double omega = 2.0 / 3.0;
  bool mg = false;
  hipStream_t stream = nullptr;
  plhr_options opt{};
  Grid g0;  // h and scale (dims per problem)
  std::vector<int> nx, ny;
  std::vector<size_t> off;
  std::vector<double> sigma;
  size_t ntot = 0;
  std::vector<size_t> ntot_l;  // packed points per level
  // device memory (one allocation)
  char* ws = nullptr;
  bool own_ws = true;  // false: the caller's workspace
  double *Z = nullptr, *QZ = nullptr, *TQZ = nullptr, *R = nullptr, *QVf = nullptr;
  double *Vfin = nullptr, *QVfin = nullptr;
  std::vector<double*> lx, lt, lr;  // per level, packed, ld 2 kint
  double *part = nullptr, *gpart = nullptr;
  // per-problem small buffers, packed with fixed strides
  double *G = nullptr, *M = nullptr, *GLR = nullptr, *Y = nullptr, *lam = nullptr,
         *relres = nullptr, *xi = nullptr, *fC = nullptr, *fth = nullptr, *vbv = nullptr,
         *work = nullptr, *HM = nullptr;
  int *keep = nullptr, *active = nullptr, *kinds = nullptr, *pair = nullptr;
  DevStatus* st = nullptr;
  DevStatus* st_host = nullptr;
  BProb *pr = nullptr, *prF = nullptr;
  std::vector<BLev*> lv;
  std::vector<RowMap*> rm;
  std::vector<int> nrows;
  Chunk* ch = nullptr;
  int nch = 0, chunk_pts = 1024, row_threads = 256;
  int max_chunks = 0;
  BatchSmall* bs = nullptr;
  BatchSmall* bsF = nullptr;  // the same with partial slots of 2k values (final step)
  const double** inv = nullptr;
  std::vector<double*> inv_store;
  const double** src = nullptr;
  double** dst = nullptr;
  const double** vbvp = nullptr;
  std::vector<std::vector<double>> pot_host;
  std::vector<const double*> pot_dev;
  // graphs
  bool use_graph = true, tuned = false;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipStream_t cap = nullptr;  // capture stream (the caller's may be the null stream)
  double tuned_ms[8] = {0};
  Prof prof;
  bool finished = false;
};

namespace {

struct ProfScopeB {
  explicit ProfScopeB(plhr_batch_s* c) { prof_attach(c ? &c->prof : nullptr); }
  ~ProfScopeB() { prof_attach(nullptr); }
};

// Chunk table for a chunk size; returns the number of chunks and sets the
// per-problem first chunk and count in the host copies of BProb.
std::vector<Chunk> make_chunks(const plhr_batch_s* c, int pts, std::vector<BProb>& prh,
                               std::vector<BProb>& prfh) {
  std::vector<Chunk> chs;
  for (int b = 0; b < c->nb; ++b) {
    const int n = c->nx[b] * c->ny[b];
    prh[b].ch0 = prfh[b].ch0 = (int)chs.size();
    for (int p0 = 0; p0 < n; p0 += pts) chs.push_back(Chunk{b, p0, std::min(n, p0 + pts)});
    prh[b].nch = prfh[b].nch = (int)chs.size() - prh[b].ch0;
  }
  return chs;
}

plhr_status upload_tables(plhr_batch_s* c, int pts) {
  PLHR_HIP_CHECK(hipStreamSynchronize(c->stream));
  std::vector<BProb> prh(c->nb), prfh(c->nb);
  PLHR_HIP_CHECK(hipMemcpy(prh.data(), c->pr, c->nb * sizeof(BProb), hipMemcpyDeviceToHost));
  PLHR_HIP_CHECK(hipMemcpy(prfh.data(), c->prF, c->nb * sizeof(BProb), hipMemcpyDeviceToHost));
  std::vector<Chunk> chs = make_chunks(c, pts, prh, prfh);
  if ((int)chs.size() > c->max_chunks) {
    set_error("batch: chunk table larger than allocated");
    return PLHR_ERR_ARG;
  }
  PLHR_HIP_CHECK(hipMemcpy(c->ch, chs.data(), chs.size() * sizeof(Chunk), hipMemcpyHostToDevice));
  PLHR_HIP_CHECK(hipMemcpy(c->pr, prh.data(), c->nb * sizeof(BProb), hipMemcpyHostToDevice));
  PLHR_HIP_CHECK(hipMemcpy(c->prF, prfh.data(), c->nb * sizeof(BProb), hipMemcpyHostToDevice));
  // the batched small kernels read the partial slots of each problem
  // (partial slots of 2 kint values in the iteration, 2 k in the final step)
  std::vector<BatchSmall> bsh(c->nb);
  PLHR_HIP_CHECK(hipMemcpy(bsh.data(), c->bs, c->nb * sizeof(BatchSmall), hipMemcpyDeviceToHost));
  for (int b = 0; b < c->nb; ++b) {
    bsh[b].part = c->part + (size_t)prh[b].ch0 * 2 * c->kint;
    bsh[b].nblk = prh[b].nch;
  }
  PLHR_HIP_CHECK(hipMemcpy(c->bs, bsh.data(), c->nb * sizeof(BatchSmall), hipMemcpyHostToDevice));
  for (int b = 0; b < c->nb; ++b) bsh[b].part = c->part + (size_t)prh[b].ch0 * 2 * c->k;
  PLHR_HIP_CHECK(hipMemcpy(c->bsF, bsh.data(), c->nb * sizeof(BatchSmall), hipMemcpyHostToDevice));
  c->nch = (int)chs.size();
  c->chunk_pts = pts;
  return PLHR_OK;
}

Grid level_grid(const plhr_batch_s* c, int lev) {
  Grid g = c->g0;
  g.dim = 2;
  for (int l = 0; l < lev; ++l) g.h *= 2.0;
  return g;
}

// One V-cycle of every problem at level lev on input r (ld ldr); at level 0
// the result goes to o0/o1 (split by column), below it stays in a level
// buffer whose address is returned.
double* mg_cycle_b(plhr_batch_s* c, int lev, const double* r, int ldr, Blk o0, Blk o1,
                   int split, int ncols) {
  hipStream_t s = c->stream;
  const Grid g = level_grid(c, lev);
  const double diag = g.diag(), off = g.off(), om = c->omega;
  const int th = c->row_threads;
  if (lev == c->levels - 1) {
    launch_dense_b(c->nb, c->lv[lev], c->pr, c->inv, r, c->lx[lev], ncols, s);
    return c->lx[lev];
  }
  double* cur = c->lx[lev];
  double* oth = c->lt[lev];
  for (int it = 0; it < c->nu; ++it) {
    launch_jacobi_b(c->rm[lev], c->nrows[lev], c->lv[lev], c->pr, diag, off, om,
                    it == 0 ? nullptr : cur, r, ldr, Blk{oth, ncols}, Blk{oth, ncols}, ncols,
                    ncols, th, s);
    std::swap(cur, oth);
  }
  launch_residual_b(c->rm[lev], c->nrows[lev], c->lv[lev], c->pr, diag, off, cur, r, ldr, oth,
                    ncols, th, s);
  launch_restrict_b(c->rm[lev + 1], c->nrows[lev + 1], c->lv[lev], c->lv[lev + 1], c->pr, oth,
                    c->lr[lev + 1], ncols, th, s);
  double* ec = mg_cycle_b(c, lev + 1, c->lr[lev + 1], ncols, Blk{nullptr, 0}, Blk{nullptr, 0},
                          ncols, ncols);
  launch_prolong_b(c->rm[lev], c->nrows[lev], c->lv[lev], c->lv[lev + 1], c->pr, ec, cur, ncols,
                   th, s);
  for (int it = 0; it < c->nu; ++it) {
    if (it == c->nu - 1 && lev == 0) {
      launch_jacobi_b(c->rm[lev], c->nrows[lev], c->lv[lev], c->pr, diag, off, om, cur, r, ldr,
                      o0, o1, split, ncols, th, s);
      return nullptr;
    }
    launch_jacobi_b(c->rm[lev], c->nrows[lev], c->lv[lev], c->pr, diag, off, om, cur, r, ldr,
                    Blk{oth, ncols}, Blk{oth, ncols}, ncols, ncols, th, s);
    std::swap(cur, oth);
  }
  return cur;
}

void precond_b(plhr_batch_s* c, const double* R, int ldr, Blk o0, Blk o1, int split, int ncols) {
  if (c->mg) {
    mg_cycle_b(c, 0, R, ldr, o0, o1, split, ncols);
  } else {
    if (split > 0) launch_copy(c->ntot, R, ldr, o0.ptr, o0.ld, split, c->stream);
    if (split < ncols) launch_copy(c->ntot, R + split, ldr, o1.ptr, o1.ld, ncols - split, c->stream);
  }
}

void fd_b(plhr_batch_s* c, const double* X, int ldx, Blk out, Blk outr, Blk outc, int ncols,
          int use_sigma, const BProb* pr) {
  const Grid& g = c->g0;
  launch_fd_b(c->rm[0], c->nrows[0], pr, g.diag(), g.off(), use_sigma, X, ldx, out, outr, outc,
              ncols, c->row_threads, c->stream);
}

void gram_b(plhr_batch_s* c, const double* X, int ldx, int mx, const double* Y1, int ldy1,
            int my1, const double* Y2, int ldy2, int my, double* out, size_t ostride) {
  launch_gram_b(c->ch, c->nch, c->nb, c->pr, X, ldx, mx, Y1, ldy1, my1, Y2, ldy2, my, c->gpart,
                out, ostride, c->ntot, c->stream);
}

// Algorithm 3, one iteration of every problem (mirrors the single-problem
// driver).
void enqueue_iteration_b(plhr_batch_s* c, bool refresh) {
  const int kint = c->kint, m = c->m;
  hipStream_t s = c->stream;
  double *Z = c->Z, *QZ = c->QZ, *TQZ = c->TQZ, *R = c->R;
  const Blk none{nullptr, 0};
  if (refresh) {
    fd_b(c, Z, m, Blk{QZ, m}, none, none, kint, 1, c->pr);
    precond_b(c, QZ, m, Blk{TQZ, m}, none, kint, kint);
  }
  fd_b(c, Z, m, Blk{c->QVf, kint}, none, none, kint, 1, c->pr);
  launch_xdots_b(c->ch, c->nch, c->pr, Z, m, c->QVf, kint, kint, c->part, s);
  launch_rq_small_b(c->bs, c->nb, 0, s);
  launch_resid_b(c->ch, c->nch, c->pr, Z, m, c->QVf, kint, R, kint, kint, c->part, s);
  launch_conv_check_b(c->bs, c->nb, s);
  precond_b(c, R, kint, Blk{Z + kint, m}, none, kint, kint);
  fd_b(c, Z + kint, m, Blk{QZ + kint, m}, Blk{R, 2 * kint}, Blk{R + kint, 2 * kint}, kint, 1,
       c->pr);
  precond_b(c, R, 2 * kint, Blk{Z + 2 * kint, m}, Blk{TQZ + kint, m}, kint, 2 * kint);
  fd_b(c, Z + 2 * kint, m, Blk{QZ + 2 * kint, m}, none, none, kint, 1, c->pr);
  precond_b(c, QZ + 2 * kint, m, Blk{TQZ + 2 * kint, m}, none, kint, kint);
  gram_b(c, Z, m, m, Z, m, m, nullptr, 0, m, c->G, (size_t)m * m);
  launch_ortho_small_b(c->bs, c->nb, m, s);
  double* arrs[3] = {Z, QZ, TQZ};
  launch_rowmul_b(c->ch, c->nch, c->pr, arrs, 3, m, m, c->M, (size_t)m * m, m, 0, 0, 0, 0,
                  nullptr, c->ntot, s);
  gram_b(c, TQZ, m, m, QZ, m, m, Z, m, 2 * m, c->GLR, (size_t)2 * m * m);
  launch_tharm_small_b(c->bs, c->nb, m, kint, s);
  launch_rowmul_b(c->ch, c->nch, c->pr, arrs, 3, m, m, c->Y, (size_t)m * kint, 2 * kint, 1, kint,
                  kint, 3 * kint, c->part, c->ntot, s);
  launch_rq_small_b(c->bs, c->nb, 1, s);
}

plhr_status read_status_b(plhr_batch_s* c) {
  PLHR_HIP_CHECK(hipMemcpyAsync(c->st_host, c->st, c->nb * sizeof(DevStatus),
                                hipMemcpyDeviceToHost, c->stream));
  PLHR_HIP_CHECK(hipStreamSynchronize(c->stream));
  return PLHR_OK;
}

void destroy_graphs(plhr_batch_s* c) {
  for (int i = 0; i < 2; ++i) {
    if (c->gexec[i]) (void)hipGraphExecDestroy(c->gexec[i]);
    if (c->graph[i]) (void)hipGraphDestroy(c->graph[i]);
    c->gexec[i] = nullptr;
    c->graph[i] = nullptr;
  }
}

// The launches are recorded on a stream of the library's own (capture is
// not allowed on the null stream) and the graphs replayed on the caller's.
plhr_status capture_graphs(plhr_batch_s* c) {
  destroy_graphs(c);
  if (!c->cap) PLHR_HIP_CHECK(hipStreamCreate(&c->cap));
  PLHR_HIP_CHECK(hipStreamSynchronize(c->stream));
  hipStream_t user = c->stream;
  c->stream = c->cap;
  hipError_t e = hipSuccess;
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) break;
    enqueue_iteration_b(c, i == 1);
    e = hipStreamEndCapture(c->cap, &c->graph[i]);
    if (e == hipSuccess) e = hipGraphInstantiate(&c->gexec[i], c->graph[i], nullptr, nullptr, 0);
  }
  c->stream = user;
  if (e != hipSuccess) {
    set_error(std::string("batch graph capture: ") + hipGetErrorString(e));
    destroy_graphs(c);
    return PLHR_ERR_HIP;
  }
  return PLHR_OK;
}

// Time `reps` repetitions of fn on the stream (ms per repetition).
template <class F>
double time_ms(hipStream_t s, int reps, F fn) {
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  fn();  // warm
  (void)hipEventRecord(a, s);
  for (int i = 0; i < reps; ++i) fn();
  (void)hipEventRecord(b, s);
  (void)hipEventSynchronize(b);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms / reps;
}

// Autotuner: the chunk size of the point-range kernels (Gram, row product,
// column sums) and the workgroup size of the grid-row kernels (stencil,
// V-cycle), each picked as the fastest of its candidates on this batch's
// own arrays (the timed kernels only read and rewrite scratch-consistent
// data: Grams into G, a transform by M into the W slot area of R and the
// V-cycle into QVf).
plhr_status autotune(plhr_batch_s* c) {
  hipStream_t s = c->stream;
  const int m = c->m, kint = c->kint;
  double best = 1e30;
  int bestpts = c->chunk_pts;
  for (int i = 0; i < 4; ++i) {
    plhr_status st = upload_tables(c, kChunkCand[i]);
    if (st != PLHR_OK) return st;
    const double ms = time_ms(s, 3, [&] {
      gram_b(c, c->TQZ, m, m, c->QZ, m, m, c->Z, m, 2 * m, c->GLR, (size_t)2 * m * m);
      launch_xdots_b(c->ch, c->nch, c->pr, c->Z, m, c->QVf, kint, kint, c->part, s);
    });
    c->tuned_ms[i] = ms;
    if (ms < best) best = ms, bestpts = kChunkCand[i];
  }
  plhr_status st = upload_tables(c, bestpts);
  if (st != PLHR_OK) return st;
  best = 1e30;
  int bestth = c->row_threads;
  for (int i = 0; i < 3; ++i) {
    c->row_threads = kRowCand[i];
    const double ms = time_ms(s, 3, [&] {
      fd_b(c, c->Z, m, Blk{c->QVf, kint}, Blk{nullptr, 0}, Blk{nullptr, 0}, kint, 1, c->pr);
      if (c->mg) precond_b(c, c->QVf, kint, Blk{c->R, kint}, Blk{nullptr, 0}, kint, kint);
    });
    c->tuned_ms[4 + i] = ms;
    if (ms < best) best = ms, bestth = kRowCand[i];
  }
  c->row_threads = bestth;
  c->tuned = true;
  PLHR_HIP_CHECK(hipGetLastError());
  return PLHR_OK;
}

plhr_status start_b(plhr_batch_s* c, const double* const* V0) {
  const int kint = c->kint, m = c->m;
  hipStream_t s = c->stream;
  PLHR_HIP_CHECK(hipMemsetAsync(c->Z, 0, c->ntot * m * sizeof(double), s));
  PLHR_HIP_CHECK(hipMemsetAsync(c->QZ, 0, c->ntot * m * sizeof(double), s));
  PLHR_HIP_CHECK(hipMemsetAsync(c->TQZ, 0, c->ntot * m * sizeof(double), s));
  PLHR_HIP_CHECK(hipMemsetAsync(c->st, 0, c->nb * sizeof(DevStatus), s));
  PLHR_HIP_CHECK(hipMemcpyAsync(c->src, V0, c->nb * sizeof(double*), hipMemcpyHostToDevice, s));
  launch_copy_in_b(c->ch, c->nch, c->pr, c->src, kint, c->Z, m, s);
  const Blk none{nullptr, 0};
  fd_b(c, c->Z, m, Blk{c->QZ, m}, none, none, kint, 1, c->pr);
  precond_b(c, c->QZ, m, Blk{c->TQZ, m}, none, kint, kint);
  launch_xdots_b(c->ch, c->nch, c->pr, c->Z, m, c->QZ, m, kint, c->part, s);
  launch_init_lam_b(c->bs, c->nb, s);
  gram_b(c, c->Z, m, kint, c->Z, m, kint, nullptr, 0, kint, c->G, (size_t)m * m);
  launch_start_check_b(c->bs, c->nb, s);
  PLHR_HIP_CHECK(hipGetLastError());
  return read_status_b(c);
}

plhr_status finish_b(plhr_batch_s* c) {
  const int kint = c->kint, k = c->k, m = c->m;
  hipStream_t s = c->stream;
  const Blk none{nullptr, 0};
  // the problems stopped at convergence: let the final steps run for all
  for (int b = 0; b < c->nb; ++b) c->st_host[b].done = 0;
  std::vector<int> err(c->nb);
  for (int b = 0; b < c->nb; ++b) err[b] = c->st_host[b].error;
  // keep failed problems halted, re-open converged and unconverged ones
  PLHR_HIP_CHECK(hipMemcpyAsync(c->st, c->st_host, c->nb * sizeof(DevStatus),
                                hipMemcpyHostToDevice, s));
  fd_b(c, c->Z, m, Blk{c->QZ, m}, none, none, kint, 1, c->pr);
  gram_b(c, c->Z, m, kint, c->QZ, m, kint, c->Z, m, 2 * kint, c->HM, (size_t)2 * kint * kint);
  launch_final_rr_b(c->bs, c->nb, kint, s);
  launch_small_gemm_b(c->ch, c->nch, c->pr, c->Z, m, kint, c->fC, (size_t)kint * kint, k,
                      c->Vfin, k, s);
  fd_b(c, c->Vfin, k, Blk{c->QVfin, k}, none, none, k, 1, c->pr);
  launch_resid_b(c->ch, c->nch, c->prF, c->Vfin, k, c->QVfin, k, nullptr, 0, k, c->part, s);
  launch_final_res_b(c->bsF, c->nb, s);
  PLHR_HIP_CHECK(hipGetLastError());
  return read_status_b(c);
}

}  // namespace

namespace {

// Validation, layout and set-up of a batch.  With `size_only` it stops after
// the layout and stores the workspace bytes there (no device call); with a
// caller `workspace` (at least that many bytes, 256-byte aligned) nothing
// is allocated on the device.
plhr_status batch_create_impl(int32_t nbatch, const plhr_op_desc* A, const plhr_prec_desc* T,
                              const double* sigma, int32_t k, const plhr_options* opt,
                              void* stream, void* workspace, size_t ws_bytes,
                              size_t* size_only, plhr_batch* out) {
  if ((!out && !size_only) || !A || !sigma || nbatch < 1) {
    set_error("plhr_batch_create: NULL argument or nbatch < 1");
    return PLHR_ERR_ARG;
  }
  if (out) *out = nullptr;
  plhr_options o;
  plhr_options_default(&o);
  if (opt) o = *opt;
  if (!(o.tol > 0.0) || o.max_iters < 0 || o.check_every < 1 || !(o.drop_tol > 0.0) ||
      o.precision != PLHR_PREC_FP64 || o.k_extra < 0 || k < 1) {
    set_error("plhr_batch_create: invalid options (FP64 only), or k < 1");
    return PLHR_ERR_ARG;
  }
  const int kint = k + o.k_extra, m = 4 * kint;
  if (m > kMaxM) {
    set_error("plhr_batch_create: 4*(k + k_extra) > 84");
    return PLHR_ERR_UNSUPPORTED;
  }
  const bool mg = T && T->kind != PLHR_PREC_IDENTITY;
  if (mg && (T->kind != PLHR_PREC_MG_VCYCLE || T->levels < 2 || T->nu_pre < 1 ||
             T->nu_pre != T->nu_post || !(T->omega > 0.0) || T->omega > 1.0)) {
    set_error("plhr_batch_create: T must be a V-cycle with levels >= 2, nu_pre == nu_post >= 1, "
              "0 < omega <= 1");
    return PLHR_ERR_ARG;
  }
  const int levels = mg ? T->levels : 1;
  const int f = 1 << (levels - 1);
  for (int b = 0; b < nbatch; ++b) {
    const plhr_op_desc& a = A[b];
    if (a.kind != PLHR_OP_FD5_2D || a.dtype != PLHR_F64 || a.nz != 1 || a.nx < 1 || a.ny < 1) {
      set_error("plhr_batch_create: every problem must be an FP64 PLHR_OP_FD5_2D operator");
      return PLHR_ERR_UNSUPPORTED;
    }
    if (a.h != A[0].h || a.scale != A[0].scale || !(a.h > 0.0) || !(a.scale > 0.0)) {
      set_error("plhr_batch_create: h and scale must be positive and equal for all problems");
      return PLHR_ERR_ARG;
    }
    if (!std::isfinite(sigma[b])) {
      set_error("plhr_batch_create: sigma must be finite");
      return PLHR_ERR_ARG;
    }
    if ((size_t)m > (size_t)a.nx * a.ny) {
      set_error("plhr_batch_create: 4*(k + k_extra) exceeds a problem's size");
      return PLHR_ERR_ARG;
    }
    if (mg && (a.nx % f || a.ny % f || (a.nx / f) * (a.ny / f) > 1024)) {
      set_error("plhr_batch_create: grid dimensions must be divisible by 2^(levels-1) and the "
                "coarsest level at most 1024 points");
      return PLHR_ERR_ARG;
    }
  }
  plhr_batch_s* c = new plhr_batch_s();
  c->nb = nbatch;
  c->k = k;
  c->kint = kint;
  c->m = m;
  c->mg = mg;
  c->levels = levels;
  if (mg) {
    c->nu = T->nu_pre;
    c->omega = T->omega;
  }
  c->opt = o;
  c->stream = (hipStream_t)stream;
  c->g0 = make_grid(&A[0]);
  for (int b = 0; b < nbatch; ++b) {
    c->nx.push_back(A[b].nx);
    c->ny.push_back(A[b].ny);
    c->off.push_back(c->ntot);
    c->ntot += (size_t)A[b].nx * A[b].ny;
    c->sigma.push_back(sigma[b]);
    c->pot_dev.push_back(A[b].potential);
  }
  // level sizes
  c->ntot_l.assign(levels, 0);
  std::vector<std::vector<BLev>> lvh(levels, std::vector<BLev>(nbatch));
  for (int l = 0; l < levels; ++l) {
    size_t o2 = 0;
    for (int b = 0; b < nbatch; ++b) {
      lvh[l][b] = BLev{c->nx[b] >> l, c->ny[b] >> l, o2};
      o2 += (size_t)(c->nx[b] >> l) * (c->ny[b] >> l);
    }
    c->ntot_l[l] = o2;
  }
  // device memory
  const size_t n = c->ntot;
  c->max_chunks = 0;
  for (int b = 0; b < nbatch; ++b) c->max_chunks += (c->nx[b] * c->ny[b] + 511) / 512;
  size_t bytes = 0;
  auto take = [&](size_t b) {
    size_t o2 = bytes;
    bytes += al(b);
    return o2;
  };
  const size_t oZ = take(n * m * 8), oQZ = take(n * m * 8), oTQZ = take(n * m * 8);
  const size_t oR = take(n * 2 * kint * 8), oQVf = take(n * kint * 8);
  const size_t oVf = take(n * k * 8), oQVfin = take(n * k * 8);
  std::vector<size_t> olx(levels), olt(levels), olr(levels);
  for (int l = 0; l < levels; ++l) {
    olx[l] = take(c->ntot_l[l] * 2 * kint * 8);
    olt[l] = take(c->ntot_l[l] * 2 * kint * 8);
    olr[l] = take(c->ntot_l[l] * 2 * kint * 8);
  }
  const size_t opart = take((size_t)c->max_chunks * 2 * kint * 8);
  const size_t ogp = take((size_t)c->max_chunks * m * 2 * m * 8);
  const size_t NB = nbatch;
  const size_t oG = take(NB * m * m * 8), oM = take(NB * m * m * 8),
               oGLR = take(NB * 2 * m * m * 8), oY = take(NB * m * kint * 8),
               olam = take(NB * kint * 8), orel = take(NB * kint * 8), oxi = take(NB * 2 * m * 8),
               ofC = take(NB * kint * kint * 8), ofth = take(NB * kint * 8),
               ovbv = take(NB * kint * 8), owork = take(NB * 4 * m * m * 8),
               oHM = take(NB * 2 * kint * kint * 8);
  const size_t okeep = take(NB * m * 4), oact = take(NB * kint * 4), okind = take(NB * kint * 4),
               opair = take(NB * kint * 4);
  const size_t ost = take(NB * sizeof(DevStatus));
  const size_t opr = take(NB * sizeof(BProb)), oprF = take(NB * sizeof(BProb));
  std::vector<size_t> olv(levels), orm(levels);
  c->nrows.assign(levels, 0);
  for (int l = 0; l < levels; ++l) {
    olv[l] = take(NB * sizeof(BLev));
    int rows = 0;
    for (int b = 0; b < nbatch; ++b) rows += c->ny[b] >> l;
    c->nrows[l] = rows;
    orm[l] = take((size_t)rows * sizeof(RowMap));
  }
  const size_t och = take((size_t)c->max_chunks * sizeof(Chunk));
  const size_t obs = take(NB * sizeof(BatchSmall)), obsF = take(NB * sizeof(BatchSmall));
  const size_t oinv = take(NB * sizeof(double*)), osrc = take(NB * sizeof(double*)),
               odst = take(NB * sizeof(double*)), ovbvp = take(NB * sizeof(double*));
  // coarse inverses, one per distinct coarsest grid (the size query only
  // counts their bytes)
  std::map<std::pair<int, int>, std::vector<double>> invs;
  std::map<std::pair<int, int>, size_t> inv_off;
  if (mg) {
    const Grid gc0 = level_grid(c, levels - 1);
    for (int b = 0; b < nbatch; ++b) {
      auto key = std::make_pair(lvh[levels - 1][b].nx, lvh[levels - 1][b].ny);
      if (invs.count(key)) continue;
      Grid gc = gc0;
      gc.nx = key.first;
      gc.ny = key.second;
      gc.nz = 1;
      std::vector<double> inv;
      if (size_only) {
        inv.assign(gc.n() * gc.n(), 0.0);
      } else if (!coarse_inverse(gc, inv)) {
        set_error("coarsest multigrid operator is not positive definite");
        delete c;
        return PLHR_ERR_NOT_HPD;
      }
      inv_off[key] = take(inv.size() * 8);
      invs[key] = std::move(inv);
    }
  }
  if (size_only) {
    *size_only = bytes;
    delete c;
    return PLHR_OK;
  }
  hipError_t e = hipSuccess;
  if (workspace) {
    if (ws_bytes < bytes || ((uintptr_t)workspace & 255)) {
      set_error("plhr_batch_create: the workspace must hold plhr_batch_workspace_size bytes "
                "and be 256-byte aligned");
      delete c;
      return PLHR_ERR_ARG;
    }
    c->ws = static_cast<char*>(workspace);
    c->own_ws = false;
  } else {
    e = hipMalloc((void**)&c->ws, bytes);
    if (e != hipSuccess) {
      set_error(std::string("plhr_batch_create: hipMalloc failed: ") + hipGetErrorString(e));
      delete c;
      return PLHR_ERR_HIP;
    }
  }
  e = hipHostMalloc((void**)&c->st_host, NB * sizeof(DevStatus), hipHostMallocDefault);
  if (e != hipSuccess) {
    set_error("plhr_batch_create: pinned status buffer");
    plhr_batch_destroy(c);
    return PLHR_ERR_HIP;
  }
  char* w = c->ws;
  c->Z = (double*)(w + oZ);
  c->QZ = (double*)(w + oQZ);
  c->TQZ = (double*)(w + oTQZ);
  c->R = (double*)(w + oR);
  c->QVf = (double*)(w + oQVf);
  c->Vfin = (double*)(w + oVf);
  c->QVfin = (double*)(w + oQVfin);
  for (int l = 0; l < levels; ++l) {
    c->lx.push_back((double*)(w + olx[l]));
    c->lt.push_back((double*)(w + olt[l]));
    c->lr.push_back((double*)(w + olr[l]));
  }
  c->part = (double*)(w + opart);
  c->gpart = (double*)(w + ogp);
  c->G = (double*)(w + oG);
  c->M = (double*)(w + oM);
  c->GLR = (double*)(w + oGLR);
  c->Y = (double*)(w + oY);
  c->lam = (double*)(w + olam);
  c->relres = (double*)(w + orel);
  c->xi = (double*)(w + oxi);
  c->fC = (double*)(w + ofC);
  c->fth = (double*)(w + ofth);
  c->vbv = (double*)(w + ovbv);
  c->work = (double*)(w + owork);
  c->HM = (double*)(w + oHM);
  c->keep = (int*)(w + okeep);
  c->active = (int*)(w + oact);
  c->kinds = (int*)(w + okind);
  c->pair = (int*)(w + opair);
  c->st = (DevStatus*)(w + ost);
  c->pr = (BProb*)(w + opr);
  c->prF = (BProb*)(w + oprF);
  for (int l = 0; l < levels; ++l) {
    c->lv.push_back((BLev*)(w + olv[l]));
    c->rm.push_back((RowMap*)(w + orm[l]));
  }
  c->ch = (Chunk*)(w + och);
  c->bs = (BatchSmall*)(w + obs);
  c->bsF = (BatchSmall*)(w + obsF);
  c->inv = (const double**)(w + oinv);
  c->src = (const double**)(w + osrc);
  c->dst = (double**)(w + odst);
  c->vbvp = (const double**)(w + ovbvp);
  plhr_status s = PLHR_OK;
  do {
    // host tables
    std::vector<BProb> prh(nbatch), prfh(nbatch);
    std::vector<BatchSmall> bsh(nbatch);
    std::vector<const double*> invp(nbatch, nullptr), vbvp(nbatch);
    for (int b = 0; b < nbatch; ++b) {
      Grid gb = c->g0;
      gb.nx = c->nx[b];
      gb.ny = c->ny[b];
      gb.nz = 1;
      std::vector<double> pot;
      if (c->pot_dev[b]) {
        pot.resize(gb.n());
        e = hipMemcpy(pot.data(), c->pot_dev[b], gb.n() * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
          set_error("plhr_batch_create: cannot read a potential");
          s = PLHR_ERR_HIP;
          break;
        }
      }
      SmallParams sp{};
      sp.kint = kint;
      sp.k = k;
      sp.m = m;
      sp.sigma = sigma[b];
      sp.tol = o.tol;
      sp.normA1 = exact_norm1(gb, pot);
      sp.normB1 = 1.0;
      sp.drop_tol = o.drop_tol;
      sp.lock = o.lock;
      SmallBufs sb{};
      sb.G = c->G + (size_t)b * m * m;
      sb.M = c->M + (size_t)b * m * m;
      sb.GLR = c->GLR + (size_t)b * 2 * m * m;
      sb.Y = c->Y + (size_t)b * m * kint;
      sb.lam = c->lam + (size_t)b * kint;
      sb.relres = c->relres + (size_t)b * kint;
      sb.xi = c->xi + (size_t)b * 2 * m;
      sb.keep = c->keep + (size_t)b * m;
      sb.active = c->active + (size_t)b * kint;
      sb.kinds = c->kinds + (size_t)b * kint;
      sb.pair = c->pair + (size_t)b * kint;
      sb.final_C = c->fC + (size_t)b * kint * kint;
      sb.final_theta = c->fth + (size_t)b * kint;
      sb.vbv = c->vbv + (size_t)b * kint;
      sb.work = c->work + (size_t)b * 4 * m * m;
      sb.scratch = nullptr;
      bsh[b] = BatchSmall{sp, sb, c->st + b, nullptr, 0, c->HM + (size_t)b * 2 * kint * kint};
      prh[b] = BProb{c->nx[b], c->ny[b], c->off[b], c->pot_dev[b], sigma[b], sb.lam,
                     c->st + b, 0, 0};
      prfh[b] = prh[b];
      prfh[b].lam = sb.final_theta;
      vbvp[b] = sb.vbv;
      if (mg) {
        auto key = std::make_pair(lvh[levels - 1][b].nx, lvh[levels - 1][b].ny);
        invp[b] = (const double*)(w + inv_off[key]);
      }
    }
    if (s != PLHR_OK) break;
    std::vector<std::vector<RowMap>> rmh(levels);
    for (int l = 0; l < levels; ++l)
      for (int b = 0; b < nbatch; ++b)
        for (int j = 0; j < (c->ny[b] >> l); ++j) rmh[l].push_back(RowMap{b, j});
#define UP(dst, src, bytes_)                                                            \
  e = hipMemcpy((void*)(dst), (const void*)(src), (bytes_), hipMemcpyHostToDevice);   \
  if (e != hipSuccess) {                                                               \
    set_error(std::string("plhr_batch_create: upload: ") + hipGetErrorString(e));     \
    s = PLHR_ERR_HIP;                                                                  \
    break;                                                                             \
  }
    UP(c->pr, prh.data(), NB * sizeof(BProb));
    UP(c->prF, prfh.data(), NB * sizeof(BProb));
    UP(c->bs, bsh.data(), NB * sizeof(BatchSmall));
    UP(c->inv, invp.data(), NB * sizeof(double*));
    UP(c->vbvp, vbvp.data(), NB * sizeof(double*));
    for (int l = 0; l < levels; ++l) {
      UP(c->lv[l], lvh[l].data(), NB * sizeof(BLev));
      UP(c->rm[l], rmh[l].data(), rmh[l].size() * sizeof(RowMap));
    }
    if (s != PLHR_OK) break;
    for (auto& kv : invs) UP(w + inv_off[kv.first], kv.second.data(), kv.second.size() * 8);
#undef UP
    if (s != PLHR_OK) break;
    s = upload_tables(c, 1024);
    if (s != PLHR_OK) break;
    e = small_set_attributes(m, kint);
    if (e == hipSuccess) e = mfma_set_attributes(m, kint);
    if (e == hipSuccess) e = batch_set_attributes(m);
    if (e != hipSuccess) {
      set_error(std::string("LDS attribute: ") + hipGetErrorString(e));
      s = PLHR_ERR_HIP;
    }
  } while (false);
  if (s != PLHR_OK) {
    plhr_batch_destroy(c);
    return s;
  }
  *out = c;
  return PLHR_OK;
}

}  // namespace

extern "C" {

plhr_status plhr_batch_workspace_size(int32_t nbatch, const plhr_op_desc* A,
                                      const plhr_prec_desc* T, const double* sigma, int32_t k,
                                      const plhr_options* opt, size_t* ws_bytes) {
  if (!ws_bytes) {
    set_error("plhr_batch_workspace_size: ws_bytes is NULL");
    return PLHR_ERR_ARG;
  }
  return batch_create_impl(nbatch, A, T, sigma, k, opt, nullptr, nullptr, 0, ws_bytes, nullptr);
}

plhr_status plhr_batch_create(int32_t nbatch, const plhr_op_desc* A, const plhr_prec_desc* T,
                              const double* sigma, int32_t k, const plhr_options* opt,
                              void* stream, void* workspace, size_t ws_bytes, plhr_batch* out) {
  return batch_create_impl(nbatch, A, T, sigma, k, opt, stream, workspace, ws_bytes, nullptr,
                           out);
}

plhr_status plhr_batch_solve(plhr_batch c, const double* const* V0, double* eigvals,
                             double* const* V, double* rel_res, int32_t* iters,
                             int32_t* status) {
  if (!c || !V0) {
    set_error("plhr_batch_solve: NULL argument");
    return PLHR_ERR_ARG;
  }
  for (int b = 0; b < c->nb; ++b)
    if (!V0[b]) {
      set_error("plhr_batch_solve: NULL start block");
      return PLHR_ERR_ARG;
    }
  ProfScopeB prof_scope(c);
  c->finished = false;
  plhr_status s = start_b(c, V0);
  if (s != PLHR_OK) return s;
  if (!c->tuned) {
    s = autotune(c);
    if (s != PLHR_OK) return s;
    // the timing runs overwrote scratch: start again
    s = start_b(c, V0);
    if (s != PLHR_OK) return s;
  }
  const bool graphs = c->use_graph && c->prof.cat == -2;
  if (graphs && !c->gexec[0]) {
    s = capture_graphs(c);
    if (s != PLHR_OK) return s;
  }
  int it = 0;
  while (it < c->opt.max_iters) {
    const int chunk = std::min(c->opt.check_every, c->opt.max_iters - it);
    for (int i = 0; i < chunk; ++i, ++it) {
      const bool refresh = (it % kRefreshB == kRefreshB - 1);
      if (graphs)
        PLHR_HIP_CHECK(hipGraphLaunch(c->gexec[refresh ? 1 : 0], c->stream));
      else
        enqueue_iteration_b(c, refresh);
    }
    PLHR_HIP_CHECK(hipGetLastError());
    s = read_status_b(c);
    if (s != PLHR_OK) return s;
    bool all = true;
    for (int b = 0; b < c->nb; ++b)
      if (!c->st_host[b].done && !c->st_host[b].error) all = false;
    if (all) break;
  }
  std::vector<int> conv(c->nb), err(c->nb), its(c->nb);
  for (int b = 0; b < c->nb; ++b) {
    conv[b] = c->st_host[b].done;
    err[b] = c->st_host[b].error;
    its[b] = c->st_host[b].iter;
  }
  s = finish_b(c);
  if (s != PLHR_OK) return s;
  const int k = c->k, kint = c->kint;
  if (eigvals)
    PLHR_HIP_CHECK(hipMemcpy2DAsync(eigvals, k * sizeof(double), c->fth, kint * sizeof(double),
                                    k * sizeof(double), c->nb, hipMemcpyDeviceToDevice,
                                    c->stream));
  if (V) {
    PLHR_HIP_CHECK(hipMemcpyAsync(c->dst, V, c->nb * sizeof(double*), hipMemcpyHostToDevice,
                                  c->stream));
    launch_copy_out_b(c->ch, c->nch, c->pr, c->Vfin, k, k, c->dst, c->stream);
  }
  std::vector<double> rr((size_t)c->nb * kint);
  PLHR_HIP_CHECK(hipMemcpyAsync(rr.data(), c->relres, rr.size() * sizeof(double),
                                hipMemcpyDeviceToHost, c->stream));
  PLHR_HIP_CHECK(hipStreamSynchronize(c->stream));
  PLHR_HIP_CHECK(hipGetLastError());
  plhr_status ret = PLHR_OK;
  int first_bad = -1;
  for (int b = 0; b < c->nb; ++b) {
    if (rel_res)
      for (int j = 0; j < k; ++j) rel_res[(size_t)b * k + j] = rr[(size_t)b * kint + j];
    if (iters) iters[b] = its[b];
    int sb = err[b] ? err[b] : (conv[b] ? PLHR_OK : PLHR_ERR_NOT_CONVERGED);
    if (c->st_host[b].error && !err[b]) sb = c->st_host[b].error;  // failed in the final step
    if (status) status[b] = sb;
    if (sb != PLHR_OK && (ret == PLHR_OK || ret == PLHR_ERR_NOT_CONVERGED)) ret = (plhr_status)sb;
    if (sb != PLHR_OK && sb != PLHR_ERR_NOT_CONVERGED && first_bad < 0) first_bad = b;
  }
  if (ret != PLHR_OK && ret != PLHR_ERR_NOT_CONVERGED)
    set_error("plhr_batch_solve: problem " + std::to_string(first_bad) + " failed: " +
              reason_text(c->st_host[first_bad].reason) + " (iteration " +
              std::to_string(c->st_host[first_bad].iter) + "; see the per-problem status)");
  else if (ret == PLHR_ERR_NOT_CONVERGED)
    set_error("plhr_batch_solve: some problems did not converge within max_iters");
  c->finished = true;
  return ret;
}

plhr_status plhr_batch_eigvals_backward(plhr_batch c, const double* dL_dlambda,
                                        double* const* dL_dpot, int32_t accumulate) {
  if (!c || !dL_dlambda || !dL_dpot) {
    set_error("plhr_batch_eigvals_backward: NULL argument");
    return PLHR_ERR_ARG;
  }
  if (!c->finished) {
    set_error("plhr_batch_eigvals_backward before plhr_batch_solve");
    return PLHR_ERR_STATE;
  }
  for (int b = 0; b < c->nb; ++b)
    if (!dL_dpot[b]) {
      set_error("plhr_batch_eigvals_backward: NULL gradient buffer");
      return PLHR_ERR_ARG;
    }
  PLHR_HIP_CHECK(hipMemcpyAsync(c->dst, dL_dpot, c->nb * sizeof(double*), hipMemcpyHostToDevice,
                                c->stream));
  launch_hf_b(c->ch, c->nch, c->pr, c->Vfin, c->k, c->k, dL_dlambda, c->vbvp, c->dst, accumulate,
              c->stream);
  PLHR_HIP_CHECK(hipStreamSynchronize(c->stream));
  PLHR_HIP_CHECK(hipGetLastError());
  return PLHR_OK;
}

plhr_status plhr_batch_apply(plhr_batch c, int32_t which, const double* const* X,
                             double* const* Y, int32_t ncols) {
  if (!c || !X || !Y || ncols < 1 || ncols > 2 * c->kint || which < 0 || which > 2) {
    set_error("plhr_batch_apply: bad argument (which 0..2, 1 <= ncols <= 2 kint)");
    return PLHR_ERR_ARG;
  }
  ProfScopeB prof_scope(c);
  hipStream_t s = c->stream;
  // no problem is halted while the operator is applied
  PLHR_HIP_CHECK(hipMemsetAsync(c->st, 0, c->nb * sizeof(DevStatus), s));
  PLHR_HIP_CHECK(hipMemcpyAsync(c->src, X, c->nb * sizeof(double*), hipMemcpyHostToDevice, s));
  PLHR_HIP_CHECK(hipMemcpyAsync(c->dst, Y, c->nb * sizeof(double*), hipMemcpyHostToDevice, s));
  launch_copy_in_b(c->ch, c->nch, c->pr, c->src, ncols, c->R, ncols, s);
  const Blk none{nullptr, 0};
  if (which == 2)
    precond_b(c, c->R, ncols, Blk{c->Z, ncols}, none, ncols, ncols);
  else
    fd_b(c, c->R, ncols, Blk{c->Z, ncols}, none, none, ncols, which, c->pr);
  launch_copy_out_b(c->ch, c->nch, c->pr, c->Z, ncols, ncols, c->dst, s);
  PLHR_HIP_CHECK(hipStreamSynchronize(s));
  PLHR_HIP_CHECK(hipGetLastError());
  return PLHR_OK;
}

plhr_status plhr_batch_tuning_info(plhr_batch c, plhr_batch_tuning* out) {
  if (!c || !out) {
    set_error("plhr_batch_tuning_info: NULL argument");
    return PLHR_ERR_ARG;
  }
  std::memset(out, 0, sizeof(*out));
  out->chunk_points = c->chunk_pts;
  out->row_threads = c->row_threads;
  out->use_graph = c->use_graph ? 1 : 0;
  out->nchunks = c->nch;
  for (int i = 0; i < 8; ++i) out->tuned_ms[i] = c->tuned_ms[i];
  return PLHR_OK;
}

plhr_status plhr_batch_set_graph(plhr_batch c, int32_t use_graph) {
  if (!c) {
    set_error("plhr_batch_set_graph: NULL batch");
    return PLHR_ERR_ARG;
  }
  c->use_graph = use_graph != 0;
  return PLHR_OK;
}

plhr_status plhr_batch_profile_start(plhr_batch c, int32_t category, int32_t max_launches) {
  if (!c) {
    set_error("plhr_batch_profile_start: NULL batch");
    return PLHR_ERR_ARG;
  }
  return prof_start(c->prof, category, max_launches);
}

plhr_status plhr_batch_profile_stop(plhr_batch c, plhr_profile* out) {
  if (!c || !out) {
    set_error("plhr_batch_profile_stop: NULL argument");
    return PLHR_ERR_ARG;
  }
  return prof_stop(c->prof, c->stream, out);
}

void plhr_batch_destroy(plhr_batch c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  destroy_graphs(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  prof_release(c->prof);
  if (c->ws && c->own_ws) (void)hipFree(c->ws);
  if (c->st_host) (void)hipHostFree(c->st_host);
  delete c;
}

}  // extern "C"
