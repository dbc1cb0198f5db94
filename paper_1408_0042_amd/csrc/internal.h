// Internal declarations shared by the HIP translation units of libplhr.
// Kernels live next to their host-side launchers; the driver (api.hip)
// only calls launchers, so no relocatable device code is needed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <string>
#include <vector>

#include "../../include/plhr.h"

namespace plhr {

// Largest trial-subspace width m = 4 (k + k_extra) handled on chip: the
// projected eigensolver keeps two m x m matrices and the selected vectors
// of the m x m problem in one workgroup's LDS (160 KiB on gfx950).
constexpr int kMaxM = 84;

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);

#define PLHR_HIP_CHECK(expr)                                                    \
  do {                                                                          \
    hipError_t _e = (expr);                                                     \
    if (_e != hipSuccess) {                                                     \
      ::plhr::set_error(std::string("HIP error in ") + #expr + ": " +          \
                        hipGetErrorString(_e));                                 \
      return PLHR_ERR_HIP;                                                      \
    }                                                                           \
  } while (0)

// ------------------------------------------------------------ device status
// One word block in device memory; every iteration kernel reads `done` and
// `error` first and returns at once when either is set, so that iterations
// enqueued past convergence leave the state untouched.
struct DevStatus {
  int done;          // the k wanted pairs met tol
  int error;         // nonzero plhr_status raised on the device
  int iter;          // iterations completed since start
  int n_active;      // columns generating W/S/P in the current iteration
  int m_kept;        // columns kept by the last B-orthonormalisation
  int have_p;        // the P block holds a conjugate direction
  int n_dropped;     // columns dropped by the last orthonormalisation
  int reason;        // which check raised `error` (kReason*)
  int n_excluded;    // slots left out of projected problems so far (G_L pivot < 0)
  int pad0;
  double max_rel_res;  // largest relative residual among the k wanted
  double reserved[3];
  long long tphase[12];  // clock stamps of the projected-solver phases
};

enum : int {
  kReasonNone = 0,
  kReasonStartRank = 1,   // the start block is rank deficient
  kReasonQR = 2,          // the projected eigensolver did not converge
  kReasonNonFinite = 3,   // a wanted residual is not finite
  kReasonFinalGram = 4,   // V^T B V of the final Rayleigh-Ritz is not HPD
  kReasonVVanished = 5    // every column of V became dependent
};
// Text of a DevStatus reason code (for error messages).
const char* reason_text(int reason);

// ---------------------------------------------------- launch profiling
// Kernel categories for per-launch HIP-event timing.  When a context turns
// profiling on for one category, every launch of that category is
// bracketed by two events on its stream and its algorithmic bytes and
// flops (what the operation must read, write and compute, not what the
// hardware moves) are accumulated.
enum KCat : int {
  KC_STENCIL = 0,        // operator block products (k_fd_apply)
  KC_JACOBI = 1,         // V-cycle weighted-Jacobi sweeps
  KC_RESIDUAL = 2,       // V-cycle residual before restriction
  KC_RESTRICT = 3,       // V-cycle restriction
  KC_PROLONG = 4,        // V-cycle prolongation and correction
  KC_COARSE = 5,         // V-cycle coarsest-level dense solve
  KC_GRAM = 6,           // Gram products (per-workgroup partials)
  KC_GRAM_REDUCE = 7,    // reduction of the Gram partials
  KC_TRANSFORM = 8,      // orthonormalising transform Z <- Z M
  KC_UPDATE = 9,         // block update V, P <- Zhat Y'
  KC_THARM_REDUCE = 10,  // Cholesky of G_L, C, Hessenberg reduction
  KC_THARM_QR = 11,      // Francis QR of the Hessenberg matrix
  KC_THARM_VECTORS = 12, // selection and eigenvectors of the projected problem
  KC_ORTHO = 13,         // Cholesky-QR factor of the Gram of Z
  KC_SMALL = 14,         // other single-workgroup kernels (RQ, convergence)
  KC_VEC = 15,           // residual formation, column reductions, copies
  KC_COUNT = 16  // PLHR_KC_COUNT
};
// Per-launch event profiling (see KCat): the entry points attach the
// active context's recorder for the duration of each call.
struct Prof {
  int cat = -2;  // -1: all categories; -2: off
  std::vector<hipEvent_t> ev;
  std::vector<int> evcat;
  size_t used = 0;
  double bytes[KC_COUNT] = {0}, flops[KC_COUNT] = {0};
  long launches[KC_COUNT] = {0};
  bool skip_end = false;
};
void prof_attach(Prof* p);
plhr_status prof_start(Prof& p, int category, int max_launches);
plhr_status prof_stop(Prof& p, hipStream_t stream, plhr_profile* out);
void prof_release(Prof& p);
void prof_begin(int cat, double bytes, double flops, hipStream_t s);
void prof_end(int cat, hipStream_t s);

// --------------------------------------------------------------- geometry
struct Grid {
  int nx = 1, ny = 1, nz = 1;
  int dim = 2;
  double h = 1.0;
  double scale = 1.0;
  // bilinear/trilinear finite elements (interior nodes, element size h);
  // the multigrid preconditioner still uses the finite-difference
  // Laplacian of this grid (diag/off below), a spectrally equivalent HPD T
  bool q1 = false;
  size_t n() const { return (size_t)nx * ny * nz; }
  double diag() const { return scale * 2.0 * dim / (h * h); }
  double off() const { return -scale / (h * h); }
};

// A block descriptor: element (p, c) lives at ptr[p * ld + c].
struct Blk {
  double* ptr;
  int ld;
};

// ------------------------------------------------------------- launchers
// Stencil: out = scale*(-Lap)X + pot.*X - shift*X  (shift = sigma for
// (A - sigma I)X, 0 for AX).  With sc != null (n doubles) the operator is
// S A S - shift I, S = diag(sc).  Optional extra outputs:
//   out_r (if ptr != null): out_r[:, c] = out[:, c] - X[:, c] * (colshift[c] - csub)
//   out_c (if ptr != null): out_c[:, c] = out[:, c]
void launch_fd_apply(const Grid& g, const double* pot, const double* sc, double shift,
                     const double* X, int ldx, Blk out, Blk out_r, const double* colshift,
                     double csub, Blk out_c, int ncols, const DevStatus* st, hipStream_t s);

// Q1 finite elements: stencil weights of scale*K and of M by offset
// (dz+1)*9 + (dy+1)*3 + (dx+1); out = (A - shift B)X with B = M when
// bmass (else I); extra outputs as for launch_fd_apply plus out_b = B X;
// out_r subtracts (B X)(colshift - csub).
struct Q1Weights {
  double a[27];
  double m[27];
};
Q1Weights q1_weights(const Grid& g);
void launch_q1_apply(const Grid& g, const double* pot, double shift, bool bmass, const double* X,
                     int ldx, Blk out, Blk out_r, const double* colshift, double csub, Blk out_c,
                     Blk out_b, int ncols, const DevStatus* st, hipStream_t s);

// General sparse matrix (CSR, device arrays); row_ptr null means absent.
struct CsrMat {
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const double* values;
  long long nnz;
};
void launch_csr_apply(int n, const CsrMat& A, const CsrMat& B, const double* pot, double shift,
                      const double* X, int ldx, Blk out, Blk out_r, const double* colshift,
                      double csub, Blk out_c, Blk out_b, int ncols, const DevStatus* st,
                      hipStream_t s);
// Y = (scale (-Laplacian_theta) + diag(pot) - shift I) X on a Bloch-periodic
// box, complex128 blocks (interleaved re, im), n x ncols point-major with
// row strides ldx, ldy in complex entries (<= 0: ncols); nothing when st
// is halted.
void launch_bloch_apply(int nx, int ny, int nz, double h, double scale, const double* theta,
                        const double* pot, double shift, const double* X, double* Y, int ncols,
                        hipStream_t s, int ldx = 0, int ldy = 0, const DevStatus* st = nullptr);
// One V-cycle of a Bloch preconditioner handle on stream s: Y = T X for
// ncols complex columns, X with row stride ldx, the result's columns
// c < split to Y0 (stride ld0), the others to Y1 (stride ld1) at column
// c - split (strides in complex entries; no overlap of X with Y0, Y1).
void bloch_prec_cycle(plhr_bloch_prec p, const double* X, int ldx, double* Y0, int ld0,
                      double* Y1, int ld1, int split, int ncols, hipStream_t s);
// Bloch V-cycle pieces (complex128 blocks, n_l x ncols point-major):
// out = alpha w + beta (r - A_l w) with A_l the level's Bloch stencil of
// coefficient cs = scale/h_l^2 (w = NULL: w = 0); rc = P^H res / 8 onto the
// coarse grid nxc x nyc x nzc; x += P ec on the fine grid nx x ny x nz;
// x = Ainv r on the coarsest level.
// Row strides (complex entries; <= 0: ncols) of a level kernel's w, r and
// out, and a second output: columns c >= split go to out1 (stride o1) at
// column c - split (out1 = null: every column to out).
struct BlochLd {
  int w = 0, r = 0, o = 0;
  double* out1 = nullptr;
  int o1 = 0, split = 0;
};
void launch_bloch_level(int nx, int ny, int nz, double cs, const double* theta, const double* w,
                        const double* r, double alpha, double beta, double* out, int ncols,
                        hipStream_t s, const BlochLd& ld = BlochLd{});
void launch_bloch_restrict(int nxc, int nyc, int nzc, const double* theta, const double* res,
                           double* rc, int ncols, hipStream_t s);
void launch_bloch_prolong_add(int nx, int ny, int nz, const double* theta, const double* ec,
                              double* x, int ncols, hipStream_t s);
void launch_bloch_dense(int nc, const double* Ainv, const double* r, double* x, int ncols,
                        hipStream_t s, const BlochLd& ld = BlochLd{});

// Multigrid V-cycle (k_mg.hip).
struct MGLevel {
  Grid g;
  double* x = nullptr;   // n_l x cmax
  double* t = nullptr;   // n_l x cmax
  double* r = nullptr;   // n_l x cmax (levels > 0)
  // three more blocks on every level of AV-MG / INV-MG (the Chebyshev
  // recurrence of a polynomial level: two terms and the sum)
  double* u0 = nullptr;
  double* u1 = nullptr;
  double* u2 = nullptr;
  // level operator B_l: 0 the Laplacian L_l, 1 L_l - sigma I, 2 the
  // polynomial p_m(L_l - sigma I); shift is subtracted from the stencil's
  // diagonal (kinds 1 and 2); w is the Richardson weight of the smoother
  int kind = 0;
  double shift = 0.0;
  double w = 0.0;
  int vtx = 0;  // the transfer to the next coarser level is vertex-centred
  std::vector<double> cheb;   // kind 2: Chebyshev coefficients c_0 .. c_m
  double ca = 0.0, cb = 0.0;  // kind 2: X = ca (L_l - sigma I) + cb I
};
// Appendix A variants: mode 0 the plain V-cycle, 1 AV-MG (Algorithm 4),
// 2 INV-MG (Algorithm 5).
struct MGOpts {
  int mode = 0;
  double sigma = 0.0;
  double delta = 0.6;
  int degree = 10;
};
struct MG {
  int levels = 0, nu_pre = 2, nu_post = 2;
  double omega = 2.0 / 3.0;
  int cmax = 0;
  MGOpts av;
  std::vector<MGLevel> lv;
  double* coarse_inv = nullptr;  // nc x nc, row-major
  float* coarse_inv32 = nullptr;  // the same in FP32
  int nc = 0;
};
// The next coarser grid of a hierarchy: all (active) dimensions even pair
// neighbouring points (cell-centred, n -> n/2); all odd and >= 3 keep every
// other point (vertex-centred, n -> (n - 1)/2, *vtx = 1); h doubles.
// False when neither applies.
bool mg_coarsen(Grid& g, int* vtx);
size_t mg_workspace_bytes(const Grid& fine, int levels, int cmax, int mode = 0);
plhr_status mg_setup(MG& mg, const Grid& fine, int levels, int nu_pre, int nu_post, double omega,
                     int cmax, char*& ws, hipStream_t s, const MGOpts& av = MGOpts{});
// X_out = T R (ncols columns).  Output may be split over two blocks:
// columns [0, split) go to out0, [split, ncols) to out1.  f32: level
// storage and arithmetic in FP32 (FP64 input and output).
void mg_apply(MG& mg, const double* R, int ldr, Blk out0, Blk out1, int split, int ncols,
              bool f32, const DevStatus* st, hipStream_t s);

// Dense level-0 helpers (k_blas.hip)
// residual prep: R[:, c] = QV[:, c] - V[:, c] * (lam[c] - sigma); partial
// sums of |R|^2 and |V|^2 per column per block written to part
// (nblk x 2c); with row weights bw != null, of bw.*R^2 and V^2./bw.
// Returns the number of blocks used.
// BV != null (ld ldb) replaces V in the shift term: R = QV - BV (lam - sigma).
int launch_resid_prep(size_t n, const double* V, int ldv, const double* QV, int ldq,
                      const double* lam, double sigma, double* R, int ldr, int ncols,
                      const double* bw, const double* BV, int ldb, double* part,
                      const DevStatus* st, hipStream_t s);
int resid_prep_blocks(size_t n);

// Split-K Gram: out(i, j) = sum_p X[p, i] * Y[p, j] for i < mx, j < my,
// where the Y columns come from up to two blocks: columns [0, my1) of Y1
// followed by [0, my - my1) of Y2.  If qshift != 0 the first block is
// formed on the fly as Y1 - qshift * Yq (Yq has the same ld as Y1).
// Partials go to part (nblk x mx x my), then a second kernel reduces them
// in a fixed order into out (mx x my, row-major).
void launch_gram(size_t n, const double* X, int ldx, int mx, const double* Y1, int ldy1,
                 int my1, const double* Y2, int ldy2, int my, double* part, int nblk, double* out,
                 const DevStatus* st, hipStream_t s);
int gram_blocks(size_t n);

// In-place right multiplication by an upper-triangular m x m matrix:
// X[p, :m] <- X[p, :m] * M for each of the nx arrays (row-wise, so
// in-place is safe).
void launch_transform(size_t n, double* const* X, int nx, int ld, int m, const double* M,
                      const DevStatus* st, hipStream_t s);

// Block update from the coefficient matrix Y (m x kc, row-major):
//   Vn = Zrow[:m] * Y ;  Pn = Zrow[kv:m] * Y[kv:m]
// written in place to columns [0,kc) (V) and [pcol, pcol+kc) (P) of the
// same arrays.  For array 0 also writes per-block partial column sums of
// v*v and v*(Q v) (from array 1) into part (nblk x 2kc).
int launch_update(size_t n, double* const* X, int nx, int ld, int m, int kv, const double* Y,
                  int kc, int pcol, double* part, const DevStatus* st, hipStream_t s);
int update_blocks(size_t n);

// Y[p, c] = X[p, c] * M  for dense (kin x kout) M; X ld ldx, Y ld ldy.
void launch_small_gemm(size_t n, const double* X, int ldx, int kin, const double* M, int kout,
                       double* Y, int ldy, hipStream_t s);

// copy n x c block with leading dimensions (nothing when st is halted)
void launch_copy(size_t n, const double* X, int ldx, double* Y, int ldy, int c, hipStream_t s,
                 const DevStatus* st = nullptr);
// Y = diag(w) X, n x c (Y may alias X with ldy == ldx; nothing when st is
// halted)
void launch_rowscale(size_t n, const double* w, const double* X, int ldx, double* Y, int ldy,
                     int c, hipStream_t s, const DevStatus* st = nullptr);

// column partial sums for final residuals (as launch_resid_prep, no R):
int launch_coldots(size_t n, const double* X, int ldx, const double* QX, int ldq, int c,
                   const double* lam, double sigma, const double* bw, const double* BX, int ldb,
                   double* part, hipStream_t s);

// partial column sums of x.(Bx) and x.y (nblk x 2c); BX null: B = I
int launch_xdots(size_t n, const double* X, int ldx, const double* Y, int ldy, int ncols,
                 double* part, hipStream_t s, const double* BX = nullptr, int ldb = 0);

// Hellmann-Feynman: g[x] (+)= sum_j dl[j] * V[x,j]^2 / vbv[j]
void launch_hf(size_t n, const double* V, int ldv, int k, const double* dl, const double* vbv,
               double* g, int accumulate, hipStream_t s);

// Up to four arrays processed by one row-product launch.
struct ArrPtrs {
  double* a[4];
  // element i by selects, not a dynamic index (which would copy the
  // by-value struct into scratch memory)
  __device__ __forceinline__ double* at(int i) const {
    return (i == 0) ? a[0] : (i == 1) ? a[1] : (i == 2) ? a[2] : a[3];
  }
};

// Matrix-core versions (k_mfma.hip); *_ok tells whether the shape fits.
int gram_mfma_ok(int mx, int my);
// G = X^H Y for complex128 blocks on the matrix cores (mx, my complex
// columns); ws holds cgram_workspace_bytes(n, mx, my) bytes.
size_t cgram_workspace_bytes(size_t n, int mx, int my);
void launch_cgram(size_t n, const double* X, int mx, const double* Y, int my, double* G,
                  double* ws, hipStream_t s);
// Complex Cholesky-QR tail: R and R^-1 from G = Z^H Z (one workgroup,
// m <= 64; *fail = 1 if G is not positive definite), then Q = Z R^-1.
hipError_t launch_cholqr_tail(size_t n, int m, const double* Z, const double* G, double* R,
                              double* Rinv, int* fail, double* Q, hipStream_t s);
// Y = Z M for complex128 blocks (Z n x m, M m x k row-major, m, k <= 64).
hipError_t launch_crowmul(size_t n, int m, int k, const double* Z, const double* M, double* Y,
                          hipStream_t s);
void launch_gram_mfma(size_t n, const double* X, int ldx, int mx, const double* Y1, int ldy1,
                      int my1, const double* Y2, int ldy2, int my, double* part, int nblk,
                      double* out, const DevStatus* st, hipStream_t s);
int rowmul_mfma_ok(int m, int kout);
void launch_rowmul_mfma(size_t n, double* const* X, int narr, int ld, int m, const double* M,
                        int kout, int mode, int kv, int kc, int pcol, double* part, int nblk,
                        const DevStatus* st, hipStream_t s);
hipError_t mfma_set_attributes(int m, int kint);

// Small single-workgroup kernels (k_small.hip)
struct SmallBufs {
  double* G;        // m x m
  double* M;        // m x m
  double* GLR;      // m x 2m : [G_L-ish | G_R] raw Gram output
  double* Y;        // m x kint
  double* lam;      // kint
  double* relres;   // kint
  double* xi;       // 2 x m (re, im) diagnostics
  int* keep;        // m
  int* active;      // kint
  int* kinds;       // kint
  int* pair;        // kint
  double* final_C;  // kint x kint
  double* final_theta;  // kint
  double* vbv;      // kint
  double* work;     // 4 m^2: projected-solver matrices between its kernels
  double* scratch;  // misc
  // automatic second Cholesky-QR pass: the first pass sets gate->done to 0
  // when it is needed (1 otherwise); the second pass's kernels take the
  // gate as their status word and return at once when it is 1
  DevStatus* gate = nullptr;
};

struct SmallParams {
  int kint, k, m;     // m = 4 * kint
  double sigma;
  double tol;
  double normA1, normB1;
  double drop_tol;
  int lock;
  int sym = 0;        // G_R symmetric (T = I or harmonic extraction, B = I)
  int pass = 0;       // Cholesky-QR pass with a gate: 1 first, 2 second; 0 none
  int cplx = 0;       // complex vectors as column pairs (re, im): 1 the
                      // single-vector iteration (Algorithm 1, kint = 2),
                      // 2 the complex block iteration (Algorithm 2)
  int plmr = 0;       // PLMR (Section 3.3): kint = 1, refinement extraction
};

// ------------------------------------------------------------- batches
// Many independent 2-D problems packed point-major one after another
// (k_batch.hip).  Tables built on the host, read by every batched launch.
struct BProb {
  int nx, ny;            // level-0 grid
  size_t off;            // first level-0 point of the problem in packed arrays
  const double* pot;     // potential (n_b values) or null
  double sigma;
  const double* lam;     // kint Rayleigh quotients used by residual epilogues
  const DevStatus* st;   // per-problem status (halted problems skip work)
  int ch0, nch;          // first point chunk and number of chunks
};
struct BLev {  // one problem at one multigrid level
  int nx, ny;
  size_t off;  // first point in the packed level arrays
};
struct RowMap {  // workgroup -> (problem, grid row)
  int b, j;
};
struct Chunk {  // workgroup -> (problem, local points [p0, p1))
  int b, p0, p1;
};

void launch_fd_b(const RowMap* rm, int nrows, const BProb* pr, double diag, double off,
                 int use_sigma, const double* X, int ldx, Blk out, Blk outr, Blk outc, int ncols,
                 int threads, hipStream_t s);
void launch_jacobi_b(const RowMap* rm, int nrows, const BLev* lv, const BProb* pr, double diag,
                     double off, double omega, const double* xin, const double* r, int ldr,
                     Blk o0, Blk o1, int split, int ncols, int threads, hipStream_t s);
void launch_residual_b(const RowMap* rm, int nrows, const BLev* lv, const BProb* pr,
                       double diag, double off, const double* x, const double* r, int ldr,
                       double* res, int ncols, int threads, hipStream_t s);
void launch_restrict_b(const RowMap* rmc, int ncrows, const BLev* lf, const BLev* lc,
                       const BProb* pr, const double* res, double* rc, int ncols, int threads,
                       hipStream_t s);
void launch_prolong_b(const RowMap* rm, int nrows, const BLev* lf, const BLev* lc,
                      const BProb* pr, const double* ec, double* x, int ncols, int threads,
                      hipStream_t s);
void launch_dense_b(int nb, const BLev* lv, const BProb* pr, const double* const* inv,
                    const double* r, double* x, int ncols, hipStream_t s);
void launch_xdots_b(const Chunk* ch, int nch, const BProb* pr, const double* X, int ldx,
                    const double* Y, int ldy, int ncols, double* part, hipStream_t s);
void launch_resid_b(const Chunk* ch, int nch, const BProb* pr, const double* V, int ldv,
                    const double* QV, int ldq, double* R, int ldr, int ncols, double* part,
                    hipStream_t s);
void launch_gram_b(const Chunk* ch, int nch, int nb, const BProb* pr, const double* X, int ldx,
                   int mx, const double* Y1, int ldy1, int my1, const double* Y2, int ldy2,
                   int my, double* gpart, double* out, size_t ostride, size_t ntot,
                   hipStream_t s);
void launch_rowmul_b(const Chunk* ch, int nch, const BProb* pr, double* const* X, int narr,
                     int ld, int m, const double* Mall, size_t mstride, int kout, int mode,
                     int kv, int kc, int pcol, double* part, size_t ntot, hipStream_t s);
void launch_small_gemm_b(const Chunk* ch, int nch, const BProb* pr, const double* X, int ldx,
                         int kin, const double* Call, size_t cstride, int kout, double* Y,
                         int ldy, hipStream_t s);
void launch_copy_in_b(const Chunk* ch, int nch, const BProb* pr, const double* const* src,
                      int c, double* Z, int ldz, hipStream_t s);
void launch_copy_out_b(const Chunk* ch, int nch, const BProb* pr, const double* X, int ldx,
                       int c, double* const* dst, hipStream_t s);
void launch_hf_b(const Chunk* ch, int nch, const BProb* pr, const double* V, int ldv, int k,
                 const double* dl, const double* const* vbv, double* const* g, int accumulate,
                 hipStream_t s);
hipError_t batch_set_attributes(int m);
Grid make_grid(const plhr_op_desc* A);
// max over rows of sum |A_ij| for the stencil plus potential (host)
double exact_norm1(const Grid& g, const std::vector<double>& pot);
// Inverse of the coarsest-level operator of a V-cycle on grid g (host,
// FP64); false if it is not positive definite.
bool coarse_inverse(const Grid& g, std::vector<double>& inv);

// One problem of a batch, for the batched single-workgroup kernels
// (workgroup b works on problem b).
struct BatchSmall {
  SmallParams p;
  SmallBufs b;
  DevStatus* st;
  const double* part;  // per-chunk partial column sums of this problem
  int nblk;            // number of chunks
  const double* HM;    // final Rayleigh-Ritz matrices
};
// Batched launchers (nb problems, device array bs).
void launch_init_lam_b(const BatchSmall* bs, int nb, hipStream_t s);
void launch_start_check_b(const BatchSmall* bs, int nb, hipStream_t s);
void launch_conv_check_b(const BatchSmall* bs, int nb, hipStream_t s);
void launch_ortho_small_b(const BatchSmall* bs, int nb, int m, hipStream_t s);
void launch_rq_small_b(const BatchSmall* bs, int nb, int end_of_iteration, hipStream_t s);
void launch_final_rr_b(const BatchSmall* bs, int nb, int kint, hipStream_t s);
void launch_final_res_b(const BatchSmall* bs, int nb, hipStream_t s);
void launch_tharm_small_b(const BatchSmall* bs, int nb, int m, int kint, hipStream_t s);

void launch_init_lam(const SmallParams& p, const double* part, int nblk, SmallBufs b,
                     DevStatus* st, hipStream_t s);
void launch_start_check(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s);
// For a small problem with B = I (vstep_small_ok): the Rayleigh quotients
// of V from (A - sigma)V, the residual block R and the convergence test in
// one single-workgroup launch (as launch_xdots, launch_rq_small,
// launch_resid_prep and launch_conv_check in sequence).
bool vstep_small_ok(size_t n, int kint);
void launch_vstep_small(const SmallParams& p, size_t n, const double* V, int ldv,
                        const double* QV, int ldq, double* R, int ldr, double* part,
                        SmallBufs b, DevStatus* st, hipStream_t s);
void launch_conv_check(const SmallParams& p, const double* part, int nblk, SmallBufs b,
                       DevStatus* st, int max_iters, hipStream_t s);
void launch_ortho_small(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s);
void launch_tharm_small(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s);
// The same step when G_R is symmetric: Cholesky, C = L^-1 G_R L^-T and
// the cyclic Jacobi method in one workgroup (k_tharm_sym.hip).
void launch_tharm_sym(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s);
hipError_t tharm_sym_set_attributes();
// Complex iterations (Algorithm 1, and Algorithm 2 with k_int complex
// columns per slot; k_complex_small.hip): the complex Cholesky-QR of
// Z = [V W S P] from the real Gram of its interleaved columns (same gating
// as launch_ortho_small), and the complex projected problem of eq. (3.5)
// with the selection of the k_int smallest |xi|.
void launch_cplx_ortho(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s);
void launch_cplx_tharm(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s);
hipError_t cplx_set_attributes();
// Final Rayleigh-Ritz of the complex block iteration from HM = the real
// Gram [V^T (A - sigma) V | V^T V] of the interleaved columns of V: the k
// pairs nearest sigma, final_C (kint x 2k real expansion of the complex
// coefficients), final_theta (2k, each value twice).
void launch_cplx_final(const SmallParams& p, const double* HM, SmallBufs b, DevStatus* st,
                       hipStream_t s);
// PLMR (Section 3.3): from [G_1 | G_2] = (T(A - lam B)Zhat)^T [(A - sigma B)Zhat | B Zhat]
// the matrix F = Zhat^T (A - lam B) T (A - lam B) Zhat = G_1^T + (sigma - lam) G_2^T,
// its smallest eigenpair by cyclic Jacobi, Y' = y (m x 1).
void launch_plmr_small(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s);
// Y = T X for a dense n x n T (row-major); columns [0, split) of Y go to
// o0, the rest to o1 (nothing when st is halted).
void launch_dense_prec(size_t n, const double* T, const double* X, int ldx, Blk o0, Blk o1,
                       int split, int ncols, const DevStatus* st, hipStream_t s);
// Rayleigh quotients from per-block partial sums [v.v | v.(A - sigma B)v];
// end_of_iteration also advances the iteration counter.
void launch_rq_small(const SmallParams& p, const double* part, int nblk, SmallBufs b,
                     DevStatus* st, int end_of_iteration, hipStream_t s);
void launch_final_rr(const SmallParams& p, const double* HM, SmallBufs b, DevStatus* st,
                     hipStream_t s);
void launch_final_res(const SmallParams& p, const double* part, int nblk, SmallBufs b,
                      hipStream_t s);
// out[c] = sum over blocks of the first of the two launch_xdots sums, c < k
void launch_colsum_first(const double* part, int nblk, int k, double* out, hipStream_t s);
hipError_t small_set_attributes(int m, int kint);
hipError_t tharm_set_attributes(int m, int kint);
// Raise a kernel's dynamic-LDS limit to the device's per-workgroup maximum.
// Limits are per function and process-wide, so they are never set to a
// size of one context (a later, smaller context would lower the limit
// under an earlier, larger one); the size a launch uses is its own.
hipError_t set_lds_limit(const void* kernel);
// Largest dynamic LDS the projected-solver kernels use at (m, kint).
size_t tharm_lds_bytes(int m, int kint);

}  // namespace plhr
