/*
 * plhr.h -- C ABI of the MI355X block PLHR eigensolver.
 *
 * Block PLHR (Vecharynski & Knyazev, "Preconditioned locally harmonic
 * residual method for computing interior eigenpairs of certain classes of
 * Hermitian matrices", arXiv:1408.0042) computes the k eigenpairs of
 *
 *     A v = lambda B v,   A = A^*,  B = B^* > 0            (eq. 1.1)
 *
 * whose eigenvalues are closest to a real shift sigma, using a Hermitian
 * positive definite preconditioner T (Section 5) and the T-harmonic
 * Rayleigh-Ritz extraction of eq. (3.5) on the trial subspace
 * span{V, W, S, P} (Algorithm 2; Algorithm 3 in real arithmetic).
 *
 * Conventions for every entry point
 *  - Block vectors are point-major: an n-by-c block is n rows of c
 *    contiguous scalars (row-major, leading dimension c).
 *  - Pointers documented as "device" must be HIP device memory on the
 *    device that was current at plhr_create; pointers documented as "host"
 *    are ordinary host memory.  All device buffers passed in are owned by
 *    the caller and must outlive the context.
 *  - Work is enqueued on the stream given to plhr_create.  Functions that
 *    return host results synchronise that stream before returning.
 *  - Every function returns a plhr_status; on failure a message describing
 *    the first error is available from plhr_last_error() (thread-local).
 *    No function throws or aborts on bad input.
 *  - Nothing here is thread-safe for a single context; distinct contexts
 *    may be used from distinct threads.
 */
#ifndef PLHR_H
#define PLHR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PLHR_OK = 0,
  PLHR_ERR_ARG = 1,           /* invalid argument or descriptor                 */
  PLHR_ERR_UNSUPPORTED = 2,   /* valid request the library does not implement   */
  PLHR_ERR_HIP = 3,           /* a HIP runtime call failed                      */
  PLHR_ERR_NOT_HPD = 4,       /* Gram/projected matrix not positive definite    */
  PLHR_ERR_BREAKDOWN = 5,     /* the V block became rank deficient              */
  PLHR_ERR_NOT_CONVERGED = 6, /* max_iters reached; outputs hold best iterate   */
  PLHR_ERR_STATE = 7          /* call out of order (e.g. backward before solve) */
} plhr_status;

/* Operator kinds (the model operators the paper uses, Section 6). */
typedef enum {
  PLHR_OP_IDENTITY = 0,
  PLHR_OP_FD5_2D = 1, /* scale*(-Laplacian) 5-point, Dirichlet, + diag(V)   */
  PLHR_OP_FD7_3D = 2, /* scale*(-Laplacian) 7-point, Dirichlet, + diag(V)  */
  PLHR_OP_DIAG = 3,   /* diag(d), d in `potential`: a lumped mass for B    */
  PLHR_OP_Q1_2D = 4,  /* scale*K, bilinear elements, Dirichlet, + diag(V)  */
  PLHR_OP_Q1_3D = 5,  /* scale*K, trilinear elements, Dirichlet, + diag(V) */
  PLHR_OP_Q1_MASS = 6, /* consistent mass M of the Q1 elements of A (B only) */
  PLHR_OP_CSR = 7,     /* general sparse symmetric matrix (CSR), A or B     */
  PLHR_OP_BLOCH7_3D = 8 /* scale*(-Laplacian_theta) 7-point, Bloch-periodic,
                           complex Hermitian, + diag(V): the solver
                           (Algorithm 2) and plhr_op_apply                */
} plhr_op_kind;

typedef enum {
  PLHR_F64 = 0, /* real double                                       */
  PLHR_C128 = 1 /* complex double, interleaved (re, im) per entry    */
} plhr_dtype;

/* Operator descriptor.  Grid points are numbered x-fastest,
 * p = i + nx*(j + ny*l); a 2-D grid has nz = 1.
 *   kind       one of plhr_op_kind
 *   dtype      PLHR_F64 (PLHR_C128 for PLHR_OP_BLOCH7_3D)
 *   nx, ny, nz interior points per direction (>= 1)
 *   h          grid spacing (> 0)
 *   scale      factor multiplying the negative discrete Laplacian (> 0)
 *   potential  device, n doubles, or NULL for none: A += diag(potential);
 *              for PLHR_OP_DIAG the diagonal itself (not NULL)
 * A PLHR_OP_DIAG descriptor is used only as B: its nx, ny, nz must be
 * those of A and every diagonal entry positive and finite (checked at
 * plhr_create, PLHR_ERR_ARG otherwise); h and scale are ignored.
 * PLHR_OP_Q1_2D/3D (the finite-element model problem of Section 6.1):
 * stiffness K of bilinear/trilinear elements of size h on a uniform mesh
 * with Dirichlet boundary, unknowns at the interior nodes (nx = elements
 * per side - 1), K = sum over directions of the tensor products of the
 * 1-D matrices (1/h)[-1 2 -1] and (h/6)[1 4 1]; the potential adds to
 * the diagonal as given (pass m_x V_x for a lumped-mass potential).
 * PLHR_OP_Q1_MASS is used only as B with a Q1 A (whose grid and h it
 * takes; its own fields are ignored): the consistent mass, the tensor
 * product of (h/6)[1 4 1].  A preconditioner with a Q1 A is the V-cycle
 * of the finite-difference Laplacian on the same nodes (spectrally
 * equivalent to K; T's scale does not change the iteration).
 * PLHR_OP_CSR: any sparse symmetric A (the potential, if given, adds to
 * its diagonal) and, as B, any sparse symmetric positive definite matrix
 * of the same n; with a CSR operator T must be the identity (the
 * multigrid preconditioner needs a grid).                              */
typedef struct {
  int32_t kind;
  int32_t dtype;
  int32_t nx, ny, nz;
  int32_t reserved0;
  double h;
  double scale;
  const double* potential;
  /* PLHR_OP_CSR only (device arrays, caller-owned, read at create and by
   * every product): n = nx rows (ny = nz = 1), row i holds the entries
   * values[row_ptr[i] .. row_ptr[i+1]) in columns col_idx[..]; the matrix
   * must be symmetric (B also positive definite); nnz = row_ptr[n].   */
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const double* values;
  int64_t nnz;
  /* PLHR_OP_BLOCH7_3D only: the Bloch phase per period in x, y, z (the
   * quasi-momentum times the box length); the other kinds ignore it.   */
  double theta[3];
} plhr_op_desc;

/* Preconditioner kinds (Section 5: T must be Hermitian positive definite). */
typedef enum {
  PLHR_PREC_IDENTITY = 0,
  PLHR_PREC_MG_VCYCLE = 1, /* one V-cycle on the Laplacian part of A            */
  PLHR_PREC_AV_MG = 2,     /* AV-MG, T ~ |L - sigma I|^-1 (Appendix A, Alg. 4)  */
  PLHR_PREC_INV_MG = 3,    /* INV-MG, T ~ (L - sigma I)^-1, indefinite (Alg. 5) */
  PLHR_PREC_DENSE = 4      /* a dense n x n matrix given by the caller        */
} plhr_prec_kind;

/* Preconditioner descriptor.
 *   kind     one of plhr_prec_kind
 *   levels   number of grid levels including the finest (>= 1).  A level
 *            whose dimensions are all even pairs neighbouring points for
 *            the next one (n -> n/2, cell-centred, trilinear interpolation
 *            3/4-1/4); one whose dimensions are all odd (>= 3) keeps every
 *            other point (n -> (n - 1)/2, vertex-centred, linear
 *            interpolation and full weighting); the coarsest level (at
 *            most 1024 points) is solved densely
 *   nu_pre, nu_post  smoothing steps before / after the coarse correction
 *            (must be equal so that T is Hermitian)
 *   omega    Jacobi weight, 0 < omega <= 2/3 keeps T positive definite
 *   delta    AV-MG only (> 0): a level of spacing h_l uses the Laplacian
 *            L_l as its operator B_l when sqrt(sigma / scale) h_l < delta
 *            and the polynomial p_m(L_l - sigma I) otherwise (default 0.6)
 *   degree   AV-MG only (1 .. 64): degree m of p_m, the Jackson-damped
 *            Chebyshev series of |x| on [-sigma, 4 d scale / h_l^2 - sigma]
 *            (default 10)
 * PLHR_PREC_MG_VCYCLE: every level the re-discretised Laplacian, weighted
 * Jacobi, the coarsest L_0^-1.  PLHR_PREC_AV_MG (Appendix A, Algorithm 4):
 * Richardson smoothing w <- w + alpha_l (r - B_l w) with alpha_l =
 * omega / diag(L_l) on the Laplacian levels and 1 / max p_m on the
 * polynomial ones, the coarsest |L_0 - sigma I_0|^-1 (a host
 * eigendecomposition at create); T is symmetric positive definite.
 * PLHR_PREC_INV_MG (Algorithm 5, the indefinite comparison of Section
 * 6.2): B_l = L_l - sigma I_l on every level, alpha_l = omega / diag(L_l),
 * the coarsest (L_0 - sigma I_0)^-1.  sigma on an eigenvalue of the
 * coarsest operator gives PLHR_ERR_ARG at create.
 * PLHR_PREC_DENSE: T is the dense symmetric positive definite matrix at
 * `matrix` (device, n x n doubles, row i at matrix + i n; caller-owned,
 * read by every application, so it must stay allocated while the context
 * is used; symmetry and definiteness are not checked).  This is the form
 * of the preconditioners of the small finite-element experiment of
 * Section 6.1, perturbations of |A - sigma B|^-1 that the caller builds.
 * levels, nu_pre, nu_post, omega, delta and degree are ignored.          */
typedef struct {
  int32_t kind;
  int32_t levels;
  int32_t nu_pre, nu_post;
  double omega;
  double delta;
  int32_t degree;
  int32_t reserved0;
  const double* matrix;
} plhr_prec_desc;

/* Arithmetic of the preconditioner.  PLHR_PREC_MIXED runs the multigrid
 * V-cycles that produce search directions (W = T R and S) in FP32
 * (storage and arithmetic on every level, FP64 input and output blocks).
 * The products that enter the T-harmonic Grams, T(A - sigma B)Z, keep the
 * FP64 V-cycle: G_L = Z^*(A - sigma B)T(A - sigma B)Z spans many orders of
 * magnitude and loses definiteness with an FP32 T.  Every other step
 * (operator products, residuals, Grams, Cholesky-QR, projected problem,
 * block updates, convergence test) stays in FP64, so the converged pairs
 * meet the same FP64 tolerance.  No effect when T is the identity.      */
typedef enum { PLHR_PREC_FP64 = 0, PLHR_PREC_MIXED = 1 } plhr_precision;

/* Extraction of the projected problem.  PLHR_EXTRACT_T_HARMONIC is the
 * method's eq. (3.5).  PLHR_EXTRACT_HARMONIC replaces T by the identity
 * inside the projection only (the search directions still use T): the
 * standard harmonic Rayleigh-Ritz of the "harm." rows of Section 6.2.    */
typedef enum { PLHR_EXTRACT_T_HARMONIC = 0, PLHR_EXTRACT_HARMONIC = 1 } plhr_extraction;

/* Iteration.  PLHR_ALG_BLOCK is the block method: in real arithmetic
 * (Algorithm 3) for the real operators, in complex arithmetic (Algorithm
 * 2) for PLHR_OP_BLOCH7_3D.  PLHR_ALG_SINGLE is the single-vector method (Algorithm
 * 1, k = 1) in complex arithmetic, as Section 3.2 prescribes even for real
 * A and B since the projected problem can have complex eigenpairs: the
 * iterate v, the directions w, s, p and their products are complex
 * vectors stored as two real columns each (real and imaginary parts, i.e.
 * the interleaved layout of a complex128 vector), every basis is
 * orthonormalised in the complex B-inner product, and the 4 x 4 (3 x 3 on
 * the first step) projected problem is solved in complex arithmetic.
 * PLHR_ALG_PLMR is the PLMR method of Section 3.3 (k = 1, real
 * arithmetic): the trial subspace of Algorithm 1 with the refinement
 * extraction, the B-unit vector v of span{v, w, s, p} of least
 * ||A v - lam B v||_T at the current Rayleigh quotient lam, i.e. the
 * eigenvector of the smallest eigenvalue of
 * Z^*(A - lam B)T(A - lam B)Z y = theta^2 Z^*BZ y.  T(A - lam B) of v and
 * w are w and s themselves, so it costs the same four preconditioner
 * applications per iteration as the T-harmonic extraction.              */
typedef enum { PLHR_ALG_BLOCK = 0, PLHR_ALG_SINGLE = 1, PLHR_ALG_PLMR = 2 } plhr_algorithm;

/* Solver options (plhr_options_default fills the defaults shown).
 *   tol          relative residual ||A v - lam B v|| /
 *                ((||A||_1 + |lam| ||B||_1) ||v||) at which a pair counts
 *                as converged                                 (1e-8)
 *   max_iters    iteration limit                              (10000)
 *   k_extra      extra block columns; 1 for real problems so that a
 *                conjugate pair is not cut (Section 4.1)      (1)
 *   precision    PLHR_PREC_FP64 or PLHR_PREC_MIXED            (FP64)
 *   lock         soft locking of converged columns            (1)
 *   check_every  iterations between host convergence checks   (1)
 *   ortho_passes Cholesky-QR passes of the B-orthonormalisation of
 *                [V W S P] per iteration: 1 one pass, 2 always a second
 *                pass on the result (CholQR2), 0 a second pass only when
 *                the first meets a pivot of the column-scaled Gram below
 *                1e-4 (one pass loses about eps / pivot of
 *                B-orthogonality, which grows when converged columns
 *                are not locked); the second pass's kernels return at
 *                once otherwise                               [0]
 *   drop_tol     squared relative norm (the pivot of the column-scaled
 *                Gram) below which a column is dropped during the
 *                B-orthonormalisation: the transform R^-1 scales by up to
 *                pivot^-1/2 and also acts on the carried products
 *                (A - sigma B)Z and T(A - sigma B)Z, so a smaller pivot
 *                amplifies their rounding-level disagreement with Z each
 *                iteration                                    [1e-10]
 *   extraction   a plhr_extraction value                      [T_HARMONIC]
 *   use_graph    1: each iteration's launches are captured once in a HIP
 *                graph (on a stream of the library's own) and replayed on
 *                the context's stream; 0: launched one by one.  Launch
 *                profiling bypasses the graphs                [0]
 *   algorithm    a plhr_algorithm value.  PLHR_ALG_SINGLE needs k = 1;
 *                k_extra and lock are then ignored, the start block is
 *                n x 2 doubles (the real and imaginary parts of the start
 *                vector), the convergence test uses the residual of the
 *                complex vector, and the returned eigenvector is real
 *                (the final Rayleigh-Ritz on the span of the two parts).
 *                PLHR_ALG_PLMR needs k = 1; k_extra, lock and extraction
 *                are ignored and the start block is n x 1   [BLOCK]   */
typedef struct {
  double tol;
  int32_t max_iters;
  int32_t k_extra;
  int32_t precision;
  int32_t lock;
  int32_t check_every;
  int32_t ortho_passes;
  double drop_tol;
  int32_t extraction;
  int32_t use_graph;
  int32_t algorithm;
  int32_t reserved0;
} plhr_options;

typedef struct plhr_ctx_s* plhr_ctx;

/* Per-call iteration report (host struct). */
typedef struct {
  int32_t iters;       /* iterations done since plhr_start                 */
  int32_t converged;   /* 1 when the k wanted pairs meet tol               */
  int32_t n_active;    /* columns still generating W/S/P                  */
  int32_t status;      /* device status word (0 = ok)                      */
  double max_rel_res;  /* largest relative residual among the k wanted     */
  int32_t n_excluded;  /* basis slots left out of projected problems since
                          plhr_start because G_L had a clearly negative
                          pivot (inconsistent carried products)           */
  int32_t reserved0;
} plhr_iter_info;

/* Library version string. */
const char* plhr_version(void);

/* Message for the most recent failure on this thread ("" if none). */
const char* plhr_last_error(void);

/* Fill *opt with defaults.  Returns PLHR_ERR_ARG if opt is NULL. */
plhr_status plhr_options_default(plhr_options* opt);

/* Bytes of device workspace plhr_create needs for these arguments.
 * Arguments as for plhr_create.  *ws_bytes (host) receives the size. */
plhr_status plhr_workspace_size(const plhr_op_desc* A, const plhr_op_desc* B,
                                const plhr_prec_desc* T, double sigma, int32_t k,
                                const plhr_options* opt, size_t* ws_bytes);

/* Create a solver for the k eigenpairs of A v = lambda B v nearest sigma
 * (Algorithm 3 for the real operators; Algorithm 1 with PLHR_ALG_SINGLE;
 * Algorithm 2 for PLHR_OP_BLOCH7_3D, see above plhr_op_apply's block).
 *   A          host descriptor of A (FD5_2D, FD7_3D, Q1_2D, Q1_3D, CSR or
 *              BLOCH7_3D)
 *   B          host descriptor of B: NULL or PLHR_OP_IDENTITY for the
 *              identity, PLHR_OP_DIAG for a positive diagonal B with a
 *              finite-difference A (the diagonal is read once at create
 *              and must stay allocated), or PLHR_OP_Q1_MASS with a Q1 A
 *   T          host descriptor of the HPD preconditioner, or NULL for I
 *   sigma      finite real shift
 *   k          wanted pairs, 1 <= k and 4*(k + k_extra) <= n; a trial
 *              subspace wider than 84 (4*(k + k_extra) > 84) gives
 *              PLHR_ERR_UNSUPPORTED; PLHR_ALG_SINGLE (its basis takes 8
 *              real columns) and PLHR_ALG_PLMR (4 columns) need k = 1 and
 *              give PLHR_ERR_ARG otherwise
 *   opt        host options, or NULL for defaults
 *   stream     HIP stream (hipStream_t) all work is enqueued on; NULL is
 *              the null stream
 *   workspace  device buffer of at least plhr_workspace_size bytes, or
 *              NULL to let the library allocate (and free at destroy)
 *   ws_bytes   size of workspace (ignored when workspace is NULL)
 *   out        host; receives the context handle                        */
plhr_status plhr_create(const plhr_op_desc* A, const plhr_op_desc* B,
                        const plhr_prec_desc* T, double sigma, int32_t k,
                        const plhr_options* opt, void* stream, void* workspace,
                        size_t ws_bytes, plhr_ctx* out);

/* Algorithm 3, steps 1-2: load the start block and B-normalise it.
 *   V0   device, n x (k + k_extra) doubles, point-major (n x 2 with
 *        PLHR_ALG_SINGLE: real and imaginary parts; n x 1 with
 *        PLHR_ALG_PLMR; n x (k + k_extra) complex128 for the Bloch
 *        operator); copied.                                              */
plhr_status plhr_start(plhr_ctx ctx, const double* V0);

/* Run up to n_steps iterations of the while-loop of Algorithm 3, stopping
 * early when the k wanted pairs converge.  info (host) may be NULL.
 * Returns PLHR_OK (also when not yet converged), or an error.            */
plhr_status plhr_iterate(plhr_ctx ctx, int32_t n_steps, plhr_iter_info* info);

/* Final standard Rayleigh-Ritz on span(V) (Algorithm 2/3, last step).
 *   eigvals  device, k doubles, ordered by |lambda - sigma| (ties: smaller)
 *   V        device, n x k doubles, B-orthonormal Ritz vectors, or NULL
 *   rel_res  host, k doubles (relative residuals recomputed from fresh
 *            operator products), or NULL                                 */
plhr_status plhr_finish(plhr_ctx ctx, double* eigvals, double* V, double* rel_res);

/* plhr_start + plhr_iterate until convergence or max_iters + plhr_finish.
 *   iters (host) receives the iteration count, may be NULL.
 * Returns PLHR_ERR_NOT_CONVERGED (outputs still written) when max_iters
 * is reached first.                                                      */
plhr_status plhr_solve(plhr_ctx ctx, const double* V0, double* eigvals, double* V,
                       double* rel_res, int32_t* iters);

/* Hellmann-Feynman gradient of L(lambda) with respect to the diagonal
 * potential of A: for A = L + diag(pot) and B independent of pot,
 *     dL/dpot_x = sum_j dL/dlambda_j * |v_j(x)|^2 / (v_j^* B v_j)
 * over the k pairs returned by the last plhr_finish.
 *   dL_dlambda  device, k doubles
 *   dL_dpot     device, n doubles; overwritten, or added to when
 *               accumulate != 0
 * PLHR_ERR_STATE if plhr_finish has not run.                              */
plhr_status plhr_eigvals_backward(plhr_ctx ctx, const double* dL_dlambda, double* dL_dpot,
                                  int32_t accumulate);

/* Apply one operator of the context to a block (no iteration state used).
 *   which  0: Y = A X;  1: Y = (A - sigma B) X;  2: Y = T X (in the
 *          precision used for search directions: FP32 V-cycle in mixed)
 *   X, Y   device, n x ncols doubles, point-major; must not overlap
 *   ncols  1 <= ncols <= 2*(k + k_extra)                                  */
plhr_status plhr_apply(plhr_ctx ctx, int32_t which, const double* X, double* Y, int32_t ncols);

/* Apply an operator given by its descriptor alone (no context, no
 * solver state):  Y = (A - shift I) X.
 * Supported: PLHR_OP_BLOCH7_3D with dtype PLHR_C128, the complex
 * Hermitian model Hamiltonian of the complex iteration (Algorithm 2,
 * Section 4) standing in for the periodic Kohn-Sham operators of
 * Section 6.3 at one quasi-momentum:
 *   scale * (-Laplacian_theta) + diag(potential) on an nx x ny x nz
 *   periodic box of spacing h, 7-point stencil; the neighbour across a
 *   face in direction d is the point at the other end times
 *   exp(+i theta[d]) going forward, exp(-i theta[d]) going backward.
 *   A          host descriptor; potential is a device array of n real
 *              doubles or NULL; h, scale > 0 and theta finite
 *   shift      real, finite
 *   X, Y       device, n x ncols complex128 entries (interleaved re, im:
 *              2*n*ncols doubles), point-major; must not overlap
 *   ncols      >= 0 (0: nothing is done); nx*ncols < 2^31
 *   stream     hipStream_t the product is enqueued on (NULL: the null
 *              stream).  Asynchronous: returns after the launch.
 * PLHR_ERR_ARG for a NULL or invalid argument, PLHR_ERR_UNSUPPORTED for
 * any other operator kind or dtype (the real operators are applied
 * through a context, plhr_apply), PLHR_ERR_HIP if the launch fails.     */
plhr_status plhr_op_apply(const plhr_op_desc* A, double shift, const void* X, void* Y,
                          int32_t ncols, void* stream);

/* The complex Hermitian Bloch operator in the solver (Algorithm 2, the
 * block iteration in complex arithmetic).  plhr_workspace_size /
 * plhr_create take A = PLHR_OP_BLOCH7_3D with dtype PLHR_C128 (phases in
 * theta, real potential or NULL) with
 *   B   NULL or PLHR_OP_IDENTITY (otherwise PLHR_ERR_UNSUPPORTED)
 *   T   NULL, PLHR_PREC_IDENTITY or PLHR_PREC_MG_VCYCLE: the Bloch V-cycle
 *       of plhr_bloch_prec_create (its rules on levels and the coarsest
 *       grid apply; its levels and coarse inverse live in the context's
 *       workspace); any other kind is PLHR_ERR_UNSUPPORTED
 *   opt algorithm PLHR_ALG_BLOCK, precision PLHR_PREC_FP64; lock locks
 *       a converged complex column (it generates no W, S or P, as in the
 *       real iteration); 8 (k + k_extra) <= 84, since each of
 *       the k + k_extra complex columns of the four slots counts as two
 *       real columns of the on-chip projected problem.
 * Blocks are complex128, interleaved, point-major: V0 of plhr_start /
 * plhr_solve is n x (k + k_extra) complex (2 n (k + k_extra) doubles),
 * V of plhr_finish / plhr_solve n x k complex; eigvals and rel_res hold
 * k values.  plhr_get_state returns 2 (k + k_extra) Rayleigh quotients
 * (each complex column's value twice) and the n x (k + k_extra) complex
 * block; plhr_apply takes n x ncols/2 complex columns (ncols even).
 * plhr_eigvals_backward returns PLHR_ERR_UNSUPPORTED.  The complex
 * columns run through the Gram, Cholesky-QR and update kernels as pairs
 * of real columns (real, imaginary part); the orthonormalisation, the
 * projected problem of eq. (3.5) and the final Rayleigh-Ritz step are
 * solved in complex arithmetic.                                          */

/* Multigrid preconditioner of the complex Bloch operator (Section 5: T
 * Hermitian positive definite; Appendix A's V-cycle on the Laplacian part
 * of the operator), standing alone for the complex iteration.  One V-cycle
 * applied to a block: every level the same Bloch stencil (spacing 2^l h,
 * the same phases, no potential), nu_pre weighted-Jacobi sweeps from zero,
 * the residual restricted by R = P^H / 8, the coarse correction, nu_post
 * sweeps; P is cell-centred trilinear interpolation (3/4 from the parent,
 * 1/4 from the parent's neighbour in each direction) and picks up
 * exp(+/- i theta[d]) across a periodic face; the coarsest level is solved
 * with the inverse of its dense matrix, formed at create.               */
typedef struct plhr_bloch_prec_s* plhr_bloch_prec;

/* Create the hierarchy.
 *   A         host descriptor, PLHR_OP_BLOCH7_3D / PLHR_C128 (potential
 *             ignored: T acts on the Laplacian part)
 *   T         host, PLHR_PREC_MG_VCYCLE; levels >= 1, nu_pre == nu_post
 *             >= 1, 0 < omega <= 1; nx, ny, nz divisible by
 *             2^(levels - 1); the coarsest grid at most 1024 points
 *   max_cols  widest block apply will take (1 .. 2^22)
 *   stream    hipStream_t of every apply (NULL: the null stream)
 *   workspace device buffer of at least plhr_bloch_prec_workspace_size
 *             bytes, 256-byte aligned, caller-owned (it must outlive the
 *             handle), or NULL: the library allocates
 *   ws_bytes  size of workspace (ignored when it is NULL)
 * The level buffers (3 blocks per coarse level, 2 on the finest, of
 * n_l x max_cols complex128) and the coarse inverse live in the workspace
 * (or in memory the library allocates on the current device and
 * plhr_bloch_prec_destroy releases).
 * PLHR_ERR_ARG / PLHR_ERR_UNSUPPORTED for bad or unsupported descriptors
 * or a workspace that is too small or misaligned, PLHR_ERR_NOT_HPD if the
 * coarsest operator is not positive definite (all phases zero),
 * PLHR_ERR_HIP if an allocation or copy fails.                          */
plhr_status plhr_bloch_prec_create(const plhr_op_desc* A, const plhr_prec_desc* T,
                                   int32_t max_cols, void* stream, void* workspace,
                                   size_t ws_bytes, plhr_bloch_prec* out);

/* Device bytes plhr_bloch_prec_create needs in a caller workspace for
 * these arguments (validated as for create; no device call).
 *   ws_bytes  host; receives the size                                    */
plhr_status plhr_bloch_prec_workspace_size(const plhr_op_desc* A, const plhr_prec_desc* T,
                                           int32_t max_cols, size_t* ws_bytes);

/* Y = T X, one V-cycle per column, enqueued on the stream given at create
 * (asynchronous).  X, Y: device, n x ncols complex128 (interleaved),
 * point-major, not overlapping; 0 <= ncols <= max_cols (0: nothing is
 * done).  Calls on one handle must not overlap in time (they share its
 * level buffers).                                                         */
plhr_status plhr_bloch_prec_apply(plhr_bloch_prec p, const void* X, void* Y, int32_t ncols);

/* Release the hierarchy (after the work enqueued on its stream is done). */
void plhr_bloch_prec_destroy(plhr_bloch_prec p);

/* Hermitian Gram product G = X^H Y of complex128 blocks on the FP64 matrix
 * cores: the Gram products of the complex iteration (Z^H B Z of the
 * orthonormalisation, Section 4; the T-harmonic Grams of eq. (3.5)).
 *   n        rows, >= 0 (0 gives G = 0)
 *   X, Y     device, n x mx and n x my complex128 (interleaved re, im),
 *            point-major; may be the same block
 *   G        device, mx x my complex128, row-major, overwritten
 *   1 <= mx, my <= 1024
 *   workspace device scratch of at least plhr_gram_c128_workspace(n, mx,
 *            my) bytes, caller-owned, contents not preserved
 *   stream   hipStream_t (NULL: the null stream); asynchronous
 * X, Y, G and the workspace must be 16-byte aligned.  The sum over rows
 * runs in a fixed order (deterministic).  PLHR_ERR_ARG for a NULL,
 * misaligned or out-of-range argument or a short workspace.              */
plhr_status plhr_gram_c128_workspace(int64_t n, int32_t mx, int32_t my, size_t* bytes);
plhr_status plhr_gram_c128(int64_t n, const void* X, int32_t mx, const void* Y, int32_t my,
                           void* G, void* workspace, size_t ws_bytes, void* stream);

/* Cholesky-QR orthonormalisation of a complex block (the orthonormalising
 * step of the complex iteration, Section 4, with B = I):
 *   Z^H Z = R^H R (R upper triangular, real positive diagonal), Q = Z R^-1,
 * so that Q^H Q = I and span Q = span Z.
 *   n        rows, >= m
 *   Z        device, n x m complex128 (interleaved), point-major; read only
 *   m        columns, 1 <= m <= 64
 *   Q        device, n x m complex128, written; must not overlap Z
 *   R        device, m x m complex128 row-major (lower part zero), or NULL;
 *            must not overlap Z, Q or the workspace
 *   workspace device scratch of plhr_cholqr_c128_workspace(n, m) bytes
 *   stream   hipStream_t (NULL: the null stream)
 * Synchronises the stream to report a breakdown: PLHR_ERR_NOT_HPD when
 * Z^H Z is not positive definite to rounding (dependent columns; Q and R
 * are then unspecified).  Pointers 16-byte aligned; PLHR_ERR_ARG for a
 * NULL, misaligned, overlapping or out-of-range argument.                */
plhr_status plhr_cholqr_c128_workspace(int64_t n, int32_t m, size_t* bytes);
plhr_status plhr_cholqr_c128(int64_t n, const void* Z, int32_t m, void* Q, void* R,
                             void* workspace, size_t ws_bytes, void* stream);

/* Complex block product Y = Z M: the block updates of the complex
 * iteration (Algorithm 2, the new V and P as combinations of the trial
 * basis with the coefficients of the projected eigenvectors).
 *   n        rows, >= 0 (0: nothing is done)
 *   Z        device, n x m complex128 (interleaved), point-major
 *   M        device, m x k complex128, row-major
 *   Y        device, n x k complex128, written; must not overlap Z or M
 *   1 <= m, k <= 64
 *   stream   hipStream_t (NULL: the null stream); asynchronous
 * Z, M and Y 16-byte aligned.  PLHR_ERR_ARG for a NULL, misaligned,
 * overlapping or out-of-range argument.                                  */
plhr_status plhr_rowmul_c128(int64_t n, const void* Z, int32_t m, const void* M, int32_t k,
                             void* Y, void* stream);

/* The projected eigenproblem of one iteration on given Gram matrices:
 * eq. (3.5), G_L y = xi G_R y, solved as in every iteration of the solver
 * (Cholesky G_L = L L^T, C = L^-1 G_R L^-T, real Schur form of C, tau =
 * 1/xi), the k_int units of smallest |xi| in the order (|xi|, Re xi,
 * -Im xi) with a conjugate pair kept together (Definition 3.1), and the
 * real coefficient basis Y' = [Y0 YR ytilde_R YI] of Algorithm 3 (the
 * real part of a selected pair's eigenvector in YR and its imaginary part
 * in YI; a pair whose conjugate would be unit k_int + 1 contributes only
 * its real part, ytilde_R).  Stands alone so that this step can be
 * checked on synthetic pencils.
 *   m        trial-subspace width, kint <= m <= 84
 *   kint     columns selected, >= 1
 *   GL, GR   device, m x m doubles, row-major: G_L symmetric positive
 *            definite (its two triangles are averaged), G_R general
 *   keep     device, m int32 (nonzero: slot used), or NULL for all; the
 *            problem is posed on the kept slots, other rows of Y are zero
 *   Y        device, m x kint doubles, row-major: Y' (each column, or each
 *            R/I pair as one complex vector, of unit 2-norm; a real
 *            column's largest entry positive)
 *   xi       device, 2 x m doubles: real parts, then imaginary parts, of
 *            the xi of the sorted units, one entry per unit (a conjugate
 *            pair by its Im > 0 member); entries past the number of
 *            units are zero
 *   kinds    device, kint int32: 0 real, 1 YR, 2 ytilde_R, 3 YI
 *   pair     device, kint int32: the partner column of a YR/YI column,
 *            -1 otherwise
 *   n_excluded host, receives the number of slots left out because G_L
 *            had a clearly negative pivot (may be NULL)
 *   workspace device scratch of plhr_projected_workspace(m, kint) bytes
 *   stream   hipStream_t (NULL: the null stream); synchronised on return
 * PLHR_ERR_ARG for a NULL, misaligned (8 bytes), overlapping or
 * out-of-range argument; PLHR_ERR_BREAKDOWN when fewer than kint slots
 * remain or the QR iteration does not converge.                          */
plhr_status plhr_projected_workspace(int32_t m, int32_t kint, size_t* bytes);
plhr_status plhr_projected_solve(int32_t m, int32_t kint, const double* GL, const double* GR,
                                 const int32_t* keep, double* Y, double* xi, int32_t* kinds,
                                 int32_t* pair, int32_t* n_excluded, void* workspace,
                                 size_t ws_bytes, void* stream);

/* The projected step of plhr_projected_solve without any allocation and
 * without a workspace argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Arguments as for plhr_projected_solve, except:
 *   status   device, 2 int32, written: the plhr_status the device raised
 *            (0 when none: PLHR_ERR_BREAKDOWN when fewer than kint slots
 *            remain or the QR iteration does not converge) and the number
 *            of slots left out (G_L pivot clearly negative)
 * Asynchronous: the work is enqueued on `stream` (NULL: the null stream)
 * and the call returns at once; it never synchronises, allocates or
 * frees.  Its scratch (the staged [G_L | G_R], the slot mask, the
 * projected-solver work area and a status block) is a file-scope device
 * array of plhr_projected_noalloc_scratch_bytes() bytes (about 332 KiB,
 * for m up to 84), one copy per device, held until the process ends; its
 * address is looked up on the first call on each device.  Every call on
 * one device shares that array: calls that overlap in time on one device
 * (different streams, or different threads without ordering) race and
 * give undefined results; calls in one stream are ordered.  Each call
 * clears the status block and restages the inputs, so the contents left
 * by an earlier call do not matter.  PLHR_ERR_ARG for the argument errors
 * of plhr_projected_solve (m <= 84) or a NULL/misaligned status.        */
size_t plhr_projected_noalloc_scratch_bytes(void);
plhr_status plhr_projected_solve_noalloc(int32_t m, int32_t kint, const double* GL,
                                         const double* GR, const int32_t* keep, double* Y,
                                         double* xi, int32_t* kinds, int32_t* pair,
                                         int32_t* status, void* stream);

/* Read back iteration state for inspection (synchronises the stream).
 *   lam      host, k + k_extra doubles (current Rayleigh quotients)
 *   V        device, n x (k + k_extra) doubles, or NULL (current block)  */
plhr_status plhr_get_state(plhr_ctx ctx, double* lam, double* V);

/* Per-kernel launch profile (HIP events around every launch).
 * Categories (PLHR_KC_*): 0 operator block products, 1 V-cycle Jacobi
 * sweeps, 2 V-cycle residual, 3 restriction, 4 prolongation,
 * 5 coarsest-level solve, 6 Gram products, 7 Gram reduction,
 * 8 orthonormalising transform, 9 block update, 10 Cholesky /
 * C / Hessenberg of the projected problem, 11 Francis QR, 12 selection
 * and eigenvectors, 13 Cholesky-QR factor, 14 other single-workgroup
 * kernels, 15 residual formation, column reductions and copies.
 * bytes/flops are algorithmic (what the operation must read, write and
 * compute; model operation counts for the single-workgroup kernels);
 * total_ms sums the event-measured kernel durations.                    */
#define PLHR_KC_COUNT 16
typedef struct {
  int32_t launches[PLHR_KC_COUNT];
  double total_ms[PLHR_KC_COUNT];
  double bytes[PLHR_KC_COUNT];
  double flops[PLHR_KC_COUNT];
  int32_t truncated;  /* 1 if more launches happened than were recorded */
  int32_t reserved0;
} plhr_profile;

/* Start recording launches of one category (-1: all) on this context, for
 * at most max_launches launches (events are created here, host side).    */
plhr_status plhr_profile_start(plhr_ctx ctx, int32_t category, int32_t max_launches);

/* Stop recording; synchronises the stream and fills *out (host).         */
plhr_status plhr_profile_stop(plhr_ctx ctx, plhr_profile* out);

/* Diagnostic read-back of internal buffers (synchronises the stream).
 *   which  0: Gram of Z (m x m); 1: orthonormalising transform M (m x m);
 *          2: [G_L | G_R] (m x 2m); 3: coefficients Y' (m x kint);
 *          4: sorted xi (2 x m: real parts, imaginary parts); 5: lambda
 *          (kint); 6: relative residuals (kint); 7: Z (n x m); 8: QZ;
 *          9: TQZ; 10: kept-slot mask (m, as doubles); 11: column kinds
 *          and partners (2 x kint, as doubles); 12: clock stamps of the
 *          phases of the last projected eigensolve (12, as doubles)
 *   dst    host buffer of `count` doubles; count must not exceed the size
 *          of the buffer named by `which` (m = 4*kint)                    */
plhr_status plhr_debug_read(plhr_ctx ctx, int32_t which, double* dst, size_t count);

/* Release the context and any workspace it allocated. NULL is ignored.   */
void plhr_destroy(plhr_ctx ctx);

/* ------------------------------------------------------------------ batch
 * Many independent problems solved together: the same iteration (Algorithm
 * 3) advances every problem, each launch covering all of them (one
 * workgroup per grid row or per chunk of points of one problem, one
 * workgroup per problem for the projected problems).  The per-iteration
 * launch sequence is captured once in a HIP graph and replayed.  The
 * chunk size of the point-range kernels and the workgroup size of the
 * grid-row kernels are picked by timing candidates on the first solve
 * (plhr_batch_tuning reports the choice).  Converged problems stop
 * working while the others continue.                                      */
typedef struct plhr_batch_s* plhr_batch;

/* Create a batch of nbatch problems A_b v = lambda v (B = I).
 *   nbatch  number of problems, >= 1
 *   A       host array of nbatch PLHR_OP_FD5_2D descriptors (each with its
 *           own grid and potential; h and scale equal for all)
 *   T       host descriptor of the V-cycle (applied to each problem's
 *           Laplacian part; levels >= 2; every grid dimension divisible by
 *           2^(levels-1), coarsest level <= 1024 points), or NULL for T = I
 *   sigma   host array of nbatch finite shifts
 *   k       wanted pairs per problem, 4 (k + k_extra) <= min n_b and <= 84
 *   opt     host options (precision FP64), or NULL for defaults
 *   stream  HIP stream for all work (NULL: the null stream)
 *   workspace  device buffer of at least plhr_batch_workspace_size bytes,
 *           256-byte aligned, caller-owned (it must outlive the handle), or
 *           NULL: the library allocates it (and frees it at destroy)
 *   ws_bytes  size of workspace (ignored when it is NULL)
 *   out     host; receives the handle
 * With a workspace the handle allocates no device memory (its host state,
 * graphs and a pinned status array are its own).  The potentials are read
 * at create and must stay valid until destroy.  A workspace that is too
 * small or misaligned gives PLHR_ERR_ARG.                                */
plhr_status plhr_batch_create(int32_t nbatch, const plhr_op_desc* A, const plhr_prec_desc* T,
                              const double* sigma, int32_t k, const plhr_options* opt,
                              void* stream, void* workspace, size_t ws_bytes, plhr_batch* out);

/* Device bytes plhr_batch_create needs in a caller workspace for these
 * arguments (validated as for create; no device call).
 *   ws_bytes  host; receives the size                                    */
plhr_status plhr_batch_workspace_size(int32_t nbatch, const plhr_op_desc* A,
                                      const plhr_prec_desc* T, const double* sigma, int32_t k,
                                      const plhr_options* opt, size_t* ws_bytes);

/* Solve every problem from its start block.
 *   V0       host array of nbatch device pointers; V0[b] is n_b x (k +
 *            k_extra) doubles, point-major, full rank
 *   eigvals  device, nbatch x k: row b holds problem b's eigenvalues
 *            ordered by |lambda - sigma_b| (ties: smaller lambda)
 *   V        host array of nbatch device pointers (n_b x k each,
 *            B-orthonormal Ritz vectors), or NULL
 *   rel_res  host, nbatch x k relative residuals, or NULL
 *   iters    host, nbatch iteration counts, or NULL
 *   status   host, nbatch per-problem status codes (PLHR_OK,
 *            PLHR_ERR_NOT_CONVERGED, PLHR_ERR_BREAKDOWN, ...), or NULL
 * Returns PLHR_OK when every problem converged, PLHR_ERR_NOT_CONVERGED
 * when some reached max_iters (outputs still written), or the first
 * device error of a problem.                                              */
plhr_status plhr_batch_solve(plhr_batch b, const double* const* V0, double* eigvals,
                             double* const* V, double* rel_res, int32_t* iters,
                             int32_t* status);

/* Hellmann-Feynman gradient of a loss of the eigenvalues with respect to
 * each problem's potential (after plhr_batch_solve).
 *   dL_dlambda  device, nbatch x k
 *   dL_dpot     host array of nbatch device pointers (n_b doubles each)
 *   accumulate  0: overwrite, 1: add                                     */
plhr_status plhr_batch_eigvals_backward(plhr_batch b, const double* dL_dlambda,
                                        double* const* dL_dpot, int32_t accumulate);

/* Apply one operator to a block of every problem (no iteration state is
 * used; the internal basis of the batch is overwritten, the results of
 * the last solve needed by the backward are not).
 *   which  0: Y = A X;  1: Y = (A - sigma B) X;  2: Y = T X
 *   X, Y   host arrays of nbatch device pointers, n_b x ncols each
 *   ncols  1 <= ncols <= 2 (k + k_extra)                                 */
plhr_status plhr_batch_apply(plhr_batch b, int32_t which, const double* const* X,
                             double* const* Y, int32_t ncols);

/* What the tuner picked (valid after the first solve). */
typedef struct {
  int32_t chunk_points;  /* points per workgroup of the point-range kernels */
  int32_t row_threads;   /* threads per workgroup of the grid-row kernels   */
  int32_t use_graph;     /* 1 when iterations replay a captured HIP graph   */
  int32_t nchunks;       /* point chunks over all problems                  */
  double tuned_ms[8];    /* timed candidates: chunk sizes 512..4096, then
                            row threads 64, 128, 256 (ms per sample)        */
} plhr_batch_tuning;
plhr_status plhr_batch_tuning_info(plhr_batch b, plhr_batch_tuning* out);

/* Use (1, default) or bypass (0) the captured iteration graph.           */
plhr_status plhr_batch_set_graph(plhr_batch b, int32_t use_graph);

/* Launch profile of the batch (as plhr_profile_start/stop); profiling
 * bypasses the graph while it is on.                                     */
plhr_status plhr_batch_profile_start(plhr_batch b, int32_t category, int32_t max_launches);
plhr_status plhr_batch_profile_stop(plhr_batch b, plhr_profile* out);

/* Release the batch. NULL is ignored. */
void plhr_batch_destroy(plhr_batch b);

#ifdef __cplusplus
}
#endif

#endif /* PLHR_H */
