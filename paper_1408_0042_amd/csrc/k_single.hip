// The refinement step of PLMR (Section 3.3, real arithmetic, one real
// column per slot) and the dense preconditioner product.
#include <cmath>

#include "common.cuh"

namespace plhr {

namespace {

constexpr int kN = 4;  // slots v, w, s, p

}  // namespace

// ------------------------------------------------ PLMR refinement step
// F = Zhat^T (A - lam B) T (A - lam B) Zhat on the kept slots from the
// Gram [G_1 | G_2] = (T(A - lam B)Zhat)^T [(A - sigma B)Zhat | B Zhat]:
// F(i, j) = G_1(j, i) + (sigma - lam) G_2(j, i), symmetrised.  Its
// eigenpairs by cyclic Jacobi (Golub & Van Loan, Sec. 8.5); the vector of
// the smallest eigenvalue theta^2 (ties: lower slot) is y, unit 2-norm,
// largest entry positive (Zhat is B-orthonormal, so v = Zhat y has
// ||v||_B = 1).
__global__ __launch_bounds__(64) void k_plmr_small(SmallParams p, SmallBufs b, DevStatus* st) {
  if (halted(st)) return;
  if (threadIdx.x != 0) return;
  const int m = p.m, ld2 = 2 * m;
  int idx[kN];
  int n = 0;
  for (int a = 0; a < m && a < kN; ++a)
    if (b.keep[a]) idx[n++] = a;
  if (n < 1) {
    st->error = PLHR_ERR_BREAKDOWN;
    st->reason = kReasonVVanished;
    return;
  }
  const double lam = b.lam[0];
  double F[kN * kN], V[kN * kN];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const int a = idx[i], c = idx[j];
      const double fij = b.GLR[(size_t)c * ld2 + a] + (p.sigma - lam) * b.GLR[(size_t)c * ld2 + m + a];
      const double fji = b.GLR[(size_t)a * ld2 + c] + (p.sigma - lam) * b.GLR[(size_t)a * ld2 + m + c];
      F[i * kN + j] = 0.5 * (fij + fji);
      V[i * kN + j] = (i == j) ? 1.0 : 0.0;
    }
  double a2 = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) a2 += F[i * kN + j] * F[i * kN + j];
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += F[i * kN + j] * F[i * kN + j];
    if (!(off > 1e-30 * a2)) break;
    for (int pp = 0; pp < n; ++pp)
      for (int q = pp + 1; q < n; ++q) {
        const double apq = F[pp * kN + q];
        if (apq == 0.0) continue;
        const double th = (F[q * kN + q] - F[pp * kN + pp]) / (2.0 * apq);
        const double t = copysign(1.0, th) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int r = 0; r < n; ++r) {  // columns pp, q
          const double x = F[r * kN + pp], y = F[r * kN + q];
          F[r * kN + pp] = c * x - sn * y;
          F[r * kN + q] = sn * x + c * y;
          const double u = V[r * kN + pp], w = V[r * kN + q];
          V[r * kN + pp] = c * u - sn * w;
          V[r * kN + q] = sn * u + c * w;
        }
        for (int r = 0; r < n; ++r) {  // rows pp, q
          const double x = F[pp * kN + r], y = F[q * kN + r];
          F[pp * kN + r] = c * x - sn * y;
          F[q * kN + r] = sn * x + c * y;
        }
      }
  }
  int js = 0;
  for (int j = 1; j < n; ++j)
    if (F[j * kN + j] < F[js * kN + js]) js = j;
  double nr2 = 0.0, big = -1.0;
  int im = 0;
  for (int i = 0; i < n; ++i) {
    const double v = V[i * kN + js];
    nr2 += v * v;
    if (fabs(v) > big) big = fabs(v), im = i;
  }
  double sc = (nr2 > 0.0) ? 1.0 / sqrt(nr2) : 0.0;
  if (V[im * kN + js] < 0.0) sc = -sc;
  for (int e = 0; e < m * p.kint; ++e) b.Y[e] = 0.0;
  for (int i = 0; i < n; ++i) b.Y[(size_t)idx[i] * p.kint] = V[i * kN + js] * sc;
  for (int r = 0; r < 2 * m; ++r) b.xi[r] = 0.0;
  b.xi[0] = F[js * kN + js];  // theta^2, the squared T-norm of the refined residual
  b.kinds[0] = 0;
  b.pair[0] = -1;
}

void launch_plmr_small(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s) {
  prof_begin(KC_THARM_QR, 2.0 * p.m * p.m * 8.0, 2000.0, s);
  hipLaunchKernelGGL(k_plmr_small, dim3(1), dim3(64), 0, s, p, b, st);
  prof_end(KC_THARM_QR, s);
}

// ------------------------------------------------ dense preconditioner
// One wavefront per row of T: lanes stride over the row (coalesced), four
// columns of X at a time, then a butterfly sum over the wavefront (a
// fixed order: deterministic).
__global__ __launch_bounds__(256) void k_dense_prec(size_t n, const double* __restrict__ T,
                                                    const double* __restrict__ X, int ldx,
                                                    double* o0, int ld0, double* o1, int ld1,
                                                    int split, int ncols, const DevStatus* st) {
  if (halted(st)) return;
  const int lane = threadIdx.x & 63;
  const size_t row = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const double* tr = T + row * n;
  for (int c0 = 0; c0 < ncols; c0 += 4) {
    const int nc = min(4, ncols - c0);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (size_t j = lane; j < n; j += 64) {
      const double t = tr[j];
      const double* x = X + j * ldx + c0;
      a0 += t * x[0];
      if (nc > 1) a1 += t * x[1];
      if (nc > 2) a2 += t * x[2];
      if (nc > 3) a3 += t * x[3];
    }
    for (int off = 32; off > 0; off >>= 1) {
      a0 += __shfl_xor(a0, off);
      a1 += __shfl_xor(a1, off);
      a2 += __shfl_xor(a2, off);
      a3 += __shfl_xor(a3, off);
    }
    if (lane < nc) {
      const double v = (lane == 0) ? a0 : (lane == 1) ? a1 : (lane == 2) ? a2 : a3;
      const int c = c0 + lane;
      if (c < split)
        o0[row * ld0 + c] = v;
      else
        o1[row * ld1 + (c - split)] = v;
    }
  }
}

void launch_dense_prec(size_t n, const double* T, const double* X, int ldx, Blk o0, Blk o1,
                       int split, int ncols, const DevStatus* st, hipStream_t s) {
  const double nn = (double)n;
  prof_begin(KC_COARSE, 8.0 * nn * nn + 16.0 * nn * ncols, 2.0 * nn * nn * ncols, s);
  const unsigned nb = (unsigned)((n + 3) / 4);
  hipLaunchKernelGGL(k_dense_prec, dim3(nb), dim3(256), 0, s, n, T, X, ldx, o0.ptr, o0.ld,
                     o1.ptr, o1.ld, split, ncols, st);
  prof_end(KC_COARSE, s);
}

}  // namespace plhr
