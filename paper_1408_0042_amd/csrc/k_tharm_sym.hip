// The projected eigenproblem of eq. (3.5) when G_R is symmetric: with
// T = I (or the harmonic extraction, T -> I in the projection) and B = I,
//     G_L = Zhat^*(A - sigma)^2 Zhat,   G_R = Zhat^*(A - sigma) Zhat,
// the Hermitian-definite harmonic Rayleigh-Ritz problem (Section 3.1):
// every xi is real.  With G_L = L L^T, C = L^-1 G_R L^-T is symmetric, so
// its eigenpairs come from the cyclic Jacobi method (Golub & Van Loan,
// Sec. 8.5) instead of a Hessenberg reduction and the nonsymmetric QR:
// each round rotates n/2 disjoint (p, q) planes of a round-robin
// tournament at once, two barriers per round; while the first wavefront
// computes a round's rotations, the other wavefronts apply the previous
// round's rotations to the eigenvector matrix.  The triangular solves (C
// from G_R, and y = L^-T u) run right-looking, one barrier per row, all
// columns at once.
// The k_int eigenvectors of smallest |xi| = 1/|tau| (ties: smaller xi)
// are y = L^-T u, scaled to unit 2-norm with their largest entry
// positive, in Y' (all columns real, no pairs).  One workgroup; C and the
// rotations in LDS.
#include <cmath>

#include "common.cuh"

namespace plhr {

namespace {

constexpr int kST = 512;

// 1/d from the hardware estimate and two Newton steps
__device__ __forceinline__ double sym_rcp(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return r;
}

// 1/sqrt(x) from the hardware estimate and two Newton steps
__device__ __forceinline__ double sym_rsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}

// Jacobi rotation (c, s) that annihilates a_pq of the 2 x 2 block
// [[a_pp, a_pq], [a_pq, a_qq]]: an entry negligible against its diagonal
// (|a_pq| below 1e-18 sqrt|a_pp a_qq|) or below 1e-150 (its square would
// lose digits) is left alone; otherwise t = tan of the angle from
// d = a_qq - a_pp, e = 2 a_pq: t = sgn(d) e / (|d| + sqrt(d^2 + e^2)), the
// smaller root, and c = 1/sqrt(1 + t^2), s = t c.
__device__ __forceinline__ void sym_rotation(double app, double aqq, double apq, double& c,
                                             double& sn) {
  c = 1.0;
  sn = 0.0;
  if (fabs(apq) > 1e-150 && apq * apq > 1e-36 * fabs(app * aqq)) {
    const double d = aqq - app, e = 2.0 * apq;
    const double r2 = fma(d, d, e * e);
    const double r = r2 * sym_rsq(r2);
    const double tt = ((d >= 0.0) ? e : -e) * sym_rcp(fabs(d) + r);
    c = sym_rsq(fma(tt, tt, 1.0));
    sn = tt * c;
  }
}

// Players of pair k in round rnd of the round-robin tournament on ne
// positions: position 0 holds player 0, position i >= 1 holds player
// 1 + (i - 1 + rnd) mod (ne - 1); pair k is positions k and ne - 1 - k.
// Returns (p, q) with p < q, q = -1 for a bye (player >= n).
__device__ __forceinline__ int2 sym_pair(int k, int rnd, int ne, int n) {
  int pa = 0;
  if (k > 0) {
    pa = k - 1 + rnd;
    if (pa >= ne - 1) pa -= ne - 1;
    ++pa;
  }
  int pb = ne - 1 - k - 1 + rnd;
  if (pb >= ne - 1) pb -= ne - 1;
  ++pb;
  const int pp = (pa < pb) ? pa : pb, qq = (pa < pb) ? pb : pa;
  return int2{pp, (qq < n) ? qq : -1};
}

__device__ double sym_block_sum(double a, double* red) {
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kST / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

}  // namespace

// LDS: C n*ld | V n*ld (L during the factorisation, later the
// eigenvectors) | 4 n doubles
__global__ __launch_bounds__(kST) void k_tharm_sym(SmallParams p, SmallBufs b, DevStatus* st) {
  if (halted(st)) return;
  extern __shared__ __attribute__((aligned(16))) double sm[];
  __shared__ int idx[kMaxM + 1];
  __shared__ int dead[kMaxM + 1];
  __shared__ int cnt_s, ndead_s;
  __shared__ double red[kST / 64];
  static_assert(kMaxM / 2 < 64 && kST > 64, "the rotations fit the first wavefront");
  // rotation tables of the current and the previous round: (c, s) and
  // (p, q) of each pair (q < 0: a bye)
  __shared__ double2 rcs[2][kMaxM / 2 + 1];
  __shared__ int2 rpq[2][kMaxM / 2 + 1];
  const int m = p.m, kint = p.kint, t = threadIdx.x;
  if (t == 0) st->tphase[0] = clock64();
  if (t == 0) {
    int c = 0;
    for (int s = 0; s < m; ++s)
      if (b.keep[s]) idx[c++] = s;
    cnt_s = c;
    ndead_s = 0;
  }
  __syncthreads();
  const int n = cnt_s;
  if (n < kint) {
    if (t == 0) {
      st->error = PLHR_ERR_BREAKDOWN;
      st->reason = kReasonVVanished;
    }
    return;
  }
  const int ld = n | 1;
  double* C = sm;
  double* V = C + n * ld;
  double* piv = V + n * ld;  // pivots, later tau
  double* aux = piv + n;     // 1/sqrt(pivot)
  double* rl = aux + n;      // 1 / L[j][j]
  const int ld2 = 2 * m;
  // symmetric parts of G_L (into V) and G_R (into C) on the kept slots
  for (int e = t; e < n * n; e += kST) {
    const int i = e / n, j = e - i * n;
    const int ia = idx[i], ja = idx[j];
    V[i * ld + j] = 0.5 * (b.GLR[(size_t)ia * ld2 + ja] + b.GLR[(size_t)ja * ld2 + ia]);
    C[i * ld + j] = 0.5 * (b.GLR[(size_t)ia * ld2 + m + ja] + b.GLR[(size_t)ja * ld2 + m + ia]);
  }
  for (int j = t; j < n; j += kST) dead[j] = 0;
  __syncthreads();
  if (t == 0) st->tphase[1] = clock64();
  // Cholesky of G_L, right-looking on unscaled columns; pivots as in the
  // general projected solver (raised to 1e-15 max diag, a clearly
  // negative one leaves its slot out)
  double maxd = 0.0;
  for (int j = 0; j < n; ++j) maxd = fmax(maxd, V[j * ld + j]);
  const double floor_ = fmax(1e-15 * maxd, 1e-300);
  for (int j = 0; j < n; ++j) {
    const double p0 = V[j * ld + j];
    if (p0 < -1e-10 * maxd) {  // uniform across the workgroup
      if (t == 0) {
        dead[j] = 1;
        ++ndead_s;
      }
      continue;
    }
    const double pp = fmax(p0, floor_);
    if (t == 0) piv[j] = pp;
    const double inv = 1.0 / pp;
    const int rem = n - j - 1;
    // exact quotient e / rem from a float reciprocal (e < 2^13)
    const float irem = 1.0f / (float)(rem > 0 ? rem : 1);
    for (int e = t; e < rem * rem; e += kST) {
      const int q = (int)(((float)e + 0.5f) * irem);
      const int i = j + 1 + q, c = j + 1 + (e - q * rem);
      if (c <= i) V[i * ld + c] -= V[i * ld + j] * inv * V[c * ld + j];
    }
    __syncthreads();
  }
  for (int j = t; j < n; j += kST) aux[j] = dead[j] ? 0.0 : 1.0 / sqrt(piv[j]);
  __syncthreads();
  // L = unscaled columns times 1/sqrt(pivot); dead slots: row and column
  // of L are e_j, G_R's row and column zero (tau = 0, never selected)
  for (int e = t; e < n * n; e += kST) {
    const int i = e / n, c = e - i * n;
    double v = 0.0;
    if (dead[i] || dead[c])
      v = (i == c) ? 1.0 : 0.0;
    else if (c == i)
      v = sqrt(piv[i]);
    else if (c < i)
      v = V[i * ld + c] * aux[c];
    V[i * ld + c] = v;
    if (c == i) rl[i] = 1.0 / v;  // the triangular solves' divisors, off their chains
    if (dead[i] || dead[c]) C[i * ld + c] = 0.0;
  }
  __syncthreads();
  if (t == 0 && ndead_s) st->n_excluded += ndead_s;
  if (ndead_s && n - ndead_s < kint) {
    if (t == 0) {
      st->error = PLHR_ERR_BREAKDOWN;
      st->reason = kReasonVVanished;
    }
    return;
  }
  if (t == 0) st->tphase[2] = clock64();
  // C <- L^-1 C: right-looking forward substitution on unscaled rows
  // (step r subtracts L[i][r] / L[r][r] times row r from the rows below;
  // row r is final after step r - 1), then every row scaled by 1 / L[r][r];
  // C <- C L^-T the same way on columns.  One barrier per step.
  const float inn = 1.0f / (float)n;  // exact float reciprocal: indices < 2^12
  for (int r = 0; r + 1 < n; ++r) {
    const double ir = rl[r];
    const int rem = n - r - 1;
    for (int e = t; e < rem * n; e += kST) {
      const int q = (int)(((float)e + 0.5f) * inn), c = e - q * n;
      const int i = r + 1 + q;
      C[i * ld + c] -= (V[i * ld + r] * ir) * C[r * ld + c];
    }
    __syncthreads();
  }
  for (int e = t; e < n * n; e += kST) {
    const int i = (int)(((float)e + 0.5f) * inn), c = e - i * n;
    C[i * ld + c] /= V[i * ld + i];
  }
  __syncthreads();
  for (int r = 0; r + 1 < n; ++r) {
    const double ir = rl[r];
    const int rem = n - r - 1;
    for (int e = t; e < rem * n; e += kST) {
      const int q = (int)(((float)e + 0.5f) * inn), i = e - q * n;
      const int c = r + 1 + q;
      C[i * ld + c] -= (V[c * ld + r] * ir) * C[i * ld + r];
    }
    __syncthreads();
  }
  for (int e = t; e < n * n; e += kST) {
    const int i = (int)(((float)e + 0.5f) * inn), c = e - i * n;
    C[i * ld + c] /= V[c * ld + c];
  }
  __syncthreads();
  // L to the work area (compact); C symmetrised; V = I
  for (int e = t; e < n * n; e += kST) {
    const int i = e / n, c = e - i * n;
    b.work[e] = V[i * ld + c];
  }
  __syncthreads();
  for (int e = t; e < n * n; e += kST) {
    const int i = e / n, c = e - i * n;
    if (c < i) {
      const double a = 0.5 * (C[i * ld + c] + C[c * ld + i]);
      C[i * ld + c] = a;
      C[c * ld + i] = a;
    }
    V[i * ld + c] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  // cyclic Jacobi, round-robin tournament over ne = n rounded up to even
  // positions (an index >= n is a bye).  The pair table of a round is
  // written by its first np threads with the rotations; the two-sided
  // update acts on the disjoint 2 x 2 blocks (pair k's rows, pair l's
  // columns) in one phase, so a round takes two barriers.
  if (t == 0) st->tphase[3] = clock64();
  const int ne = n + (n & 1), np = ne / 2;
  // exact float reciprocals for the block and row indices (e < 2^12)
  const float inp = 1.0f / (float)np;
  // the eigenvector columns of a round's rotations (V <- V J), applied by
  // the threads t >= np while the next round's rotations are computed
  auto rotate_vectors = [&](int bb, int t0, int nt) {
    for (int e = t - t0; e < np * n; e += nt) {
      const int l = (int)(((float)e + 0.5f) * inn), i = e - l * n;
      const int2 pq = rpq[bb][l];
      const int pc = pq.x, qc = pq.y;
      if (qc < 0) continue;
      const double2 cs = rcs[bb][l];
      const double cl = cs.x, sl = cs.y;
      const double vp = V[i * ld + pc], vq = V[i * ld + qc];
      V[i * ld + pc] = cl * vp - sl * vq;
      V[i * ld + qc] = sl * vp + cl * vq;
    }
  };
  int pend = -1;  // table whose vector rotations are still to be applied
  int cur = 0;
  int sweep = 0;
  for (; sweep < 30; ++sweep) {
    double a2 = 0.0, o2 = 0.0;
    for (int e = t; e < n * n; e += kST) {
      const int i = (int)(((float)e + 0.5f) * inn), c = e - i * n;
      const double v = C[i * ld + c];
      if (i == c)
        a2 += v * v;
      else
        o2 += v * v;
    }
    a2 = sym_block_sum(a2, red);
    o2 = sym_block_sum(o2, red);
    // off(C) at the rounding level of ||C|| (a rotation leaves about
    // eps max(|a_pp|, |a_qq|) behind)
    if (!(o2 > 1e-28 * a2)) break;  // uniform
    for (int rnd = 0; rnd < ne - 1; ++rnd) {
      // wavefront 0 computes the rotations (np <= 42 lanes), the other
      // wavefronts apply the previous round's to the eigenvectors
      if (t < np) {
        const int2 pq = sym_pair(t, rnd, ne, n);
        double c = 1.0, sn = 0.0;
        if (pq.y >= 0)
          sym_rotation(C[pq.x * ld + pq.x], C[pq.y * ld + pq.y], C[pq.x * ld + pq.y], c, sn);
        rcs[cur][t] = double2{c, sn};
        rpq[cur][t] = pq;
      } else if (t >= 64 && pend >= 0) {
        rotate_vectors(pend, 64, kST - 64);
      }
      __syncthreads();
      // C <- J^T C J on the 2 x 2 blocks (rows of pair k, columns of pair
      // l), which are disjoint; one phase.  Every load of a thread's items
      // is issued before the first store.
      {
        double* __restrict__ Cw = C;
        for (int e = t; e < np * np; e += kST) {
          const int k = (int)(((float)e + 0.5f) * inp), l = e - k * np;
          const int2 pqk = rpq[cur][k], pql = rpq[cur][l];
          const double2 csk = rcs[cur][k], csl = rcs[cur][l];
          const int pr = pqk.x, qr = pqk.y, pc = pql.x, qc = pql.y;
          const double ck = csk.x, sk = csk.y, cl = csl.x, sl = csl.y;
          const int qrr = (qr >= 0) ? qr : pr, qcc = (qc >= 0) ? qc : pc;
          const double a = Cw[pr * ld + pc], bb = Cw[pr * ld + qcc];
          const double cc = Cw[qrr * ld + pc], dd = Cw[qrr * ld + qcc];
          const double a1 = ck * a - sk * cc, b1 = ck * bb - sk * dd;
          const double c1 = sk * a + ck * cc, d1 = sk * bb + ck * dd;
          // a bye (q < 0) has c = 1, s = 0, so its row or column is copied
          // through unchanged and only the existing entries are stored
          Cw[pr * ld + pc] = cl * a1 - sl * b1;
          if (qc >= 0) Cw[pr * ld + qc] = sl * a1 + cl * b1;
          if (qr >= 0) Cw[qr * ld + pc] = cl * c1 - sl * d1;
          if (qr >= 0 && qc >= 0) Cw[qr * ld + qc] = sl * c1 + cl * d1;
        }
      }
      __syncthreads();
      pend = cur;
      cur ^= 1;
    }
  }
  if (pend >= 0) {  // the last round's vector rotations, all threads
    rotate_vectors(pend, 0, kST);
    __syncthreads();
  }
  if (t == 0) {
    st->tphase[4] = clock64();
    st->tphase[10] = sweep;
  }
  // tau and the ranks of xi = 1/tau by (|xi|, xi, index); tau = 0 last
  // (|xi| once per eigenvalue; xi = 1/tau is |xi| with the sign of tau,
  // exactly, since a quotient's rounding does not depend on signs)
  double* xabs = rl + n;
  for (int i = t; i < n; i += kST) {
    const double ti = C[i * ld + i];
    piv[i] = ti;
    xabs[i] = (ti != 0.0) ? 1.0 / fabs(ti) : INFINITY;
  }
  __syncthreads();
  int* rank = reinterpret_cast<int*>(aux);  // n ints fit in n doubles
  for (int i = t; i < n; i += kST) {
    const double ti = piv[i];
    const double xa = xabs[i];
    const double xs = (ti != 0.0) ? copysign(xa, ti) : INFINITY;
    int r = 0;
    for (int o = 0; o < n; ++o) {
      if (o == i) continue;
      const double to = piv[o];
      const double oa = xabs[o];
      const double os = (to != 0.0) ? copysign(oa, to) : INFINITY;
      r += (oa < xa || (oa == xa && (os < xs || (os == xs && o < i)))) ? 1 : 0;
    }
    rank[i] = r;
  }
  __syncthreads();
  // sorted xi for the host, Y' cleared, kinds and partners
  for (int i = t; i < n; i += kST) {
    const double ti = piv[i];
    b.xi[rank[i]] = (ti != 0.0) ? 1.0 / ti : INFINITY;
    b.xi[m + rank[i]] = 0.0;
  }
  for (int r = n + t; r < m; r += kST) {
    b.xi[r] = 0.0;
    b.xi[m + r] = 0.0;
  }
  for (int e = t; e < m * kint; e += kST) b.Y[e] = 0.0;
  for (int c = t; c < kint; c += kST) {
    b.kinds[c] = 0;
    b.pair[c] = -1;
  }
  if (t == 0) st->tphase[5] = clock64();
  // L back into the C region (C's diagonal is saved in piv)
  for (int e = t; e < n * n; e += kST) {
    const int i = e / n, c = e - i * n;
    C[i * ld + c] = b.work[e];
  }
  __syncthreads();
  // Y = L^-T U for all eigenvector columns at once: right-looking back
  // substitution on unscaled rows (step r subtracts L[r][q] / L[r][r]
  // times row r from the rows q < r; row r is final after step r + 1),
  // then every row scaled by 1 / L[r][r].  One barrier per step.
  for (int r = n - 1; r > 0; --r) {
    const double ir = rl[r];  // C holds L here
    for (int e = t; e < r * n; e += kST) {
      const int q = (int)(((float)e + 0.5f) * inn), c = e - q * n;
      V[q * ld + c] -= (C[r * ld + q] * ir) * V[r * ld + c];
    }
    __syncthreads();
  }
  for (int e = t; e < n * n; e += kST) {
    const int i = (int)(((float)e + 0.5f) * inn), c = e - i * n;
    V[i * ld + c] /= C[i * ld + i];
  }
  __syncthreads();
  // the selected columns, unit 2-norm, largest entry positive, written as
  // column `rank` of Y', one thread each
  for (int i = t; i < n; i += kST) {
    const int col = rank[i];
    if (col >= kint) continue;
    const double* u = V + i;  // column i of V, stride ld
    double nr2 = 0.0, big = -1.0;
    int im = 0;
    for (int r = 0; r < n; ++r) {
      const double v = u[r * ld];
      nr2 += v * v;
      if (fabs(v) > big) big = fabs(v), im = r;
    }
    double sc = (nr2 > 0.0) ? 1.0 / sqrt(nr2) : 0.0;
    if (u[im * ld] < 0.0) sc = -sc;
    for (int r = 0; r < n; ++r) b.Y[(size_t)idx[r] * kint + col] = u[r * ld] * sc;
  }
  __syncthreads();
  if (t == 0) st->tphase[6] = clock64();
}

static size_t sym_lds(int m) { return ((size_t)2 * m * (m | 1) + 4 * (size_t)m) * sizeof(double); }

hipError_t tharm_sym_set_attributes() { return set_lds_limit((const void*)k_tharm_sym); }

void launch_tharm_sym(const SmallParams& p, SmallBufs b, DevStatus* st, hipStream_t s) {
  const double m3 = (double)p.m * p.m * p.m, mm = (double)p.m * p.m;
  // model counts: Cholesky m^3/3, C 2 m^3, Jacobi ~8 sweeps of 4 m^3,
  // eigenvectors m^2 kint
  prof_begin(KC_THARM_QR, 3.0 * mm * 8.0, (1.0 / 3.0 + 2.0 + 32.0) * m3 + mm * p.kint, s);
  hipLaunchKernelGGL(k_tharm_sym, dim3(1), dim3(kST), sym_lds(p.m), s, p, b, st);
  prof_end(KC_THARM_QR, s);
}

}  // namespace plhr
