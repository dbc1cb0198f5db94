// Device helpers shared by the kernels of libplhr (header-only, inlined).
#pragma once
#include <hip/hip_runtime.h>
#include "internal.h"

namespace plhr {

// MI355X dispatches consecutive workgroup ids round-robin over its 8 XCDs,
// each with a private L2.  Renumber blocks so that every XCD walks one
// contiguous range of logical blocks: neighbouring grid rows (stencil
// halos) then stay in the same L2.
__device__ __forceinline__ int xcd_logical_block(int b, int nb) {
  const int nx = 8;
  int xcd = b % nx, local = b / nx;
  int per = nb / nx, rem = nb % nx;
  return xcd * per + (xcd < rem ? xcd : rem) + local;
}

__device__ __forceinline__ bool halted(const DevStatus* st) {
  return st != nullptr && (st->done | st->error);
}

// Copy a compact n x n matrix from global memory into LDS with row stride
// ld, every thread of the workgroup taking elements t, t + nt, ...; eight
// loads are in flight before the stores, and the (row, column) of an
// element is advanced incrementally instead of divided out.
__device__ __forceinline__ void load_square(const double* __restrict__ g, double* s, int n,
                                            int ld) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int tot = n * n;
  const int di = nt / n, dj = nt - di * n;
  int e = t, i = t / n, j = t - (t / n) * n;
  for (; e + 7 * nt < tot; e += 8 * nt) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = g[e + u * nt];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      s[i * ld + j] = v[u];
      i += di;
      j += dj;
      if (j >= n) {
        j -= n;
        ++i;
      }
    }
  }
  for (; e < tot; e += nt) {
    s[i * ld + j] = g[e];
    i += di;
    j += dj;
    if (j >= n) {
      j -= n;
      ++i;
    }
  }
}

// The reverse: LDS (row stride ld) to a compact n x n matrix in global
// memory, with the same incremental indexing.
__device__ __forceinline__ void store_square(const double* s, double* __restrict__ g, int n,
                                             int ld) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int tot = n * n;
  const int di = nt / n, dj = nt - di * n;
  int i = t / n, j = t - (t / n) * n;
  for (int e = t; e < tot; e += nt) {
    g[e] = s[i * ld + j];
    i += di;
    j += dj;
    if (j >= n) {
      j -= n;
      ++i;
    }
  }
}

}  // namespace plhr
