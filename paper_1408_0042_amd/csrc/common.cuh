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

}  // namespace plhr
