// The projected eigenproblem of one iteration as a stand-alone entry
// point: eq. (3.5) on given Gram matrices, followed by the selection of
// Algorithm 3, on the same three single-workgroup kernels the solver
// launches every iteration (k_tharm.hip).  It exists so that the
// projected step can be checked on synthetic pencils with a prescribed
// spectrum (conjugate pairs cut by the block size, ties, a nearly
// singular G_R) independently of the rest of the iteration.
#include <cstdint>
#include <mutex>
#include <string>

#include "internal.h"

using namespace plhr;

namespace {
constexpr size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct ProjLayout {
  size_t glr, keep, work, st, total;
};

constexpr ProjLayout proj_layout(int m) {
  ProjLayout L{};
  size_t o = 0;
  L.glr = o;
  o += al256((size_t)m * 2 * m * sizeof(double));
  L.keep = o;
  o += al256((size_t)m * sizeof(int));
  L.work = o;
  o += al256((size_t)4 * m * m * sizeof(double));
  L.st = o;
  o += al256(sizeof(DevStatus));
  L.total = o;
  return L;
}

// Stage the inputs for the projected-solver kernels: [G_L | G_R] side by
// side (m x 2m), the slot mask (all slots when keep is null) and a
// cleared status block.  One kernel instead of copies and fills, so that
// the sequence holds kernel launches only.
__global__ __launch_bounds__(256) void k_proj_stage(int m, const double* __restrict__ GL,
                                                    const double* __restrict__ GR,
                                                    const int* __restrict__ keep,
                                                    double* __restrict__ GLR, int* __restrict__ kp,
                                                    DevStatus* st) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  const int tot = 2 * m * m;
  for (int e = tid; e < tot; e += nt) {
    const int i = e / (2 * m), j = e - i * 2 * m;
    GLR[e] = (j < m) ? GL[i * m + j] : GR[i * m + (j - m)];
  }
  for (int e = tid; e < m; e += nt) kp[e] = keep ? keep[e] : 1;
  if (tid == 0) {
    DevStatus z{};
    *st = z;
  }
}

// The device status of the projected step as two int32: the raised
// plhr_status (0: none) and the number of slots left out.
__global__ void k_proj_status(const DevStatus* st, int32_t* out) {
  if (threadIdx.x == 0) {
    out[0] = st->error;
    out[1] = st->n_excluded;
  }
}

// Checks shared by both entry points (workspace excluded).
plhr_status proj_check(const char* name, int m, int kint, const double* GL, const double* GR,
                       const int32_t* keep, const double* Y, const double* xi,
                       const int32_t* kinds, const int32_t* pair, const void* extra,
                       size_t extra_bytes) {
  if (kint < 1 || m < kint || m > kMaxM) {
    set_error(std::string(name) + ": need 1 <= kint <= m <= " + std::to_string(kMaxM));
    return PLHR_ERR_ARG;
  }
  if (!GL || !GR || !Y || !xi || !kinds || !pair) {
    set_error(std::string(name) + ": NULL argument");
    return PLHR_ERR_ARG;
  }
  if (((uintptr_t)GL | (uintptr_t)GR | (uintptr_t)Y | (uintptr_t)xi) & 7 ||
      ((uintptr_t)keep | (uintptr_t)kinds | (uintptr_t)pair) & 3) {
    set_error(std::string(name) + ": misaligned argument (8 bytes for doubles, 4 for int32)");
    return PLHR_ERR_ARG;
  }
  struct Span {
    const char* p;
    size_t b;
  };
  const size_t mm = (size_t)m * m * sizeof(double);
  const Span in[3] = {{(const char*)GL, mm}, {(const char*)GR, mm},
                      {(const char*)keep, keep ? (size_t)m * 4 : 0}};
  const Span out[5] = {{(const char*)Y, (size_t)m * kint * sizeof(double)},
                       {(const char*)xi, (size_t)2 * m * sizeof(double)},
                       {(const char*)kinds, (size_t)kint * 4},
                       {(const char*)pair, (size_t)kint * 4},
                       {(const char*)extra, extra ? extra_bytes : 0}};
  for (const Span& a : in)
    for (const Span& b : out)
      if (a.b && b.b && a.p < b.p + b.b && b.p < a.p + a.b) {
        set_error(std::string(name) + ": an input overlaps an output");
        return PLHR_ERR_ARG;
      }
  for (int i = 0; i < 5; ++i)
    for (int j = i + 1; j < 5; ++j)
      if (out[i].b && out[j].b && out[i].p < out[j].p + out[j].b &&
          out[j].p < out[i].p + out[i].b) {
        set_error(std::string(name) + ": outputs overlap each other");
        return PLHR_ERR_ARG;
      }
  int dev = 0, lim = 0;
  PLHR_HIP_CHECK(hipGetDevice(&dev));
  PLHR_HIP_CHECK(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  int optin = 0;
  if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) ==
          hipSuccess &&
      optin > lim)
    lim = optin;
  // headroom for the kernels' static LDS (index lists, reduction slots)
  if (tharm_lds_bytes(m, kint) + 8192 > (size_t)lim) {
    set_error(std::string(name) + ": kint too large for m (the selected vectors do not fit "
              "one workgroup's LDS)");
    return PLHR_ERR_ARG;
  }
  return PLHR_OK;
}

// Enqueue staging and the three projected-solver kernels on s, with the
// scratch area at w (proj_layout(m).total bytes).
plhr_status proj_enqueue(int m, int kint, const double* GL, const double* GR,
                         const int32_t* keep, double* Y, double* xi, int32_t* kinds,
                         int32_t* pair, char* w, hipStream_t s, DevStatus** st_out) {
  const ProjLayout L = proj_layout(m);
  SmallBufs sb{};
  sb.GLR = (double*)(w + L.glr);
  sb.keep = (int*)(w + L.keep);
  sb.work = (double*)(w + L.work);
  sb.Y = Y;
  sb.xi = xi;
  sb.kinds = kinds;
  sb.pair = pair;
  DevStatus* st = (DevStatus*)(w + L.st);
  SmallParams sp{};
  sp.m = m;
  sp.kint = kint;
  const int blocks = (2 * m * m + 255) / 256;
  hipLaunchKernelGGL(k_proj_stage, dim3(blocks), dim3(256), 0, s, m, GL, GR, keep, sb.GLR,
                     sb.keep, st);
  launch_tharm_small(sp, sb, st, s);
  PLHR_HIP_CHECK(hipGetLastError());
  *st_out = st;
  return PLHR_OK;
}

// ---- the allocation-free variant: a file-scope scratch area per device
constexpr size_t kNoAllocScratch = proj_layout(kMaxM).total;
__device__ __align__(256) char scratch[kNoAllocScratch];
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per
// device (with that device current) and kept; the kernels' LDS limits are
// raised at the same time.
plhr_status scratch_for_current_device(char** out) {
  int dev = 0;
  PLHR_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("plhr_projected_solve_noalloc: device index out of range");
    return PLHR_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    PLHR_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    PLHR_HIP_CHECK(tharm_set_attributes(kMaxM, 1));
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<char*>(g_scratch_ptr[dev]);
  return PLHR_OK;
}
}  // namespace

extern "C" {

plhr_status plhr_projected_workspace(int32_t m, int32_t kint, size_t* bytes) {
  if (!bytes || kint < 1 || m < kint || m > kMaxM) {
    set_error("plhr_projected_workspace: need bytes != NULL and 1 <= kint <= m <= " +
              std::to_string(kMaxM));
    return PLHR_ERR_ARG;
  }
  *bytes = proj_layout(m).total;
  return PLHR_OK;
}

plhr_status plhr_projected_solve(int32_t m, int32_t kint, const double* GL, const double* GR,
                                 const int32_t* keep, double* Y, double* xi, int32_t* kinds,
                                 int32_t* pair, int32_t* n_excluded, void* workspace,
                                 size_t ws_bytes, void* stream) {
  size_t need = 0;
  const plhr_status s0 = plhr_projected_workspace(m, kint, &need);
  if (s0 != PLHR_OK) return s0;
  if (!workspace) {
    set_error("plhr_projected_solve: NULL workspace");
    return PLHR_ERR_ARG;
  }
  if (ws_bytes < need) {
    set_error("plhr_projected_solve: workspace smaller than plhr_projected_workspace");
    return PLHR_ERR_ARG;
  }
  if ((uintptr_t)workspace & 255) {
    set_error("plhr_projected_solve: workspace must be 256-byte aligned");
    return PLHR_ERR_ARG;
  }
  plhr_status c = proj_check("plhr_projected_solve", m, kint, GL, GR, keep, Y, xi, kinds, pair,
                             workspace, need);
  if (c != PLHR_OK) return c;
  hipStream_t s = static_cast<hipStream_t>(stream);
  PLHR_HIP_CHECK(tharm_set_attributes(m, kint));
  DevStatus* st = nullptr;
  c = proj_enqueue(m, kint, GL, GR, keep, Y, xi, kinds, pair, static_cast<char*>(workspace), s,
                   &st);
  if (c != PLHR_OK) return c;
  DevStatus host{};
  PLHR_HIP_CHECK(hipMemcpyAsync(&host, st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
  PLHR_HIP_CHECK(hipStreamSynchronize(s));
  if (n_excluded) *n_excluded = host.n_excluded;
  if (host.error) {
    set_error(std::string("plhr_projected_solve: ") + reason_text(host.reason));
    return (plhr_status)host.error;
  }
  return PLHR_OK;
}

size_t plhr_projected_noalloc_scratch_bytes(void) { return kNoAllocScratch; }

plhr_status plhr_projected_solve_noalloc(int32_t m, int32_t kint, const double* GL,
                                         const double* GR, const int32_t* keep, double* Y,
                                         double* xi, int32_t* kinds, int32_t* pair,
                                         int32_t* status, void* stream) {
  if (!status || ((uintptr_t)status & 3)) {
    set_error("plhr_projected_solve_noalloc: status must be a 4-byte aligned device pointer");
    return PLHR_ERR_ARG;
  }
  plhr_status c = proj_check("plhr_projected_solve_noalloc", m, kint, GL, GR, keep, Y, xi, kinds,
                             pair, status, 2 * sizeof(int32_t));
  if (c != PLHR_OK) return c;
  char* w = nullptr;
  c = scratch_for_current_device(&w);
  if (c != PLHR_OK) return c;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevStatus* st = nullptr;
  c = proj_enqueue(m, kint, GL, GR, keep, Y, xi, kinds, pair, w, s, &st);
  if (c != PLHR_OK) return c;
  hipLaunchKernelGGL(k_proj_status, dim3(1), dim3(64), 0, s, st, status);
  PLHR_HIP_CHECK(hipGetLastError());
  return PLHR_OK;
}

}  // extern "C"
