// The projected eigenproblem of one iteration as a stand-alone entry
// point: eq. (3.5) on given Gram matrices, followed by the selection of
// Algorithm 3, on the same three single-workgroup kernels the solver
// launches every iteration (k_tharm.hip).  It exists so that the
// projected step can be checked on synthetic pencils with a prescribed
// spectrum (conjugate pairs cut by the block size, ties, a nearly
// singular G_R) independently of the rest of the iteration.
#include <cstdint>
#include <string>
#include <vector>

#include "internal.h"

using namespace plhr;

namespace {
size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct ProjLayout {
  size_t glr, keep, work, st, total;
};

ProjLayout proj_layout(int m) {
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
  if (!GL || !GR || !Y || !xi || !kinds || !pair || !workspace) {
    set_error("plhr_projected_solve: NULL argument");
    return PLHR_ERR_ARG;
  }
  if (ws_bytes < need) {
    set_error("plhr_projected_solve: workspace smaller than plhr_projected_workspace");
    return PLHR_ERR_ARG;
  }
  if (((uintptr_t)GL | (uintptr_t)GR | (uintptr_t)Y | (uintptr_t)xi | (uintptr_t)workspace) & 7) {
    set_error("plhr_projected_solve: matrices and workspace must be 8-byte aligned");
    return PLHR_ERR_ARG;
  }
  // inputs must not overlap the outputs or the workspace
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
                       {(const char*)workspace, need}};
  for (const Span& a : in)
    for (const Span& b : out)
      if (a.b && b.b && a.p < b.p + b.b && b.p < a.p + a.b) {
        set_error("plhr_projected_solve: an input overlaps an output or the workspace");
        return PLHR_ERR_ARG;
      }
  for (int i = 0; i < 5; ++i)
    for (int j = i + 1; j < 5; ++j)
      if (out[i].p < out[j].p + out[j].b && out[j].p < out[i].p + out[i].b) {
        set_error("plhr_projected_solve: outputs overlap each other or the workspace");
        return PLHR_ERR_ARG;
      }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const ProjLayout L = proj_layout(m);
  char* w = static_cast<char*>(workspace);
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
  PLHR_HIP_CHECK(tharm_set_attributes(m, kint));
  const size_t row = (size_t)m * sizeof(double);
  PLHR_HIP_CHECK(hipMemcpy2DAsync(sb.GLR, 2 * row, GL, row, row, m, hipMemcpyDeviceToDevice, s));
  PLHR_HIP_CHECK(
      hipMemcpy2DAsync(sb.GLR + m, 2 * row, GR, row, row, m, hipMemcpyDeviceToDevice, s));
  std::vector<int> ones(m, 1);
  if (keep)
    PLHR_HIP_CHECK(hipMemcpyAsync(sb.keep, keep, (size_t)m * 4, hipMemcpyDeviceToDevice, s));
  else
    PLHR_HIP_CHECK(hipMemcpyAsync(sb.keep, ones.data(), (size_t)m * 4, hipMemcpyHostToDevice, s));
  PLHR_HIP_CHECK(hipMemsetAsync(st, 0, sizeof(DevStatus), s));
  launch_tharm_small(sp, sb, st, s);
  PLHR_HIP_CHECK(hipGetLastError());
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

}  // extern "C"
