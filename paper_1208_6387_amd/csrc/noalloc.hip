// FP64 interface operator Y = F X that allocates no device memory: the W-format workspace of the
// gather, the product and its split-K slabs lives in one fixed device array per GPU, reserved when
// the library's code object is loaded on that GPU and held until the process ends.
#include "common.hpp"
#include "problem.hpp"

#include <mutex>

namespace {
constexpr int64_t SCRATCH_DOUBLES = RPF_NOALLOC_SCRATCH_BYTES / 8;
constexpr int MAX_DEVICES = 64;

// Host code must not pass this name to a kernel: on the host it is a stand-in, not a device
// address.  Its address on a device comes from hipGetSymbolAddress, taken once per device.
__device__ __align__(256) double scratch[SCRATCH_DOUBLES];

std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {};

// the device address of `scratch` on the current device, looked up on the first call there
double* scratch_on_current_device() {
  int dev = -1;
  RPF_HIP(hipGetDevice(&dev));
  RPF_CHECK(dev >= 0 && dev < MAX_DEVICES, RPF_EINVAL, "feti_apply_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[dev] == nullptr) {
    void* p = nullptr;
    RPF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    RPF_CHECK(p != nullptr, RPF_EHIP, "feti_apply_noalloc: no device address for the scratch array");
    g_ptr[dev] = static_cast<double*>(p);
  }
  return g_ptr[dev];
}
}  // namespace

extern "C" rpf_status feti_apply_noalloc(rpf_problem pb, const rpf_pattern* patterns, int32_t m, const double* X,
                                         int64_t ldx, double* Y, int64_t ldy, int32_t prec, uint32_t flags,
                                         void* stream) {
  using namespace rpf;
  return guarded([&] {
    RPF_CHECK(pb != nullptr, RPF_EINVAL, "feti_apply_noalloc: NULL structure");
    RPF_CHECK(m >= 1 && ldx >= m && ldy >= m && X && Y, RPF_EINVAL, "feti_apply_noalloc: bad block arguments");
    RPF_CHECK(prec == RPF_FP64, RPF_EINVAL, "feti_apply_noalloc: only the FP64 product is available");
    RPF_CHECK(flags == 0, RPF_EINVAL,
              "feti_apply_noalloc: no flags are accepted (the coarse projector allocates its space)");
    check_patterns(pb, patterns, RPF_FP64);
    if (pb->n_lambda == 0) return;
    const F64Plan pl = plan_F64(pb, patterns, m, schedule_for(pb, m, RPF_FP64));
    const int64_t xn = cdiv(pl.xneed, 32) * 32;  // keeps the result slabs 256-byte aligned
    const int64_t need = xn + pl.yneed;
    RPF_CHECK(need <= SCRATCH_DOUBLES, RPF_EINVAL,
              "feti_apply_noalloc: the block needs " + std::to_string(need * 8) + " bytes of workspace, above the " +
                  std::to_string((int64_t)RPF_NOALLOC_SCRATCH_BYTES) + "-byte limit; use fewer columns per call");
    double* base = scratch_on_current_device();
    hipStream_t s = (hipStream_t)stream;
    const YLoc yl = run_F64(pb, patterns, pl, m, X, ldx, base, base + xn, s, OP_FLEX, false);
    scatter_all(pb, yl, m, Y, ldy, 0.0, s);
  });
}
