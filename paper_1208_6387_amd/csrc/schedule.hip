// Schedules of the flexibility products (section 3.2: S+ W for all occurrences of a pattern) and
// their autotuner.  A schedule names the workgroup tile of the products and the work target that
// sets each pattern's K split; tiles 64 and 128 put every pattern of the structure into one
// grouped persistent launch.  The tuner times every candidate on the structure itself (the whole
// operator: gather, products, scatter) and installs the fastest; the size rule (tile 0) is one of
// the candidates, so a tuned structure is never slower than an untuned one at the tuning width.
#include "common.hpp"
#include "problem.hpp"

#include <algorithm>

namespace rpf {
namespace {

// deterministic test block (splitmix64 of the entry index), values in [-1, 1)
__global__ void k_fill_hash(double* X, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  X[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

bool valid_schedule(rpf_problem pb, const rpf_pattern* pats, int prec, int tile, int work) {
  if (work < 1) return false;
  if (tile == 0) return true;
  if (prec == RPF_FP32) return false;  // the FP32 product has no grouped or large-tile form
  if (tile == 64 || tile == 128) return true;
  if (tile == 256) {
    if (pb->n_pat != 1) return false;
    return prec != RPF_FP64 || pats[0]->n_b % 2 == 0;
  }
  return false;
}
}  // namespace
}  // namespace rpf

using namespace rpf;

extern "C" rpf_status problem_set_schedule(rpf_problem pb, int32_t m, int32_t prec, int32_t tile, int32_t work) {
  return guarded([&] {
    RPF_CHECK(pb != nullptr, RPF_EINVAL, "problem_set_schedule: NULL structure");
    RPF_CHECK(m >= 1, RPF_EINVAL, "problem_set_schedule: m < 1");
    RPF_CHECK(prec >= RPF_FP64 && prec <= RPF_BF16, RPF_EINVAL, "problem_set_schedule: precision");
    RPF_CHECK(tile == 0 || tile == 64 || tile == 128 || tile == 256, RPF_EINVAL,
              "problem_set_schedule: tile must be 0, 64, 128 or 256");
    RPF_CHECK(work >= 1, RPF_EINVAL, "problem_set_schedule: work < 1");
    RPF_CHECK(!(tile == 256 && pb->n_pat != 1), RPF_EINVAL,
              "problem_set_schedule: the 256 tile is for single-pattern structures");
    RPF_CHECK(!(prec == RPF_FP32 && tile != 0), RPF_EINVAL, "problem_set_schedule: FP32 takes the size rule only");
    if (tile == 0) pb->sched.erase({m, prec});
    else pb->sched[{m, prec}] = Schedule{tile, work};
  });
}

extern "C" rpf_status problem_tune(rpf_problem pb, const rpf_pattern* patterns, int32_t m, int32_t prec, int32_t reps,
                                   rpf_schedule_entry* out, int32_t max_out, int32_t* n_out, void* stream) {
  return guarded([&] {
    RPF_CHECK(pb != nullptr, RPF_EINVAL, "problem_tune: NULL structure");
    RPF_CHECK(m >= 1 && reps >= 1, RPF_EINVAL, "problem_tune: m and reps must be positive");
    RPF_CHECK(prec >= RPF_FP64 && prec <= RPF_BF16, RPF_EINVAL, "problem_tune: precision");
    check_patterns(pb, patterns, prec);
    hipStream_t s = (hipStream_t)stream;
    const int64_t N = pb->n_lambda;
    RPF_CHECK(N > 0, RPF_EINVAL, "problem_tune: structure without multipliers");
    std::vector<Schedule> cand;
    cand.push_back(Schedule{0, 1024});
    for (int tile : {64, 128})
      for (int work : {256, 512, 1024, 2048, 4096})
        if (valid_schedule(pb, patterns, prec, tile, work)) cand.push_back(Schedule{tile, work});
    if (valid_schedule(pb, patterns, prec, 256, 1)) cand.push_back(Schedule{256, 1});
    DevBuf<double> X((size_t)N * m), Y((size_t)N * m);
    hipLaunchKernelGGL(k_fill_hash, dim3((unsigned)cdiv(N * m, 256)), dim3(256), 0, s, X.p, N * m);
    RPF_LAUNCH_CHECK();
    hipEvent_t e0, e1;
    RPF_HIP(hipEventCreate(&e0));
    RPF_HIP(hipEventCreate(&e1));
    const auto saved = pb->sched;
    std::vector<double> ms(cand.size(), 0.0);
    try {
      for (size_t c = 0; c < cand.size(); ++c) {
        if (cand[c].tile == 0) pb->sched.erase({m, prec});
        else pb->sched[{m, prec}] = cand[c];
        apply_F(pb, patterns, m, X.p, m, Y.p, m, prec, false, s);  // warm-up (workspace sizes)
        RPF_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) apply_F(pb, patterns, m, X.p, m, Y.p, m, prec, false, s);
        RPF_HIP(hipEventRecord(e1, s));
        RPF_HIP(hipEventSynchronize(e1));
        float t = 0.f;
        RPF_HIP(hipEventElapsedTime(&t, e0, e1));
        ms[c] = (double)t / reps;
      }
    } catch (...) {
      pb->sched = saved;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    pb->sched = saved;
    const size_t best = (size_t)(std::min_element(ms.begin(), ms.end()) - ms.begin());
    if (cand[best].tile == 0) pb->sched.erase({m, prec});
    else pb->sched[{m, prec}] = cand[best];
    if (n_out) *n_out = (int32_t)cand.size();
    if (out)
      for (size_t c = 0; c < cand.size() && (int32_t)c < max_out; ++c)
        out[c] = rpf_schedule_entry{cand[c].tile, cand[c].work, ms[c], c == best ? 1 : 0};
  });
}
