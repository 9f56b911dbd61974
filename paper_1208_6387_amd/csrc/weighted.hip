// Non-Boolean assembly (section 5: assembly operators built from a mortar coupling of non-matching
// pattern meshes, which carry interface values from one discretisation to another the way the
// rotations carry them from one frame to another).  Each side of a multiplier couples several
// boundary nodes of its occurrence with real weights:
//   (A^(s) v)[(i, c)] = sum_k w_k sum_c2 O^(s)[c][c2] v[(bn_k, c2)]      over the entries k of side (i, s)
// These kernels are the general form of the gather A^(s)T, the scatter A^(s), the rows of G = A Z,
// G^T x and G^T G; a structure described with weights takes them instead of the signed Boolean ones.
#include "common.hpp"
#include "problem.hpp"

namespace rpf {
namespace {

__device__ inline uint16_t w_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float w_bf16_val(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// X_loc = A^(s)T lambda for the occurrences of one pattern, W format (column q m + j, row bn dpn + c).
// One thread per (boundary node, column) of occurrence slot q = blockIdx.y.  MODE 2: FP64 X64;
// 0: FP32 Xf; 1: bf16 high and low parts Xh, Xl.
template <int DPN, int MODE>
__global__ __launch_bounds__(256) void k_wgather(int nbn, int m, const int* occ_list, const int* slot_off,
                                                 const int* wl_ptr, const int* wl_mult, const double* wl_w,
                                                 const double* rot, const double* lam, int64_t ldl, double* X64,
                                                 float* Xf, uint16_t* Xh, uint16_t* Xl, int64_t ldx) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nbn * m) return;
  const int bn = (int)(t / m), j = (int)(t % m);
  const int q = blockIdx.y;
  const int s = occ_list[q];
  const int slot = slot_off[s] + bn;
  double g[DPN];
#pragma unroll
  for (int c = 0; c < DPN; ++c) g[c] = 0.0;
  for (int k = wl_ptr[slot]; k < wl_ptr[slot + 1]; ++k) {
    const int64_t i = wl_mult[k];
    const double w = wl_w[k];
#pragma unroll
    for (int c = 0; c < DPN; ++c) g[c] += w * lam[(i * DPN + c) * ldl + j];
  }
  const double* O = rot ? rot + 9 * (int64_t)s : nullptr;
#pragma unroll
  for (int c2 = 0; c2 < DPN; ++c2) {
    const double v = (DPN == 3 && O) ? O[c2] * g[0] + O[3 + c2] * g[1 % DPN] + O[6 + c2] * g[2 % DPN] : g[c2];
    const int64_t o = ((int64_t)q * m + j) * ldx + (int64_t)bn * DPN + c2;
    if (MODE == 2) {
      X64[o] = v;
    } else if (MODE == 0) {
      Xf[o] = (float)v;
    } else {
      const uint16_t h = w_bf16((float)v);
      Xh[o] = h;
      Xl[o] = w_bf16((float)(v - (double)w_bf16_val(h)));
    }
  }
}

// Y = A Y_loc: one thread per (multiplier, column); the local results are column-major per pattern
// (column q m + j, row bn dpn + c), nsplit partial slabs `slab` apart, in FP64 or FP32.
template <int DPN, typename T>
__global__ __launch_bounds__(256) void k_wscatter(int n_mult, int m, const int* ep_q, const int* ep_occ,
                                                  const int8_t* ep_pat, const int* wm_ptr, const int* wm_bn,
                                                  const double* wm_w, const double* rot, WLoc<T> yl, double* Y,
                                                  int64_t ldy) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n_mult * m) return;
  const int64_t i = t / m;
  const int j = (int)(t % m);
  double acc[DPN];
#pragma unroll
  for (int c = 0; c < DPN; ++c) acc[c] = 0.0;
  for (int e = 0; e < 2; ++e) {
    const int s = ep_occ[2 * i + e];
    if (s < 0) continue;
    const int p = ep_pat[2 * i + e];
    const T* base = yl.base[p] + ((int64_t)ep_q[2 * i + e] * m + j) * yl.ld[p];
    double v[DPN];
#pragma unroll
    for (int c = 0; c < DPN; ++c) v[c] = 0.0;
    for (int k = wm_ptr[2 * i + e]; k < wm_ptr[2 * i + e + 1]; ++k) {
      const int64_t row = (int64_t)wm_bn[k] * DPN;
      const double w = wm_w[k];
#pragma unroll
      for (int c = 0; c < DPN; ++c) {
        double y = (double)base[row + c];  // slab 0, then the other K splits (none when nsplit <= 1)
        for (int z = 1; z < yl.nsplit[p]; ++z) y += (double)base[(int64_t)z * yl.slab[p] + row + c];
        v[c] += w * y;
      }
    }
    const double* O = rot ? rot + 9 * (int64_t)s : nullptr;
#pragma unroll
    for (int c = 0; c < DPN; ++c)
      acc[c] += (DPN == 3 && O) ? O[3 * c] * v[0] + O[3 * c + 1] * v[1 % DPN] + O[3 * c + 2] * v[2 % DPN] : v[c];
  }
#pragma unroll
  for (int c = 0; c < DPN; ++c) Y[(i * DPN + c) * ldy + j] = acc[c];
}

// rows of G = A Z per (multiplier, side): Grow[((i 2 + e) DPN + c) km + r] = sum_k w_k (O Z[bn_k])[c][r]
template <int DPN>
__global__ void k_wbuild_grows(int n_mult, int km, const int* ep_occ, const int* occ_pat, const int* nbn_p,
                               const double* const* Zp, const int* kp, const int* goff, const int* wm_ptr,
                               const int* wm_bn, const double* wm_w, const double* rot, double* Grow, int* ep_goff) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = 2 * DPN * km;
  if (t >= (int64_t)n_mult * per) return;
  const int r = (int)(t % km), c = (int)((t / km) % DPN), e = (int)((t / (km * DPN)) % 2);
  const int64_t i = t / per;
  const int s = ep_occ[2 * i + e];
  double v = 0.0;
  if (s >= 0) {
    const int p = occ_pat[s];
    if (r < kp[p]) {
      const int64_t ldz = (int64_t)nbn_p[p] * DPN;
      const double* O = rot ? rot + 9 * (int64_t)s : nullptr;
      for (int k = wm_ptr[2 * i + e]; k < wm_ptr[2 * i + e + 1]; ++k) {
        const double* zr = Zp[p] + (int64_t)wm_bn[k] * DPN + r * ldz;
        const double z = (DPN == 3 && O) ? O[3 * c] * zr[0] + O[3 * c + 1] * zr[1 % DPN] + O[3 * c + 2] * zr[2 % DPN]
                                          : zr[c];
        v += wm_w[k] * z;
      }
    }
  }
  Grow[t] = v;
  if (r == 0 && c == 0) ep_goff[2 * i + e] = s >= 0 ? goff[s] : -1;
}

// c = G^T x (n_G x m row-major) from the stored rows of G: one workgroup per occurrence, its k x m
// entries over the threads, the multiplier sides that touch it in a fixed order
template <int DPN>
__global__ __launch_bounds__(256) void k_wcoarse_gt(int km, const int* occ_pat, const int* kp, const int* goff,
                                                    const int* wo_ptr, const int* wo_me, const double* Grow,
                                                    const double* x, int64_t ldx, int m, double* cc) {
  const int o = blockIdx.x;
  const int k = kp[occ_pat[o]];
  for (int t = threadIdx.x; t < k * m; t += blockDim.x) {
    const int a = t / m, j = t % m;
    double acc = 0.0;
    for (int u = wo_ptr[o]; u < wo_ptr[o + 1]; ++u) {
      const int64_t me = wo_me[u], i = me >> 1;
      const double* g = Grow + me * DPN * km;
#pragma unroll
      for (int c = 0; c < DPN; ++c) acc += g[c * km + a] * x[(i * DPN + c) * ldx + j];
    }
    cc[((int64_t)goff[o] + a) * m + j] = acc;
  }
}

// G^T G from the stored rows of G.  Diagonal block of occurrence o: sum over its sides of
// G_side^T G_side; block of a pair (A, B): sum over the multipliers joining them of
// G_(i, side on A)^T G_(i, side on B).  One workgroup per occurrence or pair, entries over threads.
template <int DPN>
__global__ __launch_bounds__(256) void k_wgtg_diag(int km, const int* occ_pat, const int* kp, const int* goff,
                                                   const int* wo_ptr, const int* wo_me, const double* Grow,
                                                   double* GtG, int64_t ldg) {
  const int o = blockIdx.x;
  const int k = kp[occ_pat[o]];
  for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
    const int a = t / k, b = t % k;
    double acc = 0.0;
    for (int u = wo_ptr[o]; u < wo_ptr[o + 1]; ++u) {
      const double* g = Grow + (int64_t)wo_me[u] * DPN * km;
#pragma unroll
      for (int c = 0; c < DPN; ++c) acc += g[c * km + a] * g[c * km + b];
    }
    GtG[((int64_t)goff[o] + b) * ldg + goff[o] + a] = acc;
  }
}

template <int DPN>
__global__ __launch_bounds__(256) void k_wgtg_pairs(int km, const int* pair_a, const int* pair_b, const int* pair_ptr,
                                                    const int* pair_mult, const int* ep_occ, const int* occ_pat,
                                                    const int* kp, const int* goff, const double* Grow, double* GtG,
                                                    int64_t ldg) {
  const int w = blockIdx.x;
  const int A = pair_a[w], B = pair_b[w];
  const int ka = kp[occ_pat[A]], kb = kp[occ_pat[B]];
  for (int t = threadIdx.x; t < ka * kb; t += blockDim.x) {
    const int a = t / kb, b = t % kb;
    double acc = 0.0;
    for (int u = pair_ptr[w]; u < pair_ptr[w + 1]; ++u) {
      const int64_t i = pair_mult[u];
      const int ea = ep_occ[2 * i] == A ? 0 : 1;
      const double* ga = Grow + (i * 2 + ea) * DPN * km;
      const double* gb = Grow + (i * 2 + (1 - ea)) * DPN * km;
#pragma unroll
      for (int c = 0; c < DPN; ++c) acc += ga[c * km + a] * gb[c * km + b];
    }
    GtG[((int64_t)goff[B] + b) * ldg + goff[A] + a] = acc;
    GtG[((int64_t)goff[A] + a) * ldg + goff[B] + b] = acc;
  }
}
}  // namespace

#define RPF_BY_DPN(D, ...) \
  switch (D) {             \
    case 1: __VA_ARGS__(1); break; \
    case 2: __VA_ARGS__(2); break; \
    default: __VA_ARGS__(3);       \
  }

void wgather(rpf_problem pb, int p, const double* lam, int64_t ldl, int m, int mode, double* X64, float* Xf,
             uint16_t* Xh, uint16_t* Xl, int64_t ldx, hipStream_t s) {
  const int nq = (int)pb->occ_of_pat[p].size(), nbn = pb->pat_nbn[p];
  if (nq == 0 || nbn == 0) return;
  const dim3 grid((unsigned)cdiv((int64_t)nbn * m, 256), (unsigned)nq);
  const int* occ = pb->d_occ_of_pat.p + pb->pat_occ_off[p];
  const double* rot = pb->has_rot ? pb->d_rot.p : nullptr;
#define RPF_WG(D, MODE)                                                                                      \
  hipLaunchKernelGGL((k_wgather<D, MODE>), grid, dim3(256), 0, s, nbn, m, occ, pb->d_slot_off.p,             \
                     pb->d_wl_ptr.p, pb->d_wl_mult.p, pb->d_wl_w.p, rot, lam, ldl, X64, Xf, Xh, Xl, ldx)
#define RPF_WG2(D) RPF_WG(D, 2)
#define RPF_WG0(D) RPF_WG(D, 0)
#define RPF_WG1(D) RPF_WG(D, 1)
  if (mode == 2) {
    RPF_BY_DPN(pb->dpn, RPF_WG2)
  } else if (mode == 0) {
    RPF_BY_DPN(pb->dpn, RPF_WG0)
  } else {
    RPF_BY_DPN(pb->dpn, RPF_WG1)
  }
#undef RPF_WG0
#undef RPF_WG1
#undef RPF_WG2
#undef RPF_WG
  RPF_LAUNCH_CHECK();
}

template <typename T>
void wscatter(rpf_problem pb, const WLoc<T>& yl, int m, double* Y, int64_t ldy, hipStream_t s) {
  if (pb->n_mult == 0) return;
  const dim3 grid((unsigned)cdiv((int64_t)pb->n_mult * m, 256));
  const double* rot = pb->has_rot ? pb->d_rot.p : nullptr;
#define RPF_WS(D)                                                                                              \
  hipLaunchKernelGGL((k_wscatter<D, T>), grid, dim3(256), 0, s, pb->n_mult, m, pb->d_ep_q.p, pb->d_ep_occ.p,    \
                     pb->d_ep_pat.p, pb->d_wm_ptr.p, pb->d_wm_bn.p, pb->d_wm_w.p, rot, yl, Y, ldy)
  RPF_BY_DPN(pb->dpn, RPF_WS)
#undef RPF_WS
  RPF_LAUNCH_CHECK();
}
template void wscatter<double>(rpf_problem, const WLoc<double>&, int, double*, int64_t, hipStream_t);
template void wscatter<float>(rpf_problem, const WLoc<float>&, int, double*, int64_t, hipStream_t);

void wcoarse_setup(rpf_problem pb, double* GtG, int64_t ldg, hipStream_t s) {
  const int km = pb->g_km;
  if (pb->n_mult > 0) {
    const int64_t tot = (int64_t)pb->n_mult * 2 * pb->dpn * km;
    pb->d_grow.ensure((size_t)tot);
    pb->d_ep_goff.ensure((size_t)2 * pb->n_mult);
    const double* rot = pb->has_rot ? pb->d_rot.p : nullptr;
#define RPF_WB(D)                                                                                              \
  hipLaunchKernelGGL(k_wbuild_grows<D>, dim3((unsigned)cdiv(tot, 256)), dim3(256), 0, s, pb->n_mult, km,          \
                     pb->d_ep_occ.p, pb->d_occ_pat.p, pb->d_nbn.p, pb->d_Zp.p, pb->d_kp.p, pb->d_goff.p,          \
                     pb->d_wm_ptr.p, pb->d_wm_bn.p, pb->d_wm_w.p, rot, pb->d_grow.p, pb->d_ep_goff.p)
    RPF_BY_DPN(pb->dpn, RPF_WB)
#undef RPF_WB
    RPF_LAUNCH_CHECK();
  }
#define RPF_WD(D)                                                                                              \
  hipLaunchKernelGGL(k_wgtg_diag<D>, dim3((unsigned)pb->n_occ), dim3(256), 0, s, km, pb->d_occ_pat.p, pb->d_kp.p,  \
                     pb->d_goff.p, pb->d_wo_ptr.p, pb->d_wo_me.p, pb->d_grow.p, GtG, ldg)
  RPF_BY_DPN(pb->dpn, RPF_WD)
#undef RPF_WD
  RPF_LAUNCH_CHECK();
  if (!pb->pair_a.empty()) {
#define RPF_WP(D)                                                                                              \
  hipLaunchKernelGGL(k_wgtg_pairs<D>, dim3((unsigned)pb->pair_a.size()), dim3(256), 0, s, km, pb->d_pair_a.p,      \
                     pb->d_pair_b.p, pb->d_pair_ptr.p, pb->d_pair_mult.p, pb->d_ep_occ.p, pb->d_occ_pat.p,          \
                     pb->d_kp.p, pb->d_goff.p, pb->d_grow.p, GtG, ldg)
    RPF_BY_DPN(pb->dpn, RPF_WP)
#undef RPF_WP
    RPF_LAUNCH_CHECK();
  }
}

void wcoarse_gt(rpf_problem pb, const double* x, int64_t ldx, int m, double* c, hipStream_t s) {
#define RPF_WT(D)                                                                                              \
  hipLaunchKernelGGL(k_wcoarse_gt<D>, dim3((unsigned)pb->n_occ), dim3(256), 0, s, pb->g_km, pb->d_occ_pat.p,       \
                     pb->d_kp.p, pb->d_goff.p, pb->d_wo_ptr.p, pb->d_wo_me.p, pb->d_grow.p, x, ldx, m, c)
  RPF_BY_DPN(pb->dpn, RPF_WT)
#undef RPF_WT
  RPF_LAUNCH_CHECK();
}
#undef RPF_BY_DPN

}  // namespace rpf
