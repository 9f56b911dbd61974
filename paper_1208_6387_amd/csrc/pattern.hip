// Pattern level: factorisation with rigid-mode detection (section 2: floating
// subdomains, kernel N, Schur complement S) and condensation to the boundary
// flexibility S+ = t K+ t^T (section 2), shared by every occurrence.
#include "pattern.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <memory>
#include <sstream>

namespace rpf {

static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }

namespace {

constexpr int KDET = 8;  // block size of the kernel detection (kernel dimension <= KDET - 1)

__global__ void k_scatter_csr(int n, const int* rowptr, const int* colind, const double* val, const int* pos,
                              double* L, int64_t ld) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int pi = pos[i];
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const int pj = pos[colind[e]];
    if (pi >= pj) L[(int64_t)pj * ld + pi] = val[e];
  }
}

__global__ void k_gather_vals(int64_t count, const int* src, const double* val, double* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) out[e] = val[src[e]];
}

// deterministic pseudo-random start block (splitmix64 of the entry index)
__global__ void k_random_block(double* V, int64_t n, int64_t ld, int k) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * k) return;
  uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull + 0x2545F4914F6CDD1Dull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  V[(i / n) * ld + (i % n)] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// column sums of |A| (one workgroup per column)
__global__ void k_colabs(const double* A, int64_t n, int64_t ld, double* out) {
  __shared__ double red[4];
  const int64_t c = blockIdx.x;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) s += fabs(A[c * ld + r]);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[c] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_max(const double* x, int64_t n, double* out) {
  __shared__ double red[4];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, x[i]);
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ void k_symmetrize(double* A, int64_t n, int64_t ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * n) return;
  const int64_t r = i % n, c = i / n;
  if (r > c) {
    const double v = 0.5 * (A[c * ld + r] + A[r * ld + c]);
    A[c * ld + r] = v;
    A[r * ld + c] = v;
  }
}

__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__global__ void k_to_f32(const double* A, int64_t count, float* f32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) f32[i] = (float)A[i];
}

// bf16 split of a symmetric n x n matrix into n rows of ldp (>= n) entries, zero padded
__global__ void k_split_bf16(const double* A, int64_t n, int64_t ldp, uint16_t* hi, uint16_t* lo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * ldp) return;
  const int64_t row = i / ldp, k = i % ldp;
  const double x = (k < n) ? A[row * n + k] : 0.0;
  const uint16_t h = bf16_rne((float)x);
  hi[i] = h;
  lo[i] = bf16_rne((float)(x - (double)bf16_to_f(h)));
}

void check_status(hipStream_t s, const int* d_status, const char* what) {
  int st = 0;
  RPF_HIP(hipMemcpyAsync(&st, d_status, sizeof(int), hipMemcpyDeviceToHost, s));
  RPF_HIP(hipStreamSynchronize(s));
  if (st != 0) {
    std::ostringstream os;
    os << what << ": non-positive pivot in diagonal block " << (st - 1);
    throw Error(RPF_ENOTSPD, os.str());
  }
}

}  // namespace
}  // namespace rpf

using namespace rpf;

extern "C" const char* rpf_last_error(void) { return rpf::g_last_error.c_str(); }
extern "C" int32_t rpf_version(void) { return 200; }

extern "C" rpf_status pattern_factor(int32_t n, const int32_t* rowptr, const int32_t* colind, const double* val,
                                     int32_t n_b, const int32_t* bdofs, int32_t dpn, double ktol,
                                     int32_t expected_kernel_dim, void* stream, rpf_pattern* out,
                                     int32_t* kernel_dim_out) {
  return guarded([&] {
    RPF_CHECK(out != nullptr, RPF_EINVAL, "pattern_factor: out is NULL");
    *out = nullptr;
    RPF_CHECK(n > 0 && rowptr && colind && val, RPF_EINVAL, "pattern_factor: empty matrix");
    RPF_CHECK(n_b >= 1 && n_b <= n && bdofs, RPF_EINVAL, "pattern_factor: bad boundary");
    RPF_CHECK(dpn >= 1 && dpn <= 3 && n % dpn == 0 && n_b % dpn == 0, RPF_EINVAL,
              "pattern_factor: dofs_per_node must divide n and n_b");
    hipStream_t s = (hipStream_t)stream;
    if (ktol <= 0) ktol = 1e-10;
    auto P = std::make_unique<rpf_pattern_s>();
    static std::atomic<uint64_t> next_uid{1};
    P->uid = next_uid.fetch_add(1);
    P->n = n;
    P->n_b = n_b;
    P->n_i = n - n_b;
    P->dpn = dpn;
    const int n_i = P->n_i;

    // ---- symbolic: ordering (interior first, boundary last), envelope, K_bi / K_ib
    std::vector<int> pos(n, -1);
    for (int b = 0; b < n_b; ++b) {
      RPF_CHECK(bdofs[b] >= 0 && bdofs[b] < n, RPF_EINVAL, "pattern_factor: boundary dof out of range");
      RPF_CHECK(b == 0 || bdofs[b] > bdofs[b - 1], RPF_EINVAL, "pattern_factor: bdofs not sorted/distinct");
      if (b % dpn == 0)
        RPF_CHECK(bdofs[b] % dpn == 0, RPF_EINVAL, "pattern_factor: bdofs must list whole nodes");
      else
        RPF_CHECK(bdofs[b] == bdofs[b - 1] + 1, RPF_EINVAL, "pattern_factor: bdofs must list whole nodes");
      pos[bdofs[b]] = n_i + b;
    }
    P->bdofs.assign(bdofs, bdofs + n_b);
    int next = 0;
    for (int i = 0; i < n; ++i)
      if (pos[i] < 0) {
        pos[i] = next++;
        P->idofs.push_back(i);
      }
    RPF_CHECK(rowptr[0] == 0 && rowptr[n] > 0, RPF_EINVAL, "pattern_factor: bad rowptr");
    const int64_t nnz = rowptr[n];
    std::vector<int> first(n_i);
    std::vector<int> kbi_ptr(n_b + 1, 0), kib_ptr(n_i + 1, 0), kbi_col, kib_col, kbi_src, kib_src;
    std::vector<int> kbb_ptr(n_b + 1, 0), kbb_col, kbb_src;
    for (int r = 0; r < n; ++r) {
      RPF_CHECK(rowptr[r + 1] >= rowptr[r], RPF_EINVAL, "pattern_factor: bad rowptr");
      const int pr = pos[r];
      int f = pr;
      bool diag = false;
      for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
        const int c = colind[e];
        RPF_CHECK(c >= 0 && c < n, RPF_EINVAL, "pattern_factor: column out of range");
        diag |= (c == r);
        const int pc = pos[c];
        if (pr < n_i) {
          if (pc < n_i) f = std::min(f, pc);
          else { kib_col.push_back(pc - n_i); kib_src.push_back(e); }
        } else if (pc < n_i) {
          kbi_col.push_back(pc);
          kbi_src.push_back(e);
        } else {
          kbb_col.push_back(pc - n_i);
          kbb_src.push_back(e);
        }
      }
      RPF_CHECK(diag, RPF_EINVAL, "pattern_factor: a row has no diagonal entry");
      if (pr < n_i) { first[pr] = f; kib_ptr[pr + 1] = (int)kib_col.size(); }
      else {
        kbi_ptr[pr - n_i + 1] = (int)kbi_col.size();
        kbb_ptr[pr - n_i + 1] = (int)kbb_col.size();
      }
    }
    const int64_t nblk = cdiv(n_i, NB);
    P->env_ii.rend.assign(nblk, 0);
    P->env_ii.cstart.assign(nblk, 0);
    {
      std::vector<int64_t> mx(nblk, 0);
      for (int i = 0; i < n_i; ++i) mx[first[i] / NB] = std::max<int64_t>(mx[first[i] / NB], i + 1);
      int64_t run = 0;
      for (int64_t t = 0; t < nblk; ++t) {
        run = std::max(run, mx[t]);
        P->env_ii.rend[t] = std::max<int64_t>(run, std::min<int64_t>(n_i, (t + 1) * NB));
        int64_t cs = (t + 1) * NB;
        for (int64_t i = t * NB; i < std::min<int64_t>(n_i, (t + 1) * NB); ++i) cs = std::min<int64_t>(cs, first[i]);
        P->env_ii.cstart[t] = cs;
      }
    }

    // ---- numeric: scatter K, partial Cholesky, Schur complement
    P->status.alloc(1);
    RPF_HIP(hipMemsetAsync(P->status.p, 0, sizeof(int), s));
    DevBuf<int> d_rowptr, d_colind, d_pos, d_src;
    d_rowptr.upload(rowptr, n + 1, s);
    d_colind.upload(colind, nnz, s);
    d_pos.upload(pos.data(), n, s);
    P->ld = n;
    P->L.alloc((size_t)n * n);
    fill(s, P->L.p, (int64_t)n * n, 0.0);
    hipLaunchKernelGGL(k_scatter_csr, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, n, d_rowptr.p, d_colind.p, val,
                       d_pos.p, P->L.p, P->ld);
    RPF_LAUNCH_CHECK();
    auto upload_csr = [&](DevBuf<int>& dptr, DevBuf<int>& dcol, DevBuf<double>& dval, const std::vector<int>& hp,
                          const std::vector<int>& hc, const std::vector<int>& hs) {
      dptr.upload(hp.data(), hp.size(), s);
      if (!hc.empty()) {
        dcol.upload(hc.data(), hc.size(), s);
        d_src.upload(hs.data(), hs.size(), s);
        dval.alloc(hc.size());
        hipLaunchKernelGGL(k_gather_vals, dim3((unsigned)cdiv((int64_t)hc.size(), 256)), dim3(256), 0, s,
                           (int64_t)hc.size(), d_src.p, val, dval.p);
        RPF_LAUNCH_CHECK();
        RPF_HIP(hipStreamSynchronize(s));  // d_src is reused
      }
    };
    upload_csr(P->kbi_ptr, P->kbi_col, P->kbi_val, kbi_ptr, kbi_col, kbi_src);
    upload_csr(P->kib_ptr, P->kib_col, P->kib_val, kib_ptr, kib_col, kib_src);
    upload_csr(P->kbb_ptr, P->kbb_col, P->kbb_val, kbb_ptr, kbb_col, kbb_src);
    P->d_bdofs.upload(P->bdofs.data(), n_b, s);
    if (n_i > 0) P->d_idofs.upload(P->idofs.data(), n_i, s);

    if (n_i > 0) {
      P->dinv_ii.alloc((size_t)nblk * NB * NB);
      potrf(s, P->L.p, P->ld, n, n_i, P->env_ii, P->dinv_ii.p, P->status.p);
      schur_update(s, P->L.p, P->ld, n, n_i);
      // L_ii^T in the (otherwise unused) upper triangle: the backward solves read it row-contiguous
      mirror_envelope(s, P->L.p, P->ld, n_i, P->env_ii);
      P->L_upper = true;
    }
    P->S.alloc((size_t)n_b * n_b);
    copy_matrix(s, P->L.p + (int64_t)n_i * P->ld + n_i, P->ld, P->S.p, n_b, n_b, n_b);
    mirror_lower(s, P->S.p, n_b, n_b);
    check_status(s, P->status.p, "pattern_factor (interior stiffness K_ii)");

    // ---- kernel detection: shifted block inverse iteration + Rayleigh-Ritz
    DevBuf<double> colsum(n_b), nrm(1);
    hipLaunchKernelGGL(k_colabs, dim3(n_b), dim3(256), 0, s, P->S.p, (int64_t)n_b, (int64_t)n_b, colsum.p);
    hipLaunchKernelGGL(k_max, dim3(1), dim3(256), 0, s, colsum.p, (int64_t)n_b, nrm.p);
    RPF_LAUNCH_CHECK();
    double normS = 0.0;
    RPF_HIP(hipMemcpyAsync(&normS, nrm.p, sizeof(double), hipMemcpyDeviceToHost, s));
    RPF_HIP(hipStreamSynchronize(s));
    RPF_CHECK(normS > 0.0 && std::isfinite(normS), RPF_ENOTSPD, "pattern_factor: Schur complement is zero or not finite");
    const int kb = std::min(KDET, n_b);
    const double sigma = 1e-9 * normS;
    DevBuf<double> C((size_t)n_b * n_b), dinvC((size_t)cdiv(n_b, NB) * NB * NB), V((size_t)n_b * kb),
        W((size_t)n_b * kb), H(kb * kb), U(kb * kb), theta(kb);
    copy_matrix(s, P->S.p, n_b, C.p, n_b, n_b, n_b);
    add_diag(s, C.p, n_b, n_b, sigma);
    const Envelope envC = Envelope::dense(n_b);
    potrf(s, C.p, n_b, n_b, n_b, envC, dinvC.p, P->status.p);
    check_status(s, P->status.p, "pattern_factor (Schur complement S + sigma I)");
    hipLaunchKernelGGL(k_random_block, dim3((unsigned)cdiv((int64_t)n_b * kb, 256)), dim3(256), 0, s, V.p,
                       (int64_t)n_b, (int64_t)n_b, kb);
    RPF_LAUNCH_CHECK();
    orthonormalize(s, V.p, n_b, n_b, kb);
    for (int it = 0; it < 3; ++it) {
      trsm(s, C.p, n_b, n_b, dinvC.p, envC, V.p, n_b, kb, false);
      trsm(s, C.p, n_b, n_b, dinvC.p, envC, V.p, n_b, kb, true);
      orthonormalize(s, V.p, n_b, n_b, kb);
    }
    dgemm(s, false, false, n_b, kb, n_b, 1.0, P->S.p, n_b, V.p, n_b, 0.0, W.p, n_b);
    dgemm(s, true, false, kb, kb, n_b, 1.0, V.p, n_b, W.p, n_b, 0.0, H.p, kb);
    syev_small(s, H.p, kb, U.p, theta.p, 1);
    std::vector<double> th(kb), hU(kb * kb);
    RPF_HIP(hipMemcpyAsync(th.data(), theta.p, kb * sizeof(double), hipMemcpyDeviceToHost, s));
    RPF_HIP(hipMemcpyAsync(hU.data(), U.p, kb * kb * sizeof(double), hipMemcpyDeviceToHost, s));
    RPF_HIP(hipStreamSynchronize(s));
    int k = 0;
    while (k < kb && th[k] < ktol * normS) ++k;
    std::ostringstream ritz;
    for (int i = 0; i < kb; ++i) ritz << (i ? ", " : "") << th[i] / normS;
    RPF_CHECK(k < kb || n_b <= KDET - 1, RPF_EKERNEL,
              "pattern_factor: kernel dimension reaches the detection block (relative Ritz values " + ritz.str() + ")");
    RPF_CHECK(expected_kernel_dim < 0 || k == expected_kernel_dim, RPF_EKERNEL,
              "pattern_factor: detected kernel dimension " + std::to_string(k) + ", expected " +
                  std::to_string(expected_kernel_dim) + " (relative Ritz values " + ritz.str() + ")");
    P->k = k;
    if (k > 0) {
      P->Z.alloc((size_t)n_b * k);
      dgemm(s, false, false, n_b, k, kb, 1.0, V.p, n_b, U.p, kb, 0.0, P->Z.p, n_b);
      orthonormalize(s, P->Z.p, n_b, n_b, k);
    }
    RPF_HIP(hipStreamSynchronize(s));
    if (kernel_dim_out) *kernel_dim_out = k;
    *out = P.release();
  });
}

extern "C" rpf_status pattern_condense(rpf_pattern p, int32_t prec, void* stream) {
  return guarded([&] {
    RPF_CHECK(p != nullptr, RPF_EINVAL, "pattern_condense: NULL pattern");
    RPF_CHECK(prec >= RPF_FP64 && prec <= RPF_BF16, RPF_EINVAL, "pattern_condense: bad precision");
    hipStream_t s = (hipStream_t)stream;
    const int nb = p->n_b;
    if (!(p->condensed & 1u)) {
      DevBuf<double> M((size_t)nb * nb), dinv((size_t)cdiv(nb, NB) * NB * NB);
      copy_matrix(s, p->S.p, nb, M.p, nb, nb, nb);
      if (p->k > 0) dgemm(s, false, true, nb, nb, p->k, 1.0, p->Z.p, nb, p->Z.p, nb, 1.0, M.p, nb);
      const Envelope env = Envelope::dense(nb);
      RPF_HIP(hipMemsetAsync(p->status.p, 0, sizeof(int), s));
      potrf(s, M.p, nb, nb, nb, env, dinv.p, p->status.p);
      p->Splus.alloc((size_t)nb * nb);
      potri_lower(s, M.p, nb, nb, dinv.p, p->Splus.p, nb);
      if (p->k > 0) dgemm(s, false, true, nb, nb, p->k, -1.0, p->Z.p, nb, p->Z.p, nb, 1.0, p->Splus.p, nb);
      hipLaunchKernelGGL(k_symmetrize, dim3((unsigned)cdiv((int64_t)nb * nb, 256)), dim3(256), 0, s, p->Splus.p,
                         (int64_t)nb, (int64_t)nb);
      RPF_LAUNCH_CHECK();
      check_status(s, p->status.p, "pattern_condense (S + Z Z^T)");
      p->condensed |= 1u;
    }
    const int64_t cnt = (int64_t)nb * nb;
    if (prec == RPF_FP32 && !(p->condensed & (1u << RPF_FP32))) {
      p->Splus32.alloc(cnt);
      hipLaunchKernelGGL(k_to_f32, dim3((unsigned)cdiv(cnt, 256)), dim3(256), 0, s, p->Splus.p, cnt, p->Splus32.p);
      p->S32.alloc(cnt);
      hipLaunchKernelGGL(k_to_f32, dim3((unsigned)cdiv(cnt, 256)), dim3(256), 0, s, p->S.p, cnt, p->S32.p);
      RPF_LAUNCH_CHECK();
      p->condensed |= 1u << RPF_FP32;
    }
    if ((prec == RPF_BF16X3 || prec == RPF_BF16) && !(p->condensed & (1u << RPF_BF16X3))) {
      p->ldlp = cdiv(nb, 64) * 64;  // 128-byte rows, the layout of the low-precision products
      const int64_t cntp = (int64_t)nb * p->ldlp;
      p->Sp_hi.alloc(cntp);
      p->Sp_lo.alloc(cntp);
      hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)cdiv(cntp, 256)), dim3(256), 0, s, p->Splus.p, (int64_t)nb,
                         p->ldlp, p->Sp_hi.p, p->Sp_lo.p);
      p->S_hi.alloc(cntp);
      p->S_lo.alloc(cntp);
      hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)cdiv(cntp, 256)), dim3(256), 0, s, p->S.p, (int64_t)nb,
                         p->ldlp, p->S_hi.p, p->S_lo.p);
      RPF_LAUNCH_CHECK();
      p->condensed |= (1u << RPF_BF16X3) | (1u << RPF_BF16);
    }
  });
}

extern "C" rpf_status pattern_info(rpf_pattern p, int32_t* n, int32_t* n_b, int32_t* k) {
  return guarded([&] {
    RPF_CHECK(p != nullptr, RPF_EINVAL, "pattern_info: NULL pattern");
    if (n) *n = p->n;
    if (n_b) *n_b = p->n_b;
    if (k) *k = p->k;
  });
}

extern "C" rpf_status pattern_export(rpf_pattern p, int32_t what, double* dst, int64_t ld, void* stream) {
  return guarded([&] {
    RPF_CHECK(p != nullptr && dst != nullptr, RPF_EINVAL, "pattern_export: NULL argument");
    RPF_CHECK(ld >= p->n_b, RPF_EINVAL, "pattern_export: ld < n_b");
    hipStream_t s = (hipStream_t)stream;
    const int nb = p->n_b;
    if (what == 0) copy_matrix(s, p->S.p, nb, dst, ld, nb, nb);
    else if (what == 1) copy_matrix(s, p->Z.p, nb, dst, ld, nb, p->k);
    else if (what == 2) {
      RPF_CHECK(p->condensed & 1u, RPF_EINVAL, "pattern_export: pattern not condensed");
      copy_matrix(s, p->Splus.p, nb, dst, ld, nb, nb);
    } else {
      throw Error(RPF_EINVAL, "pattern_export: unknown quantity");
    }
  });
}

extern "C" void pattern_free(rpf_pattern p) { delete p; }

// ---------------------------------------------------------------------------- dense helpers (C ABI)
extern "C" rpf_status rpf_dgemm(int32_t ta, int32_t tb, int64_t M, int64_t N, int64_t K, double alpha,
                                const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                                int64_t ldc, void* stream) {
  return guarded([&] {
    RPF_CHECK(M >= 0 && N >= 0 && K >= 0, RPF_EINVAL, "rpf_dgemm: negative size");
    rpf::dgemm((hipStream_t)stream, ta != 0, tb != 0, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  });
}

extern "C" rpf_status rpf_dposv(int64_t n, double* A, int64_t lda, int64_t nrhs, double* B, int64_t ldb,
                                void* stream) {
  return guarded([&] {
    RPF_CHECK(n > 0 && lda >= n, RPF_EINVAL, "rpf_dposv: bad size");
    hipStream_t s = (hipStream_t)stream;
    DevBuf<double> dinv((size_t)cdiv(n, NB) * NB * NB);
    DevBuf<int> st(1);
    RPF_HIP(hipMemsetAsync(st.p, 0, sizeof(int), s));
    const Envelope env = Envelope::dense(n);
    potrf(s, A, lda, n, n, env, dinv.p, st.p);
    if (nrhs > 0) {
      trsm(s, A, lda, n, dinv.p, env, B, ldb, nrhs, false);
      trsm(s, A, lda, n, dinv.p, env, B, ldb, nrhs, true);
    }
    check_status(s, st.p, "rpf_dposv");
  });
}

extern "C" rpf_status rpf_rows_gemm(int64_t N, int32_t a, int32_t b, double alpha, const double* X, int64_t ldx,
                                    const double* M, int64_t mrow, double beta, double* Y, int64_t ldy,
                                    void* stream) {
  return guarded([&] {
    RPF_CHECK(N >= 0 && a >= 1 && b >= 0, RPF_EINVAL, "rpf_rows_gemm: bad size");
    RPF_CHECK(ldx >= a && ldy >= b && (mrow == 0 || mrow >= b), RPF_EINVAL, "rpf_rows_gemm: leading dimension");
    if (N == 0 || b == 0) return;
    rows_gemm((hipStream_t)stream, N, a, b, alpha, X, ldx, M, beta, Y, ldy, mrow);
  });
}

extern "C" rpf_status rpf_gram(int64_t N, int32_t a, int32_t b, const double* X, int64_t ldx, const double* Y,
                               int64_t ldy, double* C, void* stream) {
  return guarded([&] {
    RPF_CHECK(N >= 0 && a >= 0 && b >= 0, RPF_EINVAL, "rpf_gram: negative size");
    RPF_CHECK(ldx >= a && ldy >= b, RPF_EINVAL, "rpf_gram: leading dimension");
    if (N == 0 || a == 0 || b == 0) return;
    hipStream_t s = (hipStream_t)stream;
    DevBuf<double> ws((size_t)gram_chunks(N, a, b) * a * b);
    gram(s, N, a, b, X, ldx, Y, ldy, C, ws.p);
    RPF_HIP(hipStreamSynchronize(s));
  });
}

extern "C" rpf_status rpf_dsyev_small(int32_t m, int32_t batch, const double* A, double* V, double* w,
                                      void* stream) {
  return guarded([&] {
    RPF_CHECK(batch >= 1, RPF_EINVAL, "rpf_dsyev_small: batch < 1");
    syev_small((hipStream_t)stream, A, m, V, w, batch);
  });
}
