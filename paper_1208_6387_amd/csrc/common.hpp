// Internal helpers of the repeated-pattern FETI library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/rpfeti.h"

namespace rpf {

typedef double v4d __attribute__((ext_vector_type(4)));

// Exact timing of one kernel: when the tracer has armed a (start, stop) pair for this thread, the
// next RPF_TIMED_LAUNCH records them around the kernel itself (hipExtLaunchKernelGGL) and disarms.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
LaunchEvents& launch_events();
#define RPF_TIMED_LAUNCH(K, G, B, SH, S, ...)                                          \
  do {                                                                                 \
    rpf::LaunchEvents& le_ = rpf::launch_events();                                     \
    if (le_.start) {                                                                   \
      hipExtLaunchKernelGGL(K, G, B, SH, S, le_.start, le_.stop, 0u, __VA_ARGS__);     \
      le_.start = le_.stop = nullptr;                                                  \
    } else {                                                                           \
      hipLaunchKernelGGL(K, G, B, SH, S, __VA_ARGS__);                                 \
    }                                                                                  \
  } while (0)

// XCD-aware tile order for 2-D GEMM grids.  Workgroups are dispatched round-robin over the 8
// XCDs, each with its own L2.  The tiles are listed group by group of CG column tiles, row tile
// by row tile inside a group, and XCD x takes the x-th contiguous eighth of that list; the
// workgroups that run together on one XCD then share their row panel of A in its L2 (and the
// group's column panels of B while they stay resident).  Identity when the counts do not divide.
template <int CG = 8>
__device__ inline void xcd_tile(int nx, int ny, int& tx, int& ty) {
  constexpr int NXCD = 8;
  const int cg = ny < CG ? ny : CG;
  const int T = nx * ny;
  if (T % NXCD != 0 || ny % cg != 0) {
    tx = blockIdx.x;
    ty = blockIdx.y;
    return;
  }
  const int w = blockIdx.x + nx * blockIdx.y;
  const int q = (w % NXCD) * (T / NXCD) + w / NXCD;
  const int cc = q % cg, r = (q / cg) % nx, g = q / (cg * nx);
  tx = r;
  ty = g * cg + cc;
}
typedef float v4f __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------------------- errors
// Errors travel as C++ exceptions inside the library and are turned into a
// status code plus a thread-local message at every C entry point.
struct Error : std::runtime_error {
  rpf_status code;
  Error(rpf_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define RPF_HIP(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::rpf::Error(RPF_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

#define RPF_CHECK(cond, code, msg)                          \
  do {                                                      \
    if (!(cond)) throw ::rpf::Error((code), (msg));         \
  } while (0)

#define RPF_LAUNCH_CHECK() RPF_HIP(hipGetLastError())

template <class F>
rpf_status guarded(F&& f) {
  try {
    f();
    return RPF_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return RPF_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return RPF_EINVAL;
  }
}

// ----------------------------------------------------------------------------- device memory
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    hipError_t e = hipMalloc((void**)&p, count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      throw Error(RPF_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    n = count;
  }
  // grow-only reallocation (contents are not preserved)
  void ensure(size_t count) { if (count > n) alloc(count); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void upload(const T* h, size_t count, hipStream_t s) {
    ensure(count);
    if (count) RPF_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
  T* get() const { return p; }
};

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ----------------------------------------------------------------------------- dense FP64 kernels
constexpr int NB = 64;  // block size of the blocked Cholesky and triangular solves

// C = alpha op(A) op(B) + beta C (column-major).  lower: only entries with m >= n are written.
void dgemm(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
           const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
           int64_t ldc, bool lower = false);

// Output tiles of the configuration dgemm picks for an M x N product.
int gemm_tiles(int64_t M, int64_t N);
// NN product split over K into `splits` partial M x N slabs part[z*M*N + n*M + m]
// (no reduction; the consumer sums the slabs).  The split boundaries are
// multiples of 16, so at most cdiv(K, 16) slabs are non-empty; callers size part
// for `splits` slabs and must read exactly splits_used(K, splits) of them.
void dgemm_partials(hipStream_t s, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* B,
                    int64_t ldb, double* part, int splits);
inline int splits_used(int64_t K, int splits) {
  if (splits <= 1) return 1;
  const int64_t kchunk = ((K + splits - 1) / splits + 15) / 16 * 16;
  return (int)((K + kchunk - 1) / kchunk);
}

// Split-K form for contractions with a long K and a small M x N output; ws holds
// splits * M * N doubles (see gemm_splitk_workspace).
int gemm_splitk_count(int64_t M, int64_t N, int64_t K);
void dgemm_splitk(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                  const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                  int64_t ldc, double* ws, int splits);

// Tall-skinny Gram C (a x b, column-major ld a) = X^T Y for row-major X (N x a, ldx)
// and Y (N x b, ldy); ws must hold gram_chunks(N, a, b) * a * b doubles.
int gram_chunks(int64_t N, int a, int b);
// C (a x (b1 + b2), column-major ld a) = X^T [Y1 | Y2]; one pass over X when a, b1, b2 <= 16.
// ws must hold gram_pair_chunks(N) * a * (b1 + b2) doubles (and what two gram calls need).
// chunks (and partial-sum slabs of a x (b1 + b2) each) of gram_pair over N rows when a, b1, b2 <= 16
int gram_pair_chunks(int64_t N);
void gram_pair(hipStream_t s, int64_t N, int a, const double* X, int64_t ldx, int b1, const double* Y1,
               int64_t ldy1, int b2, const double* Y2, int64_t ldy2, double* C, double* ws);
void gram(hipStream_t s, int64_t N, int a, int b, const double* X, int64_t ldx, const double* Y, int64_t ldy,
          double* C, double* ws);

// Row-block product for tall interface blocks: Y (N x b, row-major ldy) = beta Y
// + alpha X (N x a, row-major ldx) M, M an a x b matrix stored column-major with
// ld a (mrow = 0) or row-major with ld mrow (mrow > 0).
void rows_gemm(hipStream_t s, int64_t N, int a, int b, double alpha, const double* X, int64_t ldx, const double* M,
               double beta, double* Y, int64_t ldy, int64_t mrow = 0);
// Y = beta Z + alpha X M with the beta term read from another block Z (a <= 64, b <= 16, M
// column-major with ld a).
void rows_gemm_from(hipStream_t s, int64_t N, int a, int b, double alpha, const double* X, int64_t ldx,
                    const double* M, double beta, const double* Z, int64_t ldz, double* Y, int64_t ldy);
// The paired product below (a, b <= 16, M column-major) that also returns the column sums of
// squares of Y2 after the update: sq[c * ldsq], c < b (part: cdiv(N, 256) * b doubles of
// workspace).  Returns false, doing nothing, when the block is too wide.
// C = alpha A B (+ beta C) on the large-problem FP64 kernel (the flexibility product): column-major,
// M and lda even, A and B 16-byte aligned, ldb a multiple of 32 with B's rows K .. ldb zero in
// every column.  lower: only the tiles that reach the lower triangle of C are computed.  Returns
// false (nothing launched) when those conditions do not hold.
bool dgemm_flex(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                const double* B, int64_t ldb, double beta, double* C, int64_t ldc, bool lower = false);
// Z = R - X M1 (b columns) and Lam += X M2 (c columns) from one read of X (N x a); a, b, c <= 16,
// M1 and M2 column-major with a rows.  Returns false (nothing launched) for other shapes.
bool rows_orth_lam(hipStream_t s, int64_t N, int a, int b, int c, const double* X, int64_t ldx, const double* M1,
                   const double* R, int64_t ldr, double* Z, int64_t ldz, const double* M2, double* Lam, int64_t ldl);
// Y = beta Y + alpha X M (a, b <= 16, b divides 256), and from the same pass: sq[c * ldsq] = the
// squared column norms of the new Y (skipped when sq is NULL) and G (a x b, column-major) =
// X^T Y_new.  sqpart and gpart are workspaces of (cdiv(N, 256) + 256) * b and
// (cdiv(N, 256) + 256) * a * b doubles.  Returns false (nothing launched) when the shape is not supported.
bool rows_update_gram(hipStream_t s, int64_t N, int a, int b, const double* M, const double* X, int64_t ldx,
                      double alpha, double beta, double* Y, int64_t ldy, double* sqpart, double* sq, int64_t ldsq,
                      double* gpart, double* G);
bool rows_gemm2_sq(hipStream_t s, int64_t N, int a, int b, const double* M, double alpha1, const double* X1,
                   int64_t ldx1, double beta1, double* Y1, int64_t ldy1, double alpha2, const double* X2,
                   int64_t ldx2, double beta2, double* Y2, int64_t ldy2, double* part, double* sq, int64_t ldsq);
// Two such products sharing M in one launch: Y1 = beta1 Y1 + alpha1 X1 M, Y2 = beta2 Y2 + alpha2 X2 M.
void rows_gemm2(hipStream_t s, int64_t N, int a, int b, const double* M, int64_t mrow, double alpha1,
                const double* X1, int64_t ldx1, double beta1, double* Y1, int64_t ldy1, double alpha2,
                const double* X2, int64_t ldx2, double beta2, double* Y2, int64_t ldy2);

// Envelope description of a lower factor: for column block t (NB columns),
// rows [t*NB+jb, rend[t]) below the diagonal block may be nonzero, and the
// rows of block t have nonzeros only from column cstart[t] on.
struct Envelope {
  std::vector<int64_t> rend, cstart;
  static Envelope dense(int64_t n);
};

// In-place blocked right-looking Cholesky of the leading n_fac columns of the
// n x n symmetric matrix A (lower triangle).  Rows >= n_fac are dense
// ("boundary") rows; the trailing block A[n_fac:, n_fac:] is NOT updated here
// (use schur_update).  dinv receives the inverse of every NB x NB diagonal
// block (cdiv(n_fac, NB) * NB * NB doubles).  A non-positive pivot sets *status.
void potrf(hipStream_t s, double* A, int64_t lda, int64_t n, int64_t n_fac, const Envelope& env,
           double* dinv, int* status);
// A[n_fac:, n_fac:] -= L_b L_b^T  with L_b = A[n_fac:, :n_fac] (lower triangle).
void schur_update(hipStream_t s, double* A, int64_t lda, int64_t n, int64_t n_fac);

// B <- L^{-1} B (trans = false) or L^{-T} B (trans = true), L = leading n x n of a factor.
// upper: the strict upper triangle of L's envelope holds L^T (mirror_envelope has run on it), so the
// transposed solve reads the rows of L^T as contiguous columns.
void trsm(hipStream_t s, const double* L, int64_t ldl, int64_t n, const double* dinv,
          const Envelope& env, double* B, int64_t ldb, int64_t nrhs, bool trans, bool upper = false);
// A[c, r] = A[r, c] for every entry r > c of the envelope of the leading n x n factor (column block
// t: rows up to env.rend[t]); the lower triangle is left as it is.
void mirror_envelope(hipStream_t s, double* A, int64_t lda, int64_t n, const Envelope& env);

// fill / copy helpers
// Y = (L L^T)^{-1} (full, symmetric) from a dense lower Cholesky factor and its inverted diagonal blocks
void potri_lower(hipStream_t s, const double* L, int64_t ldl, int64_t n, const double* dinv, double* Y,
                 int64_t ldy);
void fill(hipStream_t s, double* p, int64_t count, double v);
void fill_matrix(hipStream_t s, double* p, int64_t rows, int64_t cols, int64_t ld, double v);
void copy_matrix(hipStream_t s, const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                 int64_t cols);
void mirror_lower(hipStream_t s, double* A, int64_t lda, int64_t n);  // upper <- lower^T
void add_diag(hipStream_t s, double* A, int64_t lda, int64_t n, double v);

// Symmetric eigen-decomposition of small m x m matrices (m <= 64), one
// workgroup each: A (m x m, ld m, column-major) -> V (columns), w ascending.
void syev_small(hipStream_t s, const double* A, int m, double* V, double* w, int batch = 1);
// Block-solver normalisation T = V diag(w^{-1/2}) over the kept eigenpairs of eta (w_i > tau *
// max(w_max, state[1])), skipped when state[0] != 0; drops counted, flag0/flag1 set when none kept.
void eta_eigen_T(hipStream_t s, const double* eta, int m, const double* state, double tau, double* T, int* drops,
                 double* flag0, double* flag1);

// Orthonormalise the k columns of Y (n x k, ld) in place (modified Gram-Schmidt, twice).
void orthonormalize(hipStream_t s, double* Y, int64_t n, int64_t ld, int k);

}  // namespace rpf
