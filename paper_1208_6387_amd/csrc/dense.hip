// Dense FP64 building blocks for gfx950: MFMA GEMM (with split-K), blocked
// band-aware Cholesky, triangular solves through inverted diagonal blocks,
// small symmetric eigen-decompositions and block orthonormalisation.
//
// The Cholesky factors of a pattern's interior stiffness, of S + Z Z^T and of
// the coarse matrix G^T G (section 2 of the paper) all run through potrf; the
// flexibility product S+ W (section 3.2) and every trailing update run through
// the same MFMA GEMM.
#include "common.hpp"
#include "problem.hpp"

#include <algorithm>
#include <cmath>

namespace rpf {

// ============================================================================ GEMM
// Column-major C = alpha op(A) op(B) + beta C with v_mfma_f64_16x16x4_f64.
// The MFMA is issued with the B fragment as its first operand, so the 16x16
// accumulator holds a transposed C block: lane l, item r is C[l % 16][l / 16 + 4 r]
// (the f64 accumulator layout strides its 4 items by 4 rows), and lanes 0..15
// of one item store 16 consecutive doubles of a column of C (coalesced).
// Operand tiles are staged through LDS (k-major); the next K tile is loaded
// into registers while the current one is consumed.
// One output tile (tx, ty) of K split z, called with the same tile by every thread of the
// workgroup (consecutive tiles of the grouped kernel reuse the LDS: the barrier that opens each k
// stage orders a tile's stores after the previous tile's reads).
template <int BM, int BN, int WGM, int WGN, bool TA, bool TB>
__device__ __forceinline__ void dgemm_tile(int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                                           int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                                           int64_t ldc, int lower, int64_t kchunk, double* part, int tx, int ty,
                                           int z) {
  constexpr int BK = 16, PAD = 2;
  constexpr int WTM = BM / WGM, WTN = BN / WGN, TM = WTM / 16, TN = WTN / 16;
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
  static_assert(WGM * WGN == 4 && TM >= 1 && TN >= 1 && EA >= 1 && EB >= 1, "bad tile");
  __shared__ double sA[BK][BM + PAD];
  __shared__ double sB[BK][BN + PAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int64_t m0 = (int64_t)tx * BM, n0 = (int64_t)ty * BN;
  if (lower && n0 >= m0 + BM) return;  // tile strictly above the diagonal
  const int64_t kbeg = (int64_t)z * kchunk;
  const int64_t kend = K < kbeg + kchunk ? K : kbeg + kchunk;

  v4d acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  double ra[EA], rb[EB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + e * 256;
      const int mm = TA ? idx / BK : idx % BM;
      const int kk = TA ? idx % BK : idx / BM;
      const int64_t gm = m0 + mm, gk = k0 + kk;
      ra[e] = (gm < M && gk < kend) ? (TA ? A[gm * lda + gk] : A[gk * lda + gm]) : 0.0;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + e * 256;
      const int nn = TB ? idx % BN : idx / BK;
      const int kk = TB ? idx / BN : idx % BK;
      const int64_t gn = n0 + nn, gk = k0 + kk;
      rb[e] = (gn < N && gk < kend) ? (TB ? B[gk * ldb + gn] : B[gn * ldb + gk]) : 0.0;
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + e * 256;
      const int mm = TA ? idx / BK : idx % BM;
      const int kk = TA ? idx % BK : idx / BM;
      sA[kk][mm] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + e * 256;
      const int nn = TB ? idx % BN : idx / BK;
      const int kk = TB ? idx / BN : idx % BK;
      sB[kk][nn] = rb[e];
    }
  };

  if (kbeg < kend) gload(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
    sstore();
    __syncthreads();
    if (k0 + BK < kend) gload(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double af[TM], bf[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = sA[kk + (lane >> 4)][wm * WTM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j) bf[j] = sB[kk + (lane >> 4)][wn * WTN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[j], af[i], acc[i][j], 0, 0, 0);
    }
  }

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * WTM + i * 16 + (lane & 15);
        const int64_t n = n0 + wn * WTN + j * 16 + (lane >> 4) + 4 * r;
        if (m < M && n < N && (!lower || m >= n)) {
          const double v = alpha * acc[i][j][r];
          if (part) {
            part[((int64_t)z * N + n) * M + m] = v;
          } else {
            double* c = C + n * ldc + m;
            *c = (beta == 0.0) ? v : v + beta * *c;
          }
        }
      }
}

template <int BM, int BN, int WGM, int WGN, bool TA, bool TB>
__global__ __launch_bounds__(256) void k_dgemm(int64_t M, int64_t N, int64_t K, double alpha,
                                               const double* A, int64_t lda, const double* B,
                                               int64_t ldb, double beta, double* C, int64_t ldc,
                                               int lower, int64_t kchunk, double* part) {
  int tx, ty;
  xcd_tile(gridDim.x, gridDim.y, tx, ty);
  dgemm_tile<BM, BN, WGM, WGN, TA, TB>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, lower, kchunk, part, tx, ty,
                                       blockIdx.z);
}

// Every pattern's FP64 flexibility product in one persistent launch (see k_gemm_bf16_group):
// C_p = A_p B_p into split-K slabs part_p (M x N each, column-major).
template <int BM, int BN>
__global__ __launch_bounds__(256) void k_dgemm_group(const DGroup g) {
  for (int t = blockIdx.x; t < g.start[g.n]; t += gridDim.x) {
    int p = 0;
    while (t >= g.start[p + 1]) ++p;
    const int l = t - g.start[p];
    const int per_z = g.tm[p] * g.tn[p];
    const int z = l / per_z, r = l - z * per_z;
    dgemm_tile<BM, BN, 2, 2, false, false>(g.M[p], g.N[p], g.K[p], 1.0, g.A[p], g.lda[p], g.B[p], g.ldb[p], 0.0,
                                           nullptr, 0, 0, g.kchunk[p], g.part[p], r % g.tm[p], r / g.tm[p], z);
  }
}

// FP64 C = alpha A B (+ beta C), column-major; A: M x K with lda, B: K x N with ldb, its k-contiguous
// columns padded with zeros to a multiple of 32; M and lda even (16-byte loads of A).  The
// flexibility product's large-problem kernel: 128 x 128 tiles, eight waves of 64 x 32 (two per
// SIMD, so one wave's LDS waits overlap the other's MFMAs), 32-k stages loaded straight into two
// LDS buffers, the next stage issued right after the barrier that opens the current one (a whole
// stage of MFMA work covers the load latency).  Same per-accumulator summation order as k_dgemm,
// so the same bits.  A stage: A as 32 k-rows of 128 doubles (+16 pad: the two k-rows a
// half-wave reads sit on opposite bank halves); B as 128 n-rows of 32 doubles with 16-byte chunk
// kc stored at kc ^ (n % 16) (conflict-free fragment reads).  Rows past M or N are clamped to the
// last row (their results are never stored); k-rows of A past K are clamped too and meet the
// zero padding of B.
template <bool BETA>
__global__ __launch_bounds__(512) void k_dgemm_big(int M, int N, int K, double alpha, const double* __restrict__ A,
                                                   int64_t lda, const double* __restrict__ B, int64_t ldb, double beta,
                                                   double* __restrict__ C, int64_t ldc, int lower) {
  constexpr int BK = 32, RA = 128 + 16, SA = BK * RA, SB = 128 * BK;
  __shared__ __attribute__((aligned(1024))) double lA0[SA];
  __shared__ __attribute__((aligned(1024))) double lA1[SA];
  __shared__ __attribute__((aligned(1024))) double lB0[SB];
  __shared__ __attribute__((aligned(1024))) double lB1[SB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;  // wave tile 64 (m) x 32 (n)
  int tx, ty;
  xcd_tile(gridDim.x, gridDim.y, tx, ty);
  const int m0 = tx * 128, n0 = ty * 128;
  // lower: only tiles that reach the lower triangle (n <= m somewhere) are computed
  if (lower && n0 > m0 + 127) return;
  const int nst = (K + BK - 1) / BK;
  // loads of a stage: wave w takes A k-rows 4w .. 4w + 3 (lane l: doubles m0 + 2l, 2l + 1) and
  // B blocks 4w .. 4w + 3 of four n-rows (lane l: n-row l / 16, chunk (l % 16) ^ (n % 16))
  const int am = min(m0 + 2 * lane, M - 2);
  const double* asrc = A + am;
  const double* bsrc[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int nl = 4 * (4 * wave + e) + (lane >> 4);
    const int n = min(n0 + nl, N - 1);
    const int kc = (lane & 15) ^ (nl & 15);
    bsrc[e] = B + (int64_t)n * ldb + 2 * kc;
  }
  auto issue = [&](double* la, double* lb, int k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int kr = 4 * wave + e;
      const int k = min(k0 + kr, K - 1);  // k past K: finite A values times zero B padding
      __builtin_amdgcn_global_load_lds((const void*)(asrc + (int64_t)k * lda), (void*)(la + kr * RA), 16, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
      __builtin_amdgcn_global_load_lds((const void*)(bsrc[e] + k0), (void*)(lb + (4 * wave + e) * 128), 16, 0, 0);
  };
  v4d acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
  const int fl = lane & 15, fk = lane >> 4;
  auto stage = [&](const double* la, const double* lb, double* na, double* nb, int s) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (s + 1 < nst) issue(na, nb, (s + 1) * BK);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int k = kk + fk;
      double af[4], bf[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = la[k * RA + wm * 64 + i * 16 + fl];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int n = wn * 32 + j * 16 + fl;
        bf[j] = lb[n * BK + (((k >> 1) ^ (n & 15)) << 1) + (k & 1)];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[j], af[i], acc[i][j], 0, 0, 0);
    }
  };
  if (nst > 0) issue(lA0, lB0, 0);
  int s = 0;
  for (; s + 1 < nst; s += 2) {
    stage(lA0, lB0, lA1, lB1, s);
    stage(lA1, lB1, lA0, lB0, s + 1);
  }
  if (s < nst) stage(lA0, lB0, lA1, lB1, s);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 64 + i * 16 + fl;
        const int n = n0 + wn * 32 + j * 16 + fk + 4 * r;
        if (m < M && n < N) {
          double* c = C + (int64_t)n * ldc + m;
          const double v = alpha * acc[i][j][r];
          *c = BETA ? v + beta * *c : v;
        }
      }
}


bool dgemm_flex(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                const double* B, int64_t ldb, double beta, double* C, int64_t ldc, bool lower) {
  if (M < 2 || N < 1 || K < 1 || (M & 1) || (lda & 1) || (ldb % 32) || K > ldb || M > INT32_MAX || N > INT32_MAX ||
      ((uintptr_t)A & 15) || ((uintptr_t)B & 15))
    return false;
  const dim3 grid((unsigned)cdiv(M, 128), (unsigned)cdiv(N, 128));
  if (beta == 0.0)
    RPF_TIMED_LAUNCH((k_dgemm_big<false>), grid, dim3(512), 0, s, (int)M, (int)N, (int)K, alpha, A, lda, B, ldb, beta,
                     C, ldc, lower ? 1 : 0);
  else
    RPF_TIMED_LAUNCH((k_dgemm_big<true>), grid, dim3(512), 0, s, (int)M, (int)N, (int)K, alpha, A, lda, B, ldb, beta,
                     C, ldc, lower ? 1 : 0);
  RPF_LAUNCH_CHECK();
  return true;
}

// Sum of the split-K partials: one wavefront per output, lanes stride over the
// splits (fixed order, so the result is deterministic).
// Few slabs, many outputs: one thread per output, slabs summed in order (coalesced over outputs).
__global__ __launch_bounds__(256) void k_splitk_reduce_thread(int64_t M, int64_t N, int splits, const double* part,
                                                              double beta, double* C, int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t MN = M * N;
  if (idx >= MN) return;
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += part[(int64_t)z * MN + idx];
  const int64_t m = idx % M, n = idx / M;
  double* c = C + n * ldc + m;
  *c = (beta == 0.0) ? s : s + beta * *c;
}

// Sum of the split partial slabs: a workgroup covers 16 consecutive outputs (lane & 15, so each
// slab row read is 128 contiguous bytes) and its 16 thread rows take every 16th slab, eight loads
// in flight at clamped (always valid) slabs; the 16 row sums are then added in LDS in a fixed
// order.  C = sum (+ beta C), M x N column-major with leading dimension ldc.
__global__ __launch_bounds__(256) void k_splitk_reduce(int64_t M, int64_t N, int splits, const double* part,
                                                       double beta, double* C, int64_t ldc) {
  __shared__ double red[16][17];
  const int tx = threadIdx.x & 15, tz = threadIdx.x >> 4;
  const int64_t MN = M * N;
  const int64_t idx = (int64_t)blockIdx.x * 16 + tx;
  const int64_t ic = min(idx, MN - 1);
  double sum = 0.0;
  constexpr int U = 8;
  for (int z0 = tz; z0 < splits; z0 += 16 * U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = part[(int64_t)min(z0 + 16 * u, splits - 1) * MN + ic];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (z0 + 16 * u < splits) sum += v[u];
  }
  red[tz][tx] = sum;
  __syncthreads();
  if (tz == 0 && idx < MN) {
    double t = 0.0;
#pragma unroll
    for (int z = 0; z < 16; ++z) t += red[z][tx];
    const int64_t m = idx % M, n = idx / M;
    double* c = C + n * ldc + m;
    *c = (beta == 0.0) ? t : t + beta * *c;
  }
}

namespace {
enum Cfg { BIG, M16, N16, SMALL };

Cfg pick_cfg(int64_t M, int64_t N) {
  if (M <= 16) return M16;
  if (N <= 16) return N16;
  if (M <= 64 && N <= 64) return SMALL;
  // 256 CUs: fall back to 64x64 tiles when 128x128 tiles cannot give two per CU
  if (cdiv(M, 128) * cdiv(N, 128) < 512) return SMALL;
  return BIG;
}

void tile_of(Cfg c, int& bm, int& bn) {
  switch (c) {
    case BIG: bm = 128; bn = 128; break;
    case M16: bm = 16; bn = 256; break;
    case N16: bm = 256; bn = 16; break;
    default: bm = 64; bn = 64; break;
  }
}

template <bool TA, bool TB>
void launch_cfg(Cfg c, dim3 grid, hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha,
                const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                int64_t ldc, int lower, int64_t kchunk, double* part) {
  switch (c) {
    case BIG:
      RPF_TIMED_LAUNCH((k_dgemm<128, 128, 2, 2, TA, TB>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B,
                         ldb, beta, C, ldc, lower, kchunk, part);
      break;
    case M16:
      RPF_TIMED_LAUNCH((k_dgemm<16, 256, 1, 4, TA, TB>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B,
                         ldb, beta, C, ldc, lower, kchunk, part);
      break;
    case N16:
      RPF_TIMED_LAUNCH((k_dgemm<256, 16, 4, 1, TA, TB>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B,
                         ldb, beta, C, ldc, lower, kchunk, part);
      break;
    default:
      RPF_TIMED_LAUNCH((k_dgemm<64, 64, 2, 2, TA, TB>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B,
                         ldb, beta, C, ldc, lower, kchunk, part);
      break;
  }
}

void launch_gemm(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                 const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                 int64_t ldc, bool lower, int splits, double* part) {
  const Cfg c = pick_cfg(M, N);
  int bm, bn;
  tile_of(c, bm, bn);
  int64_t kchunk = K;
  if (splits > 1) kchunk = cdiv(cdiv(K, splits), 16) * 16;
  const int64_t gz = splits > 1 ? cdiv(K, kchunk) : 1;
  RPF_CHECK(cdiv(N, bn) <= 65535 && gz <= 65535, RPF_EINVAL, "dgemm: grid too large");
  dim3 grid((unsigned)cdiv(M, bm), (unsigned)cdiv(N, bn), (unsigned)gz);
  const int low = lower ? 1 : 0;
  if (!ta && !tb) launch_cfg<false, false>(c, grid, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, low, kchunk, part);
  else if (!ta && tb) launch_cfg<false, true>(c, grid, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, low, kchunk, part);
  else if (ta && !tb) launch_cfg<true, false>(c, grid, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, low, kchunk, part);
  else launch_cfg<true, true>(c, grid, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, low, kchunk, part);
  RPF_LAUNCH_CHECK();
}
}  // namespace

void dgemm(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
           int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, bool lower) {
  if (M <= 0 || N <= 0) return;
  if (K <= 0 && beta == 1.0) return;  // nothing to add; K = 0 otherwise scales C by beta
  launch_gemm(s, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, lower, 1, nullptr);
}

// resident workgroups of a kernel on the whole device (occupancy times compute units), cached
template <typename Kern>
static int resident_blocks(Kern k, int threads) {
  int per_cu = 0, dev = 0;
  RPF_HIP(hipGetDevice(&dev));
  RPF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads, 0));
  hipDeviceProp_t prop;
  RPF_HIP(hipGetDeviceProperties(&prop, dev));
  return std::max(1, per_cu) * std::max(1, prop.multiProcessorCount);
}

void dgemm_group(hipStream_t s, int tile, const DGroup& g) {
  const int total = g.start[g.n];
  if (total == 0) return;
  if (tile == 128) {
    static const int cap = resident_blocks(k_dgemm_group<128, 128>, 256);
    RPF_TIMED_LAUNCH((k_dgemm_group<128, 128>), dim3((unsigned)std::min(total, cap)), dim3(256), 0, s, g);
  } else {
    RPF_CHECK(tile == 64, RPF_EINVAL, "dgemm_group: tile must be 64 or 128");
    static const int cap = resident_blocks(k_dgemm_group<64, 64>, 256);
    RPF_TIMED_LAUNCH((k_dgemm_group<64, 64>), dim3((unsigned)std::min(total, cap)), dim3(256), 0, s, g);
  }
  RPF_LAUNCH_CHECK();
}

int gemm_tiles(int64_t M, int64_t N) {
  const Cfg c = pick_cfg(M, N);
  int bm, bn;
  tile_of(c, bm, bn);
  return (int)(cdiv(M, bm) * cdiv(N, bn));
}

void dgemm_partials(hipStream_t s, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* B,
                    int64_t ldb, double* part, int splits) {
  if (M <= 0 || N <= 0) return;
  launch_gemm(s, false, false, M, N, K, 1.0, A, lda, B, ldb, 0.0, nullptr, 0, false, splits, part);
}

int gemm_splitk_count(int64_t M, int64_t N, int64_t K) {
  const Cfg c = pick_cfg(M, N);
  int bm, bn;
  tile_of(c, bm, bn);
  const int64_t tiles = cdiv(M, bm) * cdiv(N, bn);
  int64_t sp = cdiv(1024, tiles);
  sp = std::min<int64_t>(sp, std::max<int64_t>(1, K / 256));
  sp = std::max<int64_t>(1, std::min<int64_t>(sp, 1024));
  return (int)sp;
}

void dgemm_splitk(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                  const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                  int64_t ldc, double* ws, int splits) {
  if (M <= 0 || N <= 0) return;
  if (splits <= 1 || K <= 0) {
    dgemm(s, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, false);
    return;
  }
  const int64_t kchunk = cdiv(cdiv(K, splits), 16) * 16;
  const int gz = (int)cdiv(K, kchunk);
  launch_gemm(s, ta, tb, M, N, K, alpha, A, lda, B, ldb, 0.0, nullptr, 0, false, splits, ws);
  if (gz <= 32)
    hipLaunchKernelGGL(k_splitk_reduce_thread, dim3((unsigned)cdiv(M * N, 256)), dim3(256), 0, s, M, N, gz, ws, beta,
                       C, ldc);
  else
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)cdiv(M * N, 16)), dim3(256), 0, s, M, N, gz, ws, beta, C,
                       ldc);
  RPF_LAUNCH_CHECK();
}

// ============================================================================ tall-skinny Gram
// Partial C (a x b) = X^T Y over a chunk of rows, X and Y row-major (N x a, N x b).
// Workgroup (tile, chunk): tile = (ti, tj) 16 x 16 block of C; each wave takes 4
// rows per v_mfma_f64_16x16x4_f64 (the k dimension of the MFMA runs over rows),
// the 4 waves are summed in LDS and the partial goes to part[chunk][j][i].
__global__ __launch_bounds__(256) void k_gram_partial(int64_t N, int a, int b, const double* X, int64_t ldx,
                                                      const double* Y, int64_t ldy, int64_t chunk, double* part) {
  __shared__ double red[4][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ta = (a + 15) / 16;
  const int i0 = (blockIdx.x % ta) * 16, j0 = (blockIdx.x / ta) * 16;
  const int64_t r_beg = (int64_t)blockIdx.y * chunk;
  const int64_t r_end = min(N, r_beg + chunk);
  const int i = i0 + (lane & 15), j = j0 + (lane & 15);
  const bool iok = i < a, jok = j < b;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  // four row groups in flight per wave (loads issued before the MFMAs consume them)
  for (int64_t r0 = r_beg + 4 * wave; r0 < r_end; r0 += 64) {
    double xa[4], yb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t row = r0 + 16 * u + (lane >> 4);
      const bool rok = row < r_end;
      xa[u] = (rok && iok) ? X[row * ldx + i] : 0.0;
      yb[u] = (rok && jok) ? Y[row * ldy + j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u], yb[u], acc, 0, 0, 0);
  }
  // accumulator item r of lane l is C[i0 + l/16 + 4r][j0 + l%16]
#pragma unroll
  for (int r = 0; r < 4; ++r) red[wave][((lane >> 4) + 4 * r) * 16 + (lane & 15)] = acc[r];
  __syncthreads();
  const int t = threadIdx.x;
  const int ci = i0 + t / 16, cj = j0 + t % 16;
  if (ci < a && cj < b)
    part[((int64_t)blockIdx.y * b + cj) * a + ci] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
}

// Pair form: C = X^T [Y1 | Y2] for a <= 16 and b1, b2 <= 16, each workgroup computing both
// 16 x 16 tiles from one read of X (the two Grams of a block step share their left operand).
// part[chunk] holds a x (b1 + b2), column-major.
__global__ __launch_bounds__(256) void k_gram_pair(int64_t N, int a, const double* X, int64_t ldx, int b1,
                                                   const double* Y1, int64_t ldy1, int b2, const double* Y2,
                                                   int64_t ldy2, int64_t chunk, double* part) {
  __shared__ double red[4][2][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r_beg = (int64_t)blockIdx.x * chunk;
  const int64_t r_end = min(N, r_beg + chunk);
  const int i = lane & 15, j = lane & 15;
  const bool iok = i < a, j1 = j < b1, j2 = j < b2;
  v4d acc1 = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
  if (b1 > 0 && b2 > 0 && r_end > r_beg) {
    // loads at clamped (always valid) rows and columns, masked afterwards, and the next group's
    // loads issued before this group's MFMAs: no load behind a branch, two groups in flight
    const int ic = min(i, a - 1), jc1 = min(j, b1 - 1), jc2 = min(j, b2 - 1);
    double xa[4], y1[4], y2[4], nx[4], n1[4], n2[4];
    auto load = [&](int64_t r0, double* x, double* p1, double* p2) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t row = min(r0 + 16 * u + (lane >> 4), r_end - 1);
        x[u] = X[row * ldx + ic];
        p1[u] = Y1[row * ldy1 + jc1];
        p2[u] = Y2[row * ldy2 + jc2];
      }
    };
    auto mma = [&](int64_t r0, const double* x, const double* p1, const double* p2) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool rok = r0 + 16 * u + (lane >> 4) < r_end;
        const double xv = (rok && iok) ? x[u] : 0.0;
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xv, (rok && j1) ? p1[u] : 0.0, acc1, 0, 0, 0);
        acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(xv, (rok && j2) ? p2[u] : 0.0, acc2, 0, 0, 0);
      }
    };
    // two register sets in turn (no copies): the loads of one group are in flight while the
    // MFMAs of the other run; a prefetch past the last group reads the clamped last row
    int64_t r0 = r_beg + 4 * wave;
    load(r0, xa, y1, y2);
    for (; r0 < r_end; r0 += 128) {
      load(r0 + 64, nx, n1, n2);
      mma(r0, xa, y1, y2);
      if (r0 + 64 >= r_end) break;
      load(r0 + 128, xa, y1, y2);
      mma(r0 + 64, nx, n1, n2);
    }
  } else {
    for (int64_t r0 = r_beg + 4 * wave; r0 < r_end; r0 += 64) {
      double xa[4], y1[4], y2[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t row = r0 + 16 * u + (lane >> 4);
        const bool rok = row < r_end;
        xa[u] = (rok && iok) ? X[row * ldx + i] : 0.0;
        y1[u] = (rok && j1) ? Y1[row * ldy1 + j] : 0.0;
        y2[u] = (rok && j2) ? Y2[row * ldy2 + j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u], y1[u], acc1, 0, 0, 0);
        acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u], y2[u], acc2, 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    red[wave][0][((lane >> 4) + 4 * r) * 16 + (lane & 15)] = acc1[r];
    red[wave][1][((lane >> 4) + 4 * r) * 16 + (lane & 15)] = acc2[r];
  }
  __syncthreads();
  const int t = threadIdx.x;
  const int ci = t / 16, cj = t % 16;
  const int bt = b1 + b2;
  double* pc = part + (int64_t)blockIdx.x * a * bt;
  if (ci < a && cj < b1) pc[(int64_t)cj * a + ci] = red[0][0][t] + red[1][0][t] + red[2][0][t] + red[3][0][t];
  if (ci < a && cj < b2) pc[(int64_t)(b1 + cj) * a + ci] = red[0][1][t] + red[1][1][t] + red[2][1][t] + red[3][1][t];
}

// Wide form (X with many columns, e.g. all stored search directions).  The a columns are split
// into ga groups of at most 32 column tiles, spread evenly; a workgroup covers one group against
// one 16-column tile of Y over a chunk of rows.  Its four waves are WT tile slices (TW tiles each)
// times 4/WT row slices: few tiles are split over rows instead of leaving waves idle, and each Y
// fragment feeds TW MFMAs.  The row slices' sums are added in LDS before the partial is written.
// With more than 4 tiles (a > 64), TW is 5 to 8.
struct WideShape {
  int ga, wt, tw;
};
static WideShape wide_shape(int a) {
  const int ta = (a + 15) / 16;
  const int ga = (ta + 31) / 32;
  const int tg = (ta + ga - 1) / ga;
  const int wt = tg <= 8 ? 1 : (tg <= 16 ? 2 : 4);
  return {ga, wt, (tg + wt - 1) / wt};
}

template <int TW>
__global__ __launch_bounds__(256) void k_gram_wide(int64_t N, int a, int b, const double* X, int64_t ldx,
                                                   const double* Y, int64_t ldy, int64_t chunk, int ga, int wt,
                                                   double* part) {
  __shared__ double red[4][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr_n = 4 / wt, wslice = wave % wt, wrow = wave / wt;
  const int grp = blockIdx.x % ga, tj = blockIdx.x / ga;
  const int ta = (a + 15) / 16, tg = (ta + ga - 1) / ga;
  const int tbase = grp * tg + wslice * TW;
  const int tend = min(ta, (grp + 1) * tg);
  const int j = tj * 16 + (lane & 15);
  const bool jok = j < b;
  const int64_t r_beg = (int64_t)blockIdx.y * chunk;
  const int64_t r_end = min(N, r_beg + chunk);
  v4d acc[TW];
#pragma unroll
  for (int t = 0; t < TW; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
  if (r_end > r_beg) {
    // loads at clamped (always valid) rows and columns, masked before the MFMAs, and the next
    // group of 8 rows loaded while this group's MFMAs run (two register sets in turn)
    const int jc = min(j, b - 1);
    int ic[TW];
    bool iok[TW];
#pragma unroll
    for (int t = 0; t < TW; ++t) {
      const int i = (tbase + t) * 16 + (lane & 15);
      ic[t] = min(i, a - 1);
      iok[t] = tbase + t < tend && i < a;
    }
    double yb[2], xa[2][TW], ny[2], nx[2][TW];
    auto load = [&](int64_t r0, double* y, double (*x)[TW]) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int64_t row = min(r0 + 4 * u + (lane >> 4), r_end - 1);
        y[u] = Y[row * ldy + jc];
#pragma unroll
        for (int t = 0; t < TW; ++t) x[u][t] = X[row * ldx + ic[t]];
      }
    };
    auto mma = [&](int64_t r0, const double* y, const double (*x)[TW]) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const bool rok = r0 + 4 * u + (lane >> 4) < r_end;
        const double yv = (rok && jok) ? y[u] : 0.0;
#pragma unroll
        for (int t = 0; t < TW; ++t)
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64((rok && iok[t]) ? x[u][t] : 0.0, yv, acc[t], 0, 0, 0);
      }
    };
    // this wave's row slice: groups of 8 rows r_beg + 8 (wrow + wr_n q), q = 0, 1, ...
    const int64_t step = 8 * (int64_t)wr_n;
    int64_t r0 = r_beg + 8 * wrow;
    if (r0 < r_end) {
      load(r0, yb, xa);
      for (; r0 < r_end; r0 += 2 * step) {
        load(r0 + step, ny, nx);
        mma(r0, yb, xa);
        if (r0 + step >= r_end) break;
        load(r0 + 2 * step, yb, xa);
        mma(r0 + step, ny, nx);
      }
    }
  }
  double* pc = part + (int64_t)blockIdx.y * a * b;
#pragma unroll
  for (int t = 0; t < TW; ++t) {
    if (wr_n > 1) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave][64 * r + lane] = acc[t][r];
      __syncthreads();
      if (wrow == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double v = red[wave][64 * r + lane];
          for (int q = 1; q < wr_n; ++q) v += red[wave + wt * q][64 * r + lane];
          acc[t][r] = v;
        }
      }
    }
    if (wrow == 0 && tbase + t < tend) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ci = (tbase + t) * 16 + (lane >> 4) + 4 * r, cj = tj * 16 + (lane & 15);
        if (ci < a && cj < b) pc[(int64_t)cj * a + ci] = acc[t][r];
      }
    }
  }
}

static bool gram_is_wide(int a) { return a > 64; }

int gram_chunks(int64_t N, int a, int b) {
  // about one to two workgroups per CU in total for the narrow form and about four for the wide
  // one, at least 256 rows per chunk
  const int64_t tiles = gram_is_wide(a) ? (int64_t)wide_shape(a).ga * cdiv(b, 16) : cdiv(a, 16) * cdiv(b, 16);
  int64_t g = cdiv(gram_is_wide(a) ? 1024 : 256, tiles);
  g = std::min<int64_t>(g, std::max<int64_t>(1, cdiv(N, 256)));
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 2048));
}

void gram(hipStream_t s, int64_t N, int a, int b, const double* X, int64_t ldx, const double* Y, int64_t ldy,
          double* C, double* ws) {
  if (a <= 0 || b <= 0) return;
  const int g = gram_chunks(N, a, b);
  const int64_t chunk = cdiv(N, g);
  const int gz = (int)cdiv(N, chunk);
  RPF_CHECK(gz <= 65535, RPF_EINVAL, "gram: too many chunks");
  if (gram_is_wide(a)) {
    const WideShape w = wide_shape(a);
    const dim3 grid((unsigned)(w.ga * cdiv(b, 16)), (unsigned)gz);
    switch (w.tw) {
#define RPF_WIDE(TW)                                                                                         \
  case TW:                                                                                                   \
    hipLaunchKernelGGL(k_gram_wide<TW>, grid, dim3(256), 0, s, N, a, b, X, ldx, Y, ldy, chunk, w.ga, w.wt, ws); \
    break;
      RPF_WIDE(5) RPF_WIDE(6) RPF_WIDE(7) RPF_WIDE(8)
#undef RPF_WIDE
      default:
        RPF_CHECK(false, RPF_EINVAL, "gram: unexpected wide shape");
    }
  } else {
    const int64_t tiles = cdiv(a, 16) * cdiv(b, 16);
    hipLaunchKernelGGL(k_gram_partial, dim3((unsigned)tiles, (unsigned)gz), dim3(256), 0, s, N, a, b, X, ldx, Y,
                       ldy, chunk, ws);
  }
  RPF_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)cdiv((int64_t)a * b, 16)), dim3(256), 0, s, (int64_t)a,
                     (int64_t)b, gz, ws, 0.0, C, (int64_t)a);
  RPF_LAUNCH_CHECK();
}

// rows per chunk of gram_pair: four workgroups per CU, since one wave per SIMD does not keep enough
// loads in flight for this memory-bound pass (the partial sums are still reduced in a fixed order)
static int64_t gram_pair_rows(int64_t N) {
  return cdiv(N, std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(N, 256))));
}
int gram_pair_chunks(int64_t N) { return (int)cdiv(N, gram_pair_rows(N)); }

void gram_pair(hipStream_t s, int64_t N, int a, const double* X, int64_t ldx, int b1, const double* Y1,
               int64_t ldy1, int b2, const double* Y2, int64_t ldy2, double* C, double* ws) {
  if (a <= 0 || b1 + b2 <= 0) return;
  if (a > 16 || b1 > 16 || b2 > 16) {
    gram(s, N, a, b1, X, ldx, Y1, ldy1, C, ws);
    gram(s, N, a, b2, X, ldx, Y2, ldy2, C + (int64_t)a * b1, ws);
    return;
  }
  const int64_t chunk = gram_pair_rows(N);
  const int gz = gram_pair_chunks(N);
  hipLaunchKernelGGL(k_gram_pair, dim3((unsigned)gz), dim3(256), 0, s, N, a, X, ldx, b1, Y1, ldy1, b2, Y2, ldy2,
                     chunk, ws);
  RPF_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)cdiv((int64_t)a * (b1 + b2), 16)), dim3(256), 0, s, (int64_t)a,
                     (int64_t)(b1 + b2), gz, ws, 0.0, C, (int64_t)a);
  RPF_LAUNCH_CHECK();
}

// ============================================================================ row-block products
// Y[l*ldy + j] = beta Y + alpha sum_i X[l*ldx + i] M[i + a*j] for N rows and a
// small a x b matrix M (column-major).  A workgroup owns 64 rows; slices of 32
// columns of X are staged through LDS with coalesced loads (consecutive lanes
// read consecutive columns of a row), M slices likewise; lane (r, q) then forms
// outputs 4q..4q+3 of row r.  Used for the block updates of the interface
// solver (rows = interface dofs, row-major blocks).
__global__ __launch_bounds__(256) void k_rows_gemm(int64_t N, int a, int b, double alpha, const double* X,
                                                   int64_t ldx, const double* Mm, int64_t mrow, double beta, double* Y,
                                                   int64_t ldy) {
  __shared__ double sx[64][33];
  __shared__ double sm[32][16];
  const int tid = threadIdx.x;
  const int r = tid & 63, q = tid >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * 64;
  const int64_t row = row0 + r;
  for (int j0 = 0; j0 < b; j0 += 16) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    // each 32-column chunk of X (and of M) is loaded into registers at clamped (always valid)
    // positions one chunk ahead, while the current chunk is multiplied from LDS: no load waits
    // behind a branch, and one chunk's loads are in flight during the other's FMAs
    double xr[8], mv[2];
    auto load = [&](int i0) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int idx = tid + 256 * e;
        const int ii = idx & 31, rr = idx >> 5;
        const int64_t gr = min(row0 + rr, N - 1);
        xr[e] = X[gr * ldx + min(i0 + ii, a - 1)];
      }
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int idx = tid + 256 * e;
        const int ic = min(i0 + (idx & 31), a - 1), jc = min(j0 + (idx >> 5), b - 1);
        mv[e] = mrow > 0 ? Mm[(int64_t)ic * mrow + jc] : Mm[(int64_t)ic + (int64_t)a * jc];
      }
    };
    load(0);
    for (int i0 = 0; i0 < a; i0 += 32) {
      __syncthreads();
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int idx = tid + 256 * e;
        const int ii = idx & 31, rr = idx >> 5;
        sx[rr][ii] = (row0 + rr < N && i0 + ii < a) ? xr[e] : 0.0;
      }
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int idx = tid + 256 * e;
        const int ii = idx & 31, jj = idx >> 5;
        sm[ii][jj] = (i0 + ii < a && j0 + jj < b) ? mv[e] : 0.0;
      }
      __syncthreads();
      load(i0 + 32);
#pragma unroll 8
      for (int ii = 0; ii < 32; ++ii) {
        const double xv = sx[r][ii];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += xv * sm[ii][4 * q + u];
      }
    }
    if (row < N) {
      // the old values of the four outputs are read together (clamped to a valid column)
      double yo[4] = {0.0, 0.0, 0.0, 0.0};
      if (beta != 0.0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) yo[u] = Y[row * ldy + min(j0 + 4 * q + u, b - 1)];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = j0 + 4 * q + u;
        if (j < b) Y[row * ldy + j] = (beta == 0.0) ? alpha * acc[u] : beta * yo[u] + alpha * acc[u];
      }
    }
  }
}

// Same product for many rows, a long inner dimension and at most 16 columns of M (e.g. the
// orthogonalisation against all stored blocks), on FP64 MFMA 16x16x4 with X rows as the M
// dimension.  A workgroup owns 64 rows and walks X in 32-column chunks.  A chunk is loaded with
// whole 128-byte lines per row (16 lanes of 16 bytes per row, four rows per load instruction; the
// MFMA operand layout, 4 lanes per row, would split every line over two instructions, which
// measured a fifth slower) into registers one chunk ahead, at clamped (always valid) positions, and
// stored masked into one of two LDS buffers with the matching 32 rows of M; wave w then multiplies
// rows 16 w .. 16 w + 15 from LDS, two accumulators in turn.  VEC: 16-byte loads (a and ldx even,
// X aligned).
template <bool VEC>
__global__ __launch_bounds__(256) void k_rows_mfma(int64_t N, int a, int b, double alpha, const double* X,
                                                   int64_t ldx, const double* Mm, int64_t mrow, double beta, double* Y,
                                                   int64_t ldy) {
  __shared__ double sx[2][64][34];
  __shared__ double sm[2][32][16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = lane & 15, q = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * 64;
  // chunk staging: piece p = tid + 256 i is row p >> 4, columns k0 + 2 (p & 15) + {0, 1}; M entry
  // e = tid + 256 i is row k0 + (e >> 4), column e & 15
  double2 xr[4];
  double mr[2];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = tid + 256 * i, r = p >> 4, sg = p & 15;
      const double* xrow = X + min(row0 + r, N - 1) * ldx;
      if (VEC) {
        xr[i] = *reinterpret_cast<const double2*>(xrow + min(k0 + 2 * sg, a - 2));
      } else {
        xr[i].x = xrow[min(k0 + 2 * sg, a - 1)];
        xr[i].y = xrow[min(k0 + 2 * sg + 1, a - 1)];
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int e = tid + 256 * i, kk = e >> 4, j = e & 15;
      const int kc = min(k0 + kk, a - 1), jc = min(j, b - 1);
      mr[i] = mrow > 0 ? Mm[(int64_t)kc * mrow + jc] : Mm[(int64_t)kc + (int64_t)a * jc];
    }
  };
  auto sstore = [&](int buf, int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = tid + 256 * i, r = p >> 4, sg = p & 15;
      const int c = k0 + 2 * sg;
      double2 v;
      v.x = c < a ? xr[i].x : 0.0;
      v.y = c + 1 < a ? xr[i].y : 0.0;
      *reinterpret_cast<double2*>(&sx[buf][r][2 * sg]) = v;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int e = tid + 256 * i, kk = e >> 4, j = e & 15;
      sm[buf][kk][j] = k0 + kk < a ? mr[i] : 0.0;
    }
  };
  v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};  // even and odd k-steps
  gload(0);
  sstore(0, 0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < a; k0 += 32) {
    // the next chunk's loads are in flight while this chunk is multiplied; they go into the other
    // buffer, whose last readers all passed the barrier that ended the previous chunk
    gload(k0 + 32);
#pragma unroll
    for (int st = 0; st < 8; st += 2) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(sx[buf][16 * wave + m][4 * st + q], sm[buf][4 * st + q][m], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(sx[buf][16 * wave + m][4 * st + 4 + q], sm[buf][4 * st + 4 + q][m], acc1,
                                                  0, 0, 0);
    }
    sstore(buf ^ 1, k0 + 32);
    __syncthreads();
    buf ^= 1;
  }
  // lane holds rows 16 w + q + 4 r, column m; the old values are read together first
  const bool jok = m < b;
  const int jc = min(m, b - 1);
  double yo[4];
  if (beta != 0.0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) yo[r] = Y[min(row0 + 16 * wave + q + 4 * r, N - 1) * ldy + jc];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = row0 + 16 * wave + q + 4 * r;
    const double v = acc0[r] + acc1[r];
    if (jok && row < N) Y[row * ldy + m] = (beta == 0.0) ? alpha * v : beta * yo[r] + alpha * v;
  }
}

// Same product for few rows and a long inner dimension (e.g. the coarse solve with the explicit
// inverse of G^T G): one wavefront per row, lanes stride the inner index (coalesced reads of the
// row of X), 16 output columns per pass reduced across the wavefront with shuffles.
__global__ __launch_bounds__(256) void k_rows_gemm_wave(int64_t N, int a, int b, double alpha, const double* X,
                                                        int64_t ldx, const double* Mm, int64_t mrow, double beta,
                                                        double* Y, int64_t ldy) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= N) return;
  const double* x = X + row * ldx;
  for (int j0 = 0; j0 < b; j0 += 16) {
    const int nj = min(16, b - j0);
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    // the 16 M entries of a step are loaded at clamped (always valid) columns and masked, so they
    // are one batch in flight instead of one load behind each column test
    for (int i = lane; i < a; i += 64) {
      const double xv = x[i];
      double mv[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int uc = min(u, nj - 1);
        mv[u] = mrow > 0 ? Mm[(int64_t)i * mrow + j0 + uc] : Mm[(int64_t)i + (int64_t)a * (j0 + uc)];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (u < nj) acc[u] += xv * mv[u];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      for (int off = 32; off > 0; off >>= 1) acc[u] += __shfl_xor(acc[u], off, 64);
    if (lane < nj) {
      double v = 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u) v = (lane == u) ? acc[u] : v;
      double* y = Y + row * ldy + j0 + lane;
      *y = (beta == 0.0) ? alpha * v : beta * *y + alpha * v;
    }
  }
}

// Thin products (a <= 64 inner, b <= 16 outputs per row): one thread per row.  M is
// staged once per workgroup in LDS (read back as broadcasts); each thread streams its
// row of X with 16-byte loads and writes its row of Y the same way, so the kernel runs
// at the memory rate.  blockIdx.y selects one of up to two (X, Y) pairs sharing M.
struct RowsPair {
  const double* X;
  double* Y;
  int64_t ldx, ldy;
  double alpha, beta;
  const double* Z;  // source of the beta term (NULL: Y itself), row stride ldz
  int64_t ldz;
};
struct RowsPairs {
  RowsPair p[2];
  double* colsq;  // optional: per-workgroup column sums of squares of pair 1's output (k_rows_tile)
};

__global__ __launch_bounds__(256) void k_rows_small(int64_t N, int a, int b, const double* Mm, int64_t mrow,
                                                    RowsPairs pr, int vec) {
  __shared__ double sm[64 * 16];
  {
    // staged from clamped (always valid) positions and masked, so the four loads are in flight together
    double mv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int ic = min(e >> 4, a - 1), jc = min(e & 15, b - 1);
      mv[q] = mrow > 0 ? Mm[(int64_t)ic * mrow + jc] : Mm[ic + (int64_t)a * jc];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q;
      sm[e] = ((e >> 4) < a && (e & 15) < b) ? mv[q] : 0.0;
    }
  }
  __syncthreads();
  const RowsPair& P = pr.p[blockIdx.y];
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (row >= N) return;
  double acc[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.0;
  const double* x = P.X + row * P.ldx;
  for (int i0 = 0; i0 < a; i0 += 8) {
    double xv[8];
    if (vec && i0 + 8 <= a) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double2 t = *reinterpret_cast<const double2*>(x + i0 + 2 * u);
        xv[2 * u] = t.x;
        xv[2 * u + 1] = t.y;
      }
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u) xv[u] = x[min(i0 + u, a - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) xv[u] = (i0 + u < a) ? xv[u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double* mr = sm + (i0 + u) * 16;
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j] += xv[u] * mr[j];
    }
  }
  double* y = P.Y + row * P.ldy;
  const double* z = P.Z ? P.Z + row * P.ldz : y;
  if (vec && (b & 1) == 0) {
    double2 zt[8];
    if (P.beta != 0.0) {
#pragma unroll
      for (int j = 0; j < 16; j += 2) zt[j / 2] = *reinterpret_cast<const double2*>(z + min(j, b - 2));
    }
#pragma unroll
    for (int j = 0; j < 16; j += 2) {
      if (j < b) {
        double2 o;
        if (P.beta == 0.0) {
          o.x = P.alpha * acc[j];
          o.y = P.alpha * acc[j + 1];
        } else {
          o.x = P.beta * zt[j / 2].x + P.alpha * acc[j];
          o.y = P.beta * zt[j / 2].y + P.alpha * acc[j + 1];
        }
        *reinterpret_cast<double2*>(y + j) = o;
      }
    }
  } else {
    double zv[16];
    if (P.beta != 0.0) {
#pragma unroll
      for (int j = 0; j < 16; ++j) zv[j] = z[min(j, b - 1)];
    }
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (j < b) y[j] = (P.beta == 0.0) ? P.alpha * acc[j] : P.beta * zv[j] + P.alpha * acc[j];
  }
}

// Narrow products (a, b <= 16): 256 rows per workgroup.  The rows of X are copied into LDS with
// lane-consecutive loads (a row is a contiguous run of a doubles), each thread then forms its row
// of the product from LDS, and the result leaves through LDS with lane-consecutive stores, so
// global traffic is coalesced in both directions.  blockIdx.y selects one of the (X, Y) pairs.
__global__ __launch_bounds__(256) void k_rows_tile(int64_t N, int a, int b, const double* Mm, int64_t mrow,
                                                   RowsPairs pr) {
  __shared__ double sm[16][16];
  __shared__ double xs[256][17];
  const int tid = threadIdx.x;
  {
    const int i = tid >> 4, j = tid & 15;
    sm[i][j] = (i < a && j < b) ? (mrow > 0 ? Mm[(int64_t)i * mrow + j] : Mm[i + (int64_t)a * j]) : 0.0;
  }
  const RowsPair& P = pr.p[blockIdx.y];
  const int64_t r0 = (int64_t)blockIdx.x * 256;
  const int rows = (int)min<int64_t>(256, N - r0);
  // full 256 x 16 tiles (the common case) issue all sixteen loads of a thread before the first
  // LDS store, so they are in flight together
  const bool full = rows == 256 && a == 16;
  if (full) {
    double t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + u * 256;
      t[u] = P.X[(r0 + (e >> 4)) * P.ldx + (e & 15)];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + u * 256;
      xs[e >> 4][e & 15] = t[u];
    }
  } else {
    for (int e = tid; e < rows * a; e += 256) {
      const int rr = e / a, cc = e - rr * a;
      xs[rr][cc] = P.X[(r0 + rr) * P.ldx + cc];
    }
  }
  __syncthreads();
  double acc[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.0;
  if (tid < rows) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if (i < a) {
        const double xv = xs[tid][i];
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] += xv * sm[i][j];
      }
    }
  }
  __syncthreads();  // xs is reused for the output rows
  if (tid < rows) {
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (j < b) xs[tid][j] = acc[j];
  }
  // with colsq (b divides 256), every element a thread writes lies in column tid % b: the thread
  // sums their squares and the column sums are formed in a fixed order (deterministic)
  const bool want_sq = pr.colsq != nullptr && blockIdx.y == 1;
  double myq = 0.0;
  __syncthreads();
  if (rows == 256 && b == 16) {
    // same element order as below; the sixteen beta-term loads go out together
    double zv[16];
    if (P.beta != 0.0) {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = tid + u * 256;
        const int64_t row = r0 + (e >> 4);
        zv[u] = P.Z ? P.Z[row * P.ldz + (e & 15)] : P.Y[row * P.ldy + (e & 15)];
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + u * 256;
      const double v = P.alpha * xs[e >> 4][e & 15];
      const double out = (P.beta == 0.0) ? v : P.beta * zv[u] + v;
      P.Y[(r0 + (e >> 4)) * P.ldy + (e & 15)] = out;
      myq += out * out;
    }
  } else {
    for (int e = tid; e < rows * b; e += 256) {
      const int rr = e / b, cc = e - rr * b;
      double* y = P.Y + (r0 + rr) * P.ldy + cc;
      const double v = P.alpha * xs[rr][cc];
      const double out = (P.beta == 0.0) ? v : P.beta * (P.Z ? P.Z[(r0 + rr) * P.ldz + cc] : *y) + v;
      *y = out;
      myq += out * out;
    }
  }
  if (want_sq) {
    __syncthreads();
    double* red = &xs[0][0];
    red[tid] = myq;
    __syncthreads();
    if (tid < b) {
      double t = 0.0;
      for (int k = tid; k < 256; k += b) t += red[k];
      pr.colsq[(int64_t)blockIdx.x * b + tid] = t;
    }
  }
}

// Residual update of a block step with both of its by-products from the same pass:
// Y = beta Y + alpha X M (X: N x a rows, M: a x b column-major, a, b <= 16), the per-workgroup
// column sums of squares of the new Y (sqpart[wg * b + c], fixed order, deterministic), and
// the per-workgroup Gram partial X^T Y_new (gpart[(wg * b + j) * a + i]) - the next step's
// X^T R, which would otherwise take another pass over both blocks.  The rows of X and of the new
// Y stay in LDS; the Gram partial is formed with v_mfma_f64_16x16x4_f64 (each wave four rows per
// MFMA over its 64 rows) and the four waves are summed in LDS.
__global__ __launch_bounds__(256) void k_rows_update_gram(int64_t N, int a, int b, const double* Mm,
                                                          const double* X, int64_t ldx, double alpha, double beta,
                                                          double* Y, int64_t ldy, double* sqpart, double* gpart) {
  __shared__ double sm[16][16];
  __shared__ double xs[256][17];
  __shared__ double ys[256][17];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  {
    const int i = tid >> 4, j = tid & 15;
    sm[i][j] = (i < a && j < b) ? Mm[i + (int64_t)a * j] : 0.0;
  }
  double myq = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * 256;
  const int rows = (int)min<int64_t>(256, N - r0);
  // whole tile of 16 columns: Y's old values are loaded together with X (one memory latency
  // instead of two in a row)
  const bool pre = rows == 256 && a == 16 && b == 16 && beta != 0.0;
  double zv[16];
  if (rows == 256 && a == 16) {
    double t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + u * 256;
      t[u] = X[(r0 + (e >> 4)) * ldx + (e & 15)];
      if (pre) zv[u] = Y[(r0 + (e >> 4)) * ldy + (e & 15)];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + u * 256;
      xs[e >> 4][e & 15] = t[u];
    }
  } else {
    for (int e = tid; e < 256 * 16; e += 256) {
      const int rr = e >> 4, cc = e & 15;
      xs[rr][cc] = (rr < rows && cc < a) ? X[(r0 + rr) * ldx + cc] : 0.0;
    }
  }
  __syncthreads();
  {
    double acc[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const double xv = xs[tid][i];
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j] += xv * sm[i][j];
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) ys[tid][j] = acc[j];
  }
  __syncthreads();
  if (rows == 256 && b == 16) {
    if (beta != 0.0 && !pre) {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = tid + u * 256;
        zv[u] = Y[(r0 + (e >> 4)) * ldy + (e & 15)];
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + u * 256;
      const double v = alpha * ys[e >> 4][e & 15];
      const double out = (beta == 0.0) ? v : beta * zv[u] + v;
      Y[(r0 + (e >> 4)) * ldy + (e & 15)] = out;
      ys[e >> 4][e & 15] = out;
      myq += out * out;
    }
  } else {
    for (int e = tid; e < 256 * b; e += 256) {
      const int rr = e / b, cc = e - rr * b;
      double out = 0.0;  // rows past N count as zero in the Gram
      if (rr < rows) {
        double* y = Y + (r0 + rr) * ldy + cc;
        const double v = alpha * ys[rr][cc];
        out = (beta == 0.0) ? v : beta * *y + v;
        *y = out;
      }
      ys[rr][cc] = out;
      myq += out * out;
    }
    for (int e = tid; e < 256 * 16; e += 256)
      if ((e & 15) >= b) ys[e >> 4][e & 15] = 0.0;
  }
  __syncthreads();
  // Gram partial over this tile's rows: wave w takes rows 64 w .. 64 w + 63
  v4d g = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int row = wave * 64 + 4 * q + (lane >> 4);
    g = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[row][lane & 15], ys[row][lane & 15], g, 0, 0, 0);
  }
  __syncthreads();  // xs becomes the reduction buffer
  double* red = &xs[0][0];
  // accumulator item r of lane l is (i = l / 16 + 4 r, j = l % 16)
#pragma unroll
  for (int r = 0; r < 4; ++r) red[wave * 256 + ((lane >> 4) + 4 * r) * 16 + (lane & 15)] = g[r];
  red[1024 + tid] = myq;
  __syncthreads();
  {
    const int i = tid >> 4, j = tid & 15;
    if (i < a && j < b)
      gpart[((int64_t)blockIdx.x * b + j) * a + i] = red[tid] + red[256 + tid] + red[512 + tid] + red[768 + tid];
  }
  // every element a thread wrote lies in column tid % b (b divides 256)
  if (tid < b) {
    double t = 0.0;
    for (int k = tid; k < 256; k += b) t += red[1024 + k];
    sqpart[(int64_t)blockIdx.x * b + tid] = t;
  }
}

// Two row-block products from one read of X (N x a, a <= 16), for the block step that starts from
// the residual: Z = R - X M1 (b columns) and Lam += X M2 (c columns), M1, M2 column-major with
// a rows (b, c <= 16).  X is the previous step's direction block: the orthogonalisation of the new
// block and the deferred solution update of the previous one share its pass.  Rows of X enter LDS
// with lane-consecutive loads, each thread forms its row of both products, and the results leave
// through LDS with lane-consecutive stores (the loads of R and Lam for a tile all in flight).
__global__ __launch_bounds__(256) void k_rows_orth_lam(int64_t N, int a, int b, int c, const double* M1,
                                                       const double* M2, const double* X, int64_t ldx,
                                                       const double* R, int64_t ldr, double* Z, int64_t ldz,
                                                       double* Lam, int64_t ldl) {
  __shared__ double sm1[16][16];
  __shared__ double sm2[16][16];
  __shared__ double xs[256][17];
  __shared__ double ys[256][17];
  const int tid = threadIdx.x;
  {
    const int i = tid >> 4, j = tid & 15;
    sm1[i][j] = (i < a && j < b) ? M1[i + (int64_t)a * j] : 0.0;
    sm2[i][j] = (i < a && j < c) ? M2[i + (int64_t)a * j] : 0.0;
  }
  const int64_t r0 = (int64_t)blockIdx.x * 256;
  const int rows = (int)min<int64_t>(256, N - r0);
  if (rows == 256 && a == 16 && b == 16 && c == 16) {
    // whole tile, 16 columns everywhere: the loads of X, R and Lam are all issued before anything
    // waits (one memory latency per workgroup instead of three in a row)
    double t[16], rv[16], lv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int64_t row = r0 + ((tid + u * 256) >> 4);
      const int col = (tid + u * 256) & 15;
      t[u] = X[row * ldx + col];
      rv[u] = R[row * ldr + col];
      lv[u] = Lam[row * ldl + col];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + u * 256;
      xs[e >> 4][e & 15] = t[u];
    }
    __syncthreads();
    double acc1[16], acc2[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) acc1[j] = acc2[j] = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const double xv = xs[tid][i];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        acc1[j] += xv * sm1[i][j];
        acc2[j] += xv * sm2[i][j];
      }
    }
    __syncthreads();  // xs is reused for the first product
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      xs[tid][j] = acc1[j];
      ys[tid][j] = acc2[j];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + u * 256;
      const int64_t row = r0 + (e >> 4);
      Z[row * ldz + (e & 15)] = rv[u] - xs[e >> 4][e & 15];
      Lam[row * ldl + (e & 15)] = lv[u] + ys[e >> 4][e & 15];
    }
    return;
  }
  if (rows == 256 && a == 16) {
    double t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + u * 256;
      t[u] = X[(r0 + (e >> 4)) * ldx + (e & 15)];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + u * 256;
      xs[e >> 4][e & 15] = t[u];
    }
  } else {
    for (int e = tid; e < 256 * 16; e += 256) {
      const int rr = e >> 4, cc = e & 15;
      xs[rr][cc] = (rr < rows && cc < a) ? X[(r0 + rr) * ldx + cc] : 0.0;
    }
  }
  __syncthreads();
  double acc1[16], acc2[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) acc1[j] = acc2[j] = 0.0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const double xv = xs[tid][i];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      acc1[j] += xv * sm1[i][j];
      acc2[j] += xv * sm2[i][j];
    }
  }
  __syncthreads();  // xs is reused for the first product
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    xs[tid][j] = acc1[j];
    ys[tid][j] = acc2[j];
  }
  __syncthreads();
  if (rows == 256 && b == 16) {
    double rv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + u * 256;
      rv[u] = R[(r0 + (e >> 4)) * ldr + (e & 15)];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + u * 256;
      Z[(r0 + (e >> 4)) * ldz + (e & 15)] = rv[u] - xs[e >> 4][e & 15];
    }
  } else {
    for (int e = tid; e < rows * b; e += 256) {
      const int rr = e / b, cc = e - rr * b;
      Z[(r0 + rr) * ldz + cc] = R[(r0 + rr) * ldr + cc] - xs[rr][cc];
    }
  }
  if (rows == 256 && c == 16) {
    double lv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + u * 256;
      lv[u] = Lam[(r0 + (e >> 4)) * ldl + (e & 15)];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + u * 256;
      Lam[(r0 + (e >> 4)) * ldl + (e & 15)] = lv[u] + ys[e >> 4][e & 15];
    }
  } else {
    for (int e = tid; e < rows * c; e += 256) {
      const int rr = e / c, cc = e - rr * c;
      Lam[(r0 + rr) * ldl + cc] += ys[rr][cc];
    }
  }
}

namespace {
bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

void launch_rows_small(hipStream_t s, int64_t N, int a, int b, const double* Mm, int64_t mrow, const RowsPairs& pr,
                       int npairs) {
  if (a <= 16 && b <= 16) {
    hipLaunchKernelGGL(k_rows_tile, dim3((unsigned)cdiv(N, 256), (unsigned)npairs), dim3(256), 0, s, N, a, b, Mm,
                       mrow, pr);
    RPF_LAUNCH_CHECK();
    return;
  }
  int vec = 1;
  for (int k = 0; k < npairs; ++k) {
    const RowsPair& q = pr.p[k];
    vec &= aligned16(q.X) && aligned16(q.Y) && (q.ldx % 2 == 0) && (q.ldy % 2 == 0) &&
           (!q.Z || (aligned16(q.Z) && q.ldz % 2 == 0));
  }
  hipLaunchKernelGGL(k_rows_small, dim3((unsigned)cdiv(N, 256), (unsigned)npairs), dim3(256), 0, s, N, a, b, Mm,
                     mrow, pr, vec);
  RPF_LAUNCH_CHECK();
}
}  // namespace

void rows_gemm_from(hipStream_t s, int64_t N, int a, int b, double alpha, const double* X, int64_t ldx,
                    const double* M, double beta, const double* Z, int64_t ldz, double* Y, int64_t ldy) {
  if (N <= 0 || b <= 0) return;
  RPF_CHECK(a <= 64 && b <= 16, RPF_EINVAL, "rows_gemm_from: block too wide");
  RowsPairs pr{};
  pr.p[0] = {X, Y, ldx, ldy, alpha, beta, Z, ldz};
  pr.p[1] = pr.p[0];
  launch_rows_small(s, N, a, b, M, 0, pr, 1);
}

// out[c * ldo] = sum_z part[z * b + c]: one workgroup per column c, a fixed partition of z over the
// threads and a fixed tree (deterministic).
__global__ __launch_bounds__(256) void k_colsum(int nz, int b, const double* part, double* out, int64_t ldo) {
  __shared__ double red[256];
  const int c = blockIdx.x, tid = threadIdx.x;
  double v = 0.0;
  for (int z = tid; z < nz; z += 256) v += part[(int64_t)z * b + c];
  red[tid] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) out[(int64_t)c * ldo] = red[0];
}

bool rows_gemm2_sq(hipStream_t s, int64_t N, int a, int b, const double* M, double alpha1, const double* X1,
                   int64_t ldx1, double beta1, double* Y1, int64_t ldy1, double alpha2, const double* X2,
                   int64_t ldx2, double beta2, double* Y2, int64_t ldy2, double* part, double* sq, int64_t ldsq) {
  if (N <= 0 || b <= 0 || a > 16 || b > 16 || 256 % b != 0) return false;
  RowsPairs pr{};
  pr.p[0] = {X1, Y1, ldx1, ldy1, alpha1, beta1, nullptr, 0};
  pr.p[1] = {X2, Y2, ldx2, ldy2, alpha2, beta2, nullptr, 0};
  pr.colsq = part;
  const unsigned nwg = (unsigned)cdiv(N, 256);
  hipLaunchKernelGGL(k_rows_tile, dim3(nwg, 2), dim3(256), 0, s, N, a, b, M, (int64_t)0, pr);
  RPF_LAUNCH_CHECK();
  // sq[c * ldsq] = sum over workgroups of part[wg * b + c]
  hipLaunchKernelGGL(k_colsum, dim3((unsigned)b), dim3(256), 0, s, (int)nwg, b, part, sq, ldsq);
  RPF_LAUNCH_CHECK();
  return true;
}

// Sum of nrec records of len <= 256 doubles (record r at part[r * len]): workgroup g sums the
// records g per .. g per + per - 1 with thread t on element t (coalesced) and writes element t
// to out[g * rstride + t * inc].  record_sum runs it over groups of records, then sums the groups
// with k_recsum_final; the order of every sum is fixed (deterministic).
__global__ __launch_bounds__(256) void k_recsum(int nrec, int len, int per, const double* part, double* out,
                                                int64_t rstride, int64_t inc) {
  const int t = threadIdx.x;
  if (t >= len) return;
  const int r0 = blockIdx.x * per, r1 = min(nrec, r0 + per);
  double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
  int r = r0;
  for (; r + 4 <= r1; r += 4) {
    v0 += part[(int64_t)r * len + t];
    v1 += part[(int64_t)(r + 1) * len + t];
    v2 += part[(int64_t)(r + 2) * len + t];
    v3 += part[(int64_t)(r + 3) * len + t];
  }
  for (; r < r1; ++r) v0 += part[(int64_t)r * len + t];
  out[(int64_t)blockIdx.x * rstride + t * inc] = (v0 + v1) + (v2 + v3);
}

// Final pass: one wavefront per element (lane l sums the records l, l + 64, ..., then a fixed
// butterfly across the lanes), so the records' loads of an element are all in flight together.
__global__ __launch_bounds__(256) void k_recsum_final(int nrec, int len, const double* part, double* out,
                                                      int64_t inc) {
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (t >= len) return;
  double v = 0.0;
  for (int r = lane; r < nrec; r += 64) v += part[(int64_t)r * len + t];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) out[t * inc] = v;
}

// out[t * inc] = sum of the nrec records; tmp holds 256 records
void record_sum(hipStream_t s, int nrec, int len, const double* part, double* tmp, double* out, int64_t inc) {
  const int groups = std::min(256, std::max(1, nrec));
  const int per = (int)cdiv(nrec, groups);
  const int g = (int)cdiv(nrec, per);
  hipLaunchKernelGGL(k_recsum, dim3((unsigned)g), dim3(256), 0, s, nrec, len, per, part, tmp, (int64_t)len,
                     (int64_t)1);
  hipLaunchKernelGGL(k_recsum_final, dim3((unsigned)cdiv(len, 4)), dim3(256), 0, s, g, len, tmp, out, inc);
  RPF_LAUNCH_CHECK();
}

bool rows_orth_lam(hipStream_t s, int64_t N, int a, int b, int c, const double* X, int64_t ldx, const double* M1,
                   const double* R, int64_t ldr, double* Z, int64_t ldz, const double* M2, double* Lam, int64_t ldl) {
  if (N <= 0 || a <= 0 || a > 16 || b <= 0 || b > 16 || c <= 0 || c > 16) return false;
  hipLaunchKernelGGL(k_rows_orth_lam, dim3((unsigned)cdiv(N, 256)), dim3(256), 0, s, N, a, b, c, M1, M2, X, ldx, R,
                     ldr, Z, ldz, Lam, ldl);
  RPF_LAUNCH_CHECK();
  return true;
}

bool rows_update_gram(hipStream_t s, int64_t N, int a, int b, const double* M, const double* X, int64_t ldx,
                      double alpha, double beta, double* Y, int64_t ldy, double* sqpart, double* sq, int64_t ldsq,
                      double* gpart, double* G) {
  if (N <= 0 || a <= 0 || b <= 0 || a > 16 || b > 16 || 256 % b != 0) return false;
  const int nwg = (int)cdiv(N, 256);
  hipLaunchKernelGGL(k_rows_update_gram, dim3((unsigned)nwg), dim3(256), 0, s, N, a, b, M, X, ldx, alpha, beta, Y,
                     ldy, sqpart, gpart);
  RPF_LAUNCH_CHECK();
  // the first-pass sums go past the partials (the workspaces hold 256 records more)
  if (sq) record_sum(s, nwg, b, sqpart, sqpart + (int64_t)nwg * b, sq, ldsq);
  record_sum(s, nwg, a * b, gpart, gpart + (int64_t)nwg * a * b, G, 1);
  return true;
}

void rows_gemm2(hipStream_t s, int64_t N, int a, int b, const double* M, int64_t mrow, double alpha1,
                const double* X1, int64_t ldx1, double beta1, double* Y1, int64_t ldy1, double alpha2,
                const double* X2, int64_t ldx2, double beta2, double* Y2, int64_t ldy2) {
  if (N <= 0 || b <= 0) return;
  if (a <= 64 && b <= 16) {
    RowsPairs pr{};
    pr.p[0] = {X1, Y1, ldx1, ldy1, alpha1, beta1, nullptr, 0};
    pr.p[1] = {X2, Y2, ldx2, ldy2, alpha2, beta2, nullptr, 0};
    launch_rows_small(s, N, a, b, M, mrow, pr, 2);
  } else {
    rows_gemm(s, N, a, b, alpha1, X1, ldx1, M, beta1, Y1, ldy1, mrow);
    rows_gemm(s, N, a, b, alpha2, X2, ldx2, M, beta2, Y2, ldy2, mrow);
  }
}

void rows_gemm(hipStream_t s, int64_t N, int a, int b, double alpha, const double* X, int64_t ldx, const double* Mm,
               double beta, double* Y, int64_t ldy, int64_t mrow) {
  if (N <= 0 || b <= 0) return;
  if (a <= 64 && b <= 16 && N >= 4096) {
    RowsPairs pr{};
    pr.p[0] = {X, Y, ldx, ldy, alpha, beta, nullptr, 0};
    pr.p[1] = pr.p[0];
    launch_rows_small(s, N, a, b, Mm, mrow, pr, 1);
    return;
  }
  if (a >= 128 && cdiv(N, 64) < 512) {
    // few row blocks: a wavefront per row keeps the whole chip busy on the inner dimension
    hipLaunchKernelGGL(k_rows_gemm_wave, dim3((unsigned)cdiv(N, 4)), dim3(256), 0, s, N, a, b, alpha, X, ldx, Mm, mrow,
                       beta, Y, ldy);
  } else if (b <= 16 && a >= 2) {
    const bool vec = (a % 2) == 0 && (ldx % 2) == 0 && (reinterpret_cast<uintptr_t>(X) % 16) == 0;
    if (vec)
      hipLaunchKernelGGL(k_rows_mfma<true>, dim3((unsigned)cdiv(N, 64)), dim3(256), 0, s, N, a, b, alpha, X, ldx, Mm,
                         mrow, beta, Y, ldy);
    else
      hipLaunchKernelGGL(k_rows_mfma<false>, dim3((unsigned)cdiv(N, 64)), dim3(256), 0, s, N, a, b, alpha, X, ldx,
                         Mm, mrow, beta, Y, ldy);
  } else {
    hipLaunchKernelGGL(k_rows_gemm, dim3((unsigned)cdiv(N, 64)), dim3(256), 0, s, N, a, b, alpha, X, ldx, Mm, mrow,
                       beta, Y, ldy);
  }
  RPF_LAUNCH_CHECK();
}

// ============================================================================ Cholesky
// One NB x NB diagonal block (NB = 64), blocked by 16: four steps, each (1) factors its 16 x 16
// diagonal block and inverts it on one wavefront (lane r holds row r in registers; the column
// values of the other rows come by cross-lane shuffles, no LDS round trips), (2) solves the panel
// below it, L21 = A21 L11^{-T}, and (3) updates the trailing lower triangle, A22 -= L21 L21^T, both
// on all 256 threads from LDS.  The inverse factor is then assembled block row by block row:
// W_ik = -W_ii sum_{j=k}^{i-1} L_ij W_jk.  A single right-looking wavefront needs either ~20k
// unrolled instructions (more than the instruction cache holds) or 64 dependent steps over LDS;
// this form has 4 short serial steps.  Rows and columns beyond jb are padded with the identity.
// Value of v in lane src of the wavefront, src uniform (here a compile-time constant once the
// loops are unrolled): two v_readlane into scalar registers, no LDS round trip as a shuffle takes.
__device__ inline double lane_value(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

__global__ __launch_bounds__(256) void k_potrf_diag(double* Ag, int64_t lda, int jb, double* dinv, int* status,
                                                    int blk) {
  static_assert(NB == 64, "k_potrf_diag assumes 64 x 64 blocks");
  constexpr int QB = 16;
  __shared__ double A[NB][NB + 1];
  __shared__ double W[NB][NB + 1];
  __shared__ double T[3][QB][QB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) bad = 0;
  {
    // all sixteen loads of a thread at clamped (always valid) addresses, issued together and
    // waited for once; values outside the lower jb x jb triangle are replaced afterwards (a load
    // behind a branch would cost one global-memory round trip each)
    double v[NB * NB / 256];
#pragma unroll
    for (int u = 0; u < NB * NB / 256; ++u) {
      const int e = tid + 256 * u;
      const int r = min(e & (NB - 1), jb - 1), c = min(e >> 6, jb - 1);
      v[u] = Ag[(int64_t)c * lda + r];
    }
#pragma unroll
    for (int u = 0; u < NB * NB / 256; ++u) {
      const int e = tid + 256 * u;
      const int r = e & (NB - 1), c = e >> 6;
      A[r][c] = (r < jb && c < jb && c <= r) ? v[u] : ((r == c) ? 1.0 : 0.0);
      W[r][c] = 0.0;
    }
  }
  __syncthreads();
  for (int kb = 0; kb < NB / QB; ++kb) {
    const int k0 = kb * QB;
    if (wave == 0) {
      // (1) 16 x 16 Cholesky and its inverse; lanes >= 16 carry zeros and are never read back
      const int r = lane & (QB - 1);
      double a[QB];
#pragma unroll
      for (int c = 0; c < QB; ++c) a[c] = (lane < QB && c <= r) ? A[k0 + r][k0 + c] : 0.0;
      double rd[QB];
      bool badw = false;
#pragma unroll
      for (int j = 0; j < QB; ++j) {
        double d = lane_value(a[j], j);
        if (!(d > 0.0)) {
          badw = true;
          d = 1.0;
        }
        const double piv = sqrt(d);
        rd[j] = 1.0 / piv;
        if (r == j) a[j] = piv;
        if (r > j) a[j] *= rd[j];
#pragma unroll
        for (int c = j + 1; c < QB; ++c) {
          const double lcj = lane_value(a[j], c);  // row c's entry in column j
          if (r >= c) a[c] -= a[j] * lcj;
        }
      }
      if (lane < QB) {
#pragma unroll
        for (int c = 0; c < QB; ++c)
          if (c <= r) A[k0 + r][k0 + c] = a[c];
      }
      // inverse, lane t = column t: x[k] *= 1/l_kk; x[i] -= l_ik x[k] for i > k
      double x[QB];
#pragma unroll
      for (int i = 0; i < QB; ++i) x[i] = (i == r) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < QB; ++k) {
        x[k] *= rd[k];
#pragma unroll
        for (int i = k + 1; i < QB; ++i) x[i] -= lane_value(a[k], i) * x[k];  // l_ik from row i's lane
      }
      if (lane < QB) {
#pragma unroll
        for (int i = 0; i < QB; ++i) W[k0 + i][k0 + r] = (i >= r) ? x[i] : 0.0;
      }
      if (badw && lane == 0) bad = 1;
    }
    __syncthreads();
    const int r0 = k0 + QB, rem = NB - r0;
    if (rem > 0) {
      // (2) panel: L[r][k0 + c] = sum_{q <= c} A[r][k0 + q] W[k0 + c][k0 + q]
      double pv[3];
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int e = tid + 256 * u;
        pv[u] = 0.0;
        if (e < rem * QB) {
          const int rr = r0 + e / QB, c = e % QB;
          double acc = 0.0;
          // fixed trip count (W is zero above its diagonal), so the LDS reads are issued together
#pragma unroll
          for (int q = 0; q < QB; ++q) acc += A[rr][k0 + q] * W[k0 + c][k0 + q];
          pv[u] = acc;
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int e = tid + 256 * u;
        if (e < rem * QB) A[r0 + e / QB][k0 + e % QB] = pv[u];
      }
      __syncthreads();
      // (3) trailing lower triangle: A[i][c] -= sum_q L[i][k0 + q] L[c][k0 + q], r0 <= c <= i
      const int ntri = rem * (rem + 1) / 2;
      for (int e = tid; e < ntri; e += 256) {
        // e -> (i, c) with i - r0 = ii, c - r0 = cc <= ii, row-wise
        int ii = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while ((ii + 1) * (ii + 2) / 2 <= e) ++ii;
        while (ii * (ii + 1) / 2 > e) --ii;
        const int cc = e - ii * (ii + 1) / 2;
        const int i = r0 + ii, c = r0 + cc;
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < QB; ++q) acc += A[i][k0 + q] * A[c][k0 + q];
        A[i][c] -= acc;
      }
      __syncthreads();
    }
  }
  // off-diagonal blocks of the inverse, block row by block row
  for (int ib = 1; ib < NB / QB; ++ib) {
    // T_k = sum_{j=k}^{ib-1} L_{ib,j} W_{j,k} for k < ib
    for (int e = tid; e < ib * QB * QB; e += 256) {
      const int k = e / (QB * QB), rr = (e / QB) % QB, cc = e % QB;
      double acc = 0.0;
      // the trip count is a multiple of 16: unrolled by 4, the LDS reads of four terms are in flight
#pragma unroll 4
      for (int q = k * QB; q < ib * QB; ++q) acc += A[ib * QB + rr][q] * W[q][k * QB + cc];
      T[k][rr][cc] = acc;
    }
    __syncthreads();
    // W_{ib,k} = -W_{ib,ib} T_k
    for (int e = tid; e < ib * QB * QB; e += 256) {
      const int k = e / (QB * QB), rr = (e / QB) % QB, cc = e % QB;
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < QB; ++q) acc += W[ib * QB + rr][ib * QB + q] * T[k][q][cc];
      W[ib * QB + rr][k * QB + cc] = -acc;
    }
    __syncthreads();
  }
  // the factor (lower part of the jb x jb block) and dinv (column-major, upper part zero)
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e & (NB - 1), c = e >> 6;
    if (r < jb && c < jb && c <= r) Ag[(int64_t)c * lda + r] = A[r][c];
    dinv[(int64_t)c * NB + r] = (r >= c) ? W[r][c] : 0.0;
  }
  if (tid == 0 && bad) atomicCAS(status, 0, blk + 1);
}

LaunchEvents& launch_events() {
  static thread_local LaunchEvents ev;
  return ev;
}

Envelope Envelope::dense(int64_t n) {
  Envelope e;
  const int64_t nb = cdiv(n, NB);
  e.rend.assign(nb, n);
  e.cstart.assign(nb, 0);
  return e;
}

// Two levels: NB-wide steps (diagonal block, panel) inside panels of PANEL = 4 NB columns.  A step
// updates only the columns of its own panel (rank NB); everything to the right of a panel gets
// one rank-PANEL update once the panel is done, so the trailing matrix and the boundary rows are
// read and written once per panel instead of once per step, by GEMMs with K = PANEL (compute-bound
// instead of memory-bound).  The result is the same factor (the updates of one column commute).
bool gemm_nt_flex(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, const double* X, int64_t ldx,
                  const double* Y, int64_t ldy, double beta, double* C, int64_t ldc, bool lower, DevBuf<double>& wa,
                  DevBuf<double>& wb);

void potrf(hipStream_t s, double* A, int64_t lda, int64_t n, int64_t n_fac, const Envelope& env, double* dinv,
           int* status) {
  constexpr int64_t PANEL = 4 * NB;
  const int64_t nblk = cdiv(n_fac, NB);
  RPF_CHECK((int64_t)env.rend.size() >= nblk, RPF_EINVAL, "potrf: envelope too short");
  DevBuf<double> wa, wb;  // operand copies of the large rank-PANEL updates
  for (int64_t P0 = 0; P0 < n_fac; P0 += PANEL) {
    const int64_t P1 = std::min<int64_t>(P0 + PANEL, n_fac);
    int64_t pend = P1;  // rows (and columns) reached by the panel's envelope
    for (int64_t j0 = P0; j0 < P1; j0 += NB) {
      const int64_t t = j0 / NB;
      const int jb = (int)std::min<int64_t>(NB, n_fac - j0);
      double* dt = dinv + t * NB * NB;
      hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, A + j0 * lda + j0, lda, jb, dt, status, (int)t);
      RPF_LAUNCH_CHECK();
      const int64_t r0 = j0 + jb;
      const int64_t rend = std::max<int64_t>(r0, std::min<int64_t>(env.rend[t], n_fac));
      pend = std::max(pend, rend);
      double* col = A + j0 * lda;
      // panel: L21 = A21 L11^{-T}, in place (one N tile covers the jb columns)
      if (rend > r0) dgemm(s, false, true, rend - r0, jb, jb, 1.0, col + r0, lda, dt, NB, 0.0, col + r0, lda);
      if (n > n_fac) dgemm(s, false, true, n - n_fac, jb, jb, 1.0, col + n_fac, lda, dt, NB, 0.0, col + n_fac, lda);
      // update of the remaining columns of this panel (rows within the envelope, boundary rows)
      const int64_t cend = std::min(rend, P1);
      if (cend > r0) {
        dgemm(s, false, true, rend - r0, cend - r0, jb, -1.0, col + r0, lda, col + r0, lda, 1.0,
              A + r0 * lda + r0, lda, true);
        if (n > n_fac)
          dgemm(s, false, true, n - n_fac, cend - r0, jb, -1.0, col + n_fac, lda, col + r0, lda, 1.0,
                A + r0 * lda + n_fac, lda);
      }
    }
    // rank-PANEL update of everything right of the panel (the boundary-boundary block is deferred);
    // rows of a step's columns past its own envelope end are zero, so one product over the
    // panel's whole envelope is exact
    if (pend > P1) {
      const int64_t K = P1 - P0;
      double* pc = A + P0 * lda;
      if (!gemm_nt_flex(s, pend - P1, pend - P1, K, -1.0, pc + P1, lda, pc + P1, lda, 1.0, A + P1 * lda + P1, lda, true,
                        wa, wb))
        dgemm(s, false, true, pend - P1, pend - P1, K, -1.0, pc + P1, lda, pc + P1, lda, 1.0, A + P1 * lda + P1, lda,
              true);
      if (n > n_fac &&
          !gemm_nt_flex(s, n - n_fac, pend - P1, K, -1.0, pc + n_fac, lda, pc + P1, lda, 1.0, A + P1 * lda + n_fac, lda,
                        false, wa, wb))
        dgemm(s, false, true, n - n_fac, pend - P1, K, -1.0, pc + n_fac, lda, pc + P1, lda, 1.0, A + P1 * lda + n_fac,
              lda);
    }
  }
  RPF_HIP(hipStreamSynchronize(s));  // the operand copies are freed on return
}

// Bt[j ldb + k] = X[j + k ldx] for j < rows, k < cols, and 0 for cols <= k < ldb: the transpose of a
// column-major rows x cols block with zero-padded rows, through 64 x 64 LDS tiles (coalesced on
// both sides).  Grid: (cdiv(ldb, 64), cdiv(rows, 64)).
__global__ __launch_bounds__(256) void k_transpose_pad(int64_t rows, int64_t cols, const double* X, int64_t ldx,
                                                       double* Bt, int64_t ldb) {
  __shared__ double t[64][65];
  const int64_t k0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int64_t k = k0 + r, j = j0 + tx;
    t[r][tx] = (k < cols && j < rows) ? X[j + k * ldx] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int64_t j = j0 + r, k = k0 + tx;
    if (j < rows && k < ldb) Bt[j * ldb + k] = t[tx][r];
  }
}

// C = alpha X Y^T + beta C (X: M x K, Y: N x K, column-major) on the large-problem kernel when the
// shape is large enough: X is used in place when its layout allows it (else copied with an even
// leading dimension), Y^T is copied with k-contiguous rows padded to 32.  wa, wb: grow-only
// workspaces kept by the caller across calls.  Returns false (nothing launched) for small shapes.
bool gemm_nt_flex(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, const double* X, int64_t ldx,
                  const double* Y, int64_t ldy, double beta, double* C, int64_t ldc, bool lower, DevBuf<double>& wa,
                  DevBuf<double>& wb) {
  if (M < 1024 || (M & 1) || N < 128 || K < 64 || M > INT32_MAX || N > INT32_MAX) return false;
  const double* Ause = X;
  int64_t lda = ldx;
  if ((ldx & 1) || ((uintptr_t)X & 15)) {
    wa.ensure((size_t)M * K);
    copy_matrix(s, X, ldx, wa.p, M, M, K);
    Ause = wa.p;
    lda = M;
  }
  const int64_t ldb = cdiv(K, 32) * 32;
  wb.ensure((size_t)N * ldb);
  hipLaunchKernelGGL(k_transpose_pad, dim3((unsigned)cdiv(ldb, 64), (unsigned)cdiv(N, 64)), dim3(256), 0, s, N, K, Y,
                     ldy, wb.p, ldb);
  RPF_LAUNCH_CHECK();
  return dgemm_flex(s, M, N, K, alpha, Ause, lda, wb.p, ldb, beta, C, ldc, lower);
}

void schur_update(hipStream_t s, double* A, int64_t lda, int64_t n, int64_t n_fac) {
  const int64_t nb = n - n_fac;
  if (nb <= 0 || n_fac <= 0) return;
  const double* Lbi = A + n_fac;  // boundary rows of the factor, nb x n_fac with ld lda
  // lower tiles only: S is symmetric and only its lower triangle is read afterwards
  DevBuf<double> wa, wb;
  const bool done = gemm_nt_flex(s, nb, nb, n_fac, -1.0, Lbi, lda, Lbi, lda, 1.0, A + n_fac * lda + n_fac, lda, true,
                                 wa, wb);
  if (done) {
    RPF_HIP(hipStreamSynchronize(s));  // the copies are freed on return
    return;
  }
  dgemm(s, false, true, nb, nb, n_fac, -1.0, Lbi, lda, Lbi, lda, 1.0, A + n_fac * lda + n_fac, lda, true);
}

// Panel triangular solve for many right-hand sides: one workgroup owns PW = 16 H columns of B and
// walks all diagonal blocks in order (persistent), left-looking: for block t it forms
// B_t - L_t,band X_band on FP64 MFMA, stages the result in LDS and multiplies it by the inverted
// diagonal block, overwriting B_t with X_t.  Forward (L X = B) uses the rows of block t from column
// lo[t]; backward (L^T X = B) the rows j0 + 64 .. hi[t] of column block t.  The band is split over
// the four waves (wave w takes every fourth group of 16 k, all 64 rows of the block and the H
// 16-column parts: 4 H independent accumulators, each L fragment used H times from registers),
// the loads of a wave's next group are in flight while the MFMAs of the current one run, and the
// four partial products are summed in LDS.  The band operands come from L2 (every workgroup reads
// the same band of L; its own panel of X was written by itself one block earlier); the band's L2
// traffic is one read per PW right-hand sides.  UP (backward only): the band of L^T is read from the
// mirrored upper triangle, L^T[row][k] = A[row + k ldl], sixteen consecutive rows per load like the
// forward solve, instead of sixteen columns of L 8 bytes each.
template <bool FWD, int H, bool UP = false>
__global__ __launch_bounds__(256) void k_trsm_panel(const double* L, int64_t ldl, int64_t n, const double* dinv,
                                                    const int64_t* lo, const int64_t* hi, double* B, int64_t ldb,
                                                    int64_t nrhs) {
  constexpr int PW = 16 * H;
  __shared__ double S[NB][PW + 1];
  __shared__ double red[4][NB][PW + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t col0 = (int64_t)blockIdx.x * PW + li;  // this lane's column in part 0 (part h: + 16 h)
  bool cok[H];
#pragma unroll
  for (int h = 0; h < H; ++h) cok[h] = col0 + 16 * h < nrhs;
  const int64_t nblk = (n + NB - 1) / NB;
  for (int64_t step = 0; step < nblk; ++step) {
    const int64_t t = FWD ? step : nblk - 1 - step;
    const int64_t j0 = t * NB;
    const int jb = (int)min<int64_t>(NB, n - j0);
    v4d acc[4][H];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int h = 0; h < H; ++h) acc[q][h] = v4d{0.0, 0.0, 0.0, 0.0};
    int64_t kb, ke;
    if (FWD) {
      kb = max<int64_t>(0, lo[t]);
      ke = j0;
    } else {
      kb = j0 + jb;
      ke = min<int64_t>(hi[t], n);
    }
    // group g covers k in [kb + 16 g, kb + 16 g + 16); wave w takes g = w, w + 4, ...
    auto load = [&](int64_t k0, double* a, double* b) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t k = k0 + 4 * u + lk;
        const bool kok = k < ke;
#pragma unroll
        for (int h = 0; h < H; ++h) b[H * u + h] = (kok && cok[h]) ? B[k + (col0 + 16 * h) * ldb] : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t row = j0 + 16 * q + li;
          a[4 * q + u] = (kok && row < j0 + jb) ? ((FWD || UP) ? L[row + k * ldl] : L[k + row * ldl]) : 0.0;
        }
      }
    };
    double a[16], b[4 * H], na[16], nb[4 * H];
    int64_t k0 = kb + 16 * w;
    if (k0 < ke) load(k0, a, b);
    for (; k0 < ke; k0 += 64) {
      const bool more = k0 + 64 < ke;
      if (more) load(k0 + 64, na, nb);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int h = 0; h < H; ++h)
            acc[q][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[4 * q + u], b[H * u + h], acc[q][h], 0, 0, 0);
      if (more) {
#pragma unroll
        for (int u = 0; u < 16; ++u) a[u] = na[u];
#pragma unroll
        for (int u = 0; u < 4 * H; ++u) b[u] = nb[u];
      }
    }
    // accumulator item r of tile (q, h), lane l: row 16 q + l/16 + 4 r, column 16 h + l % 16
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int h = 0; h < H; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[w][16 * q + lk + 4 * r][16 * h + li] = acc[q][h][r];
    __syncthreads();
    for (int e = tid; e < NB * PW; e += 256) {
      const int ri = e / PW, cj = e % PW;
      const int64_t gc = (int64_t)blockIdx.x * PW + cj;
      const double bv = (ri < jb && gc < nrhs) ? B[j0 + ri + gc * ldb] : 0.0;
      S[ri][cj] = bv - (red[0][ri][cj] + red[1][ri][cj] + red[2][ri][cj] + red[3][ri][cj]);
    }
    __syncthreads();
    // X_t = inv(L_tt) S (forward) or inv(L_tt)^T S (backward): dinv column-major NB x NB; wave w
    // forms rows 16 w .. 16 w + 15 of every column part
    v4d x[H];
#pragma unroll
    for (int h = 0; h < H; ++h) x[h] = v4d{0.0, 0.0, 0.0, 0.0};
    const double* D = dinv + t * NB * NB;
#pragma unroll 4
    for (int kk = 0; kk < NB; kk += 4) {
      const int k = kk + lk, i = 16 * w + li;
      const double av = FWD ? D[i + k * NB] : D[k + i * NB];
#pragma unroll
      for (int h = 0; h < H; ++h) x[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, S[k][16 * h + li], x[h], 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ri = 16 * w + lk + 4 * r;
      if (ri < jb) {
#pragma unroll
        for (int h = 0; h < H; ++h)
          if (cok[h]) B[j0 + ri + (col0 + 16 * h) * ldb] = x[h][r];
      }
    }
    __syncthreads();  // X_t is read by the band products of the following blocks
  }
}

void trsm(hipStream_t s, const double* L, int64_t ldl, int64_t n, const double* dinv, const Envelope& env,
          double* B, int64_t ldb, int64_t nrhs, bool trans, bool upper) {
  if (n <= 0 || nrhs <= 0) return;
  const int64_t nblk = cdiv(n, NB);
  bool dense = true;
  for (int64_t t = 0; t < nblk && dense; ++t) dense = env.cstart[t] <= 0 && env.rend[t] >= n;
  if (!dense && nrhs >= 2048) {
    // banded factor, many right-hand sides: one persistent pass per 16- or 32-column panel
    std::vector<int64_t> bounds(2 * nblk);
    for (int64_t t = 0; t < nblk; ++t) {
      bounds[t] = env.cstart[t];
      bounds[nblk + t] = env.rend[t];
    }
    DevBuf<int64_t> db;
    db.upload(bounds.data(), bounds.size(), s);
    // 16 columns per workgroup, two workgroups per CU, where the band of L (or of the mirrored L^T)
    // is read sixteen rows at a time: 12.7 ms each way at 8192 columns of the 20^3 pattern (32
    // columns, one workgroup per CU: 14 ms forward, 14.3 ms backward).  Without the mirror the
    // backward reads columns of L, and 32 columns per workgroup halve that less efficient band
    // traffic (15.5 ms; 21 ms at 16).
    if (!trans)
      hipLaunchKernelGGL((k_trsm_panel<true, 1>), dim3((unsigned)cdiv(nrhs, 16)), dim3(256), 0, s, L, ldl, n, dinv,
                         db.p, db.p + nblk, B, ldb, nrhs);
    else if (upper)
      hipLaunchKernelGGL((k_trsm_panel<false, 1, true>), dim3((unsigned)cdiv(nrhs, 16)), dim3(256), 0, s, L, ldl, n,
                         dinv, db.p, db.p + nblk, B, ldb, nrhs);
    else
      hipLaunchKernelGGL((k_trsm_panel<false, 2>), dim3((unsigned)cdiv(nrhs, 32)), dim3(256), 0, s, L, ldl, n, dinv,
                         db.p, db.p + nblk, B, ldb, nrhs);
    RPF_LAUNCH_CHECK();
    RPF_HIP(hipStreamSynchronize(s));  // the bounds buffer is freed on return
    return;
  }
  if (dense && nrhs >= 4096) {
    // Full factor, many right-hand sides (the identity of the condensation): left-looking by row
    // blocks.  Block t first takes the contributions of all solved blocks, B_t -= L_t,prev X_prev
    // (one product with a long inner dimension, split over K when its output tiles alone cannot
    // fill the chip), then X_t = inv(L_tt) B_t; B is read once per block instead of rewritten for
    // every trailing update.
    // the split-K workspace is sized once for the largest block: growing it inside the loop would
    // free and reallocate it (a device-wide synchronisation) at every larger block
    DevBuf<double> ws;
    {
      size_t most = 0;
      for (int64_t t = 0; t < nblk; ++t) {
        const int64_t j0 = t * NB;
        const int jb = (int)std::min<int64_t>(NB, n - j0);
        const int64_t kdim = trans ? n - j0 - jb : j0;
        const int sp = kdim > 0 ? gemm_splitk_count(jb, nrhs, kdim) : 1;
        if (sp > 1) most = std::max(most, (size_t)sp * jb * nrhs);
      }
      ws.ensure(most);
    }
    auto update = [&](bool ta, int jb, int64_t kdim, const double* A, const double* Bsrc, double* C) {
      if (kdim <= 0) return;
      const int sp = gemm_splitk_count(jb, nrhs, kdim);
      if (sp > 1) {
        ws.ensure((size_t)sp * jb * nrhs);
        dgemm_splitk(s, ta, false, jb, nrhs, kdim, -1.0, A, ldl, Bsrc, ldb, 1.0, C, ldb, ws.p, sp);
      } else {
        dgemm(s, ta, false, jb, nrhs, kdim, -1.0, A, ldl, Bsrc, ldb, 1.0, C, ldb);
      }
    };
    if (!trans) {
      for (int64_t t = 0; t < nblk; ++t) {
        const int64_t j0 = t * NB;
        const int jb = (int)std::min<int64_t>(NB, n - j0);
        update(false, jb, j0, L + j0, B, B + j0);
        // in place: the single row tile of this product reads all of B_t before writing it
        dgemm(s, false, false, jb, nrhs, jb, 1.0, dinv + t * NB * NB, NB, B + j0, ldb, 0.0, B + j0, ldb);
      }
    } else {
      for (int64_t t = nblk - 1; t >= 0; --t) {
        const int64_t j0 = t * NB;
        const int jb = (int)std::min<int64_t>(NB, n - j0);
        const int64_t r0 = j0 + jb;
        update(true, jb, n - r0, L + j0 * ldl + r0, B + r0, B + j0);
        dgemm(s, true, false, jb, nrhs, jb, 1.0, dinv + t * NB * NB, NB, B + j0, ldb, 0.0, B + j0, ldb);
      }
    }
    return;
  }
  // Banded factors: right-looking, each solved block updates the rows of its envelope below.
  if (!trans) {
    for (int64_t t = 0; t < nblk; ++t) {
      const int64_t j0 = t * NB;
      const int jb = (int)std::min<int64_t>(NB, n - j0);
      const double* dt = dinv + t * NB * NB;
      dgemm(s, false, false, jb, nrhs, jb, 1.0, dt, NB, B + j0, ldb, 0.0, B + j0, ldb);
      const int64_t r0 = j0 + jb;
      const int64_t rend = std::min<int64_t>(env.rend[t], n);
      if (rend > r0)
        dgemm(s, false, false, rend - r0, nrhs, jb, -1.0, L + j0 * ldl + r0, ldl, B + j0, ldb, 1.0, B + r0, ldb);
    }
  } else {
    for (int64_t t = nblk - 1; t >= 0; --t) {
      const int64_t j0 = t * NB;
      const int jb = (int)std::min<int64_t>(NB, n - j0);
      const double* dt = dinv + t * NB * NB;
      dgemm(s, true, false, jb, nrhs, jb, 1.0, dt, NB, B + j0, ldb, 0.0, B + j0, ldb);
      const int64_t cs = std::max<int64_t>(0, env.cstart[t]);
      if (j0 > cs)
        dgemm(s, true, false, j0 - cs, nrhs, jb, -1.0, L + cs * ldl + j0, ldl, B + j0, ldb, 1.0, B + cs, ldb);
    }
  }
}

// Y = (L L^T)^{-1} from a dense lower Cholesky factor L (n x n, ld ldl) and its inverted diagonal
// blocks: the forward solve L X = I, then L^T Y = X, skipping what is known to be zero or not
// needed.  X = L^{-1} is lower triangular, so block row t of the forward solve only involves the
// columns left of its diagonal block and the diagonal block itself; Y is symmetric, so the backward
// solve forms its lower triangle only (block row t: the columns up to its diagonal block, which need
// only lower-triangle entries of the rows below), and the upper triangle is mirrored at the end.
// Same arithmetic as the full solves with identity right-hand sides, about a quarter of the flops.
void potri_lower(hipStream_t s, const double* L, int64_t ldl, int64_t n, const double* dinv, double* Y,
                 int64_t ldy) {
  if (n <= 0) return;
  const int64_t nblk = cdiv(n, NB);
  fill_matrix(s, Y, n, n, ldy, 0.0);
  add_diag(s, Y, ldy, n, 1.0);
  // the split-K workspace is sized once for the largest block (see trsm)
  DevBuf<double> ws;
  {
    size_t most = 0;
    for (int64_t t = 0; t < nblk; ++t) {
      const int64_t j0 = t * NB;
      const int jb = (int)std::min<int64_t>(NB, n - j0);
      const int64_t fw[2][2] = {{j0, j0}, {j0 + jb, n - j0 - jb}};  // (ncol, kdim) forward, backward
      for (const auto& d : fw) {
        if (d[0] <= 0 || d[1] <= 0) continue;
        const int sp = gemm_splitk_count(jb, d[0], d[1]);
        if (sp > 1) most = std::max(most, (size_t)sp * jb * d[0]);
      }
    }
    ws.ensure(most);
  }
  auto update = [&](bool ta, int jb, int64_t ncol, int64_t kdim, const double* A, const double* Bsrc, double* C) {
    if (kdim <= 0 || ncol <= 0) return;
    const int sp = gemm_splitk_count(jb, ncol, kdim);
    if (sp > 1) {
      ws.ensure((size_t)sp * jb * ncol);
      dgemm_splitk(s, ta, false, jb, ncol, kdim, -1.0, A, ldl, Bsrc, ldy, 1.0, C, ldy, ws.p, sp);
    } else {
      dgemm(s, ta, false, jb, ncol, kdim, -1.0, A, ldl, Bsrc, ldy, 1.0, C, ldy);
    }
  };
  // forward: X_t = inv(L_tt) (I_t - L_t,prev X_prev), nonzero in columns [0, j0 + jb)
  for (int64_t t = 0; t < nblk; ++t) {
    const int64_t j0 = t * NB;
    const int jb = (int)std::min<int64_t>(NB, n - j0);
    update(false, jb, j0, j0, L + j0, Y, Y + j0);
    // in place: the single row tile of this product reads all of its rows before writing them
    dgemm(s, false, false, jb, j0 + jb, jb, 1.0, dinv + t * NB * NB, NB, Y + j0, ldy, 0.0, Y + j0, ldy);
  }
  // backward, lower triangle: Y_t = inv(L_tt)^T (X_t - L_below,t^T Y_below) in columns [0, j0 + jb)
  for (int64_t t = nblk - 1; t >= 0; --t) {
    const int64_t j0 = t * NB;
    const int jb = (int)std::min<int64_t>(NB, n - j0);
    const int64_t r0 = j0 + jb;
    update(true, jb, j0 + jb, n - r0, L + j0 * ldl + r0, Y + r0, Y + j0);
    dgemm(s, true, false, jb, j0 + jb, jb, 1.0, dinv + t * NB * NB, NB, Y + j0, ldy, 0.0, Y + j0, ldy);
  }
  mirror_lower(s, Y, ldy, n);
  RPF_HIP(hipStreamSynchronize(s));  // the split-K workspace is freed on return
}

// ============================================================================ elementwise helpers
__global__ void k_fill(double* p, int64_t count, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

__global__ void k_fill_matrix(double* p, int64_t rows, int64_t cols, int64_t ld, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < rows * cols) p[(i / rows) * ld + (i % rows)] = v;
}

__global__ void k_copy_matrix(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows, int64_t cols) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < rows * cols) {
    const int64_t r = i % rows, c = i / rows;
    dst[c * ldd + r] = src[c * lds + r];
  }
}

__global__ void k_mirror_lower(double* A, int64_t lda, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * n) {
    const int64_t r = i % n, c = i / n;
    if (r < c) A[c * lda + r] = A[r * lda + c];
  }
}

__global__ void k_add_diag(double* A, int64_t lda, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) A[i * lda + i] += v;
}

void fill(hipStream_t s, double* p, int64_t count, double v) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)cdiv(count, 256)), dim3(256), 0, s, p, count, v);
  RPF_LAUNCH_CHECK();
}

void fill_matrix(hipStream_t s, double* p, int64_t rows, int64_t cols, int64_t ld, double v) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(k_fill_matrix, dim3((unsigned)cdiv(rows * cols, 256)), dim3(256), 0, s, p, rows, cols, ld, v);
  RPF_LAUNCH_CHECK();
}

void copy_matrix(hipStream_t s, const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                 int64_t cols) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(k_copy_matrix, dim3((unsigned)cdiv(rows * cols, 256)), dim3(256), 0, s, src, lds, dst, ldd,
                     rows, cols);
  RPF_LAUNCH_CHECK();
}

// One 64 x 64 tile of column block t (blockIdx.y), rows r0 = t 64 + 64 blockIdx.x up to rend[t]: read
// down the columns, written along the rows (both coalesced, through LDS); only entries below the
// diagonal are copied, so the lower triangle is untouched.
__global__ __launch_bounds__(256) void k_mirror_env(double* A, int64_t lda, int64_t n, const int64_t* rend) {
  __shared__ double t[64][65];
  const int64_t j0 = (int64_t)blockIdx.y * 64;
  const int64_t r0 = j0 + (int64_t)blockIdx.x * 64;
  const int64_t re = min(rend[blockIdx.y], n);
  if (r0 >= re) return;
  const int jb = (int)min<int64_t>(64, n - j0);
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int c = ty; c < jb; c += 4) {
    const int64_t r = r0 + tx;
    t[c][tx] = r < re ? A[r + (j0 + c) * lda] : 0.0;
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const int64_t r = r0 + i;
    const int c = tx;
    if (r < re && c < jb && r > j0 + c) A[(j0 + c) + r * lda] = t[c][i];
  }
}

void mirror_envelope(hipStream_t s, double* A, int64_t lda, int64_t n, const Envelope& env) {
  if (n <= 0) return;
  const int64_t nblk = cdiv(n, NB);
  RPF_CHECK((int64_t)env.rend.size() >= nblk, RPF_EINVAL, "mirror_envelope: envelope too short");
  std::vector<int64_t> re(env.rend.begin(), env.rend.begin() + nblk);
  int64_t tiles = 1;
  for (int64_t t = 0; t < nblk; ++t) tiles = std::max<int64_t>(tiles, cdiv(std::min(re[t], n) - t * NB, NB));
  DevBuf<int64_t> d;
  d.upload(re.data(), re.size(), s);
  hipLaunchKernelGGL(k_mirror_env, dim3((unsigned)tiles, (unsigned)nblk), dim3(256), 0, s, A, lda, n, d.p);
  RPF_LAUNCH_CHECK();
  RPF_HIP(hipStreamSynchronize(s));  // the bounds buffer is freed on return
}

void mirror_lower(hipStream_t s, double* A, int64_t lda, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mirror_lower, dim3((unsigned)cdiv(n * n, 256)), dim3(256), 0, s, A, lda, n);
  RPF_LAUNCH_CHECK();
}

void add_diag(hipStream_t s, double* A, int64_t lda, int64_t n, double v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_add_diag, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, A, lda, n, v);
  RPF_LAUNCH_CHECK();
}

// ============================================================================ small eigenproblems
// Parallel cyclic Jacobi (Brent-Luk ordering: m/2 disjoint rotations per step,
// m-1 steps per sweep), one workgroup per matrix, m <= 64.
constexpr int EIG_MAX = 64;

// TMODE: the matrix is eta of the block solver and the kernel writes T = V diag(w^{-1/2}) over the
// kept eigenpairs (w_i > tau * max(w_max, state[1]); the others are counted in *drops and, when
// none is kept, 1 is written to flag0 and flag1); it returns at once when state[0] != 0 (T was
// already formed from a Cholesky factor of eta).
template <bool TMODE>
__global__ __launch_bounds__(256) void k_syev_jacobi(const double* Ain, int m, double* Vout, double* wout,
                                                     const double* state, double tau, double* T, int* drops,
                                                     double* flag0, double* flag1) {
  if (TMODE && state[0] != 0.0) return;
  __shared__ double a[EIG_MAX][EIG_MAX + 1];
  __shared__ double v[EIG_MAX][EIG_MAX + 1];
  __shared__ int pp[EIG_MAX / 2], qq[EIG_MAX / 2];
  __shared__ double cc[EIG_MAX / 2], ss[EIG_MAX / 2];

  __shared__ int order[EIG_MAX];
  const int tid = threadIdx.x;
  const double* A = Ain + (int64_t)blockIdx.x * m * m;
  double* V = Vout + (int64_t)blockIdx.x * m * m;
  double* w = wout + (int64_t)blockIdx.x * m;
  const int nth = blockDim.x;
  for (int i = tid; i < m * m; i += nth) {
    const int r = i % m, c = i / m;
    a[r][c] = 0.5 * (A[c * m + r] + A[r * m + c]);
    v[r][c] = (r == c) ? 1.0 : 0.0;
  }
  const int me = m + (m & 1);  // even count for the round-robin schedule
  const int npair = me / 2;
  __shared__ int nrot;
  __shared__ double floor_abs;
  __syncthreads();
  // threshold Jacobi: a pair is rotated only while |a_pq| > 1e-13 sqrt(|a_pp a_qq|) (relative
  // accuracy of the eigenvalues to about 1e-13, ample for eta^{-1/2}) and |a_pq| > 1e-15
  // max_i |a_ii| (eigenvalues below 1e-12 of the largest are dropped by the caller, and
  // below this floor a rotation only moves rounding noise); the sweeps stop once a whole
  // sweep rotates nothing
  for (int sweep = 0; sweep < 30 && m >= 2; ++sweep) {
    if (tid == 0) {
      nrot = 0;
      double d = 0.0;
      for (int i = 0; i < m; ++i) d = fmax(d, fabs(a[i][i]));
      floor_abs = fmax(1e-15 * d, 1e-300);
    }
    __syncthreads();
    for (int step = 0; step < me - 1; ++step) {
      // circle method: indices 0..me-2 rotate, me-1 is fixed
      if (tid < npair) {
        int i, j;
        if (tid == 0) {
          i = step;
          j = me - 1;
        } else {
          i = (step + tid) % (me - 1);
          j = (step - tid + (me - 1)) % (me - 1);
        }
        const int p = i < j ? i : j, q = i < j ? j : i;
        double c = 1.0, sn = 0.0;
        if (q < m) {
          const double apq = a[p][q];
          if (fabs(apq) > 1e-13 * sqrt(fabs(a[p][p] * a[q][q])) && fabs(apq) > floor_abs) {
            atomicAdd(&nrot, 1);
            const double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
            const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = t * c;
          }
        }
        pp[tid] = p;
        qq[tid] = q;
        cc[tid] = c;
        ss[tid] = sn;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int idx = tid; idx < npair * m; idx += nth) {
        const int k = idx / m, r = idx % m;
        const int p = pp[k], q = qq[k];
        if (q >= m) continue;
        const double c = cc[k], sn = ss[k];
        const double x = a[r][p], y = a[r][q];
        a[r][p] = c * x - sn * y;
        a[r][q] = sn * x + c * y;
        const double vx = v[r][p], vy = v[r][q];
        v[r][p] = c * vx - sn * vy;
        v[r][q] = sn * vx + c * vy;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int idx = tid; idx < npair * m; idx += nth) {
        const int k = idx / m, col = idx % m;
        const int p = pp[k], q = qq[k];
        if (q >= m) continue;
        const double c = cc[k], sn = ss[k];
        const double x = a[p][col], y = a[q][col];
        a[p][col] = c * x - sn * y;
        a[q][col] = sn * x + c * y;
      }
      __syncthreads();
    }
    if (nrot == 0) break;  // uniform: read after the last barrier of the sweep
    __syncthreads();
  }
  __syncthreads();
  if (tid == 0) {
    for (int i = 0; i < m; ++i) order[i] = i;
    for (int i = 0; i < m; ++i) {
      int best = i;
      for (int j = i + 1; j < m; ++j)
        if (a[order[j]][order[j]] < a[order[best]][order[best]]) best = j;
      const int t = order[i];
      order[i] = order[best];
      order[best] = t;
    }
  }
  __syncthreads();
  if (!TMODE) {
    for (int i = tid; i < m * m; i += nth) {
      const int r = i % m, c = i / m;
      V[c * m + r] = v[r][order[c]];
    }
    for (int i = tid; i < m; i += nth) w[i] = a[order[i]][order[i]];
  } else {
    __shared__ double scale[EIG_MAX];
    __shared__ int kept;
    if (tid == 0) kept = 0;
    __syncthreads();
    const double ref = fmax(a[order[m - 1]][order[m - 1]], state[1]);
    if (tid < m) {
      const double wi = a[order[tid]][order[tid]];
      const bool keep = wi > 0.0 && wi > tau * ref;
      scale[tid] = keep ? 1.0 / sqrt(wi) : 0.0;
      if (keep) atomicAdd(&kept, 1);
      else atomicAdd(drops, 1);
    }
    __syncthreads();
    if (tid == 0 && kept == 0) {
      flag0[0] = 1.0;
      flag1[0] = 1.0;
    }
    for (int i = tid; i < m * m; i += nth) {
      const int r = i % m, c = i / m;
      T[c * m + r] = v[r][order[c]] * scale[c];
    }
  }
}

void syev_small(hipStream_t s, const double* A, int m, double* V, double* w, int batch) {
  RPF_CHECK(m >= 1 && m <= EIG_MAX, RPF_EINVAL, "syev_small: m out of range");
  // one wavefront is enough (and its barriers are cheapest) while m/2 * m <= 128 work items
  const int threads = (m <= 16) ? 64 : 256;
  hipLaunchKernelGGL(k_syev_jacobi<false>, dim3(batch), dim3(threads), 0, s, A, m, V, w, (const double*)nullptr, 0.0,
                     (double*)nullptr, (int*)nullptr, (double*)nullptr, (double*)nullptr);
  RPF_LAUNCH_CHECK();
}

void eta_eigen_T(hipStream_t s, const double* eta, int m, const double* state, double tau, double* T, int* drops,
                 double* flag0, double* flag1) {
  RPF_CHECK(m >= 1 && m <= EIG_MAX, RPF_EINVAL, "eta_eigen_T: m out of range");
  const int threads = (m <= 16) ? 64 : 256;
  hipLaunchKernelGGL(k_syev_jacobi<true>, dim3(1), dim3(threads), 0, s, eta, m, (double*)nullptr, (double*)nullptr,
                     state, tau, T, drops, flag0, flag1);
  RPF_LAUNCH_CHECK();
}

// ============================================================================ orthonormalisation
__device__ inline double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (tid == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    red[16] = t;
  }
  __syncthreads();
  t = red[16];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(1024) void k_mgs2(double* Y, int64_t n, int64_t ld, int k) {
  __shared__ double red[17];
  const int tid = threadIdx.x;
  for (int j = 0; j < k; ++j) {
    double* yj = Y + (int64_t)j * ld;
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i < j; ++i) {
        const double* yi = Y + (int64_t)i * ld;
        double d = 0.0;
        for (int64_t r = tid; r < n; r += blockDim.x) d += yi[r] * yj[r];
        d = block_sum(d, red);
        for (int64_t r = tid; r < n; r += blockDim.x) yj[r] -= d * yi[r];
        __syncthreads();
      }
    }
    double nn = 0.0;
    for (int64_t r = tid; r < n; r += blockDim.x) nn += yj[r] * yj[r];
    nn = block_sum(nn, red);
    const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    for (int64_t r = tid; r < n; r += blockDim.x) yj[r] *= inv;
    __syncthreads();
  }
}

void orthonormalize(hipStream_t s, double* Y, int64_t n, int64_t ld, int k) {
  if (k <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_mgs2, dim3(1), dim3(1024), 0, s, Y, n, ld, k);
  RPF_LAUNCH_CHECK();
}

}  // namespace rpf
