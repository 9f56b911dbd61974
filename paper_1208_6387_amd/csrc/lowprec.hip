// Low-precision flexibility products for the mixed forms: Y_loc = S+ X_loc with
// FP32 operands (v_mfma_f32_16x16x4_f32) or with bf16 high/low splits of both
// operands (v_mfma_f32_16x16x32_bf16, three cross products hi*hi + hi*lo + lo*hi),
// FP32 accumulation in both cases.  The gather writes the W format directly in
// the low-precision layout and the scatter reads FP32 and assembles in FP64.
#include "problem.hpp"

namespace rpf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_val(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// ---------------------------------------------------------------------------- gather (low precision out)
// mode 0: FP32 out (Xf); mode 1: bf16 split out (Xh, Xl)
template <int DPN, int MODE>
__global__ __launch_bounds__(128) void k_gather_lp(int nbn, const int* occ_list, const int* slot_off,
                                                   const int* l2m_ptr, const int* l2m_code, const double* rot,
                                                   const double* lam, int64_t ldl, int m, float* Xf, uint16_t* Xh,
                                                   uint16_t* Xl, int64_t ldx) {
  const int bn = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (bn >= nbn) return;
  const int s = occ_list[q];
  const int slot = slot_off[s] + bn;
  const int e0 = l2m_ptr[slot], e1 = l2m_ptr[slot + 1];
  double O[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) O[i] = rot ? rot[9 * s + i] : ((i % 4 == 0) ? 1.0 : 0.0);
  for (int j0 = 0; j0 < m; j0 += 8) {
    const int jn = min(8, m - j0);
    double acc[DPN][8];
#pragma unroll
    for (int c = 0; c < DPN; ++c)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[c][j] = 0.0;
    for (int e = e0; e < e1; ++e) {
      const int code = l2m_code[e];
      const double sg = (code & 1) ? -1.0 : 1.0;
      const int64_t mult = code >> 1;
#pragma unroll
      for (int c = 0; c < DPN; ++c) {
        const double* row = lam + (mult * DPN + c) * ldl + j0;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (j < jn) acc[c][j] += sg * row[j];
      }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j >= jn) break;
      const int64_t base = ((int64_t)q * m + j0 + j) * ldx + (int64_t)bn * DPN;
#pragma unroll
      for (int c2 = 0; c2 < DPN; ++c2) {
        double v;
        if (DPN == 3) v = O[c2] * acc[0][j] + O[3 + c2] * acc[1 % DPN][j] + O[6 + c2] * acc[2 % DPN][j];
        else v = acc[c2][j];
        if (MODE == 0) {
          Xf[base + c2] = (float)v;
        } else {
          const uint16_t h = bf16_bits((float)v);
          Xh[base + c2] = h;
          Xl[base + c2] = bf16_bits((float)(v - (double)bf16_val(h)));
        }
      }
    }
  }
}

// Gather with lanes over interface columns: a group of JW lanes takes one boundary node and sums
// the signed multiplier rows at it (each row read as JW consecutive doubles), turned into the
// pattern frame; the workgroup collects a tile of NBK nodes x JW columns in LDS and writes it
// out column by column with consecutive lanes on consecutive dofs.  mode 0: FP32 (Xf), 1: bf16
// hi/lo split (Xh, Xl), 2: FP64 (X64).  Grid: (node blocks, occurrences of the pattern).
template <int DPN, int MODE, int JW>
__global__ __launch_bounds__(256) void k_gather_rows(int nbn, const int* occ_list, const int* slot_off,
                                                     const int* l2m_ptr, const int* l2m_code, const double* rot,
                                                     const double* lam, int64_t ldl, int m, double* X64, float* Xf,
                                                     uint16_t* Xh, uint16_t* Xl, int64_t ldx) {
  constexpr int NG = 256 / JW, NBK = 64;
  constexpr int NPG = NBK / NG;  // nodes per lane group
  constexpr int UM = 2;          // incidences per node fetched in the batch (faces 1, edges 2, corners 3)
  __shared__ double tile[JW][NBK * DPN + 1];
  __shared__ int sptr[NBK + 1];
  const int q = blockIdx.y, s = occ_list[q];
  const int n0 = blockIdx.x * NBK;
  const int nn = min(NBK, nbn - n0);
  const int tid = threadIdx.x, g = tid / JW, jl = tid % JW;
  const int base_slot = slot_off[s] + n0;
  double O[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) O[i] = rot ? rot[9 * s + i] : ((i % 4 == 0) ? 1.0 : 0.0);
  if (tid <= nn) sptr[tid] = l2m_ptr[base_slot + tid];
  __syncthreads();
  // the block's incidences are one contiguous run [eb, ee) of the slot lists: every code and
  // multiplier-row load below goes to a clamped index inside it (always valid: a node's own last
  // incidence, so a surplus load re-reads a row already being read) and is masked afterwards, so a
  // group's codes, then all their rows, are each one batch of loads in flight
  const int eb = sptr[0], ee = sptr[nn];
  const int nd = nn * DPN;
  for (int j0 = 0; j0 < m; j0 += JW) {
    const int j = j0 + jl;
    const bool jok = j < m;
    const int jc = min(j, m - 1);
    double xg[NPG][DPN];
#pragma unroll
    for (int i = 0; i < NPG; ++i)
#pragma unroll
      for (int c = 0; c < DPN; ++c) xg[i][c] = 0.0;
    if (ee > eb) {
      int e0[NPG], e1[NPG], code[NPG][UM];
#pragma unroll
      for (int i = 0; i < NPG; ++i) {
        const int b = g + NG * i;
        e0[i] = b < nn ? sptr[b] : 0;
        e1[i] = b < nn ? sptr[b + 1] : 0;
#pragma unroll
        for (int u = 0; u < UM; ++u) code[i][u] = l2m_code[e1[i] > e0[i] ? min(e0[i] + u, e1[i] - 1) : eb];
      }
      double v[NPG][UM][DPN];
#pragma unroll
      for (int i = 0; i < NPG; ++i)
#pragma unroll
        for (int u = 0; u < UM; ++u)
#pragma unroll
          for (int c = 0; c < DPN; ++c) v[i][u][c] = lam[((int64_t)(code[i][u] >> 1) * DPN + c) * ldl + jc];
#pragma unroll
      for (int i = 0; i < NPG; ++i) {
#pragma unroll
        for (int u = 0; u < UM; ++u) {
          if (jok && e0[i] + u < e1[i]) {
            const double sg = (code[i][u] & 1) ? -1.0 : 1.0;
#pragma unroll
            for (int c = 0; c < DPN; ++c) xg[i][c] += sg * v[i][u][c];
          }
        }
        // nodes with more incidences than the batch takes (none in the brick structures)
        for (int e = e0[i] + UM; e < e1[i]; ++e) {
          const int cd = l2m_code[e];
          const double sg = (cd & 1) ? -1.0 : 1.0;
          const int64_t mult = cd >> 1;
          if (jok) {
#pragma unroll
            for (int c = 0; c < DPN; ++c) xg[i][c] += sg * lam[(mult * DPN + c) * ldl + j];
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NPG; ++i) {
      const int b = g + NG * i;
      if (b < nn) {
#pragma unroll
        for (int c2 = 0; c2 < DPN; ++c2) {
          const double vv = (DPN == 3) ? O[c2] * xg[i][0] + O[3 + c2] * xg[i][1 % DPN] + O[6 + c2] * xg[i][2 % DPN]
                                       : xg[i][c2];
          tile[jl][b * DPN + c2] = vv;
        }
      }
    }
    __syncthreads();
    if (MODE == 1 && nd % 4 == 0 && ldx % 4 == 0) {
      // bf16 hi/lo: four consecutive dofs per thread, one 8-byte store per array (n0 DPN and ldx are
      // multiples of 4, so every group of four starts 8-byte aligned)
      const int nd4 = nd / 4;
      for (int e = tid; e < JW * nd4; e += 256) {
        const int jj = e / nd4, t = 4 * (e - jj * nd4);
        if (j0 + jj < m) {
          const int64_t o = ((int64_t)q * m + j0 + jj) * ldx + (int64_t)n0 * DPN + t;
          uint16_t h[4], l[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double v = tile[jj][t + r];
            h[r] = bf16_bits((float)v);
            l[r] = bf16_bits((float)(v - (double)bf16_val(h[r])));
          }
          *reinterpret_cast<uint2*>(Xh + o) = uint2{(uint32_t)h[0] | ((uint32_t)h[1] << 16),
                                                    (uint32_t)h[2] | ((uint32_t)h[3] << 16)};
          *reinterpret_cast<uint2*>(Xl + o) = uint2{(uint32_t)l[0] | ((uint32_t)l[1] << 16),
                                                    (uint32_t)l[2] | ((uint32_t)l[3] << 16)};
        }
      }
    } else {
      for (int e = tid; e < JW * nd; e += 256) {
        const int jj = e / nd, t = e - jj * nd;
        if (j0 + jj < m) {
          const double v = tile[jj][t];
          const int64_t o = ((int64_t)q * m + j0 + jj) * ldx + (int64_t)n0 * DPN + t;
          if (MODE == 2) {
            X64[o] = v;
          } else if (MODE == 0) {
            Xf[o] = (float)v;
          } else {
            const uint16_t h = bf16_bits((float)v);
            Xh[o] = h;
            Xl[o] = bf16_bits((float)(v - (double)bf16_val(h)));
          }
        }
      }
    }
    __syncthreads();
  }
}

// zero the rows [nb, ld) of every column of the bf16 hi/lo W-format blocks
__global__ void k_zero_pad(uint16_t* Xh, uint16_t* Xl, int64_t ld, int nb, int cols) {
  const int64_t pad = ld - nb;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pad * cols) return;
  const int64_t o = (i / pad) * ld + nb + (i % pad);
  Xh[o] = 0;
  Xl[o] = 0;
}

void gather_rows(rpf_problem pb, int p, const double* lam, int64_t ldl, int m, int mode, double* X64, float* Xf,
                 uint16_t* Xh, uint16_t* Xl, int64_t ldx, hipStream_t s) {
  const int nq = (int)pb->occ_of_pat[p].size(), nbn = pb->pat_nbn[p];
  if (nq == 0 || nbn == 0) return;
  dim3 grid((unsigned)cdiv(nbn, 64), (unsigned)nq);
  const int* occ = pb->d_occ_of_pat.p + pb->pat_occ_off[p];
  const double* rot = pb->has_rot ? pb->d_rot.p : nullptr;
  const bool w16 = m > 8;
#define RPF_GR(D, MD, JW)                                                                                     \
  hipLaunchKernelGGL((k_gather_rows<D, MD, JW>), grid, dim3(256), 0, s, nbn, occ, pb->d_slot_off.p,             \
                     pb->d_l2m_ptr.p, pb->d_l2m_code.p, rot, lam, ldl, m, X64, Xf, Xh, Xl, ldx)
#define RPF_GRM(D)                                          \
  if (mode == 0) { if (w16) RPF_GR(D, 0, 16); else RPF_GR(D, 0, 8); } \
  else if (mode == 1) { if (w16) RPF_GR(D, 1, 16); else RPF_GR(D, 1, 8); } \
  else { if (w16) RPF_GR(D, 2, 16); else RPF_GR(D, 2, 8); }
  switch (pb->dpn) {
    case 1: RPF_GRM(1); break;
    case 2: RPF_GRM(2); break;
    default: RPF_GRM(3);
  }
#undef RPF_GRM
#undef RPF_GR
  RPF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------- FP32 MFMA GEMM
// C (M x N, FP32, col-major ldc) = A (M x K, symmetric S+ read as k-contiguous rows, lda) * B (K x N, col-major)
// Tile 64x64, 4 waves of 32x32, BK = 16.  Like the FP64 kernel the B fragment is
// the first MFMA operand so that lanes 0..15 of an accumulator item hold 16 rows
// of one column of C.
template <int BM, int BN>
__global__ __launch_bounds__(256) void k_sgemm_sym(int M, int N, int Kfull, const float* A, int64_t lda,
                                                   const float* B, int64_t ldb, float* C, int64_t ldc, int kchunk,
                                                   int64_t slab) {
  constexpr int BK = 16, PAD = 4;
  // split-K: this workgroup covers k in [kb, K) and writes slab blockIdx.z
  const int kb = blockIdx.z * kchunk;
  const int K = min(Kfull, kb + kchunk);
  C += (int64_t)blockIdx.z * slab;
  constexpr int WTM = BM / 2, WTN = BN / 2, TM = WTM / 16, TN = WTN / 16;
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
  __shared__ float sA[BK][BM + PAD];
  __shared__ float sB[BK][BN + PAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % 2, wn = wave / 2;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  float ra[EA], rb[EB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + e * 256;
      const int kk = idx % BK, mm = idx / BK;  // A symmetric: row m is k-contiguous
      const int gm = m0 + mm, gk = k0 + kk;
      ra[e] = (gm < M && gk < K) ? A[(int64_t)gm * lda + gk] : 0.f;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + e * 256;
      const int kk = idx % BK, nn = idx / BK;
      const int gn = n0 + nn, gk = k0 + kk;
      rb[e] = (gn < N && gk < K) ? B[(int64_t)gn * ldb + gk] : 0.f;
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + e * 256;
      sA[idx % BK][idx / BK] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + e * 256;
      sB[idx % BK][idx / BK] = rb[e];
    }
  };
  if (kb < K) gload(kb);
  for (int k0 = kb; k0 < K; k0 += BK) {
    __syncthreads();
    sstore();
    __syncthreads();
    if (k0 + BK < K) gload(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      float af[TM], bf[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = sA[kk + (lane >> 4)][wm * WTM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j) bf[j] = sB[kk + (lane >> 4)][wn * WTN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[j], af[i], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * WTM + i * 16 + (lane & 15);
        const int n = n0 + wn * WTN + j * 16 + 4 * (lane >> 4) + r;
        if (m < M && n < N) C[(int64_t)n * ldc + m] = acc[i][j][r];
      }
}

// ---------------------------------------------------------------------------- bf16x3 MFMA GEMM
// Same product with both operands split into bf16 hi + lo; 16x16x32 MFMA, BK = 32.
// LDS holds rows of 32 k-values (64 bytes, padded) so a lane reads its 8
// consecutive k of one row as one 16-byte access.
// One output tile (tx, ty) of K split z; every thread of the workgroup calls it with the same
// tile (the grouped kernel below runs several tiles one after another through the same LDS: the
// barrier that opens each k stage keeps a tile's stores behind the previous tile's reads).
template <int BM, int BN, bool X3>
__device__ __forceinline__ void gemm_bf16_tile(int M, int N, int K, const uint16_t* Ah, const uint16_t* Al,
                                               int64_t lda, const uint16_t* Bh, const uint16_t* Bl, int64_t ldb,
                                               float* C, int64_t ldc, int kchunk, int64_t slab, int tx, int ty,
                                               int z) {
  constexpr int BK = 64, RS = BK + 8;  // row stride in bf16 elements (144 bytes)
  const int kbeg = z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  C += (int64_t)z * slab;
  constexpr int WTM = BM / 2, WTN = BN / 2, TM = WTM / 16, TN = WTN / 16;
  constexpr int NA = BM * BK / 8 / 256, NB = BN * BK / 8 / 256;  // 16-byte chunks per thread
  static_assert(NA >= 1 && NB >= 1, "tile too small");
  __shared__ __attribute__((aligned(16))) uint16_t sAh[BM * RS];
  __shared__ __attribute__((aligned(16))) uint16_t sAl[BM * RS];
  __shared__ __attribute__((aligned(16))) uint16_t sBh[BN * RS];
  __shared__ __attribute__((aligned(16))) uint16_t sBl[BN * RS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % 2, wn = wave / 2;
  const int m0 = tx * BM, n0 = ty * BN;
  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  uint4 rah[NA], ral[NA], rbh[NB], rbl[NB];
  // a 16-byte chunk = 8 consecutive k of one row; chunk c of the tile: row c / 8, k offset 8 (c % 8)
  auto load_chunk = [&](const uint16_t* P, int64_t ld, int row, int nrow, int k, int krem, uint4& out) {
    if (row < nrow && krem >= 8) {
      out = *reinterpret_cast<const uint4*>(P + (int64_t)row * ld + k);
    } else {
      uint16_t t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = (row < nrow && u < krem) ? P[(int64_t)row * ld + k + u] : (uint16_t)0;
      out = *reinterpret_cast<uint4*>(t);
    }
  };
  // Interior tiles (the workgroup-uniform common case) take unconditional 16-byte loads in one
  // straight-line block, so all of a stage's loads are in flight together; edge tiles go through
  // the guarded path.
  const bool rows_full = (m0 + BM <= M) && (n0 + BN <= N);
  auto gload = [&](int k0) {
    if (rows_full && k0 + BK <= kend) {
#pragma unroll
      for (int e = 0; e < NA; ++e) {
        const int c = tid + e * 256, row = c / 8, kk = 8 * (c % 8);
        const int64_t o = (int64_t)(m0 + row) * lda + k0 + kk;
        rah[e] = *reinterpret_cast<const uint4*>(Ah + o);
        if (X3) ral[e] = *reinterpret_cast<const uint4*>(Al + o);
      }
#pragma unroll
      for (int e = 0; e < NB; ++e) {
        const int c = tid + e * 256, row = c / 8, kk = 8 * (c % 8);
        const int64_t o = (int64_t)(n0 + row) * ldb + k0 + kk;
        rbh[e] = *reinterpret_cast<const uint4*>(Bh + o);
        if (X3) rbl[e] = *reinterpret_cast<const uint4*>(Bl + o);
      }
    } else {
#pragma unroll
      for (int e = 0; e < NA; ++e) {
        const int c = tid + e * 256, row = c / 8, kk = 8 * (c % 8);
        load_chunk(Ah, lda, m0 + row, M, k0 + kk, kend - (k0 + kk), rah[e]);
        if (X3) load_chunk(Al, lda, m0 + row, M, k0 + kk, kend - (k0 + kk), ral[e]);
      }
#pragma unroll
      for (int e = 0; e < NB; ++e) {
        const int c = tid + e * 256, row = c / 8, kk = 8 * (c % 8);
        load_chunk(Bh, ldb, n0 + row, N, k0 + kk, kend - (k0 + kk), rbh[e]);
        if (X3) load_chunk(Bl, ldb, n0 + row, N, k0 + kk, kend - (k0 + kk), rbl[e]);
      }
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int c = tid + e * 256, row = c / 8, kk = 8 * (c % 8);
      *reinterpret_cast<uint4*>(&sAh[row * RS + kk]) = rah[e];
      if (X3) *reinterpret_cast<uint4*>(&sAl[row * RS + kk]) = ral[e];
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int c = tid + e * 256, row = c / 8, kk = 8 * (c % 8);
      *reinterpret_cast<uint4*>(&sBh[row * RS + kk]) = rbh[e];
      if (X3) *reinterpret_cast<uint4*>(&sBl[row * RS + kk]) = rbl[e];
    }
  };
  // the 16-byte alignment of the vector loads needs lda, ldb, kchunk multiples of 8: guaranteed by the host
  if (kbeg < kend) gload(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
    sstore();
    __syncthreads();
    if (k0 + BK < kend) gload(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 32) {
      const int ko = ks + 8 * (lane >> 4);
      bf16x8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int row = wm * WTM + i * 16 + (lane & 15);
        ah[i] = *reinterpret_cast<const bf16x8*>(&sAh[row * RS + ko]);
        if (X3) al[i] = *reinterpret_cast<const bf16x8*>(&sAl[row * RS + ko]);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int row = wn * WTN + j * 16 + (lane & 15);
        bh[j] = *reinterpret_cast<const bf16x8*>(&sBh[row * RS + ko]);
        if (X3) bl[j] = *reinterpret_cast<const bf16x8*>(&sBl[row * RS + ko]);
      }
      // the three products of one accumulator are issued TM*TN MFMAs apart (independent chains)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], ah[i], acc[i][j], 0, 0, 0);
      if (X3) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl[j], ah[i], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], al[i], acc[i][j], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * WTM + i * 16 + (lane & 15);
        const int n = n0 + wn * WTN + j * 16 + 4 * (lane >> 4) + r;
        if (m < M && n < N) C[(int64_t)n * ldc + m] = acc[i][j][r];
      }
}

template <int BM, int BN, bool X3>
__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const uint16_t* Ah, const uint16_t* Al,
                                                   int64_t lda, const uint16_t* Bh, const uint16_t* Bl, int64_t ldb,
                                                   float* C, int64_t ldc, int kchunk, int64_t slab) {
  int tx, ty;
  xcd_tile(gridDim.x, gridDim.y, tx, ty);
  gemm_bf16_tile<BM, BN, X3>(M, N, K, Ah, Al, lda, Bh, Bl, ldb, C, ldc, kchunk, slab, tx, ty, blockIdx.z);
}

// Every pattern's product in one persistent launch: the workgroups walk the group's tile list
// (pattern by pattern in the order the host gave, split by split, then column tile by column
// tile), tile t, t + gridDim.x, ..., so a launch sized to the resident workgroups covers patterns
// of any size without a tail launch per pattern.
template <int BM, int BN, bool X3>
__global__ __launch_bounds__(256) void k_gemm_bf16_group(const BfGroup g) {
  for (int t = blockIdx.x; t < g.start[g.n]; t += gridDim.x) {
    int p = 0;
    while (t >= g.start[p + 1]) ++p;
    const int l = t - g.start[p];
    const int per_z = g.tm[p] * g.tn[p];
    const int z = l / per_z, r = l - z * per_z;
    gemm_bf16_tile<BM, BN, X3>(g.M[p], g.N[p], g.K[p], g.Ah[p], g.Al[p], g.lda[p], g.Bh[p], g.Bl[p], g.ldb[p],
                               g.C[p], g.ldc[p], g.kchunk[p], g.slab[p], r % g.tm[p], r / g.tm[p], z);
  }
}

// ---------------------------------------------------------------------------- bf16 MFMA GEMM, 256 x 256 tiles
// The large-problem form of the product above (same operands, same per-accumulator summation
// order, so the same bits), with a row-major result (see the scatter): 512 threads, eight waves of 128 x 64, k stages of 32 fed by direct
// global-to-LDS 16-byte loads into two LDS buffers (64 KiB per stage for hi + lo of both
// operands).  A stage's loads are issued right after the barrier that opens the previous stage,
// so a whole stage of MFMA work covers their latency, and no staging registers are needed.
// The two buffers are distinct LDS objects so the compiler can tell that the fragment reads of
// one stage do not depend on the loads in flight into the other.  Requirements (host-checked):
// lda, ldb, kchunk and K multiples of 32 with zeros in the padded k range, so every stage is
// whole; rows past M (or N) are clamped to the last row and their results are never stored.
// LDS layout of one operand stage: 16 blocks of 16 rows x 64 bytes; the four 16-byte k chunks of
// row r sit in the order kc ^ swz4(r), which makes the fragment reads (16 rows x one chunk per
// quarter wave) free of bank conflicts.
__device__ inline int swz4(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }

template <bool X3>
__global__ __launch_bounds__(512) void k_gemm_bf16_big(int M, int N, int K, const uint16_t* __restrict__ Ah,
                                                       const uint16_t* __restrict__ Al, int64_t lda,
                                                       const uint16_t* __restrict__ Bh,
                                                       const uint16_t* __restrict__ Bl, int64_t ldb,
                                                       float* __restrict__ C, int64_t ldc, int kchunk,
                                                       int64_t slab) {
  constexpr int BK = 32, NARR = X3 ? 4 : 2, AB = 256 * 64;  // bytes of one operand stage
  constexpr int WPA = 8 / NARR, EPW = 16 / WPA;            // waves per operand, 1 KiB blocks per wave
  __shared__ __attribute__((aligned(1024))) uint8_t lds0[NARR * AB];
  __shared__ __attribute__((aligned(1024))) uint8_t lds1[NARR * AB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  int tx, ty;
  xcd_tile<4>(gridDim.x, gridDim.y, tx, ty);  // column groups of 4: measured ~1.5 % faster than 8
  const int m0 = tx * 256, n0 = ty * 256;
  const int kbeg = blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
  C += (int64_t)blockIdx.z * slab;
  const int nst = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  // this wave loads operand la (Ah, Al, Bh, Bl; or Ah, Bh), 16-row blocks lb0 .. lb0 + EPW - 1;
  // lane l of a block load fetches row l / 4, chunk (l % 4) ^ swz4(row)
  const int la = wave / WPA, lb0 = (wave % WPA) * EPW;
  const bool isA = la < NARR / 2;
  const uint16_t* P = X3 ? (la == 0 ? Ah : la == 1 ? Al : la == 2 ? Bh : Bl) : (la == 0 ? Ah : Bh);
  const int64_t ld = isA ? lda : ldb;
  const int base = isA ? m0 : n0, lim = isA ? M : N;
  const int lr = lane >> 2, lkc = (lane & 3) ^ swz4(lr);
  const uint16_t* src[EPW];
#pragma unroll
  for (int e = 0; e < EPW; ++e) {
    const int row = min(base + (lb0 + e) * 16 + lr, lim - 1);
    src[e] = P + (int64_t)row * ld + kbeg + 8 * lkc;
  }
  auto issue = [&](uint8_t* buf, int k) {
#pragma unroll
    for (int e = 0; e < EPW; ++e)
      __builtin_amdgcn_global_load_lds((const void*)(src[e] + k), (void*)(buf + la * AB + (lb0 + e) * 1024), 16, 0, 0);
  };
  const int fr = lane & 15, foff = fr * 64 + (((lane >> 4) ^ swz4(fr)) * 16);
  auto frag = [&](const uint8_t* buf, int a, int row0) -> bf16x8 {
    return *reinterpret_cast<const bf16x8*>(buf + a * AB + row0 * 64 + foff);
  };
  constexpr int IAH = 0, IAL = 1, IBH = X3 ? 2 : 1, IBL = 3;
  f32x4 acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // one stage: wait for this stage's loads, barrier (all waves are also done with the other
  // buffer), start the next stage's loads into the other buffer, then read fragments and multiply
  auto stage = [&](const uint8_t* cur, uint8_t* nxt, int s) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (s + 1 < nst) issue(nxt, (s + 1) * BK);
    __builtin_amdgcn_sched_barrier(0);
    bf16x8 bh[4], bl[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bh[j] = frag(cur, IBH, wn * 64 + j * 16);
      if (X3) bl[j] = frag(cur, IBL, wn * 64 + j * 16);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      bf16x8 ah[4], al[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ah[i] = frag(cur, IAH, wm * 128 + (h * 4 + i) * 16);
        if (X3) al[i] = frag(cur, IAL, wm * 128 + (h * 4 + i) * 16);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[h * 4 + i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], ah[i], acc[h * 4 + i][j], 0, 0, 0);
      if (X3) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[h * 4 + i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl[j], ah[i], acc[h * 4 + i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[h * 4 + i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], al[i], acc[h * 4 + i][j], 0, 0, 0);
      }
    }
  };
  if (nst > 0) issue(lds0, 0);
  int s = 0;
  for (; s + 1 < nst; s += 2) {
    stage(lds0, lds1, s);
    stage(lds1, lds0, s + 1);
  }
  if (s < nst) stage(lds0, lds1, s);
  // row-major result (C[m * ldc + n], ldc a multiple of 4): a lane holds four consecutive n of one
  // row m, written as one 16-byte store
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = m0 + wm * 128 + i * 16 + (lane & 15);
      const int n = n0 + wn * 64 + j * 16 + 4 * (lane >> 4);
      if (m >= M) continue;
      float* row = C + (int64_t)m * ldc;
      if (n + 3 < N) {
        *reinterpret_cast<f32x4*>(row + n) = acc[i][j];
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (n + r < N) row[n + r] = acc[i][j][r];
      }
    }
}

// ---------------------------------------------------------------------------- scatter from FP32
// Local results of the low-precision product, per pattern: column-major (row r of column q m + j
// at base[(q m + j) ld + r], nsplit slabs of partial sums slab apart) or, from the 256 x 256
// kernel, row-major (base[r ld + q m + j], one slab), where the m columns of an occurrence are
// contiguous for the scatter.
struct YLoc32 {
  const float* base[MAXP];
  int64_t ld[MAXP];
  int64_t slab[MAXP];
  int nsplit[MAXP];
  int rowmajor[MAXP];
};

// JB columns per pass (8: the whole pass stays in registers)
template <int DPN, int JB>
__global__ __launch_bounds__(128) void k_scatter_f32(int n_mult, const int* ep_q, const int* ep_bn,
                                                     const int8_t* ep_pat, const int8_t* ep_sign, const int* ep_occ,
                                                     const double* rot, YLoc32 yl, int m, double* Y, int64_t ldy) {
  const int mult = blockIdx.x * blockDim.x + threadIdx.x;
  if (mult >= n_mult) return;
  for (int j0 = 0; j0 < m; j0 += JB) {
    const int jn = min(JB, m - j0);
    double acc[DPN][JB];
#pragma unroll
    for (int c = 0; c < DPN; ++c)
#pragma unroll
      for (int j = 0; j < JB; ++j) acc[c][j] = 0.0;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int q = ep_q[2 * mult + e];
      if (q < 0) continue;
      const int p = ep_pat[2 * mult + e];
      const double sg = (double)ep_sign[2 * mult + e];
      const int64_t ld = yl.ld[p];
      const bool rm = yl.rowmajor[p] != 0;
      const int64_t bn = ep_bn[2 * mult + e];
      const float* base = rm ? yl.base[p] + bn * DPN * ld + (int64_t)q * m + j0
                             : yl.base[p] + ((int64_t)q * m + j0) * ld + bn * DPN;
      // element (c, j) of this endpoint: base[c sc + j sj]
      const int64_t sc = rm ? ld : 1, sj = rm ? 1 : ld;
      double O[9];
      const int s = ep_occ[2 * mult + e];
#pragma unroll
      for (int i = 0; i < 9; ++i) O[i] = rot ? rot[9 * s + i] : ((i % 4 == 0) ? 1.0 : 0.0);
      // row-major with whole, 16-byte aligned groups: JB / 4 vector loads per dof
      float yv[DPN][JB];
      if (rm && jn == JB && (m & 3) == 0) {
#pragma unroll
        for (int c = 0; c < DPN; ++c)
#pragma unroll
          for (int v4 = 0; v4 < JB / 4; ++v4) {
            const f32x4 t = *reinterpret_cast<const f32x4*>(base + c * ld + 4 * v4);
#pragma unroll
            for (int u = 0; u < 4; ++u) yv[c][4 * v4 + u] = t[u];
          }
      } else {
#pragma unroll
        for (int c = 0; c < DPN; ++c)
#pragma unroll
          for (int j = 0; j < JB; ++j) yv[c][j] = j < jn ? base[c * sc + j * sj] : 0.f;
      }
#pragma unroll
      for (int j = 0; j < JB; ++j) {
        if (j >= jn) break;
        double v[DPN];
#pragma unroll
        for (int c = 0; c < DPN; ++c) v[c] = (double)yv[c][j];
        for (int z = 1; z < yl.nsplit[p]; ++z)
#pragma unroll
          for (int c = 0; c < DPN; ++c) v[c] += (double)base[z * yl.slab[p] + c * sc + j * sj];
        if (DPN == 3) {
#pragma unroll
          for (int c = 0; c < 3; ++c)
            acc[c % DPN][j] += sg * (O[3 * c] * v[0] + O[3 * c + 1] * v[1 % DPN] + O[3 * c + 2] * v[2 % DPN]);
        } else {
#pragma unroll
          for (int c = 0; c < DPN; ++c) acc[c][j] += sg * v[c];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < DPN; ++c) {
      double* row = Y + ((int64_t)mult * DPN + c) * ldy + j0;
#pragma unroll
      for (int j = 0; j < JB; ++j)
        if (j < jn) row[j] = acc[c][j];
    }
  }
}

// Scatter from the row-major result of the 256 x 256 kernel with one thread per (multiplier, 4
// consecutive columns): per endpoint one 16-byte load per dof row, the output rows leave as
// 16-byte stores, and four threads share a multiplier's index loads (m a multiple of 4).
template <int DPN>
__global__ __launch_bounds__(256) void k_scatter_f32_quad(int n_mult, const int* ep_q, const int* ep_bn,
                                                          const int8_t* ep_pat, const int8_t* ep_sign,
                                                          const int* ep_occ, const double* rot, YLoc32 yl, int m,
                                                          double* Y, int64_t ldy) {
  const int mq = m >> 2;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n_mult * mq) return;
  const int mult = (int)(idx / mq), j0 = (int)(idx % mq) * 4;
  int q[2], bn[2], pt[2], so[2];
  double sg[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    q[e] = ep_q[2 * mult + e];
    bn[e] = ep_bn[2 * mult + e];
    pt[e] = ep_pat[2 * mult + e];
    sg[e] = (double)ep_sign[2 * mult + e];
    so[e] = ep_occ[2 * mult + e];
  }
  f32x4 yv[2][DPN];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const bool ok = q[e] >= 0;
    const int p = ok ? pt[e] : 0;
    const float* base = yl.base[p] + (int64_t)(ok ? bn[e] : 0) * DPN * yl.ld[p] + (int64_t)(ok ? q[e] : 0) * m + j0;
#pragma unroll
    for (int c = 0; c < DPN; ++c)
      yv[e][c] = ok ? *reinterpret_cast<const f32x4*>(base + c * yl.ld[p]) : f32x4{0.f, 0.f, 0.f, 0.f};
  }
  double acc[DPN][4];
#pragma unroll
  for (int c = 0; c < DPN; ++c)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[c][u] = 0.0;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    if (q[e] < 0) continue;
    double O[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) O[i] = rot ? rot[9 * so[e] + i] : ((i % 4 == 0) ? 1.0 : 0.0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (DPN == 3) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
          acc[c % DPN][u] += sg[e] * (O[3 * c] * (double)yv[e][0][u] + O[3 * c + 1] * (double)yv[e][1 % DPN][u] +
                                      O[3 * c + 2] * (double)yv[e][2 % DPN][u]);
      } else {
#pragma unroll
        for (int c = 0; c < DPN; ++c) acc[c][u] += sg[e] * (double)yv[e][c][u];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < DPN; ++c) {
    double* row = Y + ((int64_t)mult * DPN + c) * ldy + j0;
    *reinterpret_cast<double2*>(row) = double2{acc[c][0], acc[c][1]};
    *reinterpret_cast<double2*>(row + 2) = double2{acc[c][2], acc[c][3]};
  }
}

// ---------------------------------------------------------------------------- grouped launch
template <typename Kern>
static int resident_blocks_lp(Kern k, int threads) {
  int per_cu = 0, dev = 0;
  RPF_HIP(hipGetDevice(&dev));
  RPF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads, 0));
  hipDeviceProp_t prop;
  RPF_HIP(hipGetDeviceProperties(&prop, dev));
  return std::max(1, per_cu) * std::max(1, prop.multiProcessorCount);
}

void gemm_bf16_group(hipStream_t s, int tile, bool x3, const BfGroup& g) {
  const int total = g.start[g.n];
  if (total == 0) return;
#define RPF_GRP(T, X)                                                                                   \
  {                                                                                                     \
    static const int cap = resident_blocks_lp(k_gemm_bf16_group<T, T, X>, 256);                         \
    RPF_TIMED_LAUNCH((k_gemm_bf16_group<T, T, X>), dim3((unsigned)std::min(total, cap)), dim3(256), 0, s, g); \
  }
  RPF_CHECK(tile == 64 || tile == 128, RPF_EINVAL, "gemm_bf16_group: tile must be 64 or 128");
  if (tile == 128) {
    if (x3) RPF_GRP(128, true) else RPF_GRP(128, false)
  } else {
    if (x3) RPF_GRP(64, true) else RPF_GRP(64, false)
  }
#undef RPF_GRP
  RPF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------- host
// W format from an FP64 column-major block (rows x cols, ld ldxin): mode 1 bf16 hi/lo, 0 FP32
__global__ void k_to_w(int rows, int64_t cols, const double* X, int64_t ldxin, int mode, float* Xf, uint16_t* Xh,
                       uint16_t* Xl, int64_t ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows * cols) return;
  const int64_t r = i % rows, c = i / rows;
  const double v = X[c * ldxin + r];
  const int64_t o = c * ld + r;
  if (mode == 1) {
    const uint16_t h = bf16_bits((float)v);
    Xh[o] = h;
    Xl[o] = bf16_bits((float)(v - (double)bf16_val(h)));
  } else {
    Xf[o] = (float)v;
  }
}

void apply_F_lowprec(rpf_problem pb, const rpf_pattern* pats, int m, const double* X, int64_t ldx, double* Y,
                     int64_t ldy, int prec, hipStream_t s, int op, const double* const* gsub) {
  const bool split = (prec == RPF_BF16X3 || prec == RPF_BF16);
  // W format with ld rounded up to a multiple of 64: every 64-k chunk of a row is one 128-byte
  // cache line (unaligned rows would make each chunk touch two lines)
  std::vector<int64_t> off(pb->n_pat + 1, 0), ld(pb->n_pat);
  // split K (chunks of multiples of 64) while the 64 x 64 output tiles alone give fewer than
  // ~4 workgroups per CU; the scatter sums the split slabs
  std::vector<int64_t> yoff(pb->n_pat + 1, 0), ldr(pb->n_pat, 0);
  std::vector<int> nsp(pb->n_pat, 1), kch(pb->n_pat, 0), tile_m(pb->n_pat, 64), tile_n(pb->n_pat, 64);
  // a grouped schedule (bf16 forms only) runs every pattern's product in one persistent launch of
  // its tile, each pattern's K split set by the schedule's work target
  const Schedule sc = schedule_for(pb, m, prec);
  const int gtile = (split && (sc.tile == 64 || sc.tile == 128)) ? sc.tile : 0;
  for (int p = 0; p < pb->n_pat; ++p) {
    const int nb = pats[p]->n_b;
    ld[p] = cdiv(nb, 64) * 64;
    const int64_t cols = (int64_t)pb->occ_of_pat[p].size() * m;
    off[p + 1] = off[p] + ld[p] * cols;
    // bf16 workgroup tile: 256 x 256 when those tiles alone fill the chip (about one per CU), else
    // 128 x 128 (64 x 64 per wave) when both sides allow it, else 64 x 64
    int tm = (split && cdiv(nb, 256) * cdiv(cols, (int64_t)256) >= 240) ? 256
             : (split && nb >= 128 && cols >= 128)                       ? 128
                                                                         : 64;
    if (gtile) tm = gtile;
    else if (split && sc.tile == 256) tm = 256;
    if (tm == 256 && pb->weighted) tm = 128;  // the non-Boolean scatter reads column-major results
    const int tn = tm;
    tile_m[p] = tm;
    tile_n[p] = tn;
    const int64_t tiles = std::max<int64_t>(1, cdiv(nb, tm) * cdiv(cols, tn));
    int sp = (int)std::min<int64_t>(std::max<int64_t>(1, 1024 / tiles), std::max<int64_t>(1, ld[p] / 256));
    sp = tm == 256 ? 1 : std::min(sp, 8);
    kch[p] = (int)(cdiv(cdiv(ld[p], sp), 64) * 64);
    if (gtile) kch[p] = (int)group_kchunk(nb, ld[p], cols, gtile, sc.work, 64);
    nsp[p] = (int)cdiv(ld[p], kch[p]);
    // the 256 x 256 kernel's row-major result: n_b rows of ldr[p] (a multiple of 16 floats)
    ldr[p] = cdiv(cols, (int64_t)16) * 16;
    yoff[p + 1] = yoff[p] + (tm == 256 ? (int64_t)nb * ldr[p] : ld[p] * cols * nsp[p]);
  }
  const int64_t tot = std::max<int64_t>(off[pb->n_pat], 8);
  pb->yloc32.ensure(std::max<int64_t>(yoff[pb->n_pat], 8));
  if (split) {
    pb->xhi.ensure(tot);
    pb->xlo.ensure(tot);
  } else {
    pb->xloc32.ensure(tot);
  }
  YLoc32 yl{};
  BfGroup grp{};
  double gflops = 0.0;
  for (int p = 0; p < pb->n_pat; ++p) {
    const rpf_pattern P = pats[p];
    const int nb = P->n_b, nq = (int)pb->occ_of_pat[p].size(), nbn = pb->pat_nbn[p];
    const int cols = nq * m;
    const int* occ = pb->d_occ_of_pat.p + pb->pat_occ_off[p];
    const double* rot = pb->has_rot ? pb->d_rot.p : nullptr;
    float* yp = pb->yloc32.p + yoff[p];
    const int64_t slab = ld[p] * (int64_t)cols;
    const bool rowmajor = tile_m[p] == 256;
    yl.base[p] = yp;
    yl.ld[p] = rowmajor ? ldr[p] : ld[p];
    yl.slab[p] = slab;
    yl.nsplit[p] = nsp[p];
    yl.rowmajor[p] = rowmajor ? 1 : 0;
    if (nq == 0) continue;
    dim3 grid((unsigned)cdiv(nbn, 128), (unsigned)nq);
#define RPF_GLP(D, MODE)                                                                                        \
  hipLaunchKernelGGL((k_gather_lp<D, MODE>), grid, dim3(128), 0, s, nbn, occ, pb->d_slot_off.p, pb->d_l2m_ptr.p, \
                     pb->d_l2m_code.p, rot, X, ldx, m, pb->xloc32.p + off[p], pb->xhi.p + off[p],                 \
                     pb->xlo.p + off[p], ld[p])
    // the padded rows between n_b and ld must hold zeros for the 16-byte loads
    if (split && ld[p] != nb) {
      const int64_t npad = (ld[p] - nb) * (int64_t)cols;
      hipLaunchKernelGGL(k_zero_pad, dim3((unsigned)cdiv(npad, 256)), dim3(256), 0, s, pb->xhi.p + off[p],
                         pb->xlo.p + off[p], ld[p], nb, cols);
    }
    if (gsub) {
      // g - A^T X: gathered in FP64 (any assembly and block width), the difference taken there and
      // rounded once into the W format, as a gathered column is
      pb->xloc.ensure((size_t)nb * cols);
      gather_pattern(pb, p, nbn, X, ldx, m, pb->xloc.p, nb, s);
      rsub_cols(s, nb, cols, gsub[p], nb, pb->xloc.p, nb);
      hipLaunchKernelGGL(k_to_w, dim3((unsigned)cdiv((int64_t)nb * cols, 256)), dim3(256), 0, s, nb, (int64_t)cols,
                         pb->xloc.p, (int64_t)nb, split ? 1 : 0, split ? nullptr : pb->xloc32.p + off[p],
                         split ? pb->xhi.p + off[p] : nullptr, split ? pb->xlo.p + off[p] : nullptr, ld[p]);
    } else if (split) {
      if (pb->weighted) {
        wgather(pb, p, X, ldx, m, 1, nullptr, nullptr, pb->xhi.p + off[p], pb->xlo.p + off[p], ld[p], s);
      } else if (m >= 8) {
        gather_rows(pb, p, X, ldx, m, 1, nullptr, nullptr, pb->xhi.p + off[p], pb->xlo.p + off[p], ld[p], s);
      } else {
        switch (pb->dpn) {
          case 1: RPF_GLP(1, 1); break;
          case 2: RPF_GLP(2, 1); break;
          default: RPF_GLP(3, 1);
        }
      }
    } else if (pb->weighted) {
      wgather(pb, p, X, ldx, m, 0, nullptr, pb->xloc32.p + off[p], nullptr, nullptr, ld[p], s);
    } else if (m >= 8) {
      gather_rows(pb, p, X, ldx, m, 0, nullptr, pb->xloc32.p + off[p], nullptr, nullptr, ld[p], s);
    } else {
      switch (pb->dpn) {
        case 1: RPF_GLP(1, 0); break;
        case 2: RPF_GLP(2, 0); break;
        default: RPF_GLP(3, 0);
      }
    }
#undef RPF_GLP
    RPF_LAUNCH_CHECK();
    const uint16_t* Ah = op == OP_FLEX ? P->Sp_hi.p : P->S_hi.p;
    const uint16_t* Al = op == OP_FLEX ? P->Sp_lo.p : P->S_lo.p;
    const float* A32 = op == OP_FLEX ? P->Splus32.p : P->S32.p;
    if (gtile) {
      // queued for the one grouped launch after the loop
      RPF_CHECK(P->ldlp == ld[p], RPF_EINVAL, "low-precision S+ layout mismatch");
      RPF_CHECK(Ah != nullptr && Al != nullptr, RPF_EINVAL, "low-precision copy of the pattern matrix missing");
      const int q = grp.n++;
      grp.M[q] = nb;
      grp.N[q] = cols;
      grp.K[q] = (int)ld[p];
      grp.kchunk[q] = kch[p];
      grp.tm[q] = (int)cdiv(nb, gtile);
      grp.tn[q] = (int)cdiv(cols, gtile);
      grp.Ah[q] = Ah;
      grp.Al[q] = Al;
      grp.lda[q] = ld[p];
      grp.Bh[q] = pb->xhi.p + off[p];
      grp.Bl[q] = pb->xlo.p + off[p];
      grp.ldb[q] = ld[p];
      grp.C[q] = yp;
      grp.ldc[q] = ld[p];
      grp.slab[q] = slab;
      grp.start[q + 1] = grp.start[q] + grp.tm[q] * grp.tn[q] * nsp[p];
      gflops += 2.0 * nb * (double)nb * (double)cols;
      continue;
    }
    // the tracer times the flexibility products only
    void* tok = op == OP_FLEX ? trace_begin(s, (int)prec) : nullptr;
    if (split) {
      RPF_CHECK(P->ldlp == ld[p], RPF_EINVAL, "low-precision S+ layout mismatch");
      RPF_CHECK(Ah != nullptr && Al != nullptr, RPF_EINVAL, "low-precision copy of the pattern matrix missing");
      const int tm = tile_m[p], tn = tile_n[p];
      dim3 g2((unsigned)cdiv(nb, tm), (unsigned)cdiv(cols, tn), (unsigned)nsp[p]);
#define RPF_BF(BM_, BN_, X3)                                                                                      \
  RPF_TIMED_LAUNCH((k_gemm_bf16<BM_, BN_, X3>), g2, dim3(256), 0, s, nb, cols, (int)ld[p], Ah, Al,               \
                     ld[p], pb->xhi.p + off[p], pb->xlo.p + off[p], ld[p], yp, ld[p], kch[p], slab)
#define RPF_BIG(X3)                                                                                            \
  RPF_TIMED_LAUNCH((k_gemm_bf16_big<X3>), g2, dim3(512), 0, s, nb, cols, (int)ld[p], Ah, Al,                  \
                     ld[p], pb->xhi.p + off[p], pb->xlo.p + off[p], ld[p], yp, ldr[p], kch[p], slab)
      if (tm == 256) {
        RPF_CHECK(ld[p] % 32 == 0 && kch[p] % 32 == 0, RPF_EINVAL, "bf16 operand layout not in 32-k stages");
        if (prec == RPF_BF16X3) RPF_BIG(true);
        else RPF_BIG(false);
      } else if (prec == RPF_BF16X3) {
        if (tm == 128) RPF_BF(128, 128, true);
        else RPF_BF(64, 64, true);
      } else {
        if (tm == 128) RPF_BF(128, 128, false);
        else RPF_BF(64, 64, false);
      }
#undef RPF_BIG
#undef RPF_BF
    } else {
      dim3 g2((unsigned)cdiv(nb, 64), (unsigned)cdiv(cols, 64), (unsigned)nsp[p]);
      RPF_CHECK(A32 != nullptr, RPF_EINVAL, "FP32 copy of the pattern matrix missing");
      RPF_TIMED_LAUNCH((k_sgemm_sym<64, 64>), g2, dim3(256), 0, s, nb, cols, nb, A32, (int64_t)nb,
                         pb->xloc32.p + off[p], ld[p], yp, ld[p], kch[p], slab);
    }
    RPF_LAUNCH_CHECK();
    if (tok) trace_end(tok, s, 2.0 * nb * (double)nb * (double)cols);
  }
  if (grp.n > 0) {
    void* tok = op == OP_FLEX ? trace_begin(s, (int)prec) : nullptr;
    gemm_bf16_group(s, gtile, prec == RPF_BF16X3, grp);
    if (tok) trace_end(tok, s, gflops);
  }
  if (pb->n_mult == 0) return;
  if (pb->weighted) {
    WLoc<float> w{};
    for (int p = 0; p < pb->n_pat; ++p) {
      RPF_CHECK(!yl.rowmajor[p] || pb->occ_of_pat[p].empty(), RPF_EINVAL, "non-Boolean scatter: row-major result");
      w.base[p] = yl.base[p];
      w.ld[p] = yl.ld[p];
      w.slab[p] = yl.slab[p];
      w.nsplit[p] = yl.nsplit[p];
    }
    wscatter(pb, w, m, Y, ldy, s);
    return;
  }
  dim3 grid((unsigned)cdiv(pb->n_mult, 128));
  const double* rot = pb->has_rot ? pb->d_rot.p : nullptr;
  bool all_rm = true;
  for (int p = 0; p < pb->n_pat; ++p) all_rm &= yl.rowmajor[p] != 0 || pb->occ_of_pat[p].empty();
  if (all_rm && m % 4 == 0 && ldy % 2 == 0 && ((uintptr_t)Y & 15) == 0) {
    dim3 gq((unsigned)cdiv((int64_t)pb->n_mult * (m / 4), 256));
#define RPF_SQ(D)                                                                                                \
  hipLaunchKernelGGL(k_scatter_f32_quad<D>, gq, dim3(256), 0, s, pb->n_mult, pb->d_ep_q.p, pb->d_ep_bn.p,       \
                     pb->d_ep_pat.p, pb->d_ep_sign.p, pb->d_ep_occ.p, rot, yl, m, Y, ldy)
    switch (pb->dpn) {
      case 1: RPF_SQ(1); break;
      case 2: RPF_SQ(2); break;
      default: RPF_SQ(3);
    }
#undef RPF_SQ
    RPF_LAUNCH_CHECK();
    return;
  }
#define RPF_SF(D, JB)                                                                                          \
  hipLaunchKernelGGL((k_scatter_f32<D, JB>), grid, dim3(128), 0, s, pb->n_mult, pb->d_ep_q.p, pb->d_ep_bn.p,    \
                     pb->d_ep_pat.p, pb->d_ep_sign.p, pb->d_ep_occ.p, rot, yl, m, Y, ldy)
  switch (pb->dpn) {
    case 1: RPF_SF(1, 8); break;
    case 2: RPF_SF(2, 8); break;
    default: RPF_SF(3, 8);
  }
#undef RPF_SF
  RPF_LAUNCH_CHECK();
}

}  // namespace rpf
