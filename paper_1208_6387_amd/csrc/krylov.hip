// Interface solver: projected multivector conjugate gradient (Table 1 of the
// paper), with the multivector built by permuting the interface partitions of
// the residual (section 3.1), full re-orthogonalisation and F-normalisation
// W <- W eta^{-1/2}, P <- P eta^{-1/2} with eta = P^T W (section 3.3), and a
// pseudo-inverse (dropped eigen-directions) when eta is singular (section
// 4.3).  Then the displacement recovery of eq. 2.
//
// Mixed forms: the inner solves use a low-precision flexibility product and
// are wrapped in FP64 iterative refinement of the interface residual
// r = Q^T (d - F lambda); the Gram matrices, eta^{-1/2}, the coarse problem and
// every update stay in FP64.
#include "problem.hpp"

#include <algorithm>
#include <chrono>
#include <map>
#include <cmath>

namespace rpf {
namespace {

// A direction of a new block is dropped when its F-energy after the orthogonalisation is below
// eta_drop(prec) times the block's energy before it (section 3.3: rank deficiency of eta).  The
// ratio is limited by the accuracy of the product: noise of relative size eps leaves an energy
// fraction of about eps^2, so the low-precision forms use larger thresholds.
constexpr double ETA_DROP = 1e-12;
inline double eta_drop(int prec) {
  switch (prec) {
    case RPF_FP32: return 1e-10;
    case RPF_BF16X3: return 1e-8;
    case RPF_BF16: return 1e-3;
    default: return ETA_DROP;
  }
}

// ---------------------------------------------------------------------------- kernels
// Zb[l*m + r*np + k] = z[src*nr + r], src = perm[k][mult]*dpn + c  (section 3.1 multivector)
// One thread per output entry (consecutive threads write consecutive entries of a row).
// With rotated occurrences (dpn 3) the value moved from multiplier src to mult is
// carried into the frame of its new place: O_t O_s^T z[src], O_t / O_s the rotations
// of the first-endpoint occurrences of mult / src (section 4.2).
__global__ void k_permute(int64_t n_lambda, int dpn, int n_mult, int nr, int np, const int* perm, const int* ep_occ,
                          const double* rot, const double* z, int64_t ldz, double* Zb, int64_t ldb) {
  const int m = nr * np;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_lambda * m) return;
  const int64_t l = idx / m;
  const int col = (int)(idx % m), r = col / np, k = col % np;
  const int64_t mult = l / dpn, c = l % dpn;
  const int64_t sm = perm ? (int64_t)perm[(int64_t)k * n_mult + mult] : mult;
  if (rot && dpn == 3 && sm != mult) {
    const double* Ot = rot + 9 * (int64_t)ep_occ[2 * mult];
    const double* Os = rot + 9 * (int64_t)ep_occ[2 * sm];
    double v = 0.0;
    for (int c2 = 0; c2 < 3; ++c2) {
      const double Rcc = Ot[3 * c] * Os[3 * c2] + Ot[3 * c + 1] * Os[3 * c2 + 1] + Ot[3 * c + 2] * Os[3 * c2 + 2];
      v += Rcc * z[(sm * 3 + c2) * ldz + r];
    }
    Zb[l * ldb + col] = v;
  } else {
    Zb[l * ldb + col] = z[(sm * dpn + c) * ldz + r];
  }
}

// Normalisation of a new block (section 3.3): T with T^T eta T = I on the kept directions.
// The energy of column c before the orthogonalisation is |B_c|^2 + eta_cc (B = P_stored^T Z,
// ka x m, ld ka; F-orthonormal stored blocks).  Diagonal form (classical CG per load case):
// T = diag(eta_cc^{-1/2}) keeping eta_cc > tau * energy_c.  Block form: the eigen rule keeps w_i >
// tau * max(w_max, max_c energy_c); when a Cholesky factor eta = L L^T exists with
// 1 / |L^{-1}|_F^2 (a lower bound of w_min) above tau * max(trace eta, max_c energy_c) (an upper
// bound of that reference), no eigenpair would be dropped and T = L^{-T} spans the same
// directions, so it is used and state[0] = 1; otherwise state[0] = 0, state[1] = max_c energy_c
// and the eigen form (eta_eigen_T) decides.  When nothing is kept, 1 goes to flag0 and flag1.
// One wavefront; MM >= m is the unrolled register length.
template <int MM>
__global__ __launch_bounds__(64) void k_eta_chol(int m, const double* eta, int diag_only, int ka, const double* B,
                                                 double tau, double* T, int* drops, double* flag0, double* flag1,
                                                 double* state) {
  __shared__ double epre[64];
  __shared__ double Ls[MM][MM + 1];
  __shared__ double es[MM * MM];
  __shared__ double rdiag[MM];
  __shared__ double emax_s, trace_s;
  __shared__ int bad_s;
  const int t = threadIdx.x;
  // eta staged in LDS, and B read, by loads at clamped (always valid) addresses whose values are
  // masked afterwards: no load sits behind a branch, so each group is issued together and waited
  // for once instead of one global-memory round trip at a time
  {
    constexpr int EU = (MM * MM + 63) / 64;
    double ev[EU];
    const int mm = m * m;
#pragma unroll
    for (int u = 0; u < EU; ++u) ev[u] = eta[min(t + 64 * u, mm - 1)];
#pragma unroll
    for (int u = 0; u < EU; ++u)
      if (t + 64 * u < MM * MM) es[t + 64 * u] = (t + 64 * u < mm) ? ev[u] : 0.0;
  }
  __syncthreads();
  {
    // squared column norms of B: every column's loads of a 64-row chunk are issued together
    double part[MM];
#pragma unroll
    for (int c = 0; c < MM; ++c) part[c] = 0.0;
    for (int i0 = 0; i0 < ka; i0 += 64) {
      const int i = i0 + t;
      const int ic = min(i, ka - 1);
      double bv[MM];
#pragma unroll
      for (int c = 0; c < MM; ++c) bv[c] = B[(int64_t)min(c, m - 1) * ka + ic];
#pragma unroll
      for (int c = 0; c < MM; ++c) {
        const double b = (c < m && i < ka) ? bv[c] : 0.0;
        part[c] += b * b;
      }
    }
    // lane t holds eta_tt; every reduction below is a butterfly across the wave (no serial loops
    // of dependent loads on one lane)
    const double dg = t < m ? es[t * m + t] : 0.0;
    // all MM butterflies in straight-line code (columns past m are zeros), so they interleave
    double mine = 0.0;
#pragma unroll
    for (int c = 0; c < MM; ++c) {
      double acc = part[c];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
      acc += __shfl(dg, c, 64);
      if (t == c) mine = acc;
    }
    if (t < m) epre[t] = mine;
    double me = mine, tr = fmax(dg, 0.0);
    for (int off = 32; off > 0; off >>= 1) {
      me = fmax(me, __shfl_xor(me, off, 64));
      tr += __shfl_xor(tr, off, 64);
    }
    if (t == 0) {
      emax_s = me;
      trace_s = tr;
      bad_s = 0;
    }
  }
  __syncthreads();
  if (diag_only) {
    bool keep = false;
    if (t < m) {
      const double wi = es[t * m + t];
      keep = wi > 0.0 && wi > tau * epre[t];
      if (!keep) atomicAdd(drops, 1);
    }
    const bool any = __any(keep);
    for (int i = t; i < m * m; i += 64) {
      const int r = i % m, c = i / m;
      const double wc = es[c * m + c];
      T[i] = (r == c && wc > 0.0 && wc > tau * epre[c]) ? 1.0 / sqrt(wc) : 0.0;
    }
    if (t == 0) {
      if (!any) {
        flag0[0] = 1.0;
        flag1[0] = 1.0;
      }
      state[0] = 1.0;
    }
    return;
  }
  // Cholesky, lane t owns row t
  double a[MM];
#pragma unroll
  for (int c = 0; c < MM; ++c) a[c] = (t < m && c < m && c <= t) ? 0.5 * (es[c * m + t] + es[t * m + c]) : 0.0;
  // (fully unrolled with compile-time indices into a[]: a loop left with a runtime bound would index
  // the register array dynamically; the column of L is read from LDS in one independent batch)
#pragma unroll
  for (int j = 0; j < MM; ++j) {
    if (j < m) {
      if (t == j) {
        double d = a[j];
        if (!(d > 0.0)) {
          bad_s = 1;
          d = 1.0;
        }
        a[j] = sqrt(d);
        rdiag[j] = 1.0 / a[j];
      }
      __syncthreads();
      if (t > j && t < m) {
        a[j] *= rdiag[j];
        Ls[t][j] = a[j];
      }
      __syncthreads();
      double lc[MM];
#pragma unroll
      for (int c = j + 1; c < MM; ++c) lc[c] = Ls[c][j];
      if (t > j && t < m) {
        const double ltj = a[j];
#pragma unroll
        for (int c = j + 1; c < MM; ++c)
          if (c <= t) a[c] -= ltj * lc[c];
      }
    }
  }
  __syncthreads();
  // column t of L^{-1}, right-looking
  double x[MM];
#pragma unroll
  for (int r = 0; r < MM; ++r) x[r] = (r == t) ? 1.0 : 0.0;
#pragma unroll
  for (int k = 0; k < MM; ++k) {
    if (k < m) {
      x[k] *= rdiag[k];
      const double xk = x[k];
#pragma unroll
      for (int r = k + 1; r < MM; ++r)
        if (r < m) x[r] -= Ls[r][k] * xk;
    }
  }
  double fro = 0.0;
#pragma unroll
  for (int r = 0; r < MM; ++r) fro += (t < m && r < m) ? x[r] * x[r] : 0.0;
  for (int off = 32; off > 0; off >>= 1) fro += __shfl_xor(fro, off, 64);
  const double ref_up = fmax(trace_s, emax_s);
  const bool ok = bad_s == 0 && fro > 0.0 && (1.0 / fro) > tau * ref_up;
  if (ok) {
    // T = L^{-T}: T[c + m r] = (L^{-1})[r][c] = x[r] of lane c
    if (t < m) {
#pragma unroll
      for (int r = 0; r < MM; ++r)
        if (r < m) T[t + (int64_t)m * r] = x[r];
    }
  }
  if (t == 0) {
    state[0] = ok ? 1.0 : 0.0;
    state[1] = emax_s;
  }
}

// Y_i = op(T_i) X_i for nb blocks: T_i is m x m column-major at Ts + i m m (op = transpose when
// trans), X and Y are (nb m) x c column-major with ld nb m.  One workgroup per block.
__global__ __launch_bounds__(256) void k_tblocks(int nb, int m, int c, const double* Ts, int trans, const double* X,
                                                 double* Y) {
  const int i = blockIdx.x;
  const int64_t ld = (int64_t)nb * m;
  const double* Ti = Ts + (int64_t)i * m * m;
  for (int e = threadIdx.x; e < m * c; e += blockDim.x) {
    const int r = e % m, col = e / m;
    double v = 0.0;
    for (int k = 0; k < m; ++k)
      v += (trans ? Ti[k + (int64_t)r * m] : Ti[r + (int64_t)k * m]) * X[(int64_t)col * ld + (int64_t)i * m + k];
    Y[(int64_t)col * ld + (int64_t)i * m + r] = v;
  }
}

// x[i] = a pseudo-random value in [-0.5, 0.5) from a hash of i (a fixed test vector)
__global__ void k_fill_hash(int64_t n, double* x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t h = (uint64_t)i * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  h ^= h >> 31;
  h *= 0xBF58476D1CE4E5B9ull;
  h ^= h >> 29;
  x[i] = (double)(h >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

// keep only the diagonal of an m x n column-major matrix (ld)
__global__ void k_mask_diag(double* A, int m, int n, int64_t ld) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m * n) return;
  const int r = i % m, c = i / m;
  if (r != c) A[c * ld + r] = 0.0;
}

__global__ void k_axpby(int64_t count, double a, const double* x, double b, double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] = (b == 0.0) ? a * x[i] : a * x[i] + b * y[i];
}

// out = sum_z b[z slab + .] (nsplit slabs of partial sums)
__global__ void k_sum_slabs(int64_t count, const double* b, int64_t slab, int nsplit, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double v = 0.0;
  for (int z = 0; z < nsplit; ++z) v += b[z * slab + i];
  out[i] = v;
}

// strided rows: y[l*ldy + j] = a x[l*ldx + j] + b y[l*ldy + j]
__global__ void k_axpby_rows(int64_t rows, int cols, double a, const double* x, int64_t ldx, double b, double* y,
                             int64_t ldy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int64_t l = i / cols, j = i % cols;
  // b = 0 overwrites (y may hold anything, NaN included)
  y[l * ldy + j] = (b == 0.0) ? a * x[l * ldx + j] : a * x[l * ldx + j] + b * y[l * ldy + j];
}

// split occurrence loads into interior / boundary W-format blocks of pattern p
__global__ void k_split_loads(int n_p, int n_i, int n_b, int nq, int nr, const int* occ_list, const int64_t* foff,
                              const int* idofs, const int* bdofs, const double* f, double* Fi, double* Fb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)n_p * nq * nr;
  if (i >= total) return;
  const int64_t col = i / n_p;  // q*nr + r
  const int row = (int)(i % n_p);
  const int q = (int)(col / nr), r = (int)(col % nr);
  const double* fs = f + foff[occ_list[q]] + (int64_t)r * n_p;
  if (row < n_i) Fi[col * n_i + row] = fs[idofs[row]];
  else Fb[col * n_b + (row - n_i)] = fs[bdofs[row - n_i]];
}

// write recovered displacements back into the occurrence layout
__global__ void k_merge_u(int n_p, int n_i, int n_b, int nq, int nr, const int* occ_list, const int64_t* foff,
                          const int* idofs, const int* bdofs, const double* Ui, const double* Ub, double* u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)n_p * nq * nr;
  if (i >= total) return;
  const int64_t col = i / n_p;
  const int row = (int)(i % n_p);
  const int q = (int)(col / nr), r = (int)(col % nr);
  double* us = u + foff[occ_list[q]] + (int64_t)r * n_p;
  if (row < n_i) us[idofs[row]] = Ui[col * n_i + row];
  else us[bdofs[row - n_i]] = Ub[col * n_b + (row - n_i)];
}

// Y[row, col] = beta Y + alpha * sum_e A_csr[row, e] X[colidx[e], col]   (CSR SpMM, column-major X, Y)
// One thread per (row, SPMM_CB consecutive columns): a CSR entry is read once for all of them and
// their SPMM_CB gathers from X are independent, so a row's walk is not a chain of one-at-a-time
// loads.  Consecutive threads take consecutive rows (coalesced stores of Y).
constexpr int SPMM_CB = 8;
__global__ void k_spmm(int rows, int64_t cols, const int* ptr, const int* idx, const double* val, const double* X,
                       int64_t ldx, double alpha, double* Y, int64_t ldy, double beta) {
  const int64_t ncb = (cols + SPMM_CB - 1) / SPMM_CB;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows * ncb) return;
  const int row = (int)(i % rows);
  const int64_t c0 = (i / rows) * SPMM_CB;
  const int cn = (int)min<int64_t>(SPMM_CB, cols - c0);
  double s[SPMM_CB];
#pragma unroll
  for (int j = 0; j < SPMM_CB; ++j) s[j] = 0.0;
  const double* Xc = X + c0 * ldx;
  const int p0 = ptr[row], p1 = ptr[row + 1];
  // four entries at a time: their indices and values, then all their gathers from X, each one
  // batch of loads at clamped (always valid) positions, masked afterwards (entries in their order,
  // as a plain walk would add them)
  constexpr int EU = 4;
  for (int e0 = p0; e0 < p1; e0 += EU) {
    int64_t k[EU];
    double v[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      const int e = min(e0 + u, p1 - 1);
      k[u] = idx[e];
      v[u] = val[e];
    }
    double xv[EU][SPMM_CB];
#pragma unroll
    for (int u = 0; u < EU; ++u)
#pragma unroll
      for (int j = 0; j < SPMM_CB; ++j) xv[u][j] = Xc[(int64_t)min(j, cn - 1) * ldx + k[u]];
#pragma unroll
    for (int u = 0; u < EU; ++u)
      if (e0 + u < p1) {
#pragma unroll
        for (int j = 0; j < SPMM_CB; ++j) s[j] += v[u] * xv[u][j];
      }
  }
  double yo[SPMM_CB];
  if (beta != 0.0) {
#pragma unroll
    for (int j = 0; j < SPMM_CB; ++j) yo[j] = Y[(c0 + min(j, cn - 1)) * ldy + row];
  }
#pragma unroll
  for (int j = 0; j < SPMM_CB; ++j)
    if (j < cn) Y[(c0 + j) * ldy + row] = (beta == 0.0) ? alpha * s[j] : beta * yo[j] + alpha * s[j];
}
inline unsigned spmm_blocks(int rows, int64_t cols) {
  return (unsigned)cdiv(std::max<int64_t>((int64_t)rows * ((cols + SPMM_CB - 1) / SPMM_CB), 1), 256);
}

// e[(goff[s] + r')*nr + r] = E_p[r' + k*(q*nr + r)]  (Z^T g of pattern p into the coarse layout)
__global__ void k_coarse_reorder(int k, int nq, int nr, const int* occ_list, const int* goff, const double* E,
                                 double* e) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k * nq * nr) return;
  const int rp = i % k, col = i / k;
  const int q = col / nr, r = col % nr;
  e[((int64_t)goff[occ_list[q]] + rp) * nr + r] = E[i];
}

// Ub[b + n_b*(q*nr + r)] += sum_r' Z[b + n_b*r'] a[(goff[s] + r')*nr + r]
__global__ void k_add_kernel_term(int n_b, int k, int nq, int nr, const int* occ_list, const int* goff,
                                  const double* Z, const double* a, double* Ub) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_b * nq * nr) return;
  const int b = (int)(i % n_b);
  const int64_t col = i / n_b;
  const int q = (int)(col / nr), r = (int)(col % nr);
  const int64_t g0 = goff[occ_list[q]];
  double s = 0.0;
  for (int rp = 0; rp < k; ++rp) s += Z[(int64_t)rp * n_b + b] * a[(g0 + rp) * nr + r];
  Ub[i] += s;
}

inline unsigned nblocks(int64_t n, int b = 256) { return (unsigned)cdiv(std::max<int64_t>(n, 1), b); }

struct Timer {
  hipEvent_t a, b;
  hipStream_t s;
  explicit Timer(hipStream_t st) : s(st) {
    RPF_HIP(hipEventCreate(&a));
    RPF_HIP(hipEventCreate(&b));
    RPF_HIP(hipEventRecord(a, s));
  }
  double stop() {
    RPF_HIP(hipEventRecord(b, s));
    RPF_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    RPF_HIP(hipEventElapsedTime(&ms, a, b));
    return ms;
  }
  ~Timer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
};

// ---------------------------------------------------------------------------- solver
struct Solver {
  rpf_problem pb;
  const rpf_pattern* pats;
  hipStream_t s;
  int nr, np, m, method;
  int64_t N;
  // interface blocks (row-major, ld = nr or m)
  // Krylov store: for every stored block j the raw directions Z_j and P_j = Q^T F Z_j (N x m each,
  // slot j of the row-major N x ldW arrays) and the normalisation T_j (m x m); the F-orthonormal
  // block is W_j = Z_j T_j with F W_j = P_j T_j, never formed explicitly.
  DevBuf<double> lam, R, Rs, tmp, Zall, Pall, Tall, dlam;
  int64_t ldW = 0;
  int max_blocks = 0;
  // small matrices
  DevBuf<double> eta, V, w, T, alpha, gam, Bt, Cb, Mo, nrm, ws, estate, sqpart, gpart, alpha_prev;
  DevBuf<int> drops;
  std::vector<double> r0n;  // ||r0_c||^2 of the FP64 residual
  int iterations = 0, rank_drops = 0;
  int pc = RPF_PRECOND_NONE;  // preconditioner of z = Q F~^{-1} r
  bool periodic = false;      // truly periodic structure: P of the multivector by permutations
  int cq = RPF_PRECOND_NONE;  // preconditioner in the projector: Q = I - F~^{-1} G H^{-1} G^T
  DevBuf<double> Zp;          // z before the permutations (N x nr)
  DevBuf<double> Pz;          // Q F z (N x nr), periodic shortcut

  Solver(rpf_problem p, const rpf_pattern* pt, hipStream_t st, int nr_, int method_)
      : pb(p), pats(pt), s(st), nr(nr_), method(method_) {
    np = (method == RPF_CLASSICAL) ? 1 : pb->n_perm;
    m = nr * np;
    N = pb->n_lambda;
  }

  // column norms^2 of an N x c row-major block -> host (synchronous)
  std::vector<double> colnorm2(const double* X, int64_t ldx, int c) {
    nrm.ensure((size_t)c * c);
    gram(X, ldx, c, X, ldx, c, nrm.p);
    std::vector<double> full((size_t)c * c), out(c);
    RPF_HIP(hipMemcpyAsync(full.data(), nrm.p, sizeof(double) * c * c, hipMemcpyDeviceToHost, s));
    RPF_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < c; ++i) out[i] = full[(size_t)i * c + i];
    return out;
  }

  // Gram C (a x b, col-major ld a) = X^T Y with X: N x a (ldx), Y: N x b (ldy), row-major blocks
  void gram(const double* X, int64_t ldx, int a, const double* Y, int64_t ldy, int b, double* C) {
    ws.ensure((size_t)gram_chunks(N, a, b) * a * b);
    rpf::gram(s, N, a, b, X, ldx, Y, ldy, C, ws.p);
  }

  // lagged convergence check: the norms of iteration i are copied to pinned memory and read
  // while iteration i+1 is already queued, so the host never drains the stream mid-solve
  // Each slot holds the nr x nr Gram of the residual and, after it, the "exhausted" flag that
  // k_make_T raises when a whole block was dropped.
  double* hnorm = nullptr;  // pinned, 2 slots of nr*nr + 1
  hipEvent_t nev[2] = {nullptr, nullptr};
  DevBuf<double> nrm2[2];

  size_t slot_len() const { return (size_t)nr * nr + 1; }
  void init_lag() {
    if (!hnorm) {
      RPF_HIP(hipHostMalloc((void**)&hnorm, sizeof(double) * 2 * slot_len(), hipHostMallocDefault));
      RPF_HIP(hipEventCreateWithFlags(&nev[0], hipEventDisableTiming));
      RPF_HIP(hipEventCreateWithFlags(&nev[1], hipEventDisableTiming));
    }
    for (int k = 0; k < 2; ++k) {
      nrm2[k].ensure(slot_len());
      fill(s, nrm2[k].p + (size_t)nr * nr, 1, 0.0);
    }
  }
  // have_sq: the diagonal of nrm2[slot] already holds the squared residual norms
  void post_norms(const double* X, int slot, bool have_sq = false) {
    if (!have_sq) gram(X, nr, nr, X, nr, nr, nrm2[slot].p);
    RPF_HIP(hipMemcpyAsync(hnorm + (size_t)slot * slot_len(), nrm2[slot].p, sizeof(double) * slot_len(),
                           hipMemcpyDeviceToHost, s));
    RPF_HIP(hipEventRecord(nev[slot], s));
  }
  // norms held in device slot dslot, copied to host slot hslot
  void post_norms_from(const double* X, int dslot, int hslot, bool have_sq) {
    if (!have_sq) gram(X, nr, nr, X, nr, nr, nrm2[dslot].p);
    RPF_HIP(hipMemcpyAsync(hnorm + (size_t)hslot * slot_len(), nrm2[dslot].p, sizeof(double) * slot_len(),
                           hipMemcpyDeviceToHost, s));
    RPF_HIP(hipEventRecord(nev[hslot], s));
  }
  // captured batches of iterations: one graph for block CG and classical, one per starting place
  // in the restart cycle for ORTHODIR (keyed by that place)
  struct Captured {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool sq = false;  // the captured last iteration leaves the squared norms in slot 0
  };
  int graph_batch = 0;        // iterations per captured batch (0: no capture)
  hipStream_t cs = nullptr;   // capture stream (default priority)
  std::map<int, Captured> graphs;
  int gprec = -1;             // inner precision the graphs were captured for
  int graph_replays = 0;
  void release_graph() {
    for (auto& kv : graphs) {
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
      if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    graphs.clear();
    gprec = -1;
  }
  // Nothing may be allocated while a stream is captured (hipMalloc fails there), and no workspace
  // may be reallocated while captured graphs refer to it: every buffer an iteration grows on demand
  // is sized once, before the first capture.  The gram workspace covers every Gram an iteration or
  // a sweep forms (ORTHODIR: up to max_blocks - 1 stored blocks against the new one).
  void presize_step_buffers(bool upd_gram) {
    size_t most = (size_t)gram_pair_chunks(N) * m * (m + nr);
    const int w = std::max(m, nr);
    most = std::max(most, (size_t)gram_chunks(N, m, w) * m * w);
    most = std::max(most, (size_t)gram_chunks(N, nr, nr) * nr * nr);
    const int top = method == RPF_ORTHODIR ? max_blocks - 1 : 1;
    for (int nb = 1; nb <= top; ++nb) most = std::max(most, (size_t)gram_chunks(N, nb * m, m) * nb * m * m);
    ws.ensure(most);
    sqpart.ensure((size_t)(cdiv(N, 256) + 256) * nr);
    if (upd_gram) gpart.ensure((size_t)(cdiv(N, 256) + 256) * m * nr);
    if (np > 1 && pc != RPF_PRECOND_NONE) Zp.ensure((size_t)N * nr);
    if (np > 1 && periodic) Pz.ensure((size_t)N * nr);
  }
  enum Check { GOING = 0, CONVERGED = 1, EXHAUSTED = 2 };
  Check read_norms(int slot, const std::vector<double>& target) {
    RPF_HIP(hipEventSynchronize(nev[slot]));
    const double* h = hnorm + (size_t)slot * slot_len();
    bool ok = true;
    for (int c = 0; c < nr; ++c) {
      const double v = h[(size_t)c * nr + c];
      RPF_CHECK(std::isfinite(v), RPF_EBREAKDOWN, "block_krylov_solve: residual is not finite");
      ok &= !(v > target[c]);
    }
    if (ok) return CONVERGED;
    return h[(size_t)nr * nr] != 0.0 ? EXHAUSTED : GOING;
  }
  ~Solver() {
    release_graph();
    if (cs) (void)hipStreamDestroy(cs);
    if (hnorm) (void)hipHostFree(hnorm);
    for (auto& e : nev)
      if (e) (void)hipEventDestroy(e);
  }

  void alloc(int64_t ld_lam_unused) {
    (void)ld_lam_unused;
    lam.ensure((size_t)N * nr);
    R.ensure((size_t)N * nr);
    Rs.ensure((size_t)N * nr);
    dlam.ensure((size_t)N * nr);
    tmp.ensure((size_t)N * std::max(nr, m));
    eta.ensure((size_t)m * (m + nr));
    V.ensure((size_t)m * m);
    w.ensure(m);
    T.ensure((size_t)m * m);
    alpha.ensure((size_t)m * nr);
    gam.ensure((size_t)m * nr);
    drops.ensure(1);
    estate.ensure(2);
  }

  void alloc_store(int want_blocks) {
    size_t free_b = 0, total_b = 0;
    RPF_HIP(hipMemGetInfo(&free_b, &total_b));
    const double per_block = 2.0 * (double)N * m * sizeof(double);
    int cap = (int)std::max(1.0, std::floor(0.5 * (double)free_b / per_block));
    max_blocks = std::max(1, std::min(want_blocks, cap));
    if (method != RPF_ORTHODIR) max_blocks = 2;
    ldW = (int64_t)max_blocks * m;
    Zall.ensure((size_t)N * ldW);
    Pall.ensure((size_t)N * ldW);
    Tall.ensure((size_t)max_blocks * m * m);
    Bt.ensure((size_t)ldW * m);
    Cb.ensure((size_t)ldW * m);
    Mo.ensure((size_t)ldW * m);
  }

  // x <- Q x (directions) and x <- Q^T x (residuals and products); the two coincide unless the
  // projector carries a preconditioner
  void projQ(double* x, int64_t ldx, int c) {
    if (cq != RPF_PRECOND_NONE) project_M(pb, pats, cq, x, ldx, c, s);
    else project(pb, x, ldx, c, s);
  }
  void projQt(double* x, int64_t ldx, int c, int prec_m = RPF_FP64) {
    if (cq != RPF_PRECOND_NONE) project_Mt(pb, pats, cq, x, ldx, c, s, prec_m);
    else project(pb, x, ldx, c, s);
  }

  // W = Q [Pi_0 z, .., Pi_{np-1} z] for the nr columns of z (N x nr), into a slot of the store
  void permute_into(const double* z, double* W) {
    hipLaunchKernelGGL(k_permute, dim3(nblocks(N * m)), dim3(256), 0, s, N, pb->dpn, pb->n_mult, nr, np, pb->d_perm.p,
                       pb->d_ep_occ.p, pb->has_rot ? pb->d_rot.p : (const double*)nullptr, z, (int64_t)nr, W, ldW);
    RPF_LAUNCH_CHECK();
    projQ(W, ldW, m);
  }

  // One inner Krylov run on F_prec: starts from residual Rs (N x nr), accumulates
  // the correction into dlam; stops when every column satisfies ||r_c||^2 <= target_c
  // (CONVERGED), when a whole block was dropped (EXHAUSTED) or after max_it iterations.
  Check inner(int prec, const std::vector<double>& target, int max_it, int check_every) {
    fill(s, dlam.p, N * nr, 0.0);
    int nst = 0;  // stored blocks
    const bool diag_only = (method == RPF_CLASSICAL);
    RPF_HIP(hipMemsetAsync(drops.p, 0, sizeof(int), s));
    Check conv = GOING;
    init_lag();
    const double tau = eta_drop(prec);
    int pending = -1, nchk = 0;
    // block CG with one permutation: the residual update also leaves the next step's P^T R in Cb,
    // and the solution update of a step is deferred into the next step's orthogonalisation pass,
    // which reads the same direction block (flushed when the loop ends)
    // (not with a preconditioner: the next block is then Q F~^{-1} R, not R)
    const bool upd_gram =
        pc == RPF_PRECOND_NONE && cq == RPF_PRECOND_NONE && method != RPF_ORTHODIR && np == 1 && m <= 16 && nr <= 16 && 256 % nr == 0;
    bool have_gram = false, lam_pending = false;
    const double* lam_dir = nullptr;  // the direction block of the pending update
    if (upd_gram) alpha_prev.ensure((size_t)m * nr);
    // One iteration (it): everything up to the residual update.  check: the residual update also
    // leaves the squared column norms in nrm_out (returns true), else the caller forms them.
    auto step = [&](int it, bool check, double* nrm_out) -> bool {
      // ORTHODIR: orthogonalise against every stored block (restart when the store is full);
      // block CG / classical: against the previous block only, two alternating slots
      int slot, first, nb;
      if (method == RPF_ORTHODIR) {
        // restart when the store is full; in a low-precision run also once the stored blocks
        // could span the whole interface space: past that point the new directions are made
        // of the product's rounding error, which F-orthogonalisation cannot remove
        if (nst == max_blocks || (prec != RPF_FP64 && (int64_t)(nst + 1) * m > N)) nst = 0;
        slot = nst;
        first = 0;
        nb = nst;
      } else {
        slot = it % 2;
        first = (it + 1) % 2;
        nb = it > 0 ? 1 : 0;
      }
      double* Zs = Zall.p + (int64_t)slot * m;  // this block's directions, row stride ldW
      double* Ps = Pall.p + (int64_t)slot * m;
      // multivector from the residual (Q R = R: the residual stays in range Q), re-projected when
      // permuted; with one permutation it is the residual itself and is read from Rs below
      const bool direct = (np == 1);
      // orthogonalised straight from Rs
      const bool fused = pc == RPF_PRECOND_NONE && cq == RPF_PRECOND_NONE && direct && nb > 0 && nb * m <= 16;
      // periodic shortcut (truly periodic structure, section 3.1): Q F of the permuted block is
      // the permuted Q F z, so the product runs on the nr columns of z only
      const bool per = periodic && !direct;
      // with the same preconditioner in the projector, applied in FP64: Q F~^{-1} = F~^{-1} Q^T and
      // Q^T r = r, so z = F~^{-1} r is already in range Q
      const bool z_in_range = cq != RPF_PRECOND_NONE && pc == cq && (pc == RPF_PRECOND_LUMPED || prec == RPF_FP64);
      if (pc != RPF_PRECOND_NONE && direct) {
        // z = Q F~^{-1} r (Table 1)
        apply_precond(pb, pats, nr, Rs.p, nr, Zs, ldW, pc, prec, s);
        if (!z_in_range) projQ(Zs, ldW, m);
      } else if (!direct) {
        // the multivector of z = Q F~^{-1} r (z = r without a preconditioner), re-projected
        const double* z = Rs.p;
        if (pc != RPF_PRECOND_NONE) {
          Zp.ensure((size_t)N * nr);
          apply_precond(pb, pats, nr, Rs.p, nr, Zp.p, nr, pc, prec, s);
          if (!z_in_range) projQ(Zp.p, nr, nr);
          z = Zp.p;
        }
        permute_into(z, Zs);
        if (per) {
          Pz.ensure((size_t)N * nr);
          apply_F(pb, pats, nr, z, nr, Pz.p, nr, prec, true, s);
          permute_into(Pz.p, Ps);
        }
      } else if (!fused) {
        hipLaunchKernelGGL(k_axpby_rows, dim3(nblocks(N * nr)), dim3(256), 0, s, N, nr, 1.0, Rs.p, (int64_t)nr, 0.0,
                           Zs, ldW);
        RPF_LAUNCH_CHECK();
        // the residual lies in range Q^T; the direction is its Q projection
        if (cq != RPF_PRECOND_NONE) projQ(Zs, ldW, m);
      }
      const double* zsrc = fused ? Rs.p : Zs;
      const int64_t ldzs = fused ? (int64_t)nr : ldW;
      if (nb > 0) {
        // F-orthogonalise against the stored blocks: with W_i = Z_i T_i and F W_i = P_i T_i,
        // B = [F W_i]^T Z = T_i^T (P_i^T Z) and Z -= sum_i Z_i (T_i B_i)
        const int ka = nb * m;
        if (!(fused && have_gram)) gram(Pall.p + (int64_t)first * m, ldW, ka, zsrc, ldzs, m, Cb.p);
        hipLaunchKernelGGL(k_tblocks, dim3(nb), dim3(256), 0, s, nb, m, m, Tall.p + (int64_t)first * m * m, 1, Cb.p,
                           Bt.p);
        if (diag_only)
          hipLaunchKernelGGL(k_mask_diag, dim3(nblocks((int64_t)ka * m)), dim3(256), 0, s, Bt.p, ka, m, (int64_t)ka);
        hipLaunchKernelGGL(k_tblocks, dim3(nb), dim3(256), 0, s, nb, m, m, Tall.p + (int64_t)first * m * m, 0, Bt.p,
                           Mo.p);
        RPF_LAUNCH_CHECK();
        if (fused && lam_pending) {
          // Z_j = R - Z_{j-1} Mo and lambda += Z_{j-1} alpha_{j-1} in one pass over Z_{j-1}
          RPF_CHECK(lam_dir == Zall.p + (int64_t)first * m, RPF_EINVAL, "block step: deferred update source");
          RPF_CHECK(rows_orth_lam(s, N, ka, m, nr, lam_dir, ldW, Mo.p, Rs.p, nr, Zs, ldW, alpha_prev.p, dlam.p, nr),
                    RPF_EINVAL, "block step: orthogonalisation shape");
          lam_pending = false;
        } else if (fused) {
          rows_gemm_from(s, N, ka, m, -1.0, Zall.p + (int64_t)first * m, ldW, Mo.p, 1.0, Rs.p, nr, Zs, ldW);
        } else {
          rows_gemm(s, N, ka, m, -1.0, Zall.p + (int64_t)first * m, ldW, Mo.p, 1.0, Zs, ldW);
        }
        // periodic shortcut: F Z_i = P_i, so P takes the same combination of the stored P_i
        if (per) rows_gemm(s, N, ka, m, -1.0, Pall.p + (int64_t)first * m, ldW, Mo.p, 1.0, Ps, ldW);
      }
      // P = Q^T F Z
      if (!per) {
        apply_F(pb, pats, m, Zs, ldW, Ps, ldW, prec, cq == RPF_PRECOND_NONE, s);
        // Q^T of the product may use the inner precision's F~^{-1}: it only moves P along range G,
        // which is orthogonal to every direction (G^T Z = 0 through the FP64 Q), and each sweep's
        // residual is projected again in FP64
        if (cq != RPF_PRECOND_NONE) projQt(Ps, ldW, m, cq == RPF_PRECOND_DIRICHLET ? prec : RPF_FP64);
      }
      // [eta | Z^T R] = Z^T [P | R] in one pass over Z; T with T^T eta T = I on the kept directions
      {
        const size_t need = std::max((size_t)gram_pair_chunks(N) * m * (m + nr),
                                     (size_t)gram_chunks(N, m, std::max(m, nr)) * m * std::max(m, nr));
        ws.ensure(need);
        gram_pair(s, N, m, Zs, ldW, m, Ps, ldW, nr, Rs.p, nr, eta.p, ws.p);
      }
      double* zr = eta.p + (int64_t)m * m;
      double* Tj = Tall.p + (int64_t)slot * m * m;
      {
        double* f0 = nrm2[0].p + (size_t)nr * nr;
        double* f1 = nrm2[1].p + (size_t)nr * nr;
        const int dg = diag_only ? 1 : 0;
#define RPF_ETA(MM)                                                                                             \
  hipLaunchKernelGGL(k_eta_chol<MM>, dim3(1), dim3(64), 0, s, m, eta.p, dg, nb * m, Bt.p, tau, Tj, drops.p, f0, f1, \
                     estate.p)
        if (m <= 8) RPF_ETA(8);
        else if (m <= 16) RPF_ETA(16);
        else if (m <= 32) RPF_ETA(32);
        else RPF_ETA(64);
#undef RPF_ETA
        RPF_LAUNCH_CHECK();
        if (!diag_only) eta_eigen_T(s, eta.p, m, estate.p, tau, Tj, drops.p, f0, f1);
      }
      // alpha = W^T R = T^T (Z^T R); gamma = T alpha; lambda += Z gamma; R -= P gamma
      hipLaunchKernelGGL(k_tblocks, dim3(1), dim3(256), 0, s, 1, m, nr, Tj, 1, zr, gam.p);
      if (diag_only) hipLaunchKernelGGL(k_mask_diag, dim3(nblocks((int64_t)m * nr)), dim3(256), 0, s, gam.p, m, nr, (int64_t)m);
      hipLaunchKernelGGL(k_tblocks, dim3(1), dim3(256), 0, s, 1, m, nr, Tj, 0, gam.p, alpha.p);
      RPF_LAUNCH_CHECK();
      // the residual update also returns the squared column norms (into the check slot)
      sqpart.ensure((size_t)cdiv(N, 256) * nr);
      bool have_sq = false;
      have_gram = false;
      if (upd_gram) {
        gpart.ensure((size_t)(cdiv(N, 256) + 256) * m * nr);
        sqpart.ensure((size_t)(cdiv(N, 256) + 256) * nr);
        // lambda += Z_j alpha_j is deferred to the next step (or the flush below); the copy is a
        // kernel, so that a captured iteration holds kernels only
        copy_matrix(s, alpha.p, m, alpha_prev.p, m, m, nr);
        lam_pending = true;
        lam_dir = Zs;
        have_gram = rows_update_gram(s, N, m, nr, alpha.p, Ps, ldW, -1.0, 1.0, Rs.p, nr, sqpart.p,
                                     check ? nrm_out : nullptr, nr + 1, gpart.p, Cb.p);
        RPF_CHECK(have_gram, RPF_EINVAL, "block step: residual update shape");
        have_sq = check;
      } else {
        have_sq = check && rows_gemm2_sq(s, N, m, nr, alpha.p, 1.0, Zs, ldW, 1.0, dlam.p, nr, -1.0, Ps, ldW, 1.0,
                                         Rs.p, nr, sqpart.p, nrm_out, nr + 1);
        if (!have_sq)
          rows_gemm2(s, N, m, nr, alpha.p, 0, 1.0, Zs, ldW, 1.0, dlam.p, nr, -1.0, Ps, ldW, 1.0, Rs.p, nr);
      }
      ++nst;
      ++iterations;
      return have_sq;
    };
    // Captured batches: gb iterations are recorded once into a graph on a capture stream and
    // replayed on s, one convergence check per replay (its norms in device slot 0, copied to the
    // lagged host slot after the replay).  Block CG and classical: the two alternating slots make
    // the launches of iterations it and it + 2 identical from it = 2 on, so one graph (gb even)
    // serves every batch.  ORTHODIR: an iteration's launches depend on its place in the restart
    // cycle (how many blocks are stored), so a batch starting at place 0, gb, 2 gb, ... is captured
    // the first time the cycle gets there (after the sweep's first iteration) and replayed at that
    // place in every later cycle; a batch that would reach a restart runs uncaptured.
    // (ORTHODIR only when a restart cycle fits in the iterations left: otherwise no place of the
    // cycle comes round twice and every graph would be recorded for one replay)
    const bool od = method == RPF_ORTHODIR;
    const int gb = (graph_batch >= 2 && !trace_on() && (!od || max_blocks < max_it))
                       ? (od ? graph_batch : graph_batch & ~1) : 0;
    if (gb && !graphs.empty() && gprec != prec) release_graph();
    if (gb) presize_step_buffers(upd_gram);
    // place in the ORTHODIR cycle of the next iteration (after its restart test), and whether the
    // gb iterations from there fit before the next restart
    auto od_place = [&](bool& fits) {
      int pos = nst;
      if (pos == max_blocks || (prec != RPF_FP64 && (int64_t)(pos + 1) * m > N)) pos = 0;
      fits = pos % gb == 0 && pos + gb <= max_blocks && (prec == RPF_FP64 || (int64_t)(pos + gb) * m <= N);
      return pos;
    };
    int it = 0;
    while (it < max_it) {
      bool cap = false;
      int key = 0;
      if (gb && it + gb <= max_it) {
        // the first iteration of a sweep always runs uncaptured: it also sizes what the kernels it
        // calls (the preconditioner's, for one) allocate on first use
        if (od) {
          key = od_place(cap);
          cap = cap && it > 0;
        } else {
          cap = it >= 2 && it % 2 == 0;
        }
      }
      if (cap) {
        Captured& g = graphs[key];
        if (!g.exec) {
          if (!cs) RPF_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
          const hipStream_t s0 = s;
          RPF_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
          s = cs;
          try {
            for (int k = 0; k < gb; ++k) g.sq = step(it + k, k == gb - 1, nrm2[0].p);
          } catch (...) {
            s = s0;
            hipGraph_t gg = nullptr;
            (void)hipStreamEndCapture(cs, &gg);
            if (gg) (void)hipGraphDestroy(gg);
            graphs.erase(key);
            throw;
          }
          s = s0;
          RPF_HIP(hipStreamEndCapture(cs, &g.graph));
          RPF_HIP(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
          gprec = prec;
          // the capture ran the host side of these iterations (an ORTHODIR restart included); the
          // replay below runs the device side
          nst -= gb;
          iterations -= gb;
        } else if (od && nst != key) {
          nst = key;  // the restart that the replayed batch starts with
        }
        RPF_HIP(hipGraphLaunch(g.exec, s));
        ++graph_replays;
        nst += gb;
        iterations += gb;
        it += gb;
        const int slot_n = nchk & 1;
        post_norms_from(Rs.p, 0, slot_n, g.sq);
        if (pending >= 0 && (conv = read_norms(pending, target)) != GOING) {
          pending = -1;
          break;
        }
        pending = slot_n;
        ++nchk;
        continue;
      }
      const bool check = (it + 1) % check_every == 0 || it + 1 == max_it;
      const int slot_n = nchk & 1;
      const bool have_sq = step(it, check, nrm2[slot_n].p);
      ++it;
      if (check) {
        post_norms(Rs.p, slot_n, have_sq);
        // the previous check is read now, while this iteration is already queued; when it
        // reports convergence the solve stops after this (extra, still valid) iteration
        if (pending >= 0 && (conv = read_norms(pending, target)) != GOING) {
          pending = -1;
          break;
        }
        pending = slot_n;
        ++nchk;
      }
    }
    // replays overwrote the local product buffers behind the host's record of the last product
    if (graph_replays) ++pb->fp64_gen;
    if (lam_pending) {
      rows_gemm(s, N, m, nr, 1.0, lam_dir, ldW, alpha_prev.p, 1.0, dlam.p, nr, 0);
      lam_pending = false;
    }
    if (conv == GOING && pending >= 0) conv = read_norms(pending, target);
    int hd = 0;
    RPF_HIP(hipMemcpyAsync(&hd, drops.p, sizeof(int), hipMemcpyDeviceToHost, s));
    RPF_HIP(hipStreamSynchronize(s));
    rank_drops += hd;
    return conv;
  }
};

}  // namespace

void spmm_csr(hipStream_t s, int rows, int64_t cols, const int* ptr, const int* idx, const double* val,
              const double* X, int64_t ldx, double alpha, double* Y, int64_t ldy, double beta) {
  if (rows == 0 || cols == 0) return;
  hipLaunchKernelGGL(k_spmm, dim3(spmm_blocks(rows, cols)), dim3(256), 0, s, rows, cols, ptr, idx, val, X, ldx, alpha,
                     Y, ldy, beta);
  RPF_LAUNCH_CHECK();
}
}  // namespace rpf

using namespace rpf;

extern "C" rpf_status block_krylov_solve(rpf_problem pb, const rpf_pattern* pats, int32_t n_rhs, const double* f_local,
                                         const rpf_solve_opts* opts, double* lambda, int64_t ld_lambda,
                                         double* u_local, rpf_solve_stats* stats, void* stream) {
  rpf_solve_stats st{};
  rpf_status code = guarded([&] {
    RPF_CHECK(pb && opts && f_local && lambda && u_local, RPF_EINVAL, "block_krylov_solve: NULL argument");
    RPF_CHECK(n_rhs >= 1 && ld_lambda >= n_rhs, RPF_EINVAL, "block_krylov_solve: bad n_rhs / ld_lambda");
    RPF_CHECK(opts->method >= RPF_CLASSICAL && opts->method <= RPF_ORTHODIR, RPF_EINVAL, "block_krylov_solve: method");
    RPF_CHECK(opts->tol > 0 && opts->max_it >= 1, RPF_EINVAL, "block_krylov_solve: tol / max_it");
    const int prec = opts->prec;
    RPF_CHECK(prec >= RPF_FP64 && prec <= RPF_BF16, RPF_EINVAL, "block_krylov_solve: precision");
    RPF_CHECK(!(pb->weighted && (opts->precond != RPF_PRECOND_NONE || opts->coarse != RPF_PRECOND_NONE)), RPF_EINVAL,
              "block_krylov_solve: a non-Boolean assembly takes no preconditioner (the multiplicity scaling is "
              "defined for the signed Boolean assembly)");
    RPF_CHECK(opts->precond >= RPF_PRECOND_NONE && opts->precond <= RPF_PRECOND_DIRICHLET, RPF_EINVAL,
              "block_krylov_solve: preconditioner");
    check_patterns(pb, pats, RPF_FP64);
    check_patterns(pb, pats, prec);
    hipStream_t s = (hipStream_t)stream;
    Solver S(pb, pats, s, n_rhs, opts->method);
    S.pc = opts->precond;
    RPF_CHECK(opts->graph_batch >= 0, RPF_EINVAL, "block_krylov_solve: graph_batch < 0");
    S.graph_batch = opts->graph_batch;
    RPF_CHECK(opts->coarse >= RPF_PRECOND_NONE && opts->coarse <= RPF_PRECOND_DIRICHLET, RPF_EINVAL,
              "block_krylov_solve: preconditioner of the projector");
    RPF_CHECK(!(opts->coarse != RPF_PRECOND_NONE && opts->periodic && S.np > 1), RPF_EINVAL,
              "block_krylov_solve: the periodic shortcut needs the plain projector (coarse = RPF_PRECOND_NONE)");
    S.cq = opts->coarse;
    RPF_CHECK(S.m <= 64, RPF_EINVAL, "block_krylov_solve: block width n_rhs * n_perm must be <= 64");
    const int nr = n_rhs;
    const int64_t N = S.N;
    S.alloc(ld_lambda);

    // ------------------------------------------------------------ loads: g and e (d is never formed)
    Timer tl(s);
    std::vector<int64_t> foff(pb->n_occ + 1, 0);
    for (int o = 0; o < pb->n_occ; ++o) foff[o + 1] = foff[o] + (int64_t)pats[pb->occ_pat[o]]->n * nr;
    DevBuf<int64_t> d_foff;
    d_foff.upload(foff.data(), foff.size(), s);
    std::vector<DevBuf<double>> Y2(pb->n_pat), G(pb->n_pat);
    for (int p = 0; p < pb->n_pat; ++p) {
      const rpf_pattern P = pats[p];
      const int nq = (int)pb->occ_of_pat[p].size();
      const int64_t cols = (int64_t)nq * nr;
      const int* occ = pb->d_occ_of_pat.p + pb->pat_occ_off[p];
      Y2[p].alloc(std::max<int64_t>((int64_t)P->n_i * cols, 1));
      G[p].alloc(std::max<int64_t>((int64_t)P->n_b * cols, 1));
      hipLaunchKernelGGL(k_split_loads, dim3(nblocks((int64_t)P->n * cols)), dim3(256), 0, s, P->n, P->n_i, P->n_b,
                         nq, nr, occ, d_foff.p, P->d_idofs.p, P->d_bdofs.p, f_local, Y2[p].p, G[p].p);
      RPF_LAUNCH_CHECK();
      if (P->n_i > 0) {
        // Y2 = K_ii^{-1} f_i ; g = f_b - K_bi Y2
        trsm(s, P->L.p, P->ld, P->n_i, P->dinv_ii.p, P->env_ii, Y2[p].p, P->n_i, cols, false);
        trsm(s, P->L.p, P->ld, P->n_i, P->dinv_ii.p, P->env_ii, Y2[p].p, P->n_i, cols, true, P->L_upper);
        hipLaunchKernelGGL(k_spmm, dim3(spmm_blocks(P->n_b, cols)), dim3(256), 0, s, P->n_b, cols,
                           P->kbi_ptr.p, P->kbi_col.p, P->kbi_val.p, Y2[p].p, (int64_t)P->n_i, -1.0, G[p].p,
                           (int64_t)P->n_b, 1.0);
        RPF_LAUNCH_CHECK();
      }
    }
    // d = sum_s A^(s) S+ g^(s) is never formed: every residual d - F lambda is the single product
    // sum_s A^(s) S+ (g^(s) - A^(s)T lambda) (apply_F with the offsets g)
    std::vector<const double*> gp(pb->n_pat);
    for (int p = 0; p < pb->n_pat; ++p) gp[p] = G[p].p;
    st.ms_loads = tl.stop();

    // ------------------------------------------------------------ coarse problem, lambda_0, r_0
    Timer tc(s);
    ensure_coarse(pb, pats, s);
    const int nG = pb->n_G;
    DevBuf<double> e(std::max<int64_t>((int64_t)nG * nr, 1)), yc(std::max<int64_t>((int64_t)nG * nr, 1));
    if (nG > 0) {
      for (int p = 0; p < pb->n_pat; ++p) {
        const rpf_pattern P = pats[p];
        if (P->k == 0) continue;
        const int nq = (int)pb->occ_of_pat[p].size();
        DevBuf<double> E((size_t)P->k * nq * nr);
        dgemm(s, true, false, P->k, (int64_t)nq * nr, P->n_b, 1.0, P->Z.p, P->n_b, G[p].p, P->n_b, 0.0, E.p, P->k);
        hipLaunchKernelGGL(k_coarse_reorder, dim3(nblocks((int64_t)P->k * nq * nr)), dim3(256), 0, s, P->k, nq, nr,
                           pb->d_occ_of_pat.p + pb->pat_occ_off[p], pb->d_goff.p, E.p, e.p);
        RPF_LAUNCH_CHECK();
        RPF_HIP(hipStreamSynchronize(s));
      }
      if (S.cq != RPF_PRECOND_NONE) {
        // lambda_0 = F~^{-1} G (G^T F~^{-1} G)^{-1} e
        ensure_coarse_M(pb, pats, S.cq, s);
        lambda0_M(pb, pats, S.cq, e.p, nr, S.lam.p, nr, s);
      } else {
        // lambda_0 = G (G^T G)^{-1} e
        coarse_solve(pb, e.p, yc.p, nr, s);
        coarse_g(pb, yc.p, nr, 1.0, S.lam.p, nr, 0.0, s);
      }
    } else {
      fill(s, S.lam.p, N * nr, 0.0);
    }
    // r_0 = Q^T (d - F lambda_0).  Here and at every later residual, S.tmp keeps the unprojected
    // d - F lambda of the current lambda, one product on g - A^T lambda: the recovery reuses it.  A
    // mixed solve forms r_0 with the low-precision product: it only seeds the first sweep, whose
    // inner solve stops at inner_tol, far above that product's error; every residual after a sweep
    // (and so every convergence decision) is FP64.
    const bool lp_r0 = prec != RPF_FP64;
    apply_F(pb, pats, nr, S.lam.p, nr, S.tmp.p, nr, lp_r0 ? prec : RPF_FP64, false, s, OP_FLEX, gp.data());
    uint64_t res_gen = lp_r0 ? ~(uint64_t)0 : pb->fp64_gen;  // the FP64 product behind S.tmp, if any
    RPF_HIP(hipMemcpyAsync(S.R.p, S.tmp.p, sizeof(double) * N * nr, hipMemcpyDeviceToDevice, s));
    S.projQt(S.R.p, nr, nr);
    S.r0n = S.colnorm2(S.R.p, nr, nr);
    const std::vector<double> r0raw = S.r0n;  // the first convergence test sees the true norms
    for (double& v : S.r0n)
      if (!(v > 0.0)) v = 1.0;  // a zero initial residual: relative to 1 (nothing to reduce)
    st.ms_coarse = tc.stop();

    // ------------------------------------------------------------ iterations (+ FP64 refinement)
    Timer ti(s);
    const double tol2 = opts->tol * opts->tol;
    const int check = std::max(1, opts->check_every);
    const bool mixed = prec != RPF_FP64;
    const double inner_tol = opts->inner_tol > 0 ? opts->inner_tol : 1e-4;
    // FP64 form: further sweeps only restart from the recomputed residual (residual replacement)
    // when the recursive residual reached the target but the true one did not
    const int max_sweeps = opts->max_sweeps > 0 ? opts->max_sweeps : (mixed ? 30 : 4);
    S.alloc_store(opts->max_blocks > 0 ? opts->max_blocks : std::min(opts->max_it, 2000) + 1);
    if (opts->periodic && S.np > 1) {
      // the shortcut holds when Q F (and the preconditioner) commute with every permutation:
      // checked once, in FP64, on a pseudo-random vector of range Q
      const int np = S.np;
      DevBuf<double> x(N), a(N), pa((size_t)N * np), px((size_t)N * np), b((size_t)N * np);
      hipLaunchKernelGGL(k_fill_hash, dim3(nblocks(N)), dim3(256), 0, s, N, x.p);
      RPF_LAUNCH_CHECK();
      project(pb, x.p, 1, 1, s);
      double worst = 0.0;
      for (int what = 0; what < (S.pc != RPF_PRECOND_NONE ? 2 : 1); ++what) {
        auto op = [&](const double* in, double* out, int cols) {
          if (what == 0) apply_F(pb, pats, cols, in, cols, out, cols, RPF_FP64, true, s);
          else apply_precond(pb, pats, cols, in, cols, out, cols, S.pc, RPF_FP64, s);
        };
        op(x.p, a.p, 1);
        hipLaunchKernelGGL(k_permute, dim3(nblocks(N * np)), dim3(256), 0, s, N, pb->dpn, pb->n_mult, 1, np,
                           pb->d_perm.p, pb->d_ep_occ.p, pb->has_rot ? pb->d_rot.p : (const double*)nullptr, a.p,
                           (int64_t)1, pa.p, (int64_t)np);
        hipLaunchKernelGGL(k_permute, dim3(nblocks(N * np)), dim3(256), 0, s, N, pb->dpn, pb->n_mult, 1, np,
                           pb->d_perm.p, pb->d_ep_occ.p, pb->has_rot ? pb->d_rot.p : (const double*)nullptr, x.p,
                           (int64_t)1, px.p, (int64_t)np);
        RPF_LAUNCH_CHECK();
        project(pb, px.p, np, np, s);
        op(px.p, b.p, np);
        std::vector<double> ha((size_t)N * np), hb((size_t)N * np);
        RPF_HIP(hipMemcpyAsync(ha.data(), pa.p, sizeof(double) * N * np, hipMemcpyDeviceToHost, s));
        RPF_HIP(hipMemcpyAsync(hb.data(), b.p, sizeof(double) * N * np, hipMemcpyDeviceToHost, s));
        RPF_HIP(hipStreamSynchronize(s));
        double dmax = 0.0, amax = 0.0;
        for (size_t i = 0; i < ha.size(); ++i) {
          dmax = std::max(dmax, std::fabs(ha[i] - hb[i]));
          amax = std::max(amax, std::fabs(ha[i]));
        }
        worst = std::max(worst, amax > 0.0 ? dmax / amax : 0.0);
      }
      RPF_CHECK(worst <= 1e-10, RPF_EINVAL,
                "block_krylov_solve: periodic shortcut requested but the structure is not periodic under its "
                "permutations (relative commutation defect " + std::to_string(worst) + ")");
      S.periodic = true;
    }
    bool converged = false;
    int sweeps = 0;
    std::vector<double> rn = r0raw;
    double rel = 1.0;
    bool fresh = true;  // S.R holds the FP64 residual of the current lambda
    for (int sw = 0; sw < max_sweeps; ++sw) {
      if (!fresh) {
        // FP64 residual of the current lambda
        apply_F(pb, pats, nr, S.lam.p, nr, S.tmp.p, nr, RPF_FP64, false, s, OP_FLEX, gp.data());
        res_gen = pb->fp64_gen;
        RPF_HIP(hipMemcpyAsync(S.R.p, S.tmp.p, sizeof(double) * N * nr, hipMemcpyDeviceToDevice, s));
        S.projQt(S.R.p, nr, nr);
        rn = S.colnorm2(S.R.p, nr, nr);
        fresh = true;
      }
      rel = 0.0;
      for (int c = 0; c < nr; ++c) rel = std::max(rel, std::sqrt(rn[c] / S.r0n[c]));
      if (rel <= opts->tol) {
        converged = true;
        break;
      }
      if (S.iterations >= opts->max_it) break;
      ++sweeps;
      std::vector<double> target(nr);
      for (int c = 0; c < nr; ++c)
        target[c] = mixed ? std::max(inner_tol * inner_tol * rn[c], 0.25 * tol2 * S.r0n[c]) : tol2 * S.r0n[c];
      RPF_HIP(hipMemcpyAsync(S.Rs.p, S.R.p, sizeof(double) * N * nr, hipMemcpyDeviceToDevice, s));
      S.inner(prec, target, opts->max_it - S.iterations, check);
      hipLaunchKernelGGL(k_axpby, dim3(nblocks(N * nr)), dim3(256), 0, s, N * nr, 1.0, S.dlam.p, 1.0, S.lam.p);
      RPF_LAUNCH_CHECK();
      fresh = false;
    }
    // final FP64 residual check (recomputed unless the loop ended on a fresh one)
    if (!fresh) {
      apply_F(pb, pats, nr, S.lam.p, nr, S.tmp.p, nr, RPF_FP64, false, s, OP_FLEX, gp.data());
      res_gen = pb->fp64_gen;
      RPF_HIP(hipMemcpyAsync(S.R.p, S.tmp.p, sizeof(double) * N * nr, hipMemcpyDeviceToDevice, s));
      S.projQt(S.R.p, nr, nr);
      rn = S.colnorm2(S.R.p, nr, nr);
    }
    rel = 0.0;
    for (int c = 0; c < nr; ++c) rel = std::max(rel, std::sqrt(rn[c] / S.r0n[c]));
    converged = rel <= opts->tol;
    st.ms_iterate = ti.stop();
    st.iterations = S.iterations;
    st.sweeps = std::max(sweeps, 1);
    st.rank_drops = S.rank_drops;
    st.graph_replays = S.graph_replays;
    st.rel_residual = rel;

    // ------------------------------------------------------------ recovery (eq. 2)
    Timer tr(s);
    // alpha = (G^T G)^{-1} G^T (F lambda - d), with d - F lambda of the final lambda in S.tmp (its
    // last FP64 residual)
    DevBuf<double> ca(std::max<int64_t>((int64_t)nG * nr, 1)), aa(std::max<int64_t>((int64_t)nG * nr, 1));
    if (nG > 0) {
      coarse_gt(pb, S.tmp.p, nr, nr, ca.p, s);
      hipLaunchKernelGGL(k_axpby, dim3(nblocks((int64_t)nG * nr)), dim3(256), 0, s, (int64_t)nG * nr, -1.0, ca.p, 0.0,
                         ca.p);
      RPF_LAUNCH_CHECK();
      coarse_solve(pb, ca.p, aa.p, nr, s);
    }
    // S+ (g - A^T lambda) of the final lambda is still in the problem's local product buffer when
    // the last FP64 product was that of the final residual (no other FP64 product since)
    const bool reuse = pb->fp64_gen == res_gen && pb->last_gsub && pb->last_x == S.lam.p && pb->last_m == nr &&
                       pb->last_ldx == nr;
    for (int p = 0; p < pb->n_pat; ++p) {
      const rpf_pattern P = pats[p];
      const int nq = (int)pb->occ_of_pat[p].size();
      const int64_t cols = (int64_t)nq * nr;
      const int* occ = pb->d_occ_of_pat.p + pb->pat_occ_off[p];
      DevBuf<double> Ub((size_t)P->n_b * cols);
      // u_b = S+ (g - A^T lambda) + Z alpha_s
      if (reuse) {
        hipLaunchKernelGGL(k_sum_slabs, dim3(nblocks((int64_t)P->n_b * cols)), dim3(256), 0, s, (int64_t)P->n_b * cols,
                           pb->last_yl.base[p], pb->last_yl.slab[p], pb->last_yl.nsplit[p], Ub.p);
        RPF_LAUNCH_CHECK();
      } else {
        DevBuf<double> X((size_t)P->n_b * cols);
        gather_pattern(pb, p, pb->pat_nbn[p], S.lam.p, nr, nr, X.p, P->n_b, s);
        hipLaunchKernelGGL(k_axpby, dim3(nblocks((int64_t)P->n_b * cols)), dim3(256), 0, s, (int64_t)P->n_b * cols,
                           1.0, G[p].p, -1.0, X.p);
        RPF_LAUNCH_CHECK();
        dgemm(s, false, false, P->n_b, cols, P->n_b, 1.0, P->Splus.p, P->n_b, X.p, P->n_b, 0.0, Ub.p, P->n_b);
      }
      if (nG > 0 && P->k > 0) {
        hipLaunchKernelGGL(k_add_kernel_term, dim3(nblocks((int64_t)P->n_b * cols)), dim3(256), 0, s, P->n_b, P->k, nq,
                           nr, occ, pb->d_goff.p, P->Z.p, aa.p, Ub.p);
        RPF_LAUNCH_CHECK();
      }
      // u_i = K_ii^{-1} f_i - K_ii^{-1} K_ib u_b
      DevBuf<double> Ti(std::max<int64_t>((int64_t)P->n_i * cols, 1));
      if (P->n_i > 0) {
        hipLaunchKernelGGL(k_spmm, dim3(spmm_blocks(P->n_i, cols)), dim3(256), 0, s, P->n_i, cols, P->kib_ptr.p,
                           P->kib_col.p, P->kib_val.p, Ub.p, (int64_t)P->n_b, 1.0, Ti.p, (int64_t)P->n_i, 0.0);
        RPF_LAUNCH_CHECK();
        trsm(s, P->L.p, P->ld, P->n_i, P->dinv_ii.p, P->env_ii, Ti.p, P->n_i, cols, false);
        trsm(s, P->L.p, P->ld, P->n_i, P->dinv_ii.p, P->env_ii, Ti.p, P->n_i, cols, true, P->L_upper);
        hipLaunchKernelGGL(k_axpby, dim3(nblocks((int64_t)P->n_i * cols)), dim3(256), 0, s, (int64_t)P->n_i * cols, 1.0,
                           Y2[p].p, -1.0, Ti.p);
        RPF_LAUNCH_CHECK();
      }
      hipLaunchKernelGGL(k_merge_u, dim3(nblocks((int64_t)P->n * cols)), dim3(256), 0, s, P->n, P->n_i, P->n_b, nq, nr,
                         occ, d_foff.p, P->d_idofs.p, P->d_bdofs.p, Ti.p, Ub.p, u_local);
      RPF_LAUNCH_CHECK();
      RPF_HIP(hipStreamSynchronize(s));
    }
    // lambda out
    hipLaunchKernelGGL(k_axpby_rows, dim3(nblocks(N * nr)), dim3(256), 0, s, N, nr, 1.0, S.lam.p, (int64_t)nr, 0.0,
                       lambda, ld_lambda);
    RPF_LAUNCH_CHECK();
    st.ms_recover = tr.stop();
    st.converged = converged ? 1 : 0;
    if (!converged) {
      char msg[160];
      snprintf(msg, sizeof msg, "block_krylov_solve: not converged (relative residual %.3e after %d iterations, %d sweeps)",
               rel, st.iterations, st.sweeps);
      throw Error(RPF_ENOCONV, msg);
    }
  });
  if (stats) *stats = st;
  return code;
}

extern "C" rpf_status feti_permute(rpf_problem pb, const rpf_pattern* pats, int32_t nr, const double* Z, int64_t ldz,
                                   double* W, int64_t ldw, uint32_t flags, void* stream) {
  return guarded([&] {
    RPF_CHECK(pb != nullptr, RPF_EINVAL, "feti_permute: NULL structure");
    const int np = pb->n_perm;
    RPF_CHECK(nr >= 1 && ldz >= nr && ldw >= (int64_t)nr * np && Z && W, RPF_EINVAL,
              "feti_permute: bad block arguments");
    const bool proj = (flags & RPF_APPLY_PROJECT) != 0;
    if (proj) check_patterns(pb, pats, RPF_FP64);
    hipStream_t s = (hipStream_t)stream;
    const int64_t N = pb->n_lambda;
    if (N == 0) return;
    const int m = nr * np;
    if (ldz == nr && ldw == m) {
      hipLaunchKernelGGL(k_permute, dim3(nblocks(N * m)), dim3(256), 0, s, N, pb->dpn, pb->n_mult, nr, np,
                         np > 1 ? pb->d_perm.p : (const int*)nullptr, pb->d_ep_occ.p,
                         pb->has_rot ? pb->d_rot.p : (const double*)nullptr, Z, (int64_t)nr, W, (int64_t)m);
      RPF_LAUNCH_CHECK();
    } else {
      // strided operands go through a packed staging pair
      DevBuf<double> zs, ws;
      zs.ensure((size_t)N * nr);
      ws.ensure((size_t)N * m);
      copy_matrix(s, Z, ldz, zs.p, nr, nr, N);  // (row-major: nr entries per row)
      hipLaunchKernelGGL(k_permute, dim3(nblocks(N * m)), dim3(256), 0, s, N, pb->dpn, pb->n_mult, nr, np,
                         np > 1 ? pb->d_perm.p : (const int*)nullptr, pb->d_ep_occ.p,
                         pb->has_rot ? pb->d_rot.p : (const double*)nullptr, zs.p, (int64_t)nr, ws.p, (int64_t)m);
      RPF_LAUNCH_CHECK();
      copy_matrix(s, ws.p, m, W, ldw, m, N);
      RPF_HIP(hipStreamSynchronize(s));  // staging buffers are freed on return
    }
    if (proj) {
      ensure_coarse(pb, pats, s);
      project(pb, W, ldw, m, s);
    }
  });
}

extern "C" int32_t problem_n_perm(rpf_problem pb) { return pb ? pb->n_perm : -1; }
