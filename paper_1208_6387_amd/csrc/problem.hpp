// Structure handle: signed Boolean assembly maps, permutation maps and the
// coarse space, plus the workspaces of the interface operator (internal).
#pragma once

#include "pattern.hpp"

#include <map>

namespace rpf {
constexpr int MAXP = 8;   // patterns per structure
constexpr int KMAX = 8;   // kernel dimension per pattern (coarse kernels)

// W-format result slabs of every pattern; a split-K product leaves nsplit partial
// slabs `slab` elements apart, summed by the scatter.
struct YLoc {
  double* base[MAXP];
  int64_t ld[MAXP];
  int64_t slab[MAXP];
  int nsplit[MAXP];
};
// Every pattern's flexibility product in one persistent launch: per pattern its operands and
// shape, its tile grid (tm x tn tiles of the kernel's size, K split into pieces of kchunk) and the
// index of its first tile in the group's tile list (start[n] = all tiles).
struct BfGroup {
  int n;
  int start[MAXP + 1];
  int M[MAXP], N[MAXP], K[MAXP], kchunk[MAXP], tm[MAXP], tn[MAXP];
  const uint16_t* Ah[MAXP];
  const uint16_t* Al[MAXP];
  const uint16_t* Bh[MAXP];
  const uint16_t* Bl[MAXP];
  int64_t lda[MAXP], ldb[MAXP], ldc[MAXP], slab[MAXP];
  float* C[MAXP];
};
struct DGroup {
  int n;
  int start[MAXP + 1];
  int M[MAXP], N[MAXP], K[MAXP], kchunk[MAXP], tm[MAXP], tn[MAXP];
  const double* A[MAXP];
  const double* B[MAXP];
  int64_t lda[MAXP], ldb[MAXP];
  double* part[MAXP];  // split-K result slabs, M x N column-major each
};

// Local results of a product for the non-Boolean scatter: column-major per pattern, nsplit
// partial slabs `slab` apart (FP64 or FP32).
template <typename T>
struct WLoc {
  const T* base[MAXP];
  int64_t ld[MAXP];
  int64_t slab[MAXP];
  int nsplit[MAXP];
};

// Schedule of the flexibility products of a structure for one block width and arithmetic: the
// workgroup tile (64 or 128 in a grouped persistent launch; 256 for the single-pattern large-tile
// kernels, 0 for the size rule) and the target count of work items (tiles times K splits) that
// sets each pattern's K split.
struct Schedule {
  int tile = 0;
  int work = 1024;
};
}  // namespace rpf

struct rpf_problem_s {
  int dpn = 1, n_pat = 0, n_occ = 0, n_mult = 0, n_perm = 1;
  int64_t n_lambda = 0;
  bool has_rot = false;
  std::vector<int> pat_nbn;                  // boundary nodes per pattern
  std::vector<int> occ_pat, occ_q, slot_off; // slot_off[s]: first boundary-node slot of s
  std::vector<std::vector<int>> occ_of_pat;  // pattern -> occurrences (q order)
  std::vector<int> pat_occ_off;              // offsets into d_occ_of_pat

  rpf::DevBuf<int> d_occ_of_pat, d_slot_off, d_occ_pat;
  rpf::DevBuf<int> d_l2m_ptr, d_l2m_code;    // per slot: multipliers (code = mult << 1 | negative)
  rpf::DevBuf<int> d_l2m_bn;                 // boundary node of every slot-list entry
  rpf::DevBuf<int> d_ep_q, d_ep_bn, d_ep_occ;  // per multiplier endpoint
  rpf::DevBuf<int8_t> d_ep_pat, d_ep_sign;
  rpf::DevBuf<double> d_rot;
  rpf::DevBuf<int> d_perm;
  // multipliers grouped by the pair of occurrences they join (coarse matrix assembly)
  std::vector<int> pair_a, pair_b, pair_ptr;
  rpf::DevBuf<int> d_pair_a, d_pair_b, d_pair_ptr, d_pair_mult;

  // W-format workspaces
  rpf::DevBuf<double> xloc, yloc;
  // the local products S+ A^T X of the last FP64 operator product (in yloc), its X, ldx and m;
  // fp64_gen counts FP64 products, so a reader can tell that yloc still holds them
  rpf::YLoc last_yl{};
  const double* last_x = nullptr;
  int64_t last_ldx = 0;
  int last_m = 0;
  bool last_gsub = false;  // the last FP64 product's input was g - A^T X (apply_F's gsub)
  uint64_t fp64_gen = 0;
  rpf::DevBuf<float> xloc32, yloc32;
  rpf::DevBuf<uint16_t> xhi, xlo;

  // scaling of the preconditioners, (A A^T)^{-1} = C^{-1} (x) I_dpn: C couples the multipliers
  // that share an endpoint (occurrence, local node), so C^{-1} is block diagonal over those
  // groups; CSR over multipliers (node level)
  rpf::DevBuf<int> d_sc_ptr, d_sc_col;
  rpf::DevBuf<double> d_sc_val;
  rpf::DevBuf<double> pcbuf;  // preconditioner workspace, N_lambda x m
  // occurrences whose boundaries meet through one of those groups (sorted, self included): the
  // scaled trace of a coarse mode of i reaches occurrence s only when i is in occ_nbr[s]
  std::vector<std::vector<int>> occ_nbr;

  // coarse space (built for one set of pattern handles)
  std::vector<uint64_t> coarse_key;  // uids of the pattern handles the coarse space was built for
  int n_G = 0;
  std::vector<int> goff;
  rpf::DevBuf<int> d_goff, d_kp, d_nbn;
  // rows of G per multiplier (2 endpoints x dpn x g_km) and each endpoint's first coarse index
  rpf::DevBuf<double> d_grow;
  rpf::DevBuf<int> d_ep_goff;
  int g_km = 0;
  rpf::DevBuf<const double*> d_Zp;
  rpf::DevBuf<double> Ginv, cbuf, ybuf, cpart, cws;
  // coarse space with a preconditioner F~^{-1} in the projector: (G^T F~^{-1} G)^{-1}, built for the
  // pattern handles and preconditioner kind in hkey, and an N_lambda x m workspace
  std::vector<uint64_t> hkey;
  rpf::DevBuf<double> Hinv, qbuf;

  // non-Boolean assembly (weights per side of a multiplier): per slot the (multiplier, weight)
  // entries (gather), per multiplier side the (boundary node, weight) entries (scatter, rows of G),
  // per occurrence the multiplier sides that touch it (G^T x, G^T G)
  bool weighted = false;
  rpf::DevBuf<int> d_wl_ptr, d_wl_mult, d_wm_ptr, d_wm_bn, d_wo_ptr, d_wo_me;
  rpf::DevBuf<double> d_wl_w, d_wm_w;

  // schedules of the flexibility products installed by problem_tune / problem_set_schedule, per
  // (block width m, arithmetic); absent: the size rule
  std::map<std::pair<int, int>, rpf::Schedule> sched;
};

namespace rpf {
// helpers shared by the operator and the solver
void check_patterns(rpf_problem pb, const rpf_pattern* pats, int prec);
// pattern matrix of a local product: S+ (the operator F) or S (the Dirichlet preconditioner)
enum LocalOp { OP_FLEX = 0, OP_SCHUR = 1 };
// Workspace plan of the FP64 operator for an m-column block: per pattern the offsets of its W
// block (leading dimension ldw, padded to 32 rows for the large-problem kernel) and of its result
// slabs (alloc_sp split-K slabs of n_b x cols, nsp of them written), and the doubles needed.
struct F64Plan {
  int64_t off[MAXP + 1], yoff[MAXP + 1], ldw[MAXP], kchunk[MAXP];
  int nsp[MAXP], alloc_sp[MAXP];
  char big[MAXP];
  int tile;  // 64 or 128: every pattern in one grouped launch of that tile; 0: per-pattern launches
  int64_t xneed, yneed;
};
// the schedule installed for (m, prec), or the size rule (tile 0)
Schedule schedule_for(rpf_problem pb, int m, int prec);
F64Plan plan_F64(rpf_problem pb, const rpf_pattern* pats, int m, const Schedule& sc);
// grouped persistent launches of the flexibility products (tile 64 or 128)
void dgemm_group(hipStream_t s, int tile, const DGroup& g);
void gemm_bf16_group(hipStream_t s, int tile, bool x3, const BfGroup& g);
// K split of one pattern in a grouped launch: the tiles of the pattern times the split reach about
// `work` items, each piece at least 256 deep, at most 8 pieces; a multiple of `align`
int64_t group_kchunk(int64_t nb_rows, int64_t K, int64_t cols, int tile, int work, int align);
// Gather and FP64 product of every pattern into the workspaces xw (plan.xneed doubles) and yw
// (plan.yneed doubles); returns the result slabs for scatter_all.  No allocation.
// gsub: optional per-pattern blocks g_p (n_b x occurrences * m, column-major, ld n_b); the
// product input of pattern p is then g_p - A^(s)T X instead of A^(s)T X.
YLoc run_F64(rpf_problem pb, const rpf_pattern* pats, const F64Plan& pl, int m, const double* X, int64_t ldx,
             double* xw, double* yw, hipStream_t s, int op, bool trace, const double* const* gsub = nullptr);
// Y = F X (W-format products on all patterns), optional projection; with op = OP_SCHUR the same
// assembled product with S in place of S+.  With gsub (see run_F64), Y = sum_s A^(s) S+ (g - A^(s)T X),
// which is d - F X for the condensed loads g (eq. 3 with d = sum_s A^(s) S+ g) without forming d.
void apply_F(rpf_problem pb, const rpf_pattern* pats, int m, const double* X, int64_t ldx, double* Y,
             int64_t ldy, int prec, bool project, hipStream_t s, int op = OP_FLEX,
             const double* const* gsub = nullptr);
// x[c ldx + r] = g[c ldg + r] - x[c ldx + r] for r < rows (column-major, cols columns)
void rsub_cols(hipStream_t s, int rows, int64_t cols, const double* g, int64_t ldg, double* x, int64_t ldx);
// Y = F~^{-1} X for the lumped (kind 1) or Dirichlet (kind 2) preconditioner, the Dirichlet
// product in precision prec; X and Y may be the same block
void apply_precond(rpf_problem pb, const rpf_pattern* pats, int m, const double* X, int64_t ldx, double* Y,
                   int64_t ldy, int kind, int prec, hipStream_t s);
// Y = beta Y + alpha A X for a CSR matrix A (rows x n) and column-major X, Y (cols columns)
void spmm_csr(hipStream_t s, int rows, int64_t cols, const int* ptr, const int* idx, const double* val,
              const double* X, int64_t ldx, double alpha, double* Y, int64_t ldy, double beta);
// A^(s)T gather of an interface block into the W format of pattern p
void gather_pattern(rpf_problem pb, int p, int nbn, const double* lam, int64_t ldl, int m, double* X,
                    int64_t ldx, hipStream_t s);
// Y = beta Y + sum_s A^(s) Y_loc
void scatter_all(rpf_problem pb, const YLoc& yl, int m, double* Y, int64_t ldy, double beta, hipStream_t s);
void ensure_coarse(rpf_problem pb, const rpf_pattern* pats, hipStream_t s);
// c = G^T x (n_G x m row-major)
void coarse_gt(rpf_problem pb, const double* x, int64_t ldx, int m, double* c, hipStream_t s);
// x = beta x + alpha G y
void coarse_g(rpf_problem pb, const double* y, int m, double alpha, double* x, int64_t ldx, double beta,
              hipStream_t s);
// x <- Q x = x - G (G^T G)^{-1} G^T x
void project(rpf_problem pb, double* x, int64_t ldx, int m, hipStream_t s);
void project_block(rpf_problem pb, double* x, int64_t ldx, int m, hipStream_t s);
void coarse_solve(rpf_problem pb, const double* c, double* y, int m, hipStream_t s);
// projector with the preconditioner of kind `kind` as F~^{-1} (section 2):
// H = G^T F~^{-1} G and its inverse (after ensure_coarse); x <- Q x = x - F~^{-1} G H^{-1} G^T x;
// x <- Q^T x = x - G H^{-1} G^T F~^{-1} x; x <- F~^{-1} G H^{-1} e (lambda_0, n_G x m e)
void ensure_coarse_M(rpf_problem pb, const rpf_pattern* pats, int kind, hipStream_t s);
void project_M(rpf_problem pb, const rpf_pattern* pats, int kind, double* x, int64_t ldx, int m, hipStream_t s);
void project_Mt(rpf_problem pb, const rpf_pattern* pats, int kind, double* x, int64_t ldx, int m, hipStream_t s,
                int prec = RPF_FP64);
void lambda0_M(rpf_problem pb, const rpf_pattern* pats, int kind, const double* e, int m, double* x, int64_t ldx,
               hipStream_t s);
// F X with a low-precision flexibility product (FP32 or bf16 split), FP64 in and out
// Gather A^(s)T lam for every occurrence of pattern p into the W format (lanes over interface
// columns; needs m >= 8 for full lanes).  mode 0: FP32 Xf, 1: bf16 hi/lo Xh/Xl, 2: FP64 X64.
void gather_rows(rpf_problem pb, int p, const double* lam, int64_t ldl, int m, int mode, double* X64, float* Xf,
                 uint16_t* Xh, uint16_t* Xl, int64_t ldx, hipStream_t s);
void apply_F_lowprec(rpf_problem pb, const rpf_pattern* pats, int m, const double* X, int64_t ldx, double* Y,
                     int64_t ldy, int prec, hipStream_t s, int op = OP_FLEX, const double* const* gsub = nullptr);
// non-Boolean assembly: gather (mode 2 FP64, 0 FP32, 1 bf16 split), scatter from column-major
// local results, rows of G with G^T G, and G^T x
void wgather(rpf_problem pb, int p, const double* lam, int64_t ldl, int m, int mode, double* X64, float* Xf,
             uint16_t* Xh, uint16_t* Xl, int64_t ldx, hipStream_t s);
template <typename T>
void wscatter(rpf_problem pb, const WLoc<T>& yl, int m, double* Y, int64_t ldy, hipStream_t s);
void wcoarse_setup(rpf_problem pb, double* GtG, int64_t ldg, hipStream_t s);
void wcoarse_gt(rpf_problem pb, const double* x, int64_t ldx, int m, double* c, hipStream_t s);
// event tracing of the flexibility products
bool trace_on();
void* trace_begin(hipStream_t s, int prec);
void trace_end(void* tok, hipStream_t s, double flops);
}  // namespace rpf
