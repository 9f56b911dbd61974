/*
 * rpfeti.h -- C ABI of the repeated-pattern FETI hot path on MI355X (gfx950).
 *
 * Method: Gosselet, Rixen, Rey, "A domain decomposition strategy to
 * efficiently solve structures containing repeated patterns".  A structure is
 * a set of occurrences of a few patterns.  All occurrences of a pattern share
 * one Neumann stiffness K, so the library factors K once per pattern,
 * condenses it to the dense boundary flexibility S+ = t K+ t^T (section 2),
 * and applies the dual operator F = sum_s A^(s) S+ A^(s)T to the interface
 * vectors of every occurrence at once as one matrix product (section 3.2).
 * The interface problem (eq. 3) is solved by projected multivector CG
 * (Table 1) with full re-orthogonalisation and F-normalisation (section 3.3).
 *
 * Conventions shared by every call:
 *  - Every call returns an rpf_status; on failure rpf_last_error() gives a
 *    thread-local message.  No C++ exception crosses the ABI.
 *  - "device" pointers are HIP device memory owned by the caller, which must
 *    stay valid until the work queued on `stream` has completed.  "host"
 *    pointers are read before the call returns and may be freed afterwards.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - Dense matrices are column-major FP64 with an explicit leading dimension.
 *    Interface (lambda-space) blocks are N_lambda x m, row-major: entry (l, j)
 *    at X[l * ldx + j], ldx >= m.
 *  - Handles (rpf_pattern, rpf_problem) own their device memory; free them
 *    with pattern_free / problem_free.  A handle may be used from one thread
 *    (and one stream) at a time.
 */
#ifndef RPFETI_H
#define RPFETI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RPF_OK = 0,
  RPF_EINVAL = -1,      /* bad argument or inconsistent sizes */
  RPF_ENOTSPD = -2,     /* non-positive pivot in a Cholesky factor that must be SPD */
  RPF_EKERNEL = -3,     /* detected kernel dimension differs from the expected one */
  RPF_EBREAKDOWN = -4,  /* every search direction of a block vanished (eta of rank 0) */
  RPF_ENOCONV = -5,     /* max_it reached; outputs hold the last iterate */
  RPF_EHIP = -6,        /* HIP runtime error */
  RPF_ENOMEM = -7       /* device allocation failed */
} rpf_status;

/* Arithmetic of the flexibility product (section 3.2 product S+ W).  FP64 is
 * the plain form.  FP32 stores S+ and W in FP32 with FP32 MFMA accumulation.
 * BF16X3 splits S+ and W into bf16 high and low parts and accumulates the
 * three leading cross products in FP32 on bf16 MFMA.  BF16 uses the high
 * parts only.  Every non-FP64 form is wrapped by FP64 iterative refinement in
 * block_krylov_solve. */
typedef enum { RPF_FP64 = 0, RPF_FP32 = 1, RPF_BF16X3 = 2, RPF_BF16 = 3 } rpf_prec;

typedef struct rpf_pattern_s* rpf_pattern;
typedef struct rpf_problem_s* rpf_problem;

/* Thread-local description of the last failure in this thread. */
const char* rpf_last_error(void);
/* ABI version (major * 100 + minor). */
int32_t rpf_version(void);

/* ------------------------------------------------------------------ patterns */

/* Factor one pattern: interior Cholesky, Schur complement and rigid-mode
 * kernel (section 2: floating subdomains, kernel N, local Schur complement S).
 *
 *  n                  pattern dofs
 *  rowptr, colind     host, CSR structure of the full symmetric K (n+1, nnz);
 *                     every row must hold its diagonal
 *  val                device, nnz FP64 values of K (Neumann stiffness)
 *  n_b, bdofs         host, the boundary dofs t (sorted, distinct, < n)
 *  dofs_per_node      1..3; bdofs must list whole nodes, components consecutive
 *  kernel_tol         Ritz values of S below kernel_tol * ||S||_inf span the
 *                     kernel (1e-10 when <= 0)
 *  expected_kernel_dim  -1 for no check, else RPF_EKERNEL on mismatch
 *  out                receives the handle; *kernel_dim_out the kernel dimension
 *
 * Interior dofs keep their input order; the interior factor exploits the
 * envelope (profile) of K_ii in that order.  Blocks the host until the kernel
 * dimension is known.  Errors: RPF_EINVAL, RPF_ENOTSPD (K_ii not SPD),
 * RPF_EKERNEL, RPF_EHIP, RPF_ENOMEM. */
rpf_status pattern_factor(int32_t n, const int32_t* rowptr, const int32_t* colind, const double* val,
                          int32_t n_b, const int32_t* bdofs, int32_t dofs_per_node, double kernel_tol,
                          int32_t expected_kernel_dim, void* stream, rpf_pattern* out,
                          int32_t* kernel_dim_out);

/* Condense a factored pattern to its boundary flexibility (section 2:
 * S+ = t K+ t^T), taken as the Moore-Penrose pseudo-inverse
 * S+ = (S + Z Z^T)^{-1} - Z Z^T with Z the orthonormal kernel basis.  Always
 * builds the FP64 S+; prec != RPF_FP64 also builds the low-precision copy used
 * by that form.  Asynchronous on `stream`.  Errors: RPF_EINVAL, RPF_ENOTSPD. */
rpf_status pattern_condense(rpf_pattern p, int32_t prec, void* stream);

/* Sizes of a pattern (any output pointer may be NULL). */
rpf_status pattern_info(rpf_pattern p, int32_t* n, int32_t* n_b, int32_t* kernel_dim);

/* Copy a pattern quantity into caller device memory (column-major, ld):
 * what = 0: S (n_b x n_b), 1: Z (n_b x k), 2: S+ (n_b x n_b, after condense).
 * Asynchronous on `stream`. */
rpf_status pattern_export(rpf_pattern p, int32_t what, double* dst, int64_t ld, void* stream);

void pattern_free(rpf_pattern p);

/* ------------------------------------------------------------------ structure */

/* Signed Boolean assembly and permutation structure (eq. 2; section 3.1;
 * section 4.2 for rotations).  All pointers are host pointers, copied by
 * problem_create.
 *
 * A multiplier (node level, dofs_per_node components each, lambda dof
 * l = mult * dofs_per_node + c, expressed in the global frame) joins endpoint
 * 0 (occurrence mult_occ[2i], local node mult_node[2i], sign mult_sign[2i])
 * and endpoint 1 (same at 2i+1; mult_occ = -1 for a single-endpoint
 * multiplier, e.g. a Dirichlet condition imposed in Total FETI fashion).
 * Each endpoint node must be a boundary node of the occurrence's pattern.
 * occ_rot: 9 doubles per occurrence, row-major rotation from the pattern
 * frame to the global frame (used when dofs_per_node == 3), or NULL for
 * identity.  perm_node: n_perm x n_mult, (Pi_k z)[mult] = z[perm_node[k*n_mult+mult]]
 * applied to every component (and, with rotations, turned into the frame of
 * the target multiplier, see feti_permute), or NULL with n_perm == 1
 * (identity).  The solver's multivector is [Pi_0 r, .., Pi_{n_perm-1} r]
 * (section 3.1), so row 0 is normally the identity. */
typedef struct {
  int32_t dofs_per_node;
  int32_t n_patterns;
  const int32_t* pat_n_nodes;    /* [n_patterns] nodes of each pattern */
  const int32_t* pat_bnode_ptr;  /* [n_patterns+1] offsets into pat_bnodes */
  const int32_t* pat_bnodes;     /* sorted boundary nodes of each pattern */
  int32_t n_occ;
  const int32_t* occ_pattern;    /* [n_occ] */
  const double* occ_rot;         /* [9*n_occ] or NULL */
  int32_t n_mult;
  const int32_t* mult_occ;       /* [2*n_mult] */
  const int32_t* mult_node;      /* [2*n_mult] */
  const int8_t* mult_sign;       /* [2*n_mult], +1 or -1 */
  int32_t n_perm;
  const int32_t* perm_node;      /* [n_perm*n_mult] or NULL */
  /* Non-Boolean assembly (section 5: operators from a mortar coupling of non-matching meshes), or
   * all NULL for the signed Boolean one given by mult_node and mult_sign.  Side e of multiplier i
   * couples the entries k = entry_ptr[2i+e] .. entry_ptr[2i+e+1]-1: local node entry_node[k] of
   * occurrence mult_occ[2i+e] with weight entry_weight[k] (the sign included), so that
   * (A^(s) v)[(i, c)] = sum_k entry_weight[k] (O^(s) v[entry_node[k]])[c].  A side has entries
   * exactly when it has an occurrence; every entry node must be a boundary node of its pattern.
   * mult_node and mult_sign stay required: they name one reference node per side, used to
   * validate the structure (the rotation of a permuted multiplier is that of its first side's
   * occurrence, as for the Boolean assembly).  A weighted structure takes no preconditioner
   * (RPF_EINVAL): its multiplicity scaling is defined for the Boolean assembly only. */
  const int32_t* entry_ptr;      /* [2*n_mult+1] or NULL */
  const int32_t* entry_node;     /* [entry_ptr[2*n_mult]] */
  const double* entry_weight;    /* [entry_ptr[2*n_mult]] */
} rpf_problem_desc;

rpf_status problem_create(const rpf_problem_desc* desc, rpf_problem* out);
int64_t problem_n_lambda(rpf_problem pb);
int32_t problem_n_perm(rpf_problem pb);  /* permutations of the structure (1: none) */
void problem_free(rpf_problem pb);

/* Schedules of the flexibility products (section 3.2: the product S+ W over
 * all occurrences of a pattern, here over all patterns at once).  A schedule
 * for block width m and arithmetic prec names the workgroup tile: 0 = the
 * built-in size rule (default); 64 or 128 = every pattern's product in one
 * grouped persistent launch of that tile, each pattern's K split into pieces so
 * that its tiles times pieces reach about `work` items (at most 8 pieces of at
 * least 256); 256 = the large-tile kernel of a single-pattern structure.
 * Schedules change the summation order of the products, so results differ in
 * the last bits between schedules, never in accuracy.  FP32 takes tile 0 only.
 * problem_set_schedule installs one (tile 0 removes it).  Errors: RPF_EINVAL. */
rpf_status problem_set_schedule(rpf_problem pb, int32_t m, int32_t prec, int32_t tile, int32_t work);

typedef struct {
  int32_t tile;
  int32_t work;
  double ms;       /* mean time of one operator application Y = F X (gather, products, scatter) */
  int32_t chosen;  /* 1 for the installed (fastest) candidate */
} rpf_schedule_entry;

/* Autotuner: time every candidate schedule (tile 0; tiles 64 and 128 with work
 * 256 .. 4096; tile 256 where it applies) on this structure for an m-column
 * block in arithmetic prec, `reps` applications each after one warm-up, on
 * `stream`, with a deterministic test block; install the fastest.  out
 * (host, max_out entries, may be NULL) receives every candidate with its time;
 * *n_out the candidate count.  Allocates two N_lambda x m blocks for the
 * duration of the call and blocks the host.  Errors: RPF_EINVAL. */
rpf_status problem_tune(rpf_problem pb, const rpf_pattern* patterns, int32_t m, int32_t prec, int32_t reps,
                        rpf_schedule_entry* out, int32_t max_out, int32_t* n_out, void* stream);

/* ------------------------------------------------------------------ operator */

#define RPF_APPLY_PROJECT 1u  /* return Q^T F X instead of F X (Q: coarse projector, F~ = I) */

/* Y = F X for an m-column interface block (section 2: F = sum_s A^(s) S+ A^(s)T,
 * computed pattern by pattern as one product S+ W over all occurrences,
 * section 3.2).  patterns: host array of the factored and condensed handles,
 * indexed like the structure's patterns.  X, Y: device, N_lambda x m
 * row-major (ldx, ldy >= m), must not overlap.  prec selects the product
 * arithmetic (the pattern must have been condensed with it).  With
 * RPF_APPLY_PROJECT the coarse projector Q = I - G (G^T G)^{-1} G^T is
 * applied to the result (built on first use).  Asynchronous.
 * Errors: RPF_EINVAL. */
rpf_status feti_apply(rpf_problem pb, const rpf_pattern* patterns, int32_t m, const double* X, int64_t ldx,
                      double* Y, int64_t ldy, int32_t prec, uint32_t flags, void* stream);

/* Y = F X in FP64 without allocating device memory, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, layouts and results as feti_apply with
 * prec = RPF_FP64 and flags = 0, on the same kernels.  The W-format workspace
 * (gathered blocks, product results and split-K slabs) lives in a fixed device
 * array of RPF_NOALLOC_SCRATCH_BYTES per GPU, reserved when the library is
 * loaded on that GPU and held until the process ends; its address is looked up
 * on the first call on each device (the current device).  Every call on a GPU
 * shares that array: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.  Each call overwrites
 * every workspace entry it reads, so nothing carries over between calls.
 * Errors: RPF_EINVAL for prec != RPF_FP64, any flag, bad blocks, patterns not
 * condensed, or a block whose workspace exceeds the limit (the message gives
 * the bytes needed; fewer columns per call fit).  Asynchronous. */
#define RPF_NOALLOC_SCRATCH_BYTES (128ll << 20)
rpf_status feti_apply_noalloc(rpf_problem pb, const rpf_pattern* patterns, int32_t m, const double* X, int64_t ldx,
                              double* Y, int64_t ldy, int32_t prec, uint32_t flags, void* stream);

/* Preconditioners of the interface problem (section 2).  F~^{-1} =
 * sum_s beta A^(s) M A^(s)T beta, with M the pattern's Schur complement S
 * (Dirichlet) or its boundary block K_bb (lumped), over the whole pattern
 * boundary and shared by every occurrence of the pattern.  The scaling beta
 * is (A A^T)^{-1}, with A = [.. A^(s) ..] the signed Boolean assembly.  Where
 * no two multipliers share an endpoint it is the diagonal multiplicity scaling
 * (1/2 on an interface multiplier, 1 on a single-endpoint one), whose sum over
 * the subdomains is the identity.  Where multipliers chained at a cross-point
 * share endpoints it couples them, and keeps sum_s beta A^(s) A^(s)T = I. */
typedef enum { RPF_PRECOND_NONE = 0, RPF_PRECOND_LUMPED = 1, RPF_PRECOND_DIRICHLET = 2 } rpf_precond;

/* Y = F~^{-1} X for an m-column interface block (section 2, preconditioners;
 * Table 1 applies it as z = Q F~^{-1} r).  kind: an rpf_precond value
 * (RPF_PRECOND_NONE copies X).  prec: the arithmetic of the Dirichlet
 * product S W (as for feti_apply; the patterns must have been condensed with
 * it); the lumped product with the sparse K_bb always runs in FP64.  With
 * RPF_APPLY_PROJECT the coarse projector Q is applied to the result.  X, Y:
 * device, N_lambda x m row-major (ldx, ldy >= m), must not overlap.  patterns
 * may be NULL only for RPF_PRECOND_NONE without projection.  Asynchronous.
 * Errors: RPF_EINVAL. */
rpf_status feti_precond(rpf_problem pb, const rpf_pattern* patterns, int32_t m, const double* X, int64_t ldx,
                        double* Y, int64_t ldy, int32_t kind, int32_t prec, uint32_t flags, void* stream);

/* Permuted multivector (section 3.1): W[:, l*n_perm + k] = Pi_k z_l for the
 * nr columns of Z and the structure's n_perm permutations (the rows of
 * perm_node; a structure created without permutations has n_perm = 1 and
 * Pi_0 = identity).  With rotated
 * occurrences each moved multiplier is turned into the frame of its new
 * place, O_t O_s^T z (O_t, O_s: rotations of the first-endpoint occurrences
 * of the target and source multipliers; section 4.2).  With
 * RPF_APPLY_PROJECT, W <- Q W (the re-projection of the solver; needs the
 * patterns, else patterns may be NULL).  Z: device, N_lambda x nr row-major
 * (ldz >= nr); W: device, N_lambda x (nr*n_perm) row-major
 * (ldw >= nr*n_perm); must not overlap.  Asynchronous.  Errors: RPF_EINVAL. */
rpf_status feti_permute(rpf_problem pb, const rpf_pattern* patterns, int32_t nr, const double* Z, int64_t ldz,
                        double* W, int64_t ldw, uint32_t flags, void* stream);

/* ------------------------------------------------------------------ solver */

typedef enum {
  RPF_CLASSICAL = 0,   /* projected CG per load case (Table 1, left column; FETI-mrhs) */
  RPF_BLOCK_CG = 1,    /* multivector CG, recurrence on the previous block (Table 1, right) */
  RPF_ORTHODIR = 2     /* multivector CG with full re-orthogonalisation (section 3.3) */
} rpf_method;

typedef struct {
  double tol;          /* stop when max_c ||r_c|| / ||r0_c|| <= tol, r = Q^T (d - F lambda) in FP64 */
  int32_t max_it;      /* total inner iterations allowed */
  int32_t method;      /* rpf_method */
  int32_t prec;        /* rpf_prec of the inner operator */
  double inner_tol;    /* relative reduction per refinement sweep (mixed forms; 0: 1e-4) */
  int32_t max_sweeps;  /* sweeps, each restarting from the FP64 residual of the current iterate
                          (0: 30 for the mixed forms, 4 for FP64, where a further sweep only runs
                          when the recursive residual met tol and the recomputed one did not) */
  int32_t check_every; /* read the convergence flag every k iterations (0: 1) */
  int32_t max_blocks;  /* ORTHODIR: stored (W, P) blocks before a restart (0: as many as max_it and
                          half of the free device memory allow) */
  int32_t precond;     /* rpf_precond: z = Q F~^{-1} r in every iteration (Table 1: initial and updated search directions);
                          the Dirichlet product runs in the inner precision prec.  The projector
                          keeps the identity in place of F~^{-1} unless coarse says otherwise. */
  int32_t periodic;    /* 1: truly periodic structure (section 3.1, after Table 1): with several
                          permutations, Q F of the multivector is the permuted Q F z of the nr
                          columns of z, and the orthogonalisation applies its coefficients to the
                          stored P blocks too, so each iteration runs one product on nr columns.
                          The commutation of Q F (and of the preconditioner) with the permutations
                          is checked once on a test vector: RPF_EINVAL when it fails.  Ignored
                          for the classical method and with one permutation. */
  int32_t coarse;      /* rpf_precond used as F~^{-1} in the projector and in lambda_0 (section 2:
                          Q = I - F~^{-1} G (G^T F~^{-1} G)^{-1} G^T, lambda_0 =
                          F~^{-1} G (G^T F~^{-1} G)^{-1} e; RPF_PRECOND_NONE: F~^{-1} = I).  With a
                          preconditioner the residuals and the products take Q^T and the
                          directions Q.  Each projection applies F~^{-1} once: in FP64 for the
                          directions and the sweeps' residuals, in the inner precision for the
                          products' Q^T (the difference lies in range G); the direction's Q is
                          skipped when precond equals coarse and F~^{-1} runs in FP64 (then
                          Q F~^{-1} r = F~^{-1} r).  G^T F~^{-1} G is assembled and inverted at
                          the first solve for the
                          pattern handles (RPF_ENOTSPD when it is not positive definite or a
                          relative pivot L_ii^2 / H_ii falls below 1e-10: with patterns that have
                          no interior dofs, S = K_bb = K annihilates the rigid traces and
                          G^T F~^{-1} G is singular).
                          RPF_EINVAL together with an active periodic shortcut. */
  int32_t graph_batch; /* 0 or 1: off.  Otherwise batches of iterations are recorded once into HIP
                          graphs on a capture stream of the library and replayed on `stream`, with
                          one convergence check per replay (so a converged run may do up to
                          2 * graph_batch extra, still valid, iterations).  Block CG and classical:
                          from the third iteration of each sweep on, one graph of graph_batch
                          iterations (rounded down to even).  ORTHODIR: one graph per starting
                          place 0, graph_batch, 2 graph_batch, ... of the restart cycle
                          (max_blocks stored blocks), each captured the first time the cycle
                          reaches it after the first iteration of the sweep; a batch that would
                          cross a restart runs uncaptured, and
                          nothing is captured when the cycle is not shorter than max_it.  Same
                          results as the uncaptured run.  Ignored while tracing is enabled. */
} rpf_solve_opts;

typedef struct {
  int32_t iterations;  /* inner iterations over all sweeps */
  int32_t sweeps;      /* FP64 refinement sweeps (1 for the FP64 form) */
  int32_t rank_drops;  /* directions dropped by the F-normalisation */
  int32_t converged;
  double rel_residual; /* final max_c ||r_c|| / ||r0_c||, recomputed in FP64 */
  double ms_loads, ms_coarse, ms_iterate, ms_recover;
  int32_t graph_replays; /* replays of captured iteration batches */
} rpf_solve_stats;

/* Solve the interface problem (eq. 3) for n_rhs load cases and recover the
 * displacements (eq. 2).  f_local: device, the loads of every occurrence in
 * its pattern frame, occurrence blocks concatenated in occurrence order, each
 * n_p x n_rhs column-major (ld n_p).  lambda: device, N_lambda x n_rhs
 * row-major (ld_lambda >= n_rhs).  u_local: device, same layout as f_local.
 * lambda_00 = 0.  Blocks until the solve completes; stats may be NULL.
 * Errors: RPF_EINVAL, RPF_EBREAKDOWN, RPF_ENOCONV (outputs hold the last
 * iterate), RPF_EHIP. */
rpf_status block_krylov_solve(rpf_problem pb, const rpf_pattern* patterns, int32_t n_rhs, const double* f_local,
                              const rpf_solve_opts* opts, double* lambda, int64_t ld_lambda, double* u_local,
                              rpf_solve_stats* stats, void* stream);

/* ------------------------------------------------------------------ tracing */

/* Kernel timing of the flexibility product (section 3.2: S+ W over all the
 * occurrences of a pattern), the hot kernel of every iteration.  While enabled,
 * every such product launched by feti_apply or block_krylov_solve is bracketed
 * by HIP events on its own stream.  rpf_trace_read synchronises those events,
 * returns the number of products computed in precision prec (an rpf_prec
 * value; prec < 0 counts every product), their summed duration in ms and their
 * algorithmic flop count (2 n_b^2 columns each), then drops every recorded
 * product, counted or not.  A low-precision solve also runs FP64 products (the
 * residuals of its refinement sweeps): read them with prec = RPF_FP64.
 * Process-wide; not meant for concurrent solves. */
rpf_status rpf_trace_enable(int32_t on);
rpf_status rpf_trace_read(int32_t prec, int64_t* count, double* total_ms, double* flops);

/* ------------------------------------------------------------------ dense helpers */

/* C = alpha op(A) op(B) + beta C, FP64 MFMA, column-major (ta, tb: 0 or 1). */
rpf_status rpf_dgemm(int32_t ta, int32_t tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                     int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                     void* stream);
/* In-place lower Cholesky of an SPD n x n matrix (device), then, when nrhs > 0,
 * B <- A^{-1} B.  Blocks the host.  RPF_ENOTSPD on a non-positive pivot. */
rpf_status rpf_dposv(int64_t n, double* A, int64_t lda, int64_t nrhs, double* B, int64_t ldb, void* stream);
/* Symmetric eigen-decomposition of batch m x m matrices (m <= 64), ascending. */
rpf_status rpf_dsyev_small(int32_t m, int32_t batch, const double* A, double* V, double* w, void* stream);
/* Row-block products of the multivector solver (section 3.3: F-orthogonalisation of a new block
 * against every stored block, and the block updates of Table 1).  X (N x a) and Y (N x b) are
 * row-major device blocks with leading dimensions ldx >= a and ldy >= b.
 * rpf_rows_gemm: Y <- beta Y + alpha X M.  M (a x b, device) is row-major with row stride
 * mrow >= b, or column-major with leading dimension a when mrow = 0.  Y must not overlap X or M;
 * with beta = 0 the old Y is not read.  Asynchronous on stream.
 * rpf_gram: C <- X^T Y, C (a x b, device) column-major with leading dimension a.  The partial
 * sums over row chunks are added in a fixed order.  Allocates its workspace and blocks the host
 * until the result is written.
 * Both: RPF_EINVAL for negative sizes (rpf_rows_gemm: a < 1) or leading dimensions below the
 * widths; nothing is done when N or b is 0, or (rpf_gram) a is 0: C is then left untouched. */
rpf_status rpf_rows_gemm(int64_t N, int32_t a, int32_t b, double alpha, const double* X, int64_t ldx,
                         const double* M, int64_t mrow, double beta, double* Y, int64_t ldy, void* stream);
rpf_status rpf_gram(int64_t N, int32_t a, int32_t b, const double* X, int64_t ldx, const double* Y, int64_t ldy,
                    double* C, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RPFETI_H */
