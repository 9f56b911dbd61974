// Pattern handle: one factored and condensed pattern (internal).
#pragma once

#include "common.hpp"

struct rpf_pattern_s {
  uint64_t uid = 0;  // unique per handle for the life of the process (cache keys)
  int n = 0, n_b = 0, n_i = 0, dpn = 1, k = 0;
  std::vector<int> bdofs, idofs;  // original dof ids of the boundary / interior rows

  // Dense factor storage, n x n column-major (ld = n), rows/cols ordered
  // interior first then boundary: L_ii (within its envelope), L_bi, and the
  // lower triangle of S in the trailing block.
  rpf::DevBuf<double> L;
  int64_t ld = 0;
  rpf::DevBuf<double> dinv_ii;  // inverses of the NB x NB diagonal blocks of L_ii
  rpf::Envelope env_ii;
  bool L_upper = false;         // the upper triangle of L_ii's envelope holds L_ii^T

  rpf::DevBuf<double> S;       // n_b x n_b, full, ld n_b
  rpf::DevBuf<double> Z;       // n_b x k orthonormal kernel basis, ld n_b
  rpf::DevBuf<double> Splus;   // n_b x n_b FP64 pseudo-inverse, ld n_b
  rpf::DevBuf<float> Splus32;  // FP32 copy
  rpf::DevBuf<uint16_t> Sp_hi, Sp_lo;  // bf16 split of S+ (bit patterns), n_b rows of ldlp, zero padded
  int64_t ldlp = 0;
  uint32_t condensed = 0;      // bit per rpf_prec built
  // the same low-precision copies of S, for the Dirichlet preconditioner of the low-precision solves
  rpf::DevBuf<float> S32;
  rpf::DevBuf<uint16_t> S_hi, S_lo;

  // K_bi (rows: boundary index, cols: interior index) and K_ib, CSR, for the
  // condensed loads g = f_b - K_bi K_ii^{-1} f_i and the interior recovery
  rpf::DevBuf<int> kbi_ptr, kbi_col, kib_ptr, kib_col;
  rpf::DevBuf<double> kbi_val, kib_val;
  // K_bb (boundary x boundary), CSR: the local matrix of the lumped preconditioner
  rpf::DevBuf<int> kbb_ptr, kbb_col;
  rpf::DevBuf<double> kbb_val;
  rpf::DevBuf<int> d_bdofs, d_idofs;

  rpf::DevBuf<int> status;
};
