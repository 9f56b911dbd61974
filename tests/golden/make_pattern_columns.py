"""Write tests/golden/elast20_pattern_columns.npz: sampled entries of the oracle's S, S+ and Z Z^T
for the 20^3-brick elasticity pattern (the 512-occurrence workload's pattern, n = 27,783,
n_b = 7,206).

Only the CPU oracle and the seeded workload generator are called (section 2: S = K_bb - K_bi
K_ii^{-1} K_ib, S+ = (S + Z Z^T)^{-1} - Z Z^T with Z an orthonormal basis of ker S).  The full
matrices are 7,206^2 each, so the file keeps, for COLS seeded columns:
  * the entries at ROWS seeded rows (and the diagonal entry of each column),
  * the 2-norm of each whole column,
  * the dot product of each whole column with a seeded N(0,1) weight vector
    (numpy Generator(PCG64(WEIGHT_SEED)).standard_normal(n_b)),
which pin every entry of those columns in aggregate and a sample of them one by one.

Usage (about ten minutes on 8 cores):  python tests/golden/make_pattern_columns.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "elast20_pattern_columns.npz")
SAMPLE_SEED = 20086387
WEIGHT_SEED = 30086387
COLS = 8
ROWS = 768


def main() -> None:
    t0 = time.time()
    p = W.config(4)
    pat = p.patterns[0]
    print(f"pattern n={pat.n} n_b={pat.n_b}", flush=True)
    po = O.PatternOracle(pat.K, pat.bdofs, pat.kernel_dim)
    print(f"oracle condensation {time.time() - t0:.1f} s, kernel dim {po.k}", flush=True)
    nb = po.n_b
    rng = np.random.default_rng(SAMPLE_SEED)
    cols = np.sort(np.concatenate([[0, nb - 1], rng.choice(np.arange(1, nb - 1), COLS - 2, replace=False)]))
    rows = np.sort(rng.choice(nb, ROWS, replace=False))
    w = np.random.default_rng(WEIGHT_SEED).standard_normal(nb)
    P = po.Z @ po.Z.T
    out = dict(cols=cols.astype(np.int64), rows=rows.astype(np.int64), n_b=np.int64(nb), kernel_dim=np.int64(po.k),
               weight_seed=np.int64(WEIGHT_SEED))
    for name, M in (("S", po.S), ("Splus", po.Splus), ("ZZt", P)):
        C = M[:, cols]
        out[name + "_rows"] = C[rows]
        out[name + "_diag"] = M[cols, cols]
        out[name + "_norm"] = np.linalg.norm(C, axis=0)
        out[name + "_wdot"] = w @ C
        out[name + "_absmax"] = np.float64(np.abs(M).max())
    np.savez_compressed(OUT, **out)
    print(f"wrote {OUT} in {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
