"""Marshal a structure description (patterns, occurrences, multipliers) into library objects.

The description is any object with the attributes of a repeated-pattern
problem statement: ``patterns`` (each with ``K`` as a SciPy CSR matrix,
``bdofs``, ``bnodes``, ``dpn``, ``n_nodes``, ``kernel_dim``), ``occ_pattern``,
``occ_rot``, ``mult_occ``, ``mult_node``, ``mult_sign``, ``perm_node``,
``f_local`` and ``n_rhs``.  Only argument marshalling happens here.
"""
from __future__ import annotations

import numpy as np
import torch

from . import FP64, Pattern, Problem, pattern_condense, pattern_factor, problem_create, problem_set_schedule


def factor_patterns(desc, check_kernel: bool = True, stream=None):
    out = []
    for pat in desc.patterns:
        K = pat.K
        val = torch.from_numpy(np.ascontiguousarray(K.data, dtype=np.float64)).cuda()
        out.append(pattern_factor(K.indptr, K.indices, val, pat.bdofs, pat.dpn,
                                  expected_kernel_dim=pat.kernel_dim if check_kernel else -1, stream=stream))
    return out


def condense_patterns(patterns, precs=(FP64,), stream=None):
    for p in patterns:
        for prec in precs:
            pattern_condense(p, prec, stream=stream)


def create_problem(desc, weighted: bool | None = None) -> Problem:
    """weighted: pass the assembly as weighted entries (None: when the description has them; True
    also describes a Boolean assembly through its one-node, signed entries)."""
    rot = desc.occ_rot if desc.has_rotation else None
    use_w = getattr(desc, "entry_ptr", None) is not None if weighted is None else weighted
    return problem_create(desc.dpn, [p.n_nodes for p in desc.patterns], [p.bnodes for p in desc.patterns],
                          desc.occ_pattern, rot, desc.mult_occ, desc.mult_node, desc.mult_sign,
                          desc.perm_node if desc.perm_node.shape[0] > 1 else None,
                          entries=desc.entries() if use_w else None)


def loads_to_device(desc) -> torch.Tensor:
    """Concatenate per-occurrence loads (n_p x n_rhs, column-major) into one device vector."""
    flat = np.concatenate([np.asarray(f, dtype=np.float64).T.ravel() for f in desc.f_local])
    return torch.from_numpy(flat).cuda()


def split_u(desc, u: torch.Tensor):
    """Inverse of loads_to_device for the displacement output: list of (n_p, n_rhs) host arrays."""
    h = u.cpu().numpy()
    out, o = [], 0
    for s, p in enumerate(desc.occ_pattern):
        n = desc.patterns[p].n
        blk = h[o:o + n * desc.n_rhs].reshape(desc.n_rhs, n).T
        out.append(blk)
        o += n * desc.n_rhs
    return out


def install_schedules(pb: Problem, desc, table: dict | None = None) -> dict:
    """Install the tuned product schedules recorded for this structure (schedules.json, written by
    python -m paper_1208_6387_amd.tune); returns {(block size, form): (tile, work)} of those installed
    (tile 0: one launch per pattern, else the grouped launch over all patterns with that tile)."""
    from .tune import FORMS, load_table, signature
    table = load_table() if table is None else table
    n_occ = list(np.bincount(desc.occ_pattern, minlength=len(desc.patterns)))
    n_b = [p.n_b for p in desc.patterns]
    done = {}
    for m in sorted({desc.n_rhs * desc.n_perm, desc.n_rhs}):
        for form, prec in FORMS.items():
            rec = table.get(signature(n_b, n_occ, m, form))
            if rec:
                problem_set_schedule(pb, m, prec, int(rec["tile"]), int(rec["work"]))
                done[(m, form)] = (int(rec["tile"]), int(rec["work"]))
    return done
