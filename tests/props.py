"""Properties that characterise the solution of a repeated-pattern structure at any size, computed on
the CPU from the problem statement alone (no FETI arithmetic, no oracle):

* interface continuity: the two endpoint displacements of every interface multiplier agree
  (eq. 2, B u = 0), in the global frame;
* the Dirichlet condition: u = 0 at the node of every single-endpoint multiplier;
* local equilibrium of every occurrence: K^(s) u^(s) = f^(s) - t^T A^(s)T lambda (the rows of
  eq. 2 of each subdomain).
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np


def stack_u(p, u):
    """(n_occ, n_nodes, dpn, n_rhs) view of the displacements (single-pattern structures)."""
    nn = p.patterns[0].n_nodes
    return np.stack(u).reshape(p.n_occ, nn, p.dpn, -1)


def continuity_gap(p, u):
    """max over interface multipliers of |O_a u_a - O_b u_b| (global frame)."""
    dpn = p.dpn
    U = stack_u(p, u)
    inter = np.nonzero(p.mult_occ[:, 1] >= 0)[0]
    gap = 0.0
    for chunk in np.array_split(inter, 16):
        sa, na = p.mult_occ[chunk, 0], p.mult_node[chunk, 0]
        sb, nb = p.mult_occ[chunk, 1], p.mult_node[chunk, 1]
        ua, ub = U[sa, na], U[sb, nb]
        if p.has_rotation:
            ua = np.einsum("kab,kbr->kar", p.occ_rot[sa][:, :dpn, :dpn], ua)
            ub = np.einsum("kab,kbr->kar", p.occ_rot[sb][:, :dpn, :dpn], ub)
        gap = max(gap, np.abs(ua - ub).max())
    return gap


def dirichlet_max(p, u):
    """max |u| over the nodes held by single-endpoint (Dirichlet) multipliers."""
    dsel = np.nonzero(p.mult_occ[:, 1] < 0)[0]
    if len(dsel) == 0:
        return 0.0
    return float(np.abs(stack_u(p, u)[p.mult_occ[dsel, 0], p.mult_node[dsel, 0]]).max())


def local_forces_all(p, lam):
    """t^T A^(s)T lambda for every occurrence (pattern frame), as (n_occ, n_nodes, dpn, n_rhs)."""
    dpn = p.dpn
    nn = p.patterns[0].n_nodes
    nr = lam.shape[1]
    out = np.zeros((p.n_occ, nn, dpn, nr))
    lm = lam.reshape(p.n_mult_nodes, dpn, nr)
    for e in range(2):
        sel = np.nonzero(p.mult_occ[:, e] >= 0)[0]
        s = p.mult_occ[sel, e]
        sg = p.mult_sign[sel, e].astype(float)
        loc = lm[sel] * sg[:, None, None]
        if p.has_rotation and dpn > 1:
            loc = np.einsum("kca,kcr->kar", p.occ_rot[s][:, :dpn, :dpn], loc)   # O^T lambda
        np.add.at(out, (s, p.mult_node[sel, e]), loc)
    return out


def equilibrium_residual(p, u, lam, threads=8):
    """max over every occurrence and load case of |K u - f + t^T A^T lambda| / max |f| (single-pattern
    structures); the sparse products run on a few host threads."""
    K = p.patterns[0].K.tocsr()
    n = K.shape[0]
    nr = lam.shape[1]
    U = np.concatenate(u, axis=1)                     # (n, n_occ * nr)
    F = np.concatenate(p.f_local, axis=1)
    B = local_forces_all(p, lam).reshape(p.n_occ, n, nr).transpose(1, 0, 2).reshape(n, -1)
    cols = U.shape[1]
    step = max(1, -(-cols // threads))

    def part(c):
        sl = slice(c, min(c + step, cols))
        return np.abs(K @ np.ascontiguousarray(U[:, sl]) - F[:, sl] + B[:, sl]).max()

    with ThreadPoolExecutor(threads) as ex:
        worst = max(ex.map(part, range(0, cols, step)))
    return float(worst / np.abs(F).max())


def rel_err(u, u_ref):
    """max |u - u_ref| / max |u_ref| over every occurrence."""
    scale = max(np.abs(x).max() for x in u_ref)
    return float(max(np.abs(a - b).max() for a, b in zip(u, u_ref)) / scale)
