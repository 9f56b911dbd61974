"""The CPU property checks used at full size (tests/props.py), pinned on small structures: they
read (near) zero on the assembled global solution with the oracle's multipliers, and they catch a
perturbed displacement, a perturbed multiplier and a wrong sign."""
import numpy as np

import oracle as O
import props
import workloads as W


def _exact(p):
    u, _, _, _ = O.global_solve(p)
    o = O.FetiOracle(p)
    lam = O.multipliers_from_displacements(o, u)
    return u, lam


def test_properties_vanish_on_the_global_solution():
    p = W.small_elast((3, 3, 3), (3, 2, 2), n_rhs=2, seed=21)
    u, lam = _exact(p)
    scale = max(np.abs(x).max() for x in u)
    assert props.equilibrium_residual(p, u, lam) <= 1e-11
    assert props.continuity_gap(p, u) <= 1e-12 * scale
    assert props.dirichlet_max(p, u) == 0.0
    assert props.rel_err(u, u) == 0.0


def test_properties_catch_mistakes():
    p = W.small_elast((3, 3, 3), (3, 2, 2), n_rhs=2, seed=22)
    u, lam = _exact(p)
    scale = max(np.abs(x).max() for x in u)
    # a displacement moved at one node of one occurrence: equilibrium there breaks
    ub = [x.copy() for x in u]
    ub[3][5] += 1e-3 * scale
    assert props.equilibrium_residual(p, ub, lam) > 1e-6
    # an interface node moved on one side only: continuity breaks
    inter = np.nonzero(p.mult_occ[:, 1] >= 0)[0][7]
    s, nd = p.mult_occ[inter, 0], p.mult_node[inter, 0]
    ub = [x.copy() for x in u]
    ub[s][nd * p.dpn] += 1e-3 * scale
    assert props.continuity_gap(p, ub) > 1e-4 * scale
    # one multiplier perturbed, or every sign flipped
    lb = lam.copy()
    lb[10] += 1e-3 * np.abs(lam).max()
    assert props.equilibrium_residual(p, u, lb) > 1e-6
    assert props.equilibrium_residual(p, u, -lam) > 1e-3
    # a clamped node moved
    d = np.nonzero(p.mult_occ[:, 1] < 0)[0][0]
    ub = [x.copy() for x in u]
    ub[p.mult_occ[d, 0]][p.mult_node[d, 0] * p.dpn + 1] = 1e-3
    assert props.dirichlet_max(p, ub) == 1e-3


def test_properties_with_rotated_occurrences():
    p = W.ring_elast(n_occ=4, n_rhs=1, seed=23)
    assert p.has_rotation
    u, lam = _exact(p)
    scale = max(np.abs(x).max() for x in u)
    assert props.equilibrium_residual(p, u, lam) <= 1e-10
    assert props.continuity_gap(p, u) <= 1e-11 * scale
