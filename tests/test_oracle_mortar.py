"""Pins of the non-Boolean (mortar) assembly of non-matching pattern meshes (section 5: non-Boolean
assembly operators transport information between discretisations as rotations do between frames).

The coupling weights come from the dual-multiplier mortar method (workloads.mortar_weights_1d).
Pinned here: exact reproduction of linear fields by the weights and by the assembled constraints,
agreement of the oracle's FETI solutions with a dense saddle-point solve of the constrained
problem (a different formulation of the same discrete problem), the exact linear solution of a
flux problem across non-matching interfaces, and, on matching meshes, the Boolean assembly."""
import dataclasses

import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.mark.parametrize("ns,nm", [(7, 9), (9, 7), (5, 13), (8, 8)])
def test_weights_reproduce_linear_fields(ns, nm):
    rng = np.random.default_rng(ns * 31 + nm)
    xs = np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0, 1, ns - 2)]))
    xm = np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0, 1, nm - 2)]))
    Wt = W.mortar_weights_1d(xs, xm)
    assert np.abs(Wt.sum(axis=1) - 1.0).max() < 1e-13
    for a, b in ((1.0, 0.0), (0.3, -2.0)):
        assert np.abs(Wt @ (a + b * xm) - (a + b * xs)).max() < 1e-13
    # not exact beyond linear fields (a real projection, not an interpolation that happens to fit)
    if ns != nm:
        assert np.abs(Wt @ xm ** 2 - xs ** 2).max() > 1e-4
    if ns == nm:
        Wm = W.mortar_weights_1d(xs, xs)
        assert np.abs(Wm - np.eye(ns)).max() < 1e-13


def _cut_field(p, fn):
    """A global field fn(x) on every occurrence, as (n_p, 1) local vectors (pattern frame = global)."""
    out = []
    for s in range(p.n_occ):
        pat = p.patterns[p.occ_pattern[s]]
        x = pat.coords.copy()
        x[:, 0] += s
        out.append(fn(x).reshape(-1, 1))
    return out


@pytest.mark.parametrize("kind", ["heat", "elast"])
def test_constraints_vanish_on_linear_fields(kind):
    """B u = sum_s A^(s) t u^(s) = 0 for every globally linear field (the mortar coupling passes the
    patch test), including rigid motions; a quadratic field violates the constraints."""
    if kind == "heat":
        p = W.mortar_row("heat", shapes=((8, 8), (6, 6)), n_occ=3)
        lin = [lambda x: 1.0 + 0 * x[:, 0], lambda x: x[:, 0] - 2 * x[:, 1] + 0.5]
        quad = lambda x: x[:, 1] ** 2
    else:
        p = W.mortar_row("elast", shapes=((3, 3, 3), (2, 2, 2)), n_occ=3)
        Amat = np.array([[0.1, -0.3, 0.2], [0.4, 0.05, -0.1], [-0.2, 0.3, 0.15]])
        lin = [lambda x: (x @ Amat.T + np.array([1.0, -2.0, 0.5])),
               lambda x: np.stack([-x[:, 1], x[:, 0], 0 * x[:, 2]], axis=1)]
        quad = lambda x: np.stack([x[:, 1] ** 2, 0 * x[:, 0], x[:, 2] * x[:, 1]], axis=1)
    o = O.FetiOracle(p)
    inter = np.repeat(p.mult_occ[:, 1] >= 0, p.dpn)   # the Dirichlet rows constrain u = 0 only

    def gap(fn):
        u = _cut_field(p, fn)
        return np.abs(sum(o.A[s] @ u[s][o.pats[p.occ_pattern[s]].b] for s in range(p.n_occ))[inter]).max()

    for fn in lin:
        assert gap(fn) < 1e-13
    assert gap(quad) > 1e-4


@pytest.mark.parametrize("kind,shapes,n_occ", [("heat", ((8, 8), (6, 6)), 4), ("heat", ((5, 7), (9, 4)), 3),
                                               ("elast", ((3, 3, 3), (2, 2, 2)), 3)])
def test_feti_equals_constrained_solve(kind, shapes, n_occ):
    """Classical and multivector FETI on non-matching occurrences reach the dense saddle-point solve
    of the constrained problem (u and lambda)."""
    p = W.mortar_row(kind, shapes=shapes, n_occ=n_occ, n_rhs=2)
    o = O.FetiOracle(p)
    ub, lb = O.constrained_solve(p, o)
    scale = max(np.abs(b).max() for b in ub)
    for meth in ("classical", "block"):
        lam, u, _ = o.solve(meth, tol=1e-12)
        assert max(np.abs(a - b).max() for a, b in zip(u, ub)) < 1e-10 * scale, meth
        assert np.abs(lam - lb).max() < 1e-9 * np.abs(lb).max(), meth


def test_flux_problem_is_exactly_linear():
    """u = 0 on x = 0, unit flux out of x = n_occ, no source, conductivity 1: the exact solution
    u = x is linear, and the mortar coupling reproduces it at every node of both meshes."""
    p = W.mortar_row("heat", shapes=((8, 8), (6, 6)), n_occ=4, load="flux")
    o = O.FetiOracle(p)
    for meth in ("classical", "block"):
        _, u, _ = o.solve(meth, tol=1e-13)
        ref = _cut_field(p, lambda x: x[:, 0])
        assert max(np.abs(a - b).max() for a, b in zip(u, ref)) < 1e-12, meth


def test_matching_meshes_give_the_boolean_assembly():
    """With equal meshes the mortar weights are the identity: the weighted assembly equals the
    signed Boolean one built from the same multipliers, and so do the solutions."""
    p = W.mortar_row("heat", shapes=((6, 6), (6, 6)), n_occ=3, n_rhs=1)
    assert np.allclose(np.abs(p.entry_weight), 1.0)
    pb = dataclasses.replace(p, entry_ptr=None, entry_node=None, entry_weight=None)
    ow, ob = O.FetiOracle(p), O.FetiOracle(pb)
    for s in range(p.n_occ):
        assert abs(ow.A[s] - ob.A[s]).max() < 1e-14
    lw, uw, _ = ow.solve("block", tol=1e-12)
    lb, ub, _ = ob.solve("block", tol=1e-12)
    assert np.abs(lw - lb).max() < 1e-12 * np.abs(lb).max()
