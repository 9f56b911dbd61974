"""The coarse operator G^T F~^{-1} G assembled from the patterns' responses to probed traces of the
coarse modes (section 4.3's pattern-frame assembly, in the form the library uses): occurrences that
meet through a scaling group are neighbours; occurrences two steps apart get different colours; one
probe column per (colour, mode); H[j, i] is the sum over the occurrences s reached by both of
C_s[colour(j), colour(i)], C_s = X_s^T M_s X_s with X_s = A_s^T beta G E.  Checked on the CPU
against the dense product G^T F~^{-1} G of the oracle, with the probes carrying several occurrences.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _groups(p):
    """Multipliers joined through a shared endpoint (occurrence, local node): the blocks of A A^T."""
    nm = p.mult_occ.shape[0]
    parent = list(range(nm))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    at = {}
    for i in range(nm):
        for e in range(2):
            if p.mult_occ[i, e] >= 0:
                at.setdefault((int(p.mult_occ[i, e]), int(p.mult_node[i, e])), []).append(i)
    for lst in at.values():
        for b in lst[1:]:
            ra, rb = find(lst[0]), find(b)
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
    groups = {}
    for i in range(nm):
        groups.setdefault(find(i), []).append(i)
    return list(groups.values())


def _probe_assembly(p, o, kind):
    no = p.n_occ
    nbr = [{s} for s in range(no)]
    for g in _groups(p):
        occs = {int(p.mult_occ[i, e]) for i in g for e in range(2) if p.mult_occ[i, e] >= 0}
        for a in occs:
            nbr[a] |= occs
    k = [int(o.coarse_off[s + 1] - o.coarse_off[s]) for s in range(no)]
    kmax = max(k)
    colour, ncol = [0] * no, 0
    for i in range(no):
        if k[i]:
            taken = {colour[j] for t in nbr[i] for j in nbr[t] if j < i and k[j]}
            c = 0
            while c in taken:
                c += 1
            colour[i], ncol = c, max(ncol, c + 1)
    nG = o.G.shape[1]
    E = np.zeros((nG, ncol * kmax))
    for i in range(no):
        for q in range(k[i]):
            E[o.coarse_off[i] + q, colour[i] * kmax + q] = 1.0
    T = o.scale(o.G @ E)
    C = []
    for s in range(no):
        X = o.A[s].T @ T
        C.append(X.T @ (o.local_precond_matrix(p.occ_pattern[s], kind) @ X))
    H = np.zeros((nG, nG))
    for i in range(no):
        if not k[i]:
            continue
        for j in {j for t in nbr[i] for j in nbr[t] if k[j]}:
            both = [u for u in nbr[i] if j in nbr[u]]
            for a in range(k[j]):
                for b in range(k[i]):
                    H[o.coarse_off[j] + a, o.coarse_off[i] + b] = sum(
                        C[u][colour[j] * kmax + a, colour[i] * kmax + b] for u in both)
    return H, ncol


CASES = {
    "elast-2cube-4x4x4": (lambda: W.small_elast((2, 2, 2), (4, 4, 4), n_rhs=1, seed=1), 27),
    "ring12-elast-rotated": (lambda: W.ring_elast(12, (1, 2, 1), n_rhs=1, n_perm=2), 3),
    "heat-6x5": (lambda: W.small_heat((3, 3), (6, 5), n_rhs=1, seed=2), None),
}


@pytest.mark.parametrize("kind", ["lumped", "dirichlet"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_probe_assembly_equals_dense_coarse_operator(case, kind):
    make, want_colours = CASES[case]
    p = make()
    o = O.FetiOracle(p, coarse=kind)
    G = o.G.toarray()
    H_ref = G.T @ o.precondition(G, kind)
    H, ncol = _probe_assembly(p, o, kind)
    assert ncol < p.n_occ                        # probes carry several occurrences
    if want_colours is not None:
        assert ncol == want_colours
    assert np.abs(H - H_ref).max() <= 1e-12 * np.abs(H_ref).max()


def test_probe_assembly_fails_with_one_step_colouring():
    """Colouring only direct neighbours apart lets two modes share a probe on some occurrence: its
    response block for that colour then mixes two occurrences' traces (the two-step rule is needed)."""
    p = W.small_elast((2, 2, 2), (4, 4, 4), n_rhs=1, seed=1)
    o = O.FetiOracle(p, coarse="lumped")
    G = o.G.toarray()
    no = p.n_occ
    nbr = [{s} for s in range(no)]
    for g in _groups(p):
        occs = {int(p.mult_occ[i, e]) for i in g for e in range(2) if p.mult_occ[i, e] >= 0}
        for a in occs:
            nbr[a] |= occs
    colour, ncol = [0] * no, 0
    for i in range(no):
        taken = {colour[j] for j in nbr[i] if j < i}
        c = 0
        while c in taken:
            c += 1
        colour[i], ncol = c, max(ncol, c + 1)
    assert ncol == 8
    # an occurrence reached by two occurrences of one colour
    s, i, i2 = next((s, a, b) for s in range(no) for a in sorted(nbr[s]) for b in sorted(nbr[s])
                    if a < b and colour[a] == colour[b])
    M = o.local_precond_matrix(p.occ_pattern[s], "lumped")
    E = np.zeros((G.shape[1], 6))
    for occ in range(no):
        if colour[occ] == colour[i]:
            E[o.coarse_off[occ]:o.coarse_off[occ + 1], :] = np.eye(6)
    Xc = o.A[s].T @ o.scale(G @ E)
    Xi = o.A[s].T @ o.scale(G[:, o.coarse_off[i]:o.coarse_off[i + 1]])
    mixed, exact = Xc.T @ (M @ Xc), Xi.T @ (M @ Xi)
    assert np.abs(mixed - exact).max() > 1e-3 * np.abs(exact).max()


@pytest.mark.parametrize("kind", ["lumped", "dirichlet"])
def test_coarse_operator_singular_without_interior_dofs(kind):
    """With no interior dofs the local matrix is K itself (S = K_bb = K): the rigid traces are in its
    kernel and G^T F~^{-1} G is singular; one interior layer makes it definite."""
    for pe, singular in [(1, True), (2, False)]:
        p = W.small_elast((pe, pe + 1, pe), (1, 1, 2), n_rhs=1, seed=0)
        o = O.FetiOracle(p, coarse=kind)
        G = o.G.toarray()
        w = np.linalg.eigvalsh(G.T @ o.precondition(G, kind))
        assert (w.min() < 1e-12 * w.max()) == singular, (pe, w.min(), w.max())
