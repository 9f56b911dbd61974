"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test names the passage it checks.  A plausible mistake in the oracle (a
dropped term, a wrong sign, a transposed operand) must fail at least one of
them; tests/test_oracle_mutations.py plants such mistakes and checks that.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W
from workloads import mesh as M


# ----------------------------------------------------------------------------- elements

def test_quad_element_closed_form():
    Ke = M.quad_laplace(0.3, 0.3)
    ref = np.array([[4, -1, -2, -1], [-1, 4, -1, -2], [-2, -1, 4, -1], [-1, -2, -1, 4]]) / 6.0
    assert np.abs(Ke - ref).max() < 1e-15


def _rigid_modes(coords):
    n = coords.shape[0]
    R = np.zeros((n, 3, 6))
    for c in range(3):
        R[:, c, c] = 1.0
    x, y, z = coords[:, 0], coords[:, 1], coords[:, 2]
    R[:, 0, 3], R[:, 1, 3] = -y, x          # about z
    R[:, 1, 4], R[:, 2, 4] = -z, y          # about x
    R[:, 0, 5], R[:, 2, 5] = z, -x          # about y
    return R.reshape(3 * n, 6)


def test_hex_element_rank_kernel_and_patch():
    Ke = M.hex_elasticity(0.1, 0.2, 0.15)
    assert np.abs(Ke - Ke.T).max() < 1e-14
    w = np.linalg.eigvalsh(Ke)
    assert (np.abs(w) < 1e-12 * w.max()).sum() == 6
    X = ((M.HEX_NODES + 1) / 2) * np.array([0.1, 0.2, 0.15])
    assert np.abs(Ke @ _rigid_modes(X)).max() < 1e-13 * np.abs(Ke).max()
    # patch test: a linear field on a 2x2x2 patch leaves no force on the centre node
    mesh = M.GridMesh((2, 2, 2), (1.0, 1.3, 0.7))
    K = M.assemble(mesh, M.hex_elasticity(*mesh.h), 3)
    Aff = np.array([[0.3, -0.2, 0.5], [0.1, 0.7, -0.4], [0.6, 0.2, 0.9]])
    u = (mesh.coords @ Aff.T).ravel()
    centre = mesh.node_id([1, 1, 1])
    assert np.abs((K @ u)[3 * centre:3 * centre + 3]).max() < 1e-13


def test_general_hex_matches_box():
    X = ((M.HEX_NODES + 1) / 2) * np.array([0.1, 0.2, 0.15])
    assert np.abs(M.hex_elasticity_general(X) - M.hex_elasticity(0.1, 0.2, 0.15)).max() < 1e-13


# ----------------------------------------------------------------------------- generator

def test_grid_structure_matches_directly_meshed_global_grid():
    """Occurrences placed on the grid assemble to the stiffness of the directly meshed domain."""
    p = W.small_elast((2, 3, 2), (2, 2, 1))
    _, _, Kocc, _ = O.global_solve(p)
    gm = M.GridMesh((4, 6, 2), (1.0, 1.0, 0.5))
    Kdir = M.assemble(gm, M.hex_elasticity(*gm.h), 3)
    assert abs(Kocc - Kdir).max() < 1e-14


def test_multiplier_counts_config1():
    p = W.config(1)
    pat = p.patterns[0]
    assert pat.n == 6591 and pat.n_b == 2598
    assert p.n_lambda == 76080 and p.n_dirichlet_mult() * 3 == 7203


# ----------------------------------------------------------------------------- pattern level

@pytest.fixture(scope="module")
def elast_small():
    p = W.small_elast((3, 3, 3), (3, 2, 2), n_rhs=2, n_perm=4)
    return p, O.FetiOracle(p)


def test_schur_equals_dense(elast_small):
    p, o = elast_small
    P = o.pats[0]
    K = p.patterns[0].K.toarray()
    b, i = P.b, P.i
    S = K[np.ix_(b, b)] - K[np.ix_(b, i)] @ np.linalg.solve(K[np.ix_(i, i)], K[np.ix_(i, b)])
    assert np.abs(S - P.S).max() < 1e-12 * np.abs(S).max()


def test_kernel_is_rigid_body_motion(elast_small):
    p, o = elast_small
    P = o.pats[0]
    pat = p.patterns[0]
    R = _rigid_modes(pat.coords)
    assert np.abs(pat.K @ R).max() < 1e-13 * abs(pat.K).max()
    assert P.k == 6
    Qr, _ = np.linalg.qr(R[P.b])
    assert np.linalg.norm(P.Z - Qr @ (Qr.T @ P.Z)) < 1e-10
    assert np.abs(P.Z.T @ P.Z - np.eye(6)).max() < 1e-13
    # N spans the kernel of K
    assert np.abs(pat.K @ P.N).max() < 1e-11


def test_heat_kernel_is_constant():
    p = W.config(0)
    P = O.PatternOracle(p.patterns[0].K, p.patterns[0].bdofs, 1)
    z = P.Z[:, 0] * np.sign(P.Z[0, 0])
    assert np.abs(z - 1 / np.sqrt(len(z))).max() < 1e-12


def test_pseudo_inverse_is_moore_penrose(elast_small):
    p, o = elast_small
    P = o.pats[0]
    assert np.abs(P.Splus - np.linalg.pinv(P.S, rcond=1e-10)).max() < 1e-9 * np.abs(P.Splus).max()
    assert np.abs(P.S @ P.Splus @ P.S - P.S).max() < 1e-10 * np.abs(P.S).max()


def test_generalized_inverse_identity(elast_small):
    """Section 2: S+ = t K+ t^T, read as S (t K^g t^T) S = S for a generalized inverse K^g."""
    p, o = elast_small
    P = o.pats[0]
    K = p.patterns[0].K.toarray()
    Kg = np.linalg.pinv(K, rcond=1e-12)
    T = Kg[np.ix_(P.b, P.b)]
    assert np.abs(P.S @ T @ P.S - P.S).max() < 1e-9 * np.abs(P.S).max()


def test_condensed_load(elast_small):
    p, o = elast_small
    P = o.pats[0]
    K = p.patterns[0].K.toarray()
    f = p.f_local[3]
    b, i = P.b, P.i
    g = f[b] - K[np.ix_(b, i)] @ np.linalg.solve(K[np.ix_(i, i)], f[i])
    assert np.abs(P.condensed_load(f) - g).max() < 1e-12 * np.abs(g).max()


# ----------------------------------------------------------------------------- interface level

def test_continuity_of_a_global_field(elast_small):
    """Eq. 2, second row: sum_s A^(s) t u^(s) = 0 for a globally continuous field."""
    p, o = elast_small
    rng = np.random.default_rng(3)
    ug = rng.standard_normal((p.n_gnodes, 3))
    total = np.zeros(p.n_lambda)
    for s in range(p.n_occ):
        us = ug[p.occ_gnode[s]].ravel()
        total += o.A[s] @ us[o.pats[0].b]
    # Dirichlet rows see u itself; zero it on Dirichlet nodes to test interfaces only
    nd = p.n_dirichlet_mult() * 3
    assert np.abs(total[:p.n_lambda - nd]).max() < 1e-14
    assert np.abs(total[p.n_lambda - nd:]).max() > 0.1


def test_ring_w_format_antisymmetry(golden_dir):
    """Section 3.2: the W format stores w^(s,s+1) and w^(s,s-1) = -w^(s-1,s) per occurrence."""
    gold = json.load(open(os.path.join(golden_dir, "ring_w_format.json")))
    p = W.ring_heat(3, (1, 1), n_perm=3)
    o = O.FetiOracle(p)
    # multipliers per node pair: interface (s,s+1) holds nodes 2*s, 2*s+1
    lam = np.zeros(p.n_lambda)
    names = gold["w"]
    vals = {names[s]: 10.0 * (s + 1) for s in range(3)}
    for s in range(3):
        lam[2 * s:2 * s + 2] = vals[names[s]]
    pat = p.patterns[0]
    for s in range(3):
        local = o.A[s].T @ lam
        right = [np.nonzero(pat.bnodes == n)[0][0] for n in (1, 3)]   # ix = 1 edge
        left = [np.nonzero(pat.bnodes == n)[0][0] for n in (0, 2)]    # ix = 0 edge
        top, bot = gold["W"][0][s], gold["W"][1][s]
        assert np.allclose(local[right], float(top[0] + "1") * vals[top[1:]])
        assert np.allclose(local[left], float(bot[0] + "1") * vals[bot[1:]])


def test_ring_multivector_is_circulant(golden_dir):
    gold = json.load(open(os.path.join(golden_dir, "ring_multivector.json")))
    p = W.ring_heat(3, (2, 2), n_perm=3)
    o = O.FetiOracle(p)
    nn = 3                      # nodes per interface edge (ny + 1)
    w = np.zeros((p.n_lambda, 1))
    names = gold["w"]
    for s in range(3):
        w[nn * s:nn * (s + 1), 0] = (s + 1) * 100 + np.arange(nn)
    Wt = o.permute(w)
    for row in range(3):
        for col in range(3):
            src = names.index(gold["w_tilde"][row][col])
            assert np.array_equal(Wt[nn * row:nn * (row + 1), col], w[nn * src:nn * (src + 1), 0])


def test_stand_interface_replicated(golden_dir):
    gold = json.load(open(os.path.join(golden_dir, "stand_multivector.json")))
    p = W.ring_heat(3, (2, 2), stand=True, n_perm=3)
    o = O.FetiOracle(p)
    w = np.arange(p.n_lambda, dtype=float)[:, None] + 1
    Wt = o.permute(w)
    ring = p.mult_occ[:, 1] < 3
    ring &= p.mult_occ[:, 0] < 3
    stand = ~ring
    # every stand multiplier (interface (3,4) and its corner links) keeps its own value
    assert stand.any()
    for col in range(3):
        assert np.array_equal(Wt[stand, col], w[stand, 0])
    # the ring interior-edge multipliers rotate as in the three-occurrence ring
    assert not np.array_equal(Wt[ring, 1], w[ring, 0])
    assert gold["w_tilde"][3] == ["34", "34", "34"]


def test_ring_coarse_G_structure(golden_dir):
    """Section 4.3: block structure and signs of G on a three-occurrence ring."""
    gold = json.load(open(os.path.join(golden_dir, "ring_coarse_G.json")))
    p = W.ring_heat(3, (2, 2), n_perm=3, dirichlet_bottom=False)
    o = O.FetiOracle(p)
    G = o.G.toarray()
    nn = 3
    z = o.pats[0].Z[0, 0]
    for row in range(3):
        for col in range(3):
            blk = G[nn * row:nn * (row + 1), col]
            want = gold["blocks"][row][col]
            if want == "0":
                assert np.all(blk == 0)
            else:
                sign = 1.0 if want[0] == "+" else -1.0
                assert np.allclose(blk, sign * z, atol=1e-14)


def test_F_symmetric_psd_and_dense(elast_small):
    p, o = elast_small
    F = o.F(np.eye(p.n_lambda))
    assert np.abs(F - F.T).max() < 1e-12 * np.abs(F).max()
    assert np.linalg.eigvalsh(F).min() > -1e-10 * np.abs(F).max()
    Fd = sum(o.A[s].toarray() @ o.pats[0].Splus @ o.A[s].toarray().T for s in range(p.n_occ))
    assert np.abs(F - Fd).max() < 1e-12 * np.abs(F).max()


def test_projector_identities(elast_small):
    """Section 2: Q^2 = Q, G^T Q = 0, G^T lambda_0 = e."""
    p, o = elast_small
    rng = np.random.default_rng(0)
    X = rng.standard_normal((p.n_lambda, 3))
    QX = o.Q(X)
    assert np.abs(o.Q(QX) - QX).max() < 1e-12 * np.abs(X).max()
    assert np.abs(o.G.T @ QX).max() < 1e-11
    g, d, e = o.loads()
    l0 = o.lambda0(e)
    assert np.abs(o.G.T @ l0 - e).max() < 1e-11 * np.abs(e).max()


def test_periodic_ring_commutation():
    """Section 3.1: on a truly periodic ring F and the permutations commute."""
    p = W.ring_heat(5, (3, 3), n_perm=5)
    o = O.FetiOracle(p)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((p.n_lambda, 1))
    Pk = p.perm_dof()
    for k in range(1, 5):
        lhs = o.F(x[Pk[k]])
        rhs = o.F(x)[Pk[k]]
        assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()


def test_rotated_ring_permutation_carries_frames():
    """Sections 3.1 and 4.2: on a periodic ring of rotated elastic sectors F commutes with the
    permutations only when each moved multiplier is turned into the frame of its new place
    (O_t O_s^T); moving the components as they are does not commute."""
    p = W.ring_elast(4, (1, 2, 1), n_perm=4, clamp=False)
    o = O.FetiOracle(p)
    x = np.random.default_rng(5).standard_normal((p.n_lambda, 1))
    z = o.permute(x)                                       # columns k = 0..3
    Fz = o.F(z)
    Fx_moved = o.permute(o.F(x))
    assert np.abs(z[:, :1] - x).max() == 0.0
    assert np.abs(Fz - Fx_moved).max() < 1e-12 * np.abs(Fx_moved).max()
    Pk = p.perm_dof()
    plain = o.F(x[Pk[1]]) - o.F(x)[Pk[1]]
    assert np.abs(plain).max() > 1e-2 * np.abs(Fz).max()
    # a rotation keeps the Euclidean norm of every multiplier
    for k in range(4):
        assert np.linalg.norm(z[:, k]) == pytest.approx(np.linalg.norm(x), rel=1e-13)


def test_rotated_ring_brute_force():
    """Section 4.2 assembly with rotated occurrences: FETI on a clamped ring of three sectors
    reproduces the directly assembled global solution and its interface forces."""
    p = W.ring_elast(3, (2, 3, 2), n_rhs=2)
    o = O.FetiOracle(p)
    ub, _, _, _ = O.global_solve(p)
    scale = max(np.abs(x).max() for x in ub)
    lam, u, st = o.solve("block", tol=1e-11)
    assert max(np.abs(ub[s] - u[s]).max() for s in range(p.n_occ)) < 1e-8 * scale
    lb = O.multipliers_from_displacements(o, ub)
    assert np.abs(lb - lam).max() < 1e-7 * np.abs(lam).max()


def test_uneven_three_patterns_brute_force():
    """Three patterns of uneven size (plates, ring sectors, a base block) joined by algebraic glue
    with rotated frames (sections 2 and 4.2): FETI reproduces the directly assembled global solution
    and its interface forces, G^T lambda = e holds, and every floating occurrence is in equilibrium
    against its rigid modes."""
    p = W.uneven_three(plate=(6, 8, 2), sector=(2, 6, 4), base=6, n_sectors=4, plates_per_sector=1, n_perm=4,
                       seed=5)
    assert [int(v) for v in np.bincount(p.occ_pattern)] == [4, 4, 1]
    o = O.FetiOracle(p)
    ub, _, _, _ = O.global_solve(p)
    scale = max(np.abs(x).max() for x in ub)
    for method in ("classical", "block"):
        lam, u, st = o.solve(method, tol=1e-11)
        assert max(np.abs(ub[s] - u[s]).max() for s in range(p.n_occ)) < 1e-9 * scale, method
    lb = O.multipliers_from_displacements(o, ub)
    assert np.abs(lb - lam).max() < 1e-8 * np.abs(lam).max()
    g, d, e = o.loads()
    assert np.abs(o.G.T @ lam - e).max() < 1e-10 * np.abs(e).max()
    for s in range(p.n_occ):
        P = o.pats[p.occ_pattern[s]]
        res = P.N.T @ p.f_local[s] - P.Z.T @ (o.A[s].T @ lam)
        assert np.abs(res).max() < 1e-9 * np.abs(p.f_local[s]).max(), s


# ----------------------------------------------------------------------------- solvers

def test_heat_row_closed_form(golden_dir):
    gold = json.load(open(os.path.join(golden_dir, "heat_row_closed_form.json")))
    p = W.config(0)
    o = O.FetiOracle(p)
    for method in ("classical", "block"):
        lam, u, st = o.solve(method)
        x = p.patterns[0].coords[:, 0]
        for s in range(4):
            xs = x + s
            assert np.abs(u[s][:, 0] - xs * (8 - xs) / 2).max() < 1e-9
    assert max(u[3][:, 0]) == pytest.approx(gold["u_max"], abs=1e-9)


def test_brute_force_elasticity(elast_small):
    p, o = elast_small
    ub, _, _, _ = O.global_solve(p)
    scale = max(np.abs(x).max() for x in ub)
    for method, fr in (("classical", True), ("block", True), ("block", False)):
        lam, u, st = o.solve(method, tol=1e-11, full_reorth=fr)
        err = max(np.abs(ub[s] - u[s]).max() for s in range(p.n_occ)) / scale
        assert err < 1e-9, (method, fr, err)
    lb = O.multipliers_from_displacements(o, ub)
    assert np.abs(lb - lam).max() < 1e-8 * np.abs(lam).max()


def test_equilibrium_and_continuity_of_solution(elast_small):
    p, o = elast_small
    lam, u, st = o.solve("block", tol=1e-11)
    g, d, e = o.loads()
    assert np.abs(o.G.T @ lam - e).max() < 1e-10 * np.abs(e).max()
    cont = sum(o.A[s] @ u[s][o.pats[0].b] for s in range(p.n_occ))
    assert np.abs(cont).max() < 1e-9 * max(np.abs(x).max() for x in u)
    # each floating occurrence is in equilibrium against its rigid modes
    for s in range(p.n_occ):
        P = o.pats[0]
        lb = o.A[s].T @ lam
        res = P.N.T @ p.f_local[s] - P.Z.T @ lb
        assert np.abs(res).max() < 1e-9 * np.abs(p.f_local[s]).max()


def test_block_single_direction_equals_classical():
    """Table 1: with one direction per iteration the multivector column reduces to the classical one."""
    p = W.small_elast((2, 2, 2), (2, 2, 1), n_rhs=1, n_perm=1)
    o = O.FetiOracle(p)
    g, d, e = o.loads()
    rc, rb = [], []
    o.solve_classical(d, e, 1e-10, record=rc)
    o.solve_block(d, e, 1e-10, full_reorth=True, record=rb)
    n = min(20, len(rc), len(rb))
    for j in range(n):
        assert np.abs(rc[j] - rb[j][:, 0]).max() < 1e-10 * np.abs(rc[j]).max()


def _krylov_minimisers(o, d, e, n_it, precond=None):
    """The iterates that define projected CG, computed from their definition and nothing else: the
    j-th is the minimiser of the F-energy of the error over lambda_0 + K_j, K_j = span{z_0, A z_0,
    .., A^{j-1} z_0} with z_0 = Q F~^{-1} r_0 and A = Q F~^{-1} Q^T F.  With V an orthonormal basis
    of K_j (range Q, where Q V = V): (V^T F V) y = V^T r_0 and lambda_j = lambda_0 + V y."""
    l0 = o.lambda0(e)[:, 0]
    r0 = o.Qt(d[:, 0] - o.F(l0))
    V, FV, out = [], [], []
    w = o.Q(o.precondition(r0, precond))
    for _ in range(n_it):
        for _ in range(2):
            for v in V:
                w = w - (v @ w) * v
        w = o.Q(w)
        V.append(w / np.linalg.norm(w))
        FV.append(o.F(V[-1]))
        Vm, FVm = np.array(V).T, np.array(FV).T
        H = Vm.T @ FVm
        y = np.linalg.solve(0.5 * (H + H.T), Vm.T @ r0)
        out.append(l0 + Vm @ y)
        w = o.Q(o.precondition(o.Qt(FV[-1]), precond))
    return out


@pytest.mark.parametrize("precond,coarse", [(None, None), ("dirichlet", None), ("lumped", "lumped")])
def test_classical_iterates_minimise_energy_over_krylov_space(precond, coarse):
    """Section 2: projected (preconditioned) CG gives, at iteration j, the F-energy minimiser over
    lambda_0 + K_j.  The oracle's recurrences reproduce the minimisers computed from that
    definition (with an orthonormal Krylov basis and a dense Galerkin solve) over the first 15
    iterations, before rounding separates the two."""
    p = W.small_elast((2, 2, 2), (2, 2, 1), n_rhs=1, n_perm=1, seed=31)
    o = O.FetiOracle(p, coarse=coarse)
    g, d, e = o.loads()
    rc = []
    o.solve_classical(d, e, 1e-14, record=rc, max_it=15, precond=precond)
    ref = _krylov_minimisers(o, d, e, min(15, len(rc)), precond)
    for j, (a, b) in enumerate(zip(rc, ref)):
        assert np.abs(a - b).max() < 1e-9 * np.abs(b).max(), j


def test_classical_converges_within_rank():
    p = W.small_heat((2, 2), (3, 1), n_rhs=1)
    o = O.FetiOracle(p)
    g, d, e = o.loads()
    lam, st = o.solve_classical(d, e, 1e-12)
    assert st["iterations"][0] <= p.n_lambda - o.G.shape[1] + 1


def test_block_not_slower_than_classical():
    """Sections 3.1 and 5: the multivector method needs no more iterations (soft check)."""
    p = W.config(0)
    o = O.FetiOracle(p)
    _, _, sc = o.solve("classical")
    _, _, sb = o.solve("block")
    assert sb["iterations"] <= max(sc["iterations"])


# ----------------------------------------------------------------------------- preconditioners (section 2)

def test_precond_mirror_pair_is_exact_inverse():
    """Two mirror-image, non-floating occurrences meeting on one edge: F = 2 S^{-1} on that edge
    and the Dirichlet preconditioner with the scaling 1/2 is (1/4)(S + S) = S / 2, its exact
    inverse; preconditioned CG then ends in one iteration.  The lumped one is not exact."""
    p = W.mirror_row_heat(2, (4, 4))
    o = O.FetiOracle(p)
    assert o.pats[0].k == 0 and len(p.patterns[0].bnodes) == 5
    I = np.eye(p.n_lambda)
    F = o.F(I)
    assert np.abs(o.precondition(F, "dirichlet") - I).max() < 1e-13
    assert np.abs(o.precondition(F, "lumped") - I).max() > 0.1
    g, d, e = o.loads()
    lam, st = o.solve_classical(d, e, 1e-12, precond="dirichlet")
    assert st["iterations"] == [1]
    ub, _, _, _ = O.global_solve(p)
    u = o.recover(lam, d, g)
    assert max(np.abs(a - b).max() for a, b in zip(u, ub)) < 1e-12 * max(np.abs(b).max() for b in ub)


def test_precond_lumped_equals_dirichlet_without_interior():
    """With no interior dof, S = K_bb and the lumped and Dirichlet preconditioners coincide."""
    p = W.mirror_row_heat(3, (1, 3))
    o = O.FetiOracle(p)
    assert len(o.pats[0].i) == 0
    X = np.random.default_rng(0).standard_normal((p.n_lambda, 3))
    a, b = o.precondition(X, "lumped"), o.precondition(X, "dirichlet")
    assert np.abs(a - b).max() < 1e-14 * np.abs(a).max()


def test_precond_scaling_is_multiplicity_away_from_cross_points():
    """The scaling is 1/2 on an interface multiplier and 1 on a Dirichlet one wherever no other
    multiplier shares an endpoint dof (the paper's diagonal beta with sum_s beta^(s) = I)."""
    p = W.small_elast((2, 2, 2), (2, 2, 2), n_rhs=1)
    o = O.FetiOracle(p)
    keys = {}
    for e in range(2):
        for i, (s, n) in enumerate(zip(p.mult_occ[:, e], p.mult_node[:, e])):
            if s >= 0:
                keys.setdefault((int(s), int(n)), []).append(i)
    shared = np.zeros(p.n_mult_nodes, bool)
    for lst in keys.values():
        if len(lst) > 1:
            shared[lst] = True
    lone = np.nonzero(~shared)[0]
    assert len(lone) > 0 and shared.any()
    X = np.eye(p.n_lambda)[:, (lone[:, None] * 3 + np.arange(3)).ravel()]
    Y = o.scale(X)
    ends = 1 + (p.mult_occ[lone, 1] >= 0)
    expect = np.repeat(1.0 / ends, 3)
    assert np.abs(Y - X * expect[None, :]).max() < 1e-14
    assert ((ends == 1).any() and (ends == 2).any())


@pytest.mark.parametrize("case", ["elast222", "ring4"])
def test_precond_spectrum_and_order(case):
    """Spectral facts of the preconditioned operator Q F~^{-1} Q F on range Q: its smallest
    eigenvalue is 1 or more for a consistent scaling (the dual Dirichlet bound), the Dirichlet
    form is the better conditioned one, and K_bb - S = K_bi K_ii^{-1} K_ib >= 0 makes the lumped
    preconditioner dominate the Dirichlet one (a nonzero positive semi-definite difference)."""
    p = W.small_elast((3, 3, 3), (2, 2, 2), n_rhs=1) if case == "elast222" else W.ring_elast(4, (1, 2, 1), n_perm=1)
    o = O.FetiOracle(p)
    I = np.eye(p.n_lambda)
    F, Q = o.F(I), o.Q(I)
    conds = {}
    Ms = {}
    for kind in (None, "lumped", "dirichlet"):
        Ms[kind] = o.precondition(I, kind)
        w = np.linalg.eigvals(Q @ Ms[kind] @ Q @ F).real
        w = np.sort(w[np.abs(w) > 1e-9 * np.abs(w).max()])
        conds[kind] = w[-1] / w[0]
        if kind is not None:
            assert w[0] > 1.0 - 1e-8, (kind, w[0])
            assert np.abs(Ms[kind] - Ms[kind].T).max() < 1e-13 * np.abs(Ms[kind]).max()
    assert conds["dirichlet"] < conds["lumped"] < conds[None] / 10
    diff = Ms["lumped"] - Ms["dirichlet"]
    ev = np.linalg.eigvalsh(0.5 * (diff + diff.T))
    assert ev[0] > -1e-12 * ev[-1] and ev[-1] > 1e-3 * np.abs(Ms["dirichlet"]).max()


def test_precond_solutions_match_brute_force():
    """Preconditioning changes the path, not the solution (eq. 1 solved by the assembled system)."""
    p = W.small_elast((3, 3, 3), (2, 2, 2), n_rhs=2, n_perm=1)
    o = O.FetiOracle(p)
    ub, _, _, _ = O.global_solve(p)
    scale = max(np.abs(x).max() for x in ub)
    _, _, s_id = o.solve("block", tol=1e-10)
    for kind in ("lumped", "dirichlet"):
        for method in ("classical", "block"):
            lam, u, st = o.solve(method, tol=1e-10, precond=kind)
            err = max(np.abs(ub[s] - u[s]).max() for s in range(p.n_occ)) / scale
            assert err < 1e-9, (kind, method, err)
            its = max(st["iterations"]) if method == "classical" else st["iterations"]
            assert its * 3 < s_id["iterations"], (kind, method, its)


# ----------------------------------------------------------------------------- academic study (section 3.4.1)

@pytest.mark.parametrize("n_occ", [5, 9])
def test_random_spd_ring_solution(n_occ):
    """A ring of a random dense SPD pattern (its Schur complement is the matrix itself): the FETI
    solution, classical and multivector, with and without the Dirichlet preconditioner, is the
    assembled solution."""
    p = W.random_spd_ring(n_occ, 24)
    o = O.FetiOracle(p)
    assert len(o.pats[0].i) == 0 and o.pats[0].k == 0 and o.G.shape[1] == 0
    assert np.abs(o.pats[0].S - p.patterns[0].K.toarray()).max() == 0.0
    ub, _, _, _ = O.global_solve(p)
    scale = max(np.abs(x).max() for x in ub)
    for method in ("classical", "block"):
        for pc in (None, "dirichlet"):
            _, u, _ = o.solve(method, tol=1e-12, precond=pc)
            assert max(np.abs(a - b).max() for a, b in zip(u, ub)) < 1e-9 * scale, (method, pc)


def test_random_spd_ring_iteration_study():
    """The paper's academic study, qualitatively: with the Dirichlet preconditioner and random
    non-periodic loads, the multivector built from the n_occ cyclic shifts needs far fewer
    iterations than classical CG, and the saving grows from five to nine repetitions (the paper
    reports about 35 % and 55 %)."""
    saving = {}
    for n_occ in (5, 9):
        p = W.random_spd_ring(n_occ, 40)
        o = O.FetiOracle(p)
        _, _, sc = o.solve("classical", tol=1e-10, precond="dirichlet")
        _, _, sb = o.solve("block", tol=1e-10, precond="dirichlet")
        saving[n_occ] = 1.0 - sb["iterations"] / sc["iterations"][0]
    assert saving[5] > 0.3 and saving[9] > saving[5], saving


# ----------------------------------------------------------------------------- periodic shortcut (section 3.1)

def _periodic_cases():
    return {"heat-ring": W.ring_heat(4, (4, 4), dirichlet_bottom="periodic", n_perm=4, n_rhs=2),
            "elast-ring-rotated": W.ring_elast(4, (1, 2, 1), clamp="periodic", n_perm=4),
            "random-spd-ring": W.random_spd_ring(5, 10)}


@pytest.mark.parametrize("name", ["heat-ring", "elast-ring-rotated", "random-spd-ring", "heat-ring-clamped-once"])
def test_periodicity_of_the_operators(name):
    """A truly periodic structure: F, Q and the Dirichlet preconditioner commute with every
    permutation (section 3.1).  Clamping one occurrence only breaks it."""
    p = _periodic_cases().get(name) or W.ring_heat(4, (4, 4), dirichlet_bottom=True, n_perm=4)
    o = O.FetiOracle(p)
    x = o.Q(np.random.default_rng(1).standard_normal((p.n_lambda, 1)))
    pairs = [(o.permute(o.Q(o.F(x))), o.Q(o.F(o.Q(o.permute(x))))),
             (o.permute(o.precondition(x, "dirichlet")), o.precondition(o.permute(x), "dirichlet")),
             (o.permute(x), o.Q(o.permute(x)))]
    devs = [np.abs(a - b).max() / np.abs(a).max() for a, b in pairs]
    if name == "heat-ring-clamped-once":
        assert devs[0] > 0.1 and devs[1] > 0.1
    else:
        assert max(devs) < 1e-13, devs


@pytest.mark.parametrize("name", ["heat-ring", "elast-ring-rotated", "random-spd-ring"])
@pytest.mark.parametrize("pc", [None, "dirichlet"])
def test_periodic_shortcut_follows_full_products(name, pc):
    """One product per iteration plus permutations gives the same iterates as the product of the
    whole multivector (full re-orthogonalisation), and the assembled solution."""
    p = _periodic_cases()[name]
    o = O.FetiOracle(p)
    g, d, e = o.loads()
    ra, rb = [], []
    _, sa = o.solve_block(d, e, 1e-11, precond=pc, record=ra)
    lb, sb = o.solve_block(d, e, 1e-11, precond=pc, record=rb, periodic=True)
    assert sa["iterations"] == sb["iterations"]
    for a, b in zip(ra, rb):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    ub, _, _, _ = O.global_solve(p)
    u = o.recover(lb, d, g)
    assert max(np.abs(x - y).max() for x, y in zip(u, ub)) < 1e-9 * max(np.abs(y).max() for y in ub)


def test_periodic_shortcut_on_a_non_periodic_structure_is_wrong():
    """Negative control: with one occurrence clamped the shortcut's products are not F W."""
    p = W.ring_heat(4, (4, 4), dirichlet_bottom=True, n_perm=4)
    o = O.FetiOracle(p)
    g, d, e = o.loads()
    lb, _ = o.solve_block(d, e, 1e-11, periodic=True, max_it=50)
    ub, _, _, _ = O.global_solve(p)
    u = o.recover(lb, d, g)
    assert max(np.abs(x - y).max() for x, y in zip(u, ub)) > 1e-3 * max(np.abs(y).max() for y in ub)


# ----------------------------------------------------------------------------- enriched multivector (section 4.1.2)

def _paper_label(p, m):
    """Interface label of multiplier m in the paper's numbering of the two-stand donut: ring pieces
    1, 2, 3 are occurrences 0, 1, 2; stand 4 (on piece 2) is occurrence 3, stand 5 (on piece 1) is 4."""
    a, b = (int(x) + 1 for x in p.mult_occ[m])
    return f"{min(a, b)}{max(a, b)}" if {a, b} != {1, 3} else "31"


def test_two_stand_enriched_multivector(golden_dir):
    gold = json.load(open(os.path.join(golden_dir, "two_stand_multivector.json")))
    p = W.ring_heat(3, (4, 4), stands=(1, 0), enriched=True)
    assert p.n_perm == 6
    o = O.FetiOracle(p)
    labels = [_paper_label(p, m) for m in range(p.n_mult_nodes)]
    code = {lab: float(i + 1) for i, lab in enumerate(gold["w"])}
    w = np.array([[code.get(lab, 100.0 + m)] for m, lab in enumerate(labels)])
    Wt = o.permute(w)
    orbit = [len(set(p.perm_node[:, m])) for m in range(p.n_mult_nodes)]
    checked = set()
    for m, lab in enumerate(labels):
        if lab not in code or orbit[m] != (3 if lab in ("12", "23", "31") else 2):
            continue                     # corner links of the chains are classes of their own
        row = gold["w"].index(lab)
        for c in range(6):
            assert Wt[m, c] == code[gold["w_tilde"][row][c]], (lab, c)
        checked.add(lab)
    assert checked == set(gold["w"])


def test_enriched_multivector_solution():
    """The enriched multivector (product of the ring and stand shifts) solves the same problem; with
    four ring pieces it has 8 columns where the synchronised shifts give 4."""
    for enriched in (False, True):
        p = W.ring_heat(4, (6, 6), stands=(1, 0), enriched=enriched, n_rhs=2, dirichlet_bottom=True)
        assert p.n_perm == (8 if enriched else 4)
        o = O.FetiOracle(p)
        ub, _, _, _ = O.global_solve(p)
        _, u, st = o.solve("block", tol=1e-11)
        assert max(np.abs(a - b).max() for a, b in zip(u, ub)) < 1e-9 * max(np.abs(b).max() for b in ub)


def test_precond_single_occurrence_is_exact():
    """One occurrence held by Dirichlet multipliers only: F = S+ on the pattern boundary and the
    Dirichlet preconditioner is S, so F~^{-1} F = S S+ is the orthogonal projector on range S and the
    preconditioned solve ends in one iteration."""
    p = W.small_elast((3, 3, 3), (1, 1, 1), n_rhs=1, seed=4)
    o = O.FetiOracle(p)
    I = np.eye(p.n_lambda)
    M = o.precondition(o.F(I), "dirichlet")
    G = o.G.toarray()                       # A Z: orthonormal columns, A a signed permutation here
    assert np.abs(M - (I - G @ G.T)).max() < 1e-11
    _, _, st = o.solve("block", tol=1e-12, precond="dirichlet")
    assert st["iterations"] == 1


# ----------------------------------------------------------------------------- preconditioner in the projector (section 2)

@pytest.mark.parametrize("case", ["elast222", "ring4"])
@pytest.mark.parametrize("coarse", ["lumped", "dirichlet"])
def test_projector_with_preconditioner(case, coarse):
    """Q = I - F~^{-1} G (G^T F~^{-1} G)^{-1} G^T: a projector (Q Q = Q) onto directions with
    G^T w = 0, Q^T its transpose, lambda_0 with G^T lambda_0 = e; with these the FETI solution is the
    assembled one, and a consistent pair (Dirichlet preconditioner in both places) needs no more
    iterations than the orthogonal projector."""
    p = W.small_elast((3, 3, 3), (2, 2, 2), n_rhs=2, seed=7) if case == "elast222" else \
        W.ring_elast(4, (1, 2, 1), n_perm=4)
    o = O.FetiOracle(p, coarse=coarse)
    I = np.eye(p.n_lambda)
    Q, Qt = o.Q(I), o.Qt(I)
    assert np.abs(o.G.T @ Q).max() < 1e-13
    assert np.abs(Q @ Q - Q).max() < 1e-12
    assert np.abs(Q.T - Qt).max() < 1e-12
    assert np.abs(Q - O.FetiOracle(p).Q(I)).max() > 1e-3      # not the orthogonal projector
    g, d, e = o.loads()
    assert np.abs(o.G.T @ o.lambda0(e) - e).max() < 1e-12 * np.abs(e).max()
    ub, _, _, _ = O.global_solve(p)
    scale = max(np.abs(x).max() for x in ub)
    for method in ("classical", "block"):
        _, u, st = o.solve(method, tol=1e-11, precond="dirichlet")
        assert max(np.abs(a - b).max() for a, b in zip(u, ub)) < 1e-9 * scale, (method, coarse)
    if coarse == "dirichlet":
        _, _, s_orth = O.FetiOracle(p).solve("block", tol=1e-11, precond="dirichlet")
        assert st["iterations"] <= s_orth["iterations"]
