"""Plant plausible mistakes in the CPU oracle and check that its pins notice them.

Every mutant lives here, on the CPU, and is applied by monkeypatching; the
oracle itself is never modified.
"""
import numpy as np
import pytest

import oracle as O
from oracle import feti as OF
import workloads as W


@pytest.fixture(scope="module")
def prob():
    return W.small_elast((2, 2, 2), (2, 2, 2), n_rhs=1, n_perm=2, seed=11)


@pytest.fixture(scope="module")
def brute(prob):
    ub, _, _, _ = O.global_solve(prob)
    return ub


def _err(u, ub):
    return max(np.abs(a - b).max() for a, b in zip(u, ub)) / max(np.abs(b).max() for b in ub)


def test_reference_passes(prob, brute):
    _, u, _ = O.FetiOracle(prob).solve("block", tol=1e-11)
    assert _err(u, brute) < 1e-9


def test_dropped_kernel_term_in_pseudo_inverse_is_caught(prob, monkeypatch):
    monkeypatch.setattr(OF, "pseudo_inverse", lambda S, Z: np.linalg.inv(S + Z @ Z.T))
    P = OF.PatternOracle(prob.patterns[0].K, prob.patterns[0].bdofs, 6)
    # the Moore-Penrose pin fails (the solution itself would not notice: Q removes G G^T)
    assert np.abs(P.Splus - np.linalg.pinv(P.S, rcond=1e-10)).max() > 1e-3 * np.abs(P.Splus).max()


def test_wrong_sign_of_kernel_term_in_recovery_is_caught(prob, brute, monkeypatch):
    o = O.FetiOracle(prob)
    orig = o.coarse_solve
    g, d, e = o.loads()
    lam, _ = o.solve_block(d, e, 1e-11)
    monkeypatch.setattr(o, "coarse_solve", lambda c: -orig(c))
    u = o.recover(lam, d, g)
    assert _err(u, brute) > 1e-3


def test_wrong_sign_in_condensed_load_is_caught(prob, brute, monkeypatch):
    def bad(self, f):
        return f[self.b] + self.Kib.T @ self.lu.solve(np.ascontiguousarray(f[self.i]))
    monkeypatch.setattr(OF.PatternOracle, "condensed_load", bad)
    _, u, _ = O.FetiOracle(prob).solve("block", tol=1e-11)
    assert _err(u, brute) > 1e-3


def test_unsigned_assembly_is_caught(prob):
    bad = prob.mult_sign.copy()
    bad[:] = np.abs(bad)
    p2 = W.small_elast((2, 2, 2), (2, 2, 2), n_rhs=1, n_perm=2, seed=11)
    p2.mult_sign = bad
    o = O.FetiOracle(p2)
    rng = np.random.default_rng(3)
    ug = rng.standard_normal((p2.n_gnodes, 3))
    total = sum(o.A[s] @ ug[p2.occ_gnode[s]].ravel()[o.pats[0].b] for s in range(p2.n_occ))
    nd = p2.n_dirichlet_mult() * 3
    assert np.abs(total[:p2.n_lambda - nd]).max() > 0.1      # continuity pin fails


def test_reversed_permutation_is_caught():
    p = W.ring_heat(3, (2, 2), n_perm=3)
    p.perm_node = p.perm_node[[0, 2, 1]]        # Pi_k -> Pi_{-k}
    o = O.FetiOracle(p)
    nn = 3
    w = np.zeros((p.n_lambda, 1))
    for s in range(3):
        w[nn * s:nn * (s + 1), 0] = s + 1
    Wt = o.permute(w)
    # paper: second column starts with w23
    assert not np.array_equal(Wt[:nn, 1], w[nn:2 * nn, 0])


def test_projector_with_wrong_sign_is_caught(prob, monkeypatch):
    o = O.FetiOracle(prob)
    monkeypatch.setattr(o, "Q", lambda X: X + o.G @ o.coarse_solve(o.G.T @ X))
    X = np.random.default_rng(0).standard_normal((prob.n_lambda, 2))
    QX = o.Q(X)
    assert np.abs(o.G.T @ QX).max() > 1e-3


def test_operator_drift_inside_block_solver_is_caught(prob, brute, monkeypatch):
    """An F that changes between iterations (e.g. a stale or mis-scaled operand) is noticed."""
    o = O.FetiOracle(prob)
    g, d, e = o.loads()
    orig_F = o.F
    calls = {"n": 0}

    def F_scaled(X):
        calls["n"] += 1
        return orig_F(X) * (1.0 if calls["n"] < 3 else 1.0 + 1e-3)   # operator drift mid-solve
    monkeypatch.setattr(o, "F", F_scaled)
    lam, st = o.solve_block(d, e, 1e-11, max_it=300)
    u = o.recover(lam, d, g)
    assert _err(u, brute) > 1e-6


def test_permutation_rotated_the_wrong_way_is_caught():
    """Moved multipliers turned by O_t^T O_s instead of O_t O_s^T break the commutation pin."""
    p = W.ring_elast(4, (1, 2, 1), n_perm=4, clamp=False)
    o = O.FetiOracle(p)
    x = np.random.default_rng(5).standard_normal((p.n_lambda, 1))
    good = o.F(o.permute(x)) - o.permute(o.F(x))
    assert np.abs(good).max() < 1e-12 * np.abs(o.F(x)).max()
    rot = p.occ_rot.copy()
    p.occ_rot = np.ascontiguousarray(np.swapaxes(rot, 1, 2))
    z_bad = o.permute(x)
    Fx_bad = o.permute(o.F(x))
    p.occ_rot = rot
    assert np.abs(o.F(z_bad) - Fx_bad).max() > 1e-2 * np.abs(Fx_bad).max()


def _min_precond_eig(o, kind):
    I = np.eye(o.n_lambda)
    F, Q = o.F(I), o.Q(I)
    w = np.linalg.eigvals(Q @ o.precondition(I, kind) @ Q @ F).real
    return np.sort(w[np.abs(w) > 1e-9 * np.abs(w).max()])[0]


def test_diagonal_half_scaling_at_cross_points_is_caught(prob, monkeypatch):
    """The diagonal 1/2 (1 on Dirichlet multipliers) applied at cross-points as well breaks the
    lower spectral bound of the preconditioned operator."""
    o = O.FetiOracle(prob)
    assert _min_precond_eig(o, "dirichlet") > 1.0 - 1e-8
    ends = np.repeat(1.0 / (1 + (prob.mult_occ[:, 1] >= 0)), 3)
    monkeypatch.setattr(o, "scale", lambda X: ends[:, None] * np.asarray(X) if np.ndim(X) == 2 else ends * X)
    assert _min_precond_eig(o, "dirichlet") < 0.5


def test_dirichlet_with_flexibility_instead_of_schur_is_caught(monkeypatch):
    p = W.mirror_row_heat(2, (4, 4))
    o = O.FetiOracle(p)
    monkeypatch.setattr(o, "local_precond_matrix", lambda pat, kind: o.pats[pat].Splus)
    I = np.eye(p.n_lambda)
    assert np.abs(o.precondition(o.F(I), "dirichlet") - I).max() > 0.1


def test_lumped_with_schur_instead_of_kbb_is_caught(monkeypatch):
    """K_bb replaced by S makes the lumped preconditioner equal to the Dirichlet one: the pin on
    their nonzero positive semi-definite difference fails."""
    p = W.ring_elast(4, (1, 2, 1), n_perm=1)
    o = O.FetiOracle(p)
    monkeypatch.setattr(o, "local_precond_matrix", lambda pat, kind: o.pats[pat].S)
    I = np.eye(p.n_lambda)
    diff = o.precondition(I, "lumped") - o.precondition(I, "dirichlet")
    assert np.abs(diff).max() < 1e-12


def test_unscaled_preconditioner_is_caught(monkeypatch):
    p = W.mirror_row_heat(2, (4, 4))
    o = O.FetiOracle(p)
    monkeypatch.setattr(o, "scale", lambda X: np.asarray(X, float))
    I = np.eye(p.n_lambda)
    assert np.abs(o.precondition(o.F(I), "dirichlet") - I).max() > 0.5


def test_projector_sides_swapped_is_caught(monkeypatch):
    """Directions projected with Q^T instead of Q leave the admissible space G^T w = 0 when F~^{-1}
    is in the projector."""
    p = W.small_elast((2, 2, 2), (2, 2, 1), n_rhs=1, seed=3)
    o = O.FetiOracle(p, coarse="dirichlet")
    I = np.eye(p.n_lambda)
    assert np.abs(o.G.T @ o.Q(I)).max() < 1e-13
    monkeypatch.setattr(o, "Q", o.Qt)
    assert np.abs(o.G.T @ o.Q(I)).max() > 1e-3
