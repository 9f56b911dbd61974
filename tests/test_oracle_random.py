"""Randomised pins of the CPU oracle: small structures drawn at random (grid shape, pattern size,
load cases, permutations, preconditioner, solver form), each solved by the oracle's FETI and
checked against the assembled global solve of eq. 1 built from the global node numbering.  The
solution does not depend on any of the drawn solver choices, so every draw must reach it.
"""
import numpy as np
import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def _check(p, method, precond, full_reorth=True):
    o = O.FetiOracle(p)
    ub, _, _, _ = O.global_solve(p)
    _, u, _ = o.solve(method, tol=1e-11, precond=precond, full_reorth=full_reorth)
    scale = max(np.abs(x).max() for x in ub)
    err = max(np.abs(a - b).max() for a, b in zip(u, ub)) / scale
    assert err < 1e-8, (p.name, method, precond, err)


@settings(max_examples=30, deadline=None, database=None)
@given(gx=st.integers(1, 3), gy=st.integers(1, 3), px=st.integers(1, 4), py=st.integers(1, 4),
       n_rhs=st.integers(1, 3), n_perm=st.integers(1, 3), seed=st.integers(0, 10_000),
       method=st.sampled_from(["classical", "block"]), precond=st.sampled_from([None, "lumped", "dirichlet"]))
def test_random_heat_grids(gx, gy, px, py, n_rhs, n_perm, seed, method, precond):
    p = W.small_heat((px, py), (gx, gy), n_rhs=n_rhs, n_perm=n_perm, seed=seed)
    _check(p, method, precond)


@settings(max_examples=15, deadline=None, database=None)
@given(gx=st.integers(1, 2), gy=st.integers(1, 2), gz=st.integers(1, 2), pe=st.integers(1, 2),
       n_rhs=st.integers(1, 2), n_perm=st.integers(1, 2), seed=st.integers(0, 10_000),
       precond=st.sampled_from([None, "lumped", "dirichlet"]), full_reorth=st.booleans())
def test_random_elastic_grids(gx, gy, gz, pe, n_rhs, n_perm, seed, precond, full_reorth):
    p = W.small_elast((pe, pe, pe), (gx, gy, gz), n_rhs=n_rhs, n_perm=n_perm, seed=seed)
    _check(p, "block", precond, full_reorth=full_reorth or n_perm > 1)


@settings(max_examples=6, deadline=None, database=None)
@given(n_occ=st.integers(3, 5), seed=st.integers(0, 10_000), precond=st.sampled_from([None, "dirichlet"]))
def test_random_rotated_rings(n_occ, seed, precond):
    p = W.ring_elast(n_occ, (1, 2, 1), n_perm=n_occ, seed=seed)
    _check(p, "block", precond)
