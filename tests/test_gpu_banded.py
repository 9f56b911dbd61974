"""The banded many-right-hand-side triangular solves of the condensed loads and the interior recovery
(section 3.2: one factorisation of the pattern, substitutions for every occurrence and load case at
once), through the C ABI, on a ragged shape: 60 occurrences of a 10^3 brick (an interior of 2,187
dofs, not a whole number of 64-row blocks) with 35 load cases (2,100 columns, not a multiple of the
16 columns a workgroup takes).  From 2,048 columns on, the library runs one persistent pass per 16
columns, the backward pass reading the mirrored L_ii^T; fewer columns take the per-block path.
Checked: local equilibrium of every occurrence and load case (which the interior solves decide),
continuity and the clamp, and the same u as two solves of 17 and 18 load cases (1,020 and 1,080
columns, the per-block path)."""
import dataclasses

import numpy as np
import pytest

import props
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    import paper_1208_6387_amd as R
    R.load()
    return R


@pytest.mark.timeout(600)
@pytest.mark.parametrize("form", ["fp64", "bf16x3"])
def test_banded_many_rhs_ragged(R, form):
    from paper_1208_6387_amd import structure as ST
    p = W.small_elast((10, 10, 10), (5, 4, 3), n_rhs=35, seed=91)
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats, (R.FP64, R.BF16X3))
    pb = ST.create_problem(p)
    prec = R.FP64 if form == "fp64" else R.BF16X3
    kw = dict(tol=1e-11, max_it=3000, method=R.BLOCK_CG, prec=prec, inner_tol=1e-4)
    assert p.n_occ * p.n_rhs >= 2048 and p.n_occ * p.n_rhs % 16 != 0
    assert (p.patterns[0].n - p.patterns[0].n_b) % 64 != 0
    res = R.block_krylov_solve(pb, pats, ST.loads_to_device(p), p.n_rhs, **kw)
    u = ST.split_u(p, res.u)
    lam = res.lam.cpu().numpy()
    scale = max(np.abs(x).max() for x in u)
    eq = props.equilibrium_residual(p, u, lam)
    gap = props.continuity_gap(p, u) / scale
    halves = []
    for a, b in ((0, 17), (17, 35)):
        q = dataclasses.replace(p, n_rhs=b - a, f_local=[f[:, a:b] for f in p.f_local])
        rq = R.block_krylov_solve(pb, pats, ST.loads_to_device(q), q.n_rhs, **kw)
        halves.append(np.concatenate([x for x in ST.split_u(q, rq.u)], axis=0))
    whole = np.concatenate(u, axis=0)
    diff = np.abs(whole - np.concatenate(halves, axis=1)).max() / scale
    print(f"[banded] {form}: its={res.stats['iterations']} res={res.stats['rel_residual']:.2e} equilibrium={eq:.2e} "
          f"continuity={gap:.2e} against halves={diff:.2e}")
    assert res.stats["rel_residual"] <= 1e-11
    assert eq <= 1e-10
    assert gap <= 1e-8
    assert props.dirichlet_max(p, u) <= 1e-8 * scale
    assert diff <= 1e-8
