"""The lumped or Dirichlet preconditioner as F~^{-1} inside the projector and lambda_0 (section 2:
Q = I - F~^{-1} G (G^T F~^{-1} G)^{-1} G^T) on the HIP path, against the CPU oracle built with the
same projector, through the C ABI.

Tolerances: displacements 1e-8 of max |u| (FP64) and 1e-6 (bf16x3 with FP64 sweeps) against the
oracle's solution at 1e-12, as for the plain projector; lambda 1e-7 of max |lambda| against the
oracle's solution with the same projector (the interface unknown is unique here: the multipliers
have full row rank); the coarse admissibility G^T lambda = e to 1e-10 of max |e|, which both
projectors keep exactly up to rounding; iteration counts within 3 of the oracle's run with the
same projector and preconditioner.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KINDS = {"none": 0, "lumped": 1, "dirichlet": 2}


@pytest.fixture(scope="module")
def R():
    import paper_1208_6387_amd as R
    R.load()
    return R


def _problem(name):
    if name == "elast-3cube-3x2x2":
        return W.small_elast((3, 3, 3), (3, 2, 2), n_rhs=2, n_perm=4, seed=7)
    if name == "heat-3x2":
        return W.small_heat((4, 4), (3, 2), n_rhs=2, n_perm=2, seed=5)
    if name == "ring-elast-rotated":
        return W.ring_elast(4, (1, 2, 1), n_rhs=2, n_perm=2)
    if name == "elast-ragged-2x3x1":
        return W.small_elast((5, 2, 3), (2, 3, 1), n_rhs=3, n_perm=1, seed=9)
    if name == "elast-2cube-4x4x4":
        # 64 occurrences in 27 colours: probe columns carry the modes of several occurrences
        return W.small_elast((2, 2, 2), (4, 4, 4), n_rhs=2, n_perm=1, seed=1)
    if name == "ring12-elast-rotated":
        # 12 rotated occurrences in 3 colours
        return W.ring_elast(12, (1, 2, 1), n_rhs=2, n_perm=2)
    raise KeyError(name)


CASES = ["elast-3cube-3x2x2", "heat-3x2", "ring-elast-rotated", "elast-ragged-2x3x1", "elast-2cube-4x4x4",
         "ring12-elast-rotated"]


@pytest.fixture(scope="module", params=CASES)
def case(request, R):
    from paper_1208_6387_amd import structure as ST
    p = _problem(request.param)
    print(f"\n[coarse-precond case {request.param}] n_lambda={p.n_lambda} n_occ={p.n_occ}", flush=True)
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats, precs=(R.FP64, R.BF16X3))
    pb = ST.create_problem(p)
    o = O.FetiOracle(p)
    lam_ref, u_ref, _ = o.solve("block", tol=1e-12)
    return request.param, p, pats, pb, u_ref


def _check(R, p, res, u_ref, oc, tol_u):
    from paper_1208_6387_amd import structure as ST
    u = ST.split_u(p, res.u)
    scale = max(np.abs(x).max() for x in u_ref)
    err = max(np.abs(a - b).max() for a, b in zip(u, u_ref)) / scale
    assert err < tol_u, (err, res.stats)
    lam = res.lam.cpu().numpy()
    _, _, e = oc.loads()
    if oc.G.shape[1]:
        adm = np.abs(oc.G.T @ lam - e).max()
        assert adm <= 1e-10 * max(np.abs(e).max(), 1.0), adm
    return lam


@pytest.mark.parametrize("coarse", ["lumped", "dirichlet"])
@pytest.mark.parametrize("precond", ["none", "same"])
@pytest.mark.parametrize("method", ["classical", "block_cg", "orthodir"])
def test_solve_coarse_precond(case, R, coarse, precond, method):
    name, p, pats, pb, u_ref = case
    from paper_1208_6387_amd import structure as ST
    pc = coarse if precond == "same" else "none"
    meth = {"classical": R.CLASSICAL, "block_cg": R.BLOCK_CG, "orthodir": R.ORTHODIR}[method]
    print(f"[coarse-precond {name} coarse={coarse} precond={pc} {method}]", flush=True)
    res = R.block_krylov_solve(pb, pats, ST.loads_to_device(p), p.n_rhs, tol=1e-11, max_it=3000, method=meth,
                               precond=KINDS[pc], coarse=KINDS[coarse])
    assert res.stats["rel_residual"] <= 1e-11
    oc = O.FetiOracle(p, coarse=coarse)
    lam = _check(R, p, res, u_ref, oc, 1e-8)
    lam_o, _, so = oc.solve("classical" if method == "classical" else "block", tol=1e-11,
                            precond=None if pc == "none" else pc, full_reorth=method != "block_cg")
    assert np.abs(lam - lam_o).max() <= 1e-7 * np.abs(lam_o).max(), np.abs(lam - lam_o).max()
    # (the classical form advances every load case together: its count is the largest per case)
    ref_it = max(so["iterations"]) if method == "classical" else so["iterations"]
    assert res.stats["iterations"] <= ref_it + 3, (res.stats["iterations"], ref_it)


def test_solve_coarse_precond_mixed(case, R):
    name, p, pats, pb, u_ref = case
    from paper_1208_6387_amd import structure as ST
    res = R.block_krylov_solve(pb, pats, ST.loads_to_device(p), p.n_rhs, tol=1e-9, max_it=3000, method=R.ORTHODIR,
                               prec=R.BF16X3, inner_tol=1e-3, precond=R.PRECOND_DIRICHLET,
                               coarse=R.PRECOND_DIRICHLET)
    assert res.stats["rel_residual"] <= 1e-9
    _check(R, p, res, u_ref, O.FetiOracle(p, coarse="dirichlet"), 1e-6)


@pytest.mark.parametrize("coarse", ["lumped", "dirichlet"])
def test_coarse_assembly_columns_matches_responses(case, R, coarse, monkeypatch):
    """The coarse matrix from the patterns' responses to the probed mode traces gives the same solve
    as the column-by-column assembly (one preconditioner application per 64 coarse unknowns)."""
    name, p, pats, pb, u_ref = case
    from paper_1208_6387_amd import structure as ST
    f = ST.loads_to_device(p)
    out = {}
    for how in ["columns", "responses"]:
        monkeypatch.setenv("RPF_COARSE_ASSEMBLY", how)
        # fresh structure: the coarse matrix is cached per structure and pattern handles
        pb2 = ST.create_problem(p)
        res = R.block_krylov_solve(pb2, pats, f, p.n_rhs, tol=1e-11, max_it=3000, method=R.BLOCK_CG,
                                   precond=KINDS[coarse], coarse=KINDS[coarse])
        out[how] = (res.lam.cpu().numpy(), res.stats["iterations"])
    (la, ia), (lb, ib) = out["columns"], out["responses"]
    # the two matrices differ by rounding only
    assert abs(ia - ib) <= 1, (ia, ib)
    assert np.abs(la - lb).max() <= 1e-8 * np.abs(la).max()


def test_coarse_precond_switch_and_plain_again(R):
    """The coarse matrix follows the kind between solves on one structure, and the plain projector
    is untouched by a solve with a preconditioned one."""
    from paper_1208_6387_amd import structure as ST
    p = W.small_elast((3, 3, 3), (2, 2, 2), n_rhs=2, n_perm=1, seed=3)
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats)
    pb = ST.create_problem(p)
    f = ST.loads_to_device(p)
    _, u_ref, _ = O.FetiOracle(p).solve("block", tol=1e-12)
    its = {}
    for coarse in ["none", "lumped", "dirichlet", "none", "dirichlet"]:
        res = R.block_krylov_solve(pb, pats, f, 2, tol=1e-11, max_it=500, method=R.BLOCK_CG,
                                   precond=R.PRECOND_DIRICHLET, coarse=KINDS[coarse])
        oc = O.FetiOracle(p, coarse=None if coarse == "none" else coarse)
        _check(R, p, res, u_ref, oc, 1e-8)
        its.setdefault(coarse, []).append(res.stats["iterations"])
    assert its["none"][0] == its["none"][1] and its["dirichlet"][0] == its["dirichlet"][1], its


def test_coarse_precond_error_paths(R):
    from paper_1208_6387_amd import structure as ST
    p = W.small_elast((3, 3, 3), (3, 2, 2), n_rhs=1, n_perm=4, seed=7)
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats)
    pb = ST.create_problem(p)
    f = ST.loads_to_device(p)
    with pytest.raises(R.RpfError, match="EINVAL.*projector"):
        R.block_krylov_solve(pb, pats, f, 1, tol=1e-8, max_it=50, coarse=3)
    with pytest.raises(R.RpfError, match="EINVAL.*periodic"):
        R.block_krylov_solve(pb, pats, f, 1, tol=1e-8, max_it=50, method=R.ORTHODIR, periodic=True,
                             coarse=R.PRECOND_LUMPED)


@pytest.mark.parametrize("coarse", ["lumped", "dirichlet"])
def test_coarse_precond_singular_refused(R, coarse):
    """A pattern with no interior dofs (one brick element): S = K_bb = K, whose kernel holds the
    rigid traces, so G^T F~^{-1} G is singular (the oracle's eigenvalues, checked on the CPU) and the
    solve is refused with RPF_ENOTSPD instead of iterating on a singular coarse problem."""
    from paper_1208_6387_amd import structure as ST
    p = W.small_elast((1, 2, 1), (1, 1, 2), n_rhs=1, n_perm=1, seed=0)
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats)
    pb = ST.create_problem(p)
    f = ST.loads_to_device(p)
    with pytest.raises(R.RpfError, match="ENOTSPD.*not positive definite"):
        R.block_krylov_solve(pb, pats, f, 1, tol=1e-10, max_it=200, coarse=KINDS[coarse])
    # the plain projector still solves it
    res = R.block_krylov_solve(pb, pats, f, 1, tol=1e-10, max_it=200)
    assert res.stats["rel_residual"] <= 1e-10
