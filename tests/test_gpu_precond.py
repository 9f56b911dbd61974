"""Lumped and Dirichlet preconditioners (section 2) on the HIP path against the CPU oracle,
through the C ABI: the operator F~^{-1} alone, then preconditioned solves.

Tolerances: F~^{-1} X in FP64 element by element relative to max |ref|, 1e-12 (a product with
S or the sparse K_bb between two scalings); low-precision Dirichlet products as the operator F
(5e-5 FP32 and bf16x3, 3e-2 bf16); solutions as for the unpreconditioned solver (1e-8 FP64,
1e-6 mixed, against the oracle solved to 1e-12).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KINDS = {"lumped": 1, "dirichlet": 2}


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
    if name == "mirror-pair":
        return W.mirror_row_heat(2, (4, 4), n_rhs=2)
    raise KeyError(name)


CASES = ["elast-3cube-3x2x2", "heat-3x2", "ring-elast-rotated", "elast-ragged-2x3x1", "mirror-pair"]


@pytest.fixture(scope="module", params=CASES)
def case(request, R):
    from paper_1208_6387_amd import structure as ST
    p = _problem(request.param)
    print(f"\n[precond case {request.param}] n_lambda={p.n_lambda} n_occ={p.n_occ}", flush=True)
    o = O.FetiOracle(p)
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats, precs=(R.FP64, R.FP32, R.BF16X3))
    pb = ST.create_problem(p)
    return request.param, p, o, pats, pb


@pytest.mark.parametrize("kind", ["lumped", "dirichlet"])
@pytest.mark.parametrize("m", [1, 8, 11])
def test_feti_precond(case, R, kind, m):
    name, p, o, pats, pb = case
    X = np.random.default_rng(20 + m).standard_normal((p.n_lambda, m))
    Xd = torch.from_numpy(X).cuda()
    Y = R.feti_precond(pb, pats, Xd, KINDS[kind]).cpu().numpy()
    ref = o.precondition(X, kind)
    assert np.abs(Y - ref).max() <= 1e-12 * np.abs(ref).max(), (kind, np.abs(Y - ref).max() / np.abs(ref).max())
    Yq = R.feti_precond(pb, pats, Xd, KINDS[kind], project=True).cpu().numpy()
    assert np.abs(Yq - o.Q(ref)).max() <= 1e-11 * np.abs(ref).max()


def test_feti_precond_none_and_strided(case, R):
    name, p, o, pats, pb = case
    rng = np.random.default_rng(7)
    big = torch.from_numpy(rng.standard_normal((p.n_lambda, 7))).cuda()
    X = big[:, 2:5]
    out = torch.full((p.n_lambda, 9), 3.0, dtype=torch.float64, device="cuda")
    R.feti_precond(pb, None, X, R.PRECOND_NONE, out=out[:, 1:4])
    got = out.cpu().numpy()
    assert np.array_equal(got[:, 1:4], X.cpu().numpy())
    R.feti_precond(pb, pats, X, R.PRECOND_DIRICHLET, out=out[:, 1:4])
    got = out.cpu().numpy()
    ref = o.precondition(X.cpu().numpy(), "dirichlet")
    assert np.abs(got[:, 1:4] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.all(got[:, 0] == 3.0) and np.all(got[:, 4:] == 3.0)


LOWPREC_TOL = {"fp32": 5e-5, "bf16x3": 5e-5, "bf16": 3e-2}


@pytest.mark.parametrize("form", ["fp32", "bf16x3", "bf16"])
@pytest.mark.parametrize("m", [1, 8])
def test_feti_precond_dirichlet_lowprec(case, R, form, m):
    name, p, o, pats, pb = case
    prec = {"fp32": R.FP32, "bf16x3": R.BF16X3, "bf16": R.BF16}[form]
    X = np.random.default_rng(40 + m).standard_normal((p.n_lambda, m))
    Y = R.feti_precond(pb, pats, torch.from_numpy(X).cuda(), R.PRECOND_DIRICHLET, prec=prec).cpu().numpy()
    ref = o.precondition(X, "dirichlet")
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    assert 0.0 < err <= LOWPREC_TOL[form], (form, err)


def test_mirror_pair_dirichlet_is_exact_inverse(R):
    """F~^{-1}_D F = I on two mirror-image non-floating occurrences (the oracle's pin, on the GPU)."""
    from paper_1208_6387_amd import structure as ST
    p = W.mirror_row_heat(2, (4, 4))
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats)
    pb = ST.create_problem(p)
    I = torch.eye(p.n_lambda, dtype=torch.float64, device="cuda")
    FI = R.feti_apply(pb, pats, I)
    M = R.feti_precond(pb, pats, FI.contiguous(), R.PRECOND_DIRICHLET).cpu().numpy()
    assert np.abs(M - np.eye(p.n_lambda)).max() < 1e-12
    res = R.block_krylov_solve(pb, pats, ST.loads_to_device(p), 1, tol=1e-12, max_it=50, method=R.CLASSICAL,
                               precond=R.PRECOND_DIRICHLET)
    assert res.stats["iterations"] <= 2


@pytest.mark.parametrize("kind", ["lumped", "dirichlet"])
@pytest.mark.parametrize("method", ["classical", "block_cg", "orthodir"])
def test_solve_preconditioned(case, R, kind, method):
    from paper_1208_6387_amd import structure as ST
    name, p, o, pats, pb = case
    meth = {"classical": R.CLASSICAL, "block_cg": R.BLOCK_CG, "orthodir": R.ORTHODIR}[method]
    f = ST.loads_to_device(p)
    res = R.block_krylov_solve(pb, pats, f, p.n_rhs, tol=1e-11, max_it=3000, method=meth, precond=KINDS[kind])
    u = ST.split_u(p, res.u)
    lam_o, u_o, st = o.solve("block", tol=1e-12)
    scale = max(np.abs(x).max() for x in u_o)
    err = max(np.abs(a - b).max() for a, b in zip(u, u_o)) / scale
    assert err < 1e-8, (kind, method, err, res.stats)
    assert res.stats["rel_residual"] <= 1e-11
    # the GPU iteration count follows the oracle's preconditioned solver
    _, _, sp = o.solve("classical" if method == "classical" else "block", tol=1e-11, precond=kind,
                       full_reorth=method != "block_cg")
    # (the classical form advances every load case together: its count is the largest per case)
    ref_it = max(sp["iterations"]) if method == "classical" else sp["iterations"]
    assert res.stats["iterations"] <= ref_it + 3, (res.stats["iterations"], ref_it)


@pytest.mark.parametrize("form", ["fp32", "bf16x3"])
@pytest.mark.parametrize("method", ["block_cg", "orthodir"])
def test_solve_preconditioned_mixed(case, R, form, method):
    from paper_1208_6387_amd import structure as ST
    name, p, o, pats, pb = case
    prec = {"fp32": R.FP32, "bf16x3": R.BF16X3}[form]
    meth = {"block_cg": R.BLOCK_CG, "orthodir": R.ORTHODIR}[method]
    f = ST.loads_to_device(p)
    res = R.block_krylov_solve(pb, pats, f, p.n_rhs, tol=1e-8, max_it=3000, method=meth, prec=prec,
                               inner_tol=1e-3, precond=R.PRECOND_DIRICHLET)
    assert res.stats["rel_residual"] <= 1e-8
    u = ST.split_u(p, res.u)
    lam_o, u_o, st = o.solve("block", tol=1e-12)
    scale = max(np.abs(x).max() for x in u_o)
    err = max(np.abs(a - b).max() for a, b in zip(u, u_o)) / scale
    assert err < 1e-6, (form, method, err, res.stats)


def test_precond_error_paths(R):
    """Bad arguments come back as RPF_EINVAL with a message, nothing is launched."""
    from paper_1208_6387_amd import structure as ST
    p = W.small_elast((2, 2, 2), (2, 1, 1), n_rhs=1)
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats)          # FP64 only
    pb = ST.create_problem(p)
    X = torch.zeros((p.n_lambda, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(R.RpfError, match="EINVAL.*kind"):
        R.feti_precond(pb, pats, X, 3)
    with pytest.raises(R.RpfError, match="EINVAL.*not condensed"):
        R.feti_precond(pb, pats, X, R.PRECOND_DIRICHLET, prec=R.BF16X3)
    with pytest.raises(R.RpfError, match="EINVAL"):
        R.feti_precond(pb, None, X, R.PRECOND_LUMPED)
    f = ST.loads_to_device(p)
    with pytest.raises(R.RpfError, match="EINVAL.*preconditioner"):
        R.block_krylov_solve(pb, pats, f, 1, tol=1e-8, max_it=50, precond=5)
    # the periodic shortcut is ignored with a single permutation
    res = R.block_krylov_solve(pb, pats, f, 1, tol=1e-10, max_it=200, method=R.BLOCK_CG, periodic=True,
                               precond=R.PRECOND_LUMPED)
    assert res.stats["rel_residual"] <= 1e-10
