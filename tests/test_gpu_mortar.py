"""Non-Boolean (mortar) assembly on the GPU through the C ABI (section 5: non-Boolean assembly
operators for non-matching pattern meshes): the operator F, its projection and the solutions on
rows of alternating non-matching patterns against the oracle (whose mortar path is pinned by the
saddle-point solve and the exact linear flux solution), and the weighted kernels on Boolean
structures against the signed Boolean ones."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = {
    "heat": dict(kind="heat", shapes=((8, 8), (6, 6)), n_occ=4),
    "heat-wide": dict(kind="heat", shapes=((24, 16), (10, 20)), n_occ=6),
    "elast": dict(kind="elast", shapes=((3, 3, 3), (2, 2, 2)), n_occ=3),
    "elast-6x4": dict(kind="elast", shapes=((6, 6, 6), (4, 4, 4)), n_occ=4),
}


@pytest.fixture(scope="module")
def R():
    import paper_1208_6387_amd as R
    R.load()
    return R


@pytest.fixture(scope="module", params=sorted(CASES))
def mortar(request, R):
    from paper_1208_6387_amd import structure as ST
    p = W.mortar_row(n_rhs=2, **CASES[request.param])
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats, (R.FP64, R.BF16X3, R.FP32))
    pb = ST.create_problem(p)
    o = O.FetiOracle(p)
    return request.param, p, o, pats, pb


@pytest.mark.parametrize("ncol", [3, 8, 40])
def test_operator_against_oracle(mortar, R, ncol):
    """F X and Q^T F X with the weighted gather and scatter, in every precision of the product."""
    name, p, o, pats, pb = mortar
    X = np.random.default_rng(ncol).standard_normal((p.n_lambda, ncol))
    Xd = torch.from_numpy(X).cuda()
    ref = o.F(X)
    scale = np.abs(ref).max()
    for prec, tol in ((R.FP64, 1e-12), (R.BF16X3, 5e-5), (R.FP32, 5e-5)):
        Y = R.feti_apply(pb, pats, Xd, prec=prec).cpu().numpy()
        assert np.abs(Y - ref).max() <= tol * scale, (name, prec)
    Yq = R.feti_apply(pb, pats, Xd, project=True).cpu().numpy()
    refq = o.Q(ref)
    assert np.abs(Yq - refq).max() <= 1e-11 * np.abs(refq).max(), name
    # G^T of the projected product vanishes (the rows of G are weighted sums of the rigid modes)
    assert np.abs(o.G.T @ Yq).max() <= 1e-10 * np.abs(refq).max() * np.sqrt(p.n_lambda)


@pytest.mark.parametrize("form,method", [("fp64", "classical"), ("fp64", "block_cg"), ("fp64", "orthodir"),
                                         ("bf16x3", "block_cg"), ("bf16x3", "orthodir")])
def test_solution_against_constrained_solve(mortar, R, form, method):
    """u and lambda on non-matching occurrences against the dense saddle-point solve of the
    constrained problem: 1e-8 at a 1e-10 residual in both forms."""
    from paper_1208_6387_amd import structure as ST
    name, p, o, pats, pb = mortar
    prec = R.FP64 if form == "fp64" else R.BF16X3
    meth = {"classical": R.CLASSICAL, "block_cg": R.BLOCK_CG, "orthodir": R.ORTHODIR}[method]
    res = R.block_krylov_solve(pb, pats, ST.loads_to_device(p), p.n_rhs, tol=1e-10, max_it=3000, method=meth,
                               prec=prec, inner_tol=1e-4)
    u = ST.split_u(p, res.u)
    ub, lb = O.constrained_solve(p, o)
    scale = max(np.abs(b).max() for b in ub)
    err = max(np.abs(a - b).max() for a, b in zip(u, ub)) / scale
    lerr = np.abs(res.lam.cpu().numpy() - lb).max() / np.abs(lb).max()
    print(f"[mortar] {name} {form} {method}: its={res.stats['iterations']} u_err={err:.2e} lam_err={lerr:.2e}")
    assert res.stats["rel_residual"] <= 1e-10
    assert err <= 1e-8 and lerr <= 1e-7, (err, lerr)


def test_flux_solution_is_linear(R):
    """The unit-flux heat row across non-matching interfaces: the GPU solution is u = x (to 1e-9 at a
    1e-11 residual; max |u| = 4)."""
    from paper_1208_6387_amd import structure as ST
    p = W.mortar_row("heat", shapes=((8, 8), (6, 6)), n_occ=4, load="flux")
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats)
    pb = ST.create_problem(p)
    res = R.block_krylov_solve(pb, pats, ST.loads_to_device(p), p.n_rhs, tol=1e-11, max_it=2000, method=R.ORTHODIR)
    u = ST.split_u(p, res.u)
    for s in range(p.n_occ):
        x = p.patterns[p.occ_pattern[s]].coords[:, 0] + s
        assert np.abs(u[s][:, 0] - x).max() < 1e-9, s


@pytest.mark.parametrize("maker", ["elast", "ring"])
def test_weighted_kernels_on_boolean_structures(R, maker):
    """A signed Boolean structure described through one-node weighted entries takes the weighted
    kernels; F X, the projection and the solve equal those of the Boolean kernels (rotated frames
    and eight permutations included)."""
    from paper_1208_6387_amd import structure as ST
    p = (W.small_elast((3, 3, 3), (3, 2, 2), n_rhs=2, n_perm=2, seed=71) if maker == "elast"
         else W.ring_elast(n_occ=4, n_rhs=1, seed=72))
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats, (R.FP64, R.BF16X3))
    pw = ST.create_problem(p, weighted=True)
    pbool = ST.create_problem(p, weighted=False)
    X = torch.from_numpy(np.random.default_rng(5).standard_normal((p.n_lambda, 8))).cuda()
    for prec, tol in ((R.FP64, 1e-13), (R.BF16X3, 1e-6)):
        for proj in (False, True):
            a = R.feti_apply(pw, pats, X, prec=prec, project=proj)
            b = R.feti_apply(pbool, pats, X, prec=prec, project=proj)
            assert (a - b).abs().max().item() <= tol * b.abs().max().item(), (prec, proj)
    f = ST.loads_to_device(p)
    rw = R.block_krylov_solve(pw, pats, f, p.n_rhs, tol=1e-10, max_it=2000, method=R.ORTHODIR)
    rb = R.block_krylov_solve(pbool, pats, f, p.n_rhs, tol=1e-10, max_it=2000, method=R.ORTHODIR)
    assert (rw.u - rb.u).abs().max().item() <= 1e-9 * rb.u.abs().max().item()


def test_grouped_schedule_with_weights(R):
    """The grouped product launch under the weighted gather and scatter."""
    from paper_1208_6387_amd import structure as ST
    p = W.mortar_row("elast", shapes=((6, 6, 6), (4, 4, 4)), n_occ=4, n_rhs=1)
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats, (R.FP64, R.BF16X3))
    pb = ST.create_problem(p)
    o = O.FetiOracle(p)
    X = np.random.default_rng(9).standard_normal((p.n_lambda, 8))
    ref = o.F(X)
    for prec, tol in ((R.FP64, 1e-12), (R.BF16X3, 5e-5)):
        for tile in (64, 128):
            R.problem_set_schedule(pb, 8, prec, tile, 1024)
            Y = R.feti_apply(pb, pats, torch.from_numpy(X).cuda(), prec=prec).cpu().numpy()
            assert np.abs(Y - ref).max() <= tol * np.abs(ref).max(), (prec, tile)


def test_weighted_refuses_preconditioners(R):
    from paper_1208_6387_amd import _lib
    from paper_1208_6387_amd import structure as ST
    p = W.mortar_row("heat", shapes=((8, 8), (6, 6)), n_occ=4)
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats)
    pb = ST.create_problem(p)
    X = torch.ones((p.n_lambda, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(R.RpfError) as e:
        R.feti_precond(pb, pats, X, R.PRECOND_DIRICHLET)
    assert e.value.code == _lib.RPF_EINVAL
    for kw in (dict(precond=R.PRECOND_LUMPED), dict(coarse=R.PRECOND_DIRICHLET)):
        with pytest.raises(R.RpfError) as e:
            R.block_krylov_solve(pb, pats, ST.loads_to_device(p), p.n_rhs, tol=1e-8, max_it=50, **kw)
        assert e.value.code == _lib.RPF_EINVAL
