"""HIP path against the CPU oracle, stage by stage and end to end (through the C ABI).

Tolerances (FP64 path):
* S, S+, F X: element by element relative to the largest entry, 1e-12 (S), 1e-9 (S+: the
  inverse of S + Z Z^T carries its condition number, ~1e3 here), 1e-11 (F X, Q F X);
* the kernel: the projector Z Z^T, 1e-10;
* solutions: displacements within 1e-8 relative to the oracle solved to 1e-12, with the GPU
  tolerance 1e-11 (two 1e-8 iterates may differ by more than 1e-8).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    import paper_1208_6387_amd as R
    R.load()
    return R


def _problem(name):
    if name == "elast-3cube-3x2x2":
        return W.small_elast((3, 3, 3), (3, 2, 2), n_rhs=2, n_perm=4, seed=7)
    if name == "heat-row":
        return W.config(0)
    if name == "ring-stand":
        return W.ring_heat(3, (4, 4), stand=True, n_rhs=2, n_perm=3, dirichlet_bottom=True)
    if name == "elast-ragged-2x3x1":
        return W.small_elast((5, 2, 3), (2, 3, 1), n_rhs=3, n_perm=2, seed=9)
    if name == "ring-elast-rotated":
        return W.ring_elast(3, (2, 3, 2), n_rhs=2, n_perm=3)
    raise KeyError(name)


CASES = ["elast-3cube-3x2x2", "heat-row", "ring-stand", "elast-ragged-2x3x1", "ring-elast-rotated"]


@pytest.fixture(scope="module", params=CASES)
def case(request, R):
    from paper_1208_6387_amd import structure as ST
    p = _problem(request.param)
    print(f"\n[case {request.param}] n_lambda={p.n_lambda} n_occ={p.n_occ}", flush=True)
    o = O.FetiOracle(p)
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats)
    pb = ST.create_problem(p)
    return p, o, pats, pb


def test_schur_and_kernel(case, R):
    p, o, pats, pb = case
    for P, Po in zip(pats, o.pats):
        S = R.pattern_export(P, "S").cpu().numpy()
        assert np.abs(S - Po.S).max() <= 1e-12 * np.abs(Po.S).max()
        assert P.kernel_dim == Po.k
        Z = R.pattern_export(P, "Z").cpu().numpy()
        assert np.abs(Z.T @ Z - np.eye(Po.k)).max() < 1e-12
        assert np.abs(Z @ Z.T - Po.Z @ Po.Z.T).max() < 1e-10


def test_pseudo_inverse(case, R):
    p, o, pats, pb = case
    for P, Po in zip(pats, o.pats):
        Sp = R.pattern_export(P, "Splus").cpu().numpy()
        assert np.abs(Sp - Po.Splus).max() <= 1e-9 * np.abs(Po.Splus).max()


@pytest.mark.parametrize("m", [1, 3, 8, 11])
def test_feti_apply(case, R, m):
    p, o, pats, pb = case
    rng = np.random.default_rng(m)
    X = rng.standard_normal((p.n_lambda, m))
    Xd = torch.from_numpy(X).cuda()
    Y = R.feti_apply(pb, pats, Xd).cpu().numpy()
    ref = o.F(X)
    assert np.abs(Y - ref).max() <= 1e-11 * np.abs(ref).max()
    Yq = R.feti_apply(pb, pats, Xd, project=True).cpu().numpy()
    refq = o.Q(ref)
    assert np.abs(Yq - refq).max() <= 1e-11 * np.abs(ref).max()


def test_feti_apply_strided_block(case, R):
    """Row stride larger than the block width (ldx > m), both for input and output."""
    p, o, pats, pb = case
    rng = np.random.default_rng(5)
    big = torch.from_numpy(rng.standard_normal((p.n_lambda, 7))).cuda()
    X = big[:, 2:5]
    out = torch.full((p.n_lambda, 9), 7.0, dtype=torch.float64, device="cuda")
    R.feti_apply(pb, pats, X, out=out[:, 1:4])
    got = out.cpu().numpy()
    ref = o.F(X.cpu().numpy())
    assert np.abs(got[:, 1:4] - ref).max() <= 1e-11 * np.abs(ref).max()
    assert np.all(got[:, 0] == 7.0) and np.all(got[:, 4:] == 7.0)


@pytest.mark.parametrize("nr", [1, 2])
def test_feti_permute(case, R, nr):
    """Permuted multivector (with the frame turn of rotated occurrences) and its re-projection."""
    p, o, pats, pb = case
    Z = np.random.default_rng(10 + nr).standard_normal((p.n_lambda, nr))
    Wg = R.feti_permute(pb, torch.from_numpy(Z).cuda()).cpu().numpy()
    ref = o.permute(Z)
    assert Wg.shape == ref.shape
    assert np.abs(Wg - ref).max() <= 1e-14 * np.abs(ref).max()
    Wq = R.feti_permute(pb, torch.from_numpy(Z).cuda(), patterns=pats, project=True).cpu().numpy()
    assert np.abs(Wq - o.Q(ref)).max() <= 1e-11 * np.abs(ref).max()
    # strided operands
    big = torch.from_numpy(np.random.default_rng(3).standard_normal((p.n_lambda, nr + 3))).cuda()
    out = torch.full((p.n_lambda, nr * pb.n_perm + 2), 5.0, dtype=torch.float64, device="cuda")
    R.feti_permute(pb, big[:, 1:1 + nr], out=out[:, 1:1 + nr * pb.n_perm])
    got = out.cpu().numpy()
    ref2 = o.permute(big[:, 1:1 + nr].cpu().numpy())
    assert np.abs(got[:, 1:1 + nr * pb.n_perm] - ref2).max() <= 1e-14 * np.abs(ref2).max()
    assert np.all(got[:, 0] == 5.0) and np.all(got[:, -1] == 5.0)


@pytest.mark.parametrize("method", ["classical", "block_cg", "orthodir"])
def test_solve(case, R, method):
    from paper_1208_6387_amd import structure as ST
    p, o, pats, pb = case
    meth = {"classical": R.CLASSICAL, "block_cg": R.BLOCK_CG, "orthodir": R.ORTHODIR}[method]
    f = ST.loads_to_device(p)
    res = R.block_krylov_solve(pb, pats, f, p.n_rhs, tol=1e-11, max_it=3000, method=meth)
    u = ST.split_u(p, res.u)
    lam = res.lam.cpu().numpy()
    lam_o, u_o, st = o.solve("block", tol=1e-12)
    scale = max(np.abs(x).max() for x in u_o)
    err = max(np.abs(a - b).max() for a, b in zip(u, u_o)) / scale
    assert err < 1e-8, (method, err, res.stats)
    assert np.abs(lam - lam_o).max() < 1e-7 * np.abs(lam_o).max()
    assert res.stats["rel_residual"] <= 1e-11
    # iterations of the GPU classical form equal the oracle's per-case CG counts up to a few
    if method == "classical" and p.n_rhs == 1:
        _, _, sc = o.solve("classical", tol=1e-11)
        assert abs(res.stats["iterations"] - max(sc["iterations"])) <= 2


# Low-precision flexibility products: relative error bounds of the operator (max-norm, relative to
# max |F X|).  FP32 and bf16x3 are limited by FP32 accumulation over n_b terms (~sqrt(n_b) 2^-24)
# and, for bf16x3, by the 16-bit split (~2^-17); plain bf16 by its 8-bit significand.
LOWPREC_TOL = {"fp32": 5e-5, "bf16x3": 5e-5, "bf16": 3e-2}


@pytest.mark.parametrize("form", ["fp32", "bf16x3", "bf16"])
@pytest.mark.parametrize("m", [1, 8, 11])
def test_feti_apply_lowprec(case, R, form, m):
    p, o, pats, pb = case
    prec = {"fp32": R.FP32, "bf16x3": R.BF16X3, "bf16": R.BF16}[form]
    for P in pats:
        R.pattern_condense(P, prec)
    rng = np.random.default_rng(100 + m)
    X = rng.standard_normal((p.n_lambda, m))
    Y = R.feti_apply(pb, pats, torch.from_numpy(X).cuda(), prec=prec).cpu().numpy()
    ref = o.F(X)
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    assert err <= LOWPREC_TOL[form], (form, err)
    assert err > 0.0   # really computed in low precision


@pytest.mark.parametrize("form", ["fp32", "bf16x3"])
def test_solve_mixed_refined(case, R, form):
    """Mixed form: low-precision inner solves + FP64 refinement reach the FP64 tolerance, and u is
    within 1e-6 of the oracle."""
    from paper_1208_6387_amd import structure as ST
    p, o, pats, pb = case
    prec = {"fp32": R.FP32, "bf16x3": R.BF16X3}[form]
    for P in pats:
        R.pattern_condense(P, prec)
    f = ST.loads_to_device(p)
    res = R.block_krylov_solve(pb, pats, f, p.n_rhs, tol=1e-8, max_it=3000, method=R.ORTHODIR, prec=prec,
                               inner_tol=1e-3)
    assert res.stats["rel_residual"] <= 1e-8
    u = ST.split_u(p, res.u)
    lam_o, u_o, st = o.solve("block", tol=1e-12)
    scale = max(np.abs(x).max() for x in u_o)
    err = max(np.abs(a - b).max() for a, b in zip(u, u_o)) / scale
    assert err < 1e-6, (form, err, res.stats)


def test_heat_row_closed_form(R):
    from paper_1208_6387_amd import structure as ST
    p = W.config(0)
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats)
    pb = ST.create_problem(p)
    for meth in (R.CLASSICAL, R.ORTHODIR):
        res = R.block_krylov_solve(pb, pats, ST.loads_to_device(p), 1, tol=1e-10, max_it=500, method=meth)
        u = ST.split_u(p, res.u)
        x = p.patterns[0].coords[:, 0]
        for s in range(4):
            xs = x + s
            assert np.abs(u[s][:, 0] - xs * (8 - xs) / 2).max() < 1e-8


def test_structure_reused_with_new_pattern_handles(R):
    """One structure, patterns factored, freed and factored again (handles may reuse addresses):
    the coarse space must be rebuilt for the new handles and both solves agree."""
    from paper_1208_6387_amd import structure as ST
    p = W.small_elast((3, 3, 3), (2, 2, 1), n_rhs=2, n_perm=2, seed=4)
    pb = ST.create_problem(p)
    f = ST.loads_to_device(p)
    outs = []
    for rep in range(3):
        pats = ST.factor_patterns(p)
        ST.condense_patterns(pats)
        res = R.block_krylov_solve(pb, pats, f, p.n_rhs, tol=1e-10, max_it=500, method=R.ORTHODIR)
        outs.append(res.u.cpu().numpy())
        for P in pats:
            P.free()
    for u in outs[1:]:
        assert np.abs(u - outs[0]).max() <= 1e-9 * np.abs(outs[0]).max()


def test_kernel_dimension_mismatch_is_reported(R):
    p = W.small_elast((2, 2, 2), (2, 1, 1))
    pat = p.patterns[0]
    val = torch.from_numpy(pat.K.data.copy()).cuda()
    with pytest.raises(R.RpfError, match="EKERNEL"):
        R.pattern_factor(pat.K.indptr, pat.K.indices, val, pat.bdofs, 3, expected_kernel_dim=5)


def test_indefinite_interior_is_reported(R):
    p = W.small_elast((3, 3, 3), (2, 1, 1))
    pat = p.patterns[0]
    K = pat.K.copy()
    K.data = -K.data
    val = torch.from_numpy(K.data.copy()).cuda()
    with pytest.raises(R.RpfError, match="ENOTSPD"):
        R.pattern_factor(K.indptr, K.indices, val, pat.bdofs, 3)


def test_noconv_reports_last_iterate(R):
    from paper_1208_6387_amd import structure as ST
    p = W.small_elast((3, 3, 3), (3, 2, 2), n_rhs=1, n_perm=1, seed=7)
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats)
    pb = ST.create_problem(p)
    res = R.block_krylov_solve(pb, pats, ST.loads_to_device(p), 1, tol=1e-12, max_it=3, method=R.ORTHODIR,
                               raise_on_noconv=False)
    assert res.status == -5
    assert res.stats["iterations"] == 3 and res.stats["rel_residual"] > 1e-12
    assert np.isfinite(res.u.cpu().numpy()).all()
