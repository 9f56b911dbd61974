"""Parity at the benchmark sizes, in the launch configuration bench.py times.

* 64-occurrence elasticity (12^3 bricks, 8 load cases): the GPU operator F X against the
  oracle's element by element, and the GPU solutions (FP64 and bf16x3 forms) checked with the
  oracle's own F and Q: the FP64 interface residual Q^T (d - F lambda) recomputed on the CPU.
* 512-occurrence elasticity (20^3 bricks, 16 load cases): too large for the oracle's condensation;
  the solution is checked through properties that characterise it at any size, computed on the
  CPU from the problem statement only (tests/props.py): interface continuity of u at every
  multiplier, u = 0 on the clamped face, and the local equilibrium K^(s) u^(s) = f^(s) - t^T A^(s)T
  lambda of every occurrence.
* uneven batch (48 plates, 16 ring sectors, one base block, rotated frames, 8 permutations): the
  operator in every precision against the oracle's F, and FP64 / mixed ORTHODIR solutions against
  the oracle's residual and displacements.
"""
import numpy as np
import pytest

import oracle as O
import props
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    import paper_1208_6387_amd as R
    R.load()
    return R


@pytest.fixture(scope="module")
def config2(R):
    from paper_1208_6387_amd import structure as ST
    p = W.config(2)
    print("\n[fullsize] 64 x 12^3 bricks, 8 load cases", flush=True)
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats, (R.FP64, R.BF16X3))
    pb = ST.create_problem(p)
    o = O.FetiOracle(p)
    return p, o, pats, pb


def test_config2_operator(config2, R):
    p, o, pats, pb = config2
    X = np.random.default_rng(2).standard_normal((p.n_lambda, 8))
    Y = R.feti_apply(pb, pats, torch.from_numpy(X).cuda()).cpu().numpy()
    ref = o.F(X)
    assert np.abs(Y - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("form,tol", [("bf16x3", 5e-5), ("bf16", 3e-2), ("fp64", 1e-11)])
@pytest.mark.parametrize("ncol", [97, 96])
def test_config2_operator_large_tiles(config2, R, form, tol, ncol):
    """97 columns per occurrence make 64 x 97 = 6208 product columns: with n_b = 2598 that is 11 x 25
    tiles of 256 x 256, enough for the large-tile bf16 kernel, and both sides are ragged (2598 =
    10 x 256 + 38, 6208 = 24 x 256 + 64); 96 columns (a multiple of 4) take the four-column scatter
    from the row-major result.  In FP64 the same shapes take the large-problem FP64 kernel (21 x 49
    tiles of 128 x 128, ragged on both sides, zero-padded W blocks).  Checked against the oracle's
    FP64 operator."""
    p, o, pats, pb = config2
    prec = {"bf16x3": R.BF16X3, "bf16": R.BF16, "fp64": R.FP64}[form]
    X = np.random.default_rng(ncol).standard_normal((p.n_lambda, ncol))
    Y = R.feti_apply(pb, pats, torch.from_numpy(X).cuda(), prec=prec).cpu().numpy()
    ref = o.F(X)
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    assert err <= tol and (form == "fp64" or err > 0.0), (form, err)
    # every column, the ragged last ones included, is within the bound on its own
    colerr = np.abs(Y - ref).max(0) / np.abs(ref).max(0)
    assert colerr.max() <= 4 * tol, (form, colerr.max(), int(colerr.argmax()))


@pytest.mark.parametrize("form,method", [("fp64", "orthodir"), ("bf16x3", "orthodir"), ("bf16x3", "block_cg")])
def test_config2_solution(config2, R, form, method):
    from paper_1208_6387_amd import structure as ST
    p, o, pats, pb = config2
    prec = R.FP64 if form == "fp64" else R.BF16X3
    meth = R.ORTHODIR if method == "orthodir" else R.BLOCK_CG
    res = R.block_krylov_solve(pb, pats, ST.loads_to_device(p), p.n_rhs, tol=1e-8, max_it=3000, method=meth,
                               prec=prec, inner_tol=1e-4)
    lam = res.lam.cpu().numpy()
    g, d, e = o.loads()
    r0 = np.linalg.norm(o.Q(d - o.F(o.lambda0(e))), axis=0)
    r = np.linalg.norm(o.Q(d - o.F(lam)), axis=0)
    assert np.max(r / r0) <= 1.05e-8, (form, method, np.max(r / r0))
    assert np.abs(o.G.T @ lam - e).max() <= 1e-9 * np.abs(e).max()
    u = ST.split_u(p, res.u)
    scale = max(np.abs(x).max() for x in u)
    assert props.continuity_gap(p, u) <= (1e-8 if form == "fp64" else 1e-6) * scale
    assert props.equilibrium_residual(p, u, lam) <= 1e-10


def test_config4_operator_forms(R):
    """512 occurrences: the low-precision products (large-tile kernels) against the FP64 one, and the
    FP64 operator's symmetry x^T F y = y^T F x (a property of F at any size)."""
    from paper_1208_6387_amd import structure as ST
    p = W.config(4)
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats, (R.FP64, R.BF16X3, R.FP32))
    pb = ST.create_problem(p)
    g = torch.Generator(device="cuda").manual_seed(4)
    X = torch.randn(pb.n_lambda, 16, dtype=torch.float64, device="cuda", generator=g)
    Y = torch.randn(pb.n_lambda, 16, dtype=torch.float64, device="cuda", generator=g)
    FX = R.feti_apply(pb, pats, X)
    FY = R.feti_apply(pb, pats, Y)
    a = (Y * FX).sum(0)
    b = (X * FY).sum(0)
    assert torch.max(torch.abs(a - b) / torch.abs(a)).item() < 1e-11
    scale = FX.abs().max().item()
    for prec, tol in ((R.BF16X3, 5e-5), (R.FP32, 5e-5)):
        Z = R.feti_apply(pb, pats, X, prec=prec)
        assert (Z - FX).abs().max().item() <= tol * scale, prec


@pytest.mark.parametrize("kind,form,tol", [("dirichlet", "fp64", 1e-12), ("dirichlet", "bf16x3", 5e-5),
                                           ("lumped", "fp64", 1e-12)])
@pytest.mark.parametrize("ncol", [8, 97])
def test_config2_preconditioner(config2, R, kind, form, tol, ncol):
    """The preconditioners at 64 occurrences against the oracle's F~^{-1}: 8 columns as in the
    solves, 97 for the large-tile product kernels (ragged 256 x 256 bf16 tiles, 128 x 128 FP64
    tiles) running with S in place of S+."""
    p, o, pats, pb = config2
    prec = R.FP64 if form == "fp64" else R.BF16X3
    k = R.PRECOND_DIRICHLET if kind == "dirichlet" else R.PRECOND_LUMPED
    X = np.random.default_rng(300 + ncol).standard_normal((p.n_lambda, ncol))
    Y = R.feti_precond(pb, pats, torch.from_numpy(X).cuda(), k, prec=prec).cpu().numpy()
    ref = o.precondition(X, kind)
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    assert err <= tol and (form == "fp64" or err > 0.0), (kind, form, err)


def test_config4_preconditioned(R):
    """512 occurrences with the Dirichlet preconditioner, as bench.py times it: the operator is
    symmetric and positive (x^T F~^{-1} x > 0 off the kernel of A^T), its bf16x3 form agrees with the
    FP64 one, and the preconditioned mixed block-CG solution satisfies continuity, the clamped face
    and local equilibrium on sampled occurrences."""
    from paper_1208_6387_amd import structure as ST
    p = W.config(4)
    print("\n[fullsize] 512 x 20^3 bricks, Dirichlet preconditioner", flush=True)
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats, (R.FP64, R.BF16X3))
    pb = ST.create_problem(p)
    g = torch.Generator(device="cuda").manual_seed(7)
    X = torch.randn(pb.n_lambda, 16, dtype=torch.float64, device="cuda", generator=g)
    Y = torch.randn(pb.n_lambda, 16, dtype=torch.float64, device="cuda", generator=g)
    MX = R.feti_precond(pb, pats, X, R.PRECOND_DIRICHLET)
    MY = R.feti_precond(pb, pats, Y, R.PRECOND_DIRICHLET)
    a = (Y * MX).sum(0)
    b = (X * MY).sum(0)
    assert torch.max(torch.abs(a - b) / torch.abs(a)).item() < 1e-11
    assert torch.min((X * MX).sum(0)).item() > 0.0
    Z = R.feti_precond(pb, pats, X, R.PRECOND_DIRICHLET, prec=R.BF16X3)
    assert (Z - MX).abs().max().item() <= 5e-5 * MX.abs().max().item()
    res = R.block_krylov_solve(pb, pats, ST.loads_to_device(p), p.n_rhs, tol=1e-8, max_it=3000,
                               method=R.BLOCK_CG, prec=R.BF16X3, inner_tol=1e-4, max_blocks=48,
                               precond=R.PRECOND_DIRICHLET)
    assert res.stats["rel_residual"] <= 1e-8
    assert res.stats["iterations"] < 80, res.stats
    lam = res.lam.cpu().numpy()
    u = ST.split_u(p, res.u)
    scale = max(np.abs(x).max() for x in u)
    assert props.continuity_gap(p, u) <= 1e-6 * scale
    assert props.dirichlet_max(p, u) <= 1e-6 * scale
    assert props.equilibrium_residual(p, u, lam) <= 1e-9


@pytest.fixture(scope="module")
def config3(R):
    from paper_1208_6387_amd import structure as ST
    p = W.config(3)
    print("\n[fullsize] uneven: 48 plates, 16 ring sectors, one base block; 8 permutations", flush=True)
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats, (R.FP64, R.BF16X3, R.FP32))
    pb = ST.create_problem(p)
    o = O.FetiOracle(p)
    lam_o, u_o, st_o = o.solve("block", tol=1e-10)
    return p, o, pats, pb, lam_o, u_o


def test_config3_operator(config3, R):
    """Uneven batch (three patterns, rotated frames): F X per precision against the oracle's F."""
    p, o, pats, pb, _, _ = config3
    X = np.random.default_rng(3).standard_normal((p.n_lambda, 8))
    ref = o.F(X)
    scale = np.abs(ref).max()
    Xd = torch.from_numpy(X).cuda()
    for prec, tol in ((R.FP64, 1e-11), (R.BF16X3, 5e-5), (R.FP32, 5e-5)):
        Y = R.feti_apply(pb, pats, Xd, prec=prec).cpu().numpy()
        err = np.abs(Y - ref).max() / scale
        assert err <= tol, (prec, err)


@pytest.mark.parametrize("form", ["fp64", "bf16x3"])
def test_config3_solution(config3, R, form):
    """Uneven batch solved with ORTHODIR over 8 permuted copies: FP64 residual at 1e-8 against the
    oracle's operator, u within 1e-8 (FP64 form) and 1e-6 (mixed form) of the oracle's solution."""
    from paper_1208_6387_amd import structure as ST
    p, o, pats, pb, lam_o, u_o = config3
    prec = R.FP64 if form == "fp64" else R.BF16X3
    res = R.block_krylov_solve(pb, pats, ST.loads_to_device(p), p.n_rhs, tol=1e-8, max_it=2000,
                               method=R.ORTHODIR, prec=prec, inner_tol=1e-4)
    lam = res.lam.cpu().numpy()
    g, d, e = o.loads()
    r0 = np.linalg.norm(o.Q(d - o.F(o.lambda0(e))), axis=0)
    r = np.linalg.norm(o.Q(d - o.F(lam)), axis=0)
    assert np.max(r / r0) <= 1.05e-8, (form, np.max(r / r0))
    u = ST.split_u(p, res.u)
    scale = max(np.abs(x).max() for x in u_o)
    err = max(np.abs(a - b).max() for a, b in zip(u, u_o)) / scale
    assert err <= (1e-8 if form == "fp64" else 1e-6), (form, err, res.stats)
