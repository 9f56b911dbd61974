"""Randomised GPU parity: small structures drawn with fixed draws (derandomised, so every run sees
the same cases), solved through the C ABI in a drawn precision, solver form and preconditioner,
against the CPU oracle's displacements (1e-8 FP64, 1e-6 mixed) and its operator (F X, F~^{-1} X).
"""
import numpy as np
import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    import paper_1208_6387_amd as R
    R.load()
    return R


def _run(R, p, prec_name, method, pc):
    from paper_1208_6387_amd import structure as ST
    prec = {"fp64": R.FP64, "bf16x3": R.BF16X3, "fp32": R.FP32}[prec_name]
    meth = {"classical": R.CLASSICAL, "block_cg": R.BLOCK_CG, "orthodir": R.ORTHODIR}[method]
    kind = {None: R.PRECOND_NONE, "lumped": R.PRECOND_LUMPED, "dirichlet": R.PRECOND_DIRICHLET}[pc]
    if p.n_perm > 1 and method == "block_cg":
        meth = R.ORTHODIR                      # the short recurrence is for one permutation
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats, (R.FP64, prec) if prec != R.FP64 else (R.FP64,))
    pb = ST.create_problem(p)
    o = O.FetiOracle(p)
    # operator parity on a drawn block
    X = np.random.default_rng(p.n_lambda).standard_normal((p.n_lambda, 3))
    Xd = torch.from_numpy(X).cuda()
    F = R.feti_apply(pb, pats, Xd).cpu().numpy()
    ref = o.F(X)
    assert np.abs(F - ref).max() <= 1e-11 * np.abs(ref).max()
    if pc is not None:
        M = R.feti_precond(pb, pats, Xd, kind).cpu().numpy()
        refm = o.precondition(X, pc)
        assert np.abs(M - refm).max() <= 1e-12 * np.abs(refm).max()
    tol = 1e-11 if prec == R.FP64 else 1e-8
    res = R.block_krylov_solve(pb, pats, ST.loads_to_device(p), p.n_rhs, tol=tol, max_it=3000, method=meth,
                               prec=prec, inner_tol=1e-3, precond=kind)
    assert res.stats["rel_residual"] <= tol
    _, u_o, _ = o.solve("block", tol=1e-12)
    u = ST.split_u(p, res.u)
    err = max(np.abs(a - b).max() for a, b in zip(u, u_o)) / max(np.abs(b).max() for b in u_o)
    assert err < (1e-8 if prec == R.FP64 else 1e-6), (p.name, prec_name, method, pc, err)


@settings(max_examples=10, deadline=None, database=None, derandomize=True)
@given(gx=st.integers(1, 3), gy=st.integers(1, 3), px=st.integers(1, 5), py=st.integers(1, 5),
       n_rhs=st.integers(1, 3), n_perm=st.integers(1, 3), seed=st.integers(0, 10_000),
       prec=st.sampled_from(["fp64", "bf16x3", "fp32"]), method=st.sampled_from(["classical", "block_cg", "orthodir"]),
       pc=st.sampled_from([None, "lumped", "dirichlet"]))
def test_random_heat(R, gx, gy, px, py, n_rhs, n_perm, seed, prec, method, pc):
    p = W.small_heat((px, py), (gx, gy), n_rhs=n_rhs, n_perm=n_perm, seed=seed)
    print(f"\n[random heat] grid {gx}x{gy} pattern {px}x{py} n_rhs {n_rhs} n_perm {n_perm} seed {seed} "
          f"{prec} {method} {pc}", flush=True)
    _run(R, p, prec, method, pc)


@settings(max_examples=6, deadline=None, database=None, derandomize=True)
@given(gx=st.integers(1, 2), gy=st.integers(1, 2), pe=st.integers(1, 3), n_rhs=st.integers(1, 2),
       n_perm=st.integers(1, 2), seed=st.integers(0, 10_000), prec=st.sampled_from(["fp64", "bf16x3"]),
       pc=st.sampled_from([None, "lumped", "dirichlet"]))
def test_random_elastic(R, gx, gy, pe, n_rhs, n_perm, seed, prec, pc):
    p = W.small_elast((pe, pe + 1, pe), (gx, gy, 2), n_rhs=n_rhs, n_perm=n_perm, seed=seed)
    print(f"\n[random elastic] grid {gx}x{gy}x2 pattern {pe}x{pe + 1}x{pe} n_rhs {n_rhs} n_perm {n_perm} "
          f"seed {seed} {prec} {pc}", flush=True)
    _run(R, p, prec, "orthodir", pc)


@settings(max_examples=10, deadline=None, database=None, derandomize=True)
@given(elastic=st.booleans(), gx=st.integers(1, 3), gy=st.integers(1, 3), pe=st.integers(1, 2),
       n_rhs=st.integers(1, 2), n_perm=st.integers(1, 2), seed=st.integers(0, 10_000),
       prec=st.sampled_from(["fp64", "bf16x3"]), method=st.sampled_from(["classical", "block_cg", "orthodir"]),
       coarse=st.sampled_from(["lumped", "dirichlet"]), same=st.booleans())
def test_random_coarse_precond(R, elastic, gx, gy, pe, n_rhs, n_perm, seed, prec, method, coarse, same):
    """The preconditioner in the projector on drawn structures: displacements against the oracle's
    (unique) solution and G^T lambda = e against the oracle's G and e."""
    from paper_1208_6387_amd import structure as ST
    if elastic:
        # patterns with interior dofs: without them S = K_bb = K annihilates the rigid traces and
        # G^T F~^{-1} G is singular (the refused case of test_gpu_coarse_precond)
        p = W.small_elast((pe + 1, pe + 1, pe + 1), (min(gx, 2), min(gy, 2), 2), n_rhs=n_rhs, n_perm=n_perm,
                          seed=seed)
    else:
        p = W.small_heat((pe + 2, pe + 1), (gx, gy), n_rhs=n_rhs, n_perm=n_perm, seed=seed)
    print(f"\n[random coarse] {p.name} n_rhs {n_rhs} n_perm {n_perm} seed {seed} {prec} {method} "
          f"coarse {coarse} same {same}", flush=True)
    kinds = {"lumped": R.PRECOND_LUMPED, "dirichlet": R.PRECOND_DIRICHLET}
    pr = {"fp64": R.FP64, "bf16x3": R.BF16X3}[prec]
    meth = {"classical": R.CLASSICAL, "block_cg": R.BLOCK_CG, "orthodir": R.ORTHODIR}[method]
    if p.n_perm > 1 and method == "block_cg":
        meth = R.ORTHODIR
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats, (R.FP64, pr) if pr != R.FP64 else (R.FP64,))
    pb = ST.create_problem(p)
    tol = 1e-11 if pr == R.FP64 else 1e-8
    res = R.block_krylov_solve(pb, pats, ST.loads_to_device(p), p.n_rhs, tol=tol, max_it=3000, method=meth, prec=pr,
                               inner_tol=1e-3, precond=kinds[coarse] if same else R.PRECOND_NONE,
                               coarse=kinds[coarse])
    assert res.stats["rel_residual"] <= tol
    _, u_o, _ = O.FetiOracle(p).solve("block", tol=1e-12)
    u = ST.split_u(p, res.u)
    err = max(np.abs(a - b).max() for a, b in zip(u, u_o)) / max(np.abs(b).max() for b in u_o)
    assert err < (1e-8 if pr == R.FP64 else 1e-6), (p.name, prec, method, coarse, same, err)
    oc = O.FetiOracle(p, coarse=coarse)
    _, _, e = oc.loads()
    if oc.G.shape[1]:
        lam = res.lam.cpu().numpy()
        assert np.abs(oc.G.T @ lam - e).max() <= 1e-10 * max(np.abs(e).max(), 1.0)
