"""Captured iteration batches (HIP graphs replayed by block_krylov_solve) through the C ABI: after every
number of replays, the captured run leaves exactly the multipliers of the uncaptured run (the same
kernels in the same order), in the FP64 and mixed forms, for block CG, classical CG, ORTHODIR (one
graph per place in the restart cycle, restarts inside and between batches) and with the Dirichlet
preconditioner; converged captured solves reach the oracle's displacements."""
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


@pytest.fixture(scope="module")
def elast(R):
    from paper_1208_6387_amd import structure as ST
    p = W.small_elast((4, 4, 4), (3, 2, 2), n_rhs=4, seed=51)
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats, (R.FP64, R.BF16X3))
    pb = ST.create_problem(p)
    return p, pats, pb, ST.loads_to_device(p)


@pytest.mark.parametrize("form,method,precond", [("fp64", "block_cg", "none"), ("bf16x3", "block_cg", "none"),
                                                 ("fp64", "classical", "none"), ("fp64", "block_cg", "dirichlet"),
                                                 ("bf16x3", "block_cg", "dirichlet")])
def test_replays_equal_eager_iterations(elast, R, form, method, precond):
    """Runs cut after 2 + 4 r iterations (r = 1..5 replays of a 4-iteration graph, each run with the
    library's eager work and host synchronisations before and after it) leave the multipliers and
    displacements of the same runs without capture.  Without a preconditioner the captured
    iterations are the eager kernels exactly (bit for bit); with one, the eager run forms the
    residual norms at every iteration in a fused variant of the residual update that the captured
    batch uses only at its end, so the two agree to rounding (1e-12)."""
    p, pats, pb, f = elast
    prec = R.FP64 if form == "fp64" else R.BF16X3
    meth = R.BLOCK_CG if method == "block_cg" else R.CLASSICAL
    pc = R.PRECOND_NONE if precond == "none" else R.PRECOND_DIRICHLET
    compared = 0
    for r in range(1, 6):
        its = 2 + 4 * r
        out = []
        for gb in (0, 4):
            res = R.block_krylov_solve(pb, pats, f, p.n_rhs, tol=1e-30, max_it=its, method=meth, prec=prec,
                                       precond=pc, graph_batch=gb, max_sweeps=1, raise_on_noconv=False)
            torch.cuda.synchronize()
            out.append((res.lam.clone(), res.u.clone(), res.stats))
        if out[0][2]["iterations"] < its:
            # the eager run ended the sweep itself (a whole block dropped: the run is exhausted);
            # the captured run notices only at the end of a batch, so the runs part here
            break
        assert out[0][2]["iterations"] == its and out[1][2]["iterations"] == its, (out[0][2], out[1][2])
        assert out[0][2]["graph_replays"] == 0 and out[1][2]["graph_replays"] == r, out[1][2]
        compared += 1
        for a, b in zip(out[0][:2], out[1][:2]):
            if precond == "none":
                assert torch.equal(a, b), (form, method, r)
            else:
                assert (a - b).abs().max().item() <= 1e-12 * a.abs().max().item(), (form, method, r)
    assert compared >= 1


def _orthodir_schedule(its, gb, max_blocks):
    """Replays of the captured ORTHODIR loop: a batch starts at places 0, gb, 2 gb, ... of the restart
    cycle when it fits before the next restart and before max_it, from the second iteration on;
    other iterations run uncaptured; nothing is captured when the cycle is not shorter than max_it."""
    if max_blocks >= its:
        return 0
    it = nst = replays = 0
    while it < its:
        pos = 0 if nst == max_blocks else nst
        if pos % gb == 0 and pos + gb <= max_blocks and it + gb <= its and it > 0:
            replays, nst, it = replays + 1, pos + gb, it + gb
        else:
            nst, it = pos + 1, it + 1
    return replays


@pytest.mark.parametrize("form,max_blocks,gb", [("fp64", 8, 4), ("bf16x3", 8, 4), ("fp64", 6, 4), ("fp64", 5, 2),
                                                ("bf16x3", 7, 3)])
def test_orthodir_replays_equal_eager_iterations(elast, R, form, max_blocks, gb):
    """ORTHODIR runs cut after 1 to 4 restart cycles and a few more iterations leave the multipliers and
    displacements of the same runs without capture.  With max_blocks a multiple of the batch and
    convergence checks every batch, the captured iterations are the eager kernels exactly (bit for
    bit); otherwise the eager run forms the residual norms at other iterations, in a fused variant of
    the residual update, and the two agree to rounding (1e-10 after up to 28 iterations)."""
    p, pats, pb, f = elast
    prec = R.FP64 if form == "fp64" else R.BF16X3
    exact = max_blocks % gb == 0
    compared = 0
    for its in (gb, max_blocks, max_blocks + gb, 2 * max_blocks + 1, 3 * max_blocks + gb, 4 * max_blocks):
        out = []
        for g in (0, gb):
            res = R.block_krylov_solve(pb, pats, f, p.n_rhs, tol=1e-30, max_it=its, method=R.ORTHODIR, prec=prec,
                                       graph_batch=g, max_sweeps=1, max_blocks=max_blocks,
                                       check_every=gb if exact else 1, raise_on_noconv=False)
            torch.cuda.synchronize()
            out.append((res.lam.clone(), res.u.clone(), res.stats))
        if out[0][2]["iterations"] < its:
            break  # the eager run was exhausted (a whole block dropped); the runs part here
        assert out[0][2]["iterations"] == its and out[1][2]["iterations"] == its, (out[0][2], out[1][2])
        assert out[0][2]["graph_replays"] == 0, out[0][2]
        assert out[1][2]["graph_replays"] == _orthodir_schedule(its, gb, max_blocks), (its, out[1][2])
        compared += 1
        for a, b in zip(out[0][:2], out[1][:2]):
            if exact:
                assert torch.equal(a, b), (form, max_blocks, gb, its)
            else:
                assert (a - b).abs().max().item() <= 1e-10 * a.abs().max().item(), (form, max_blocks, gb, its)
    assert compared >= 3


@pytest.mark.parametrize("method,form,precond", [("block_cg", "fp64", "none"), ("block_cg", "bf16x3", "none"),
                                                 ("block_cg", "bf16x3", "dirichlet"), ("orthodir", "fp64", "none"),
                                                 ("orthodir", "bf16x3", "none"), ("orthodir", "bf16x3", "dirichlet")])
@pytest.mark.parametrize("gb", [2, 8])
def test_captured_solve_against_oracle(elast, R, method, form, precond, gb):
    """Converged captured solves (several refinement sweeps in the mixed form reuse the graphs):
    u within 1e-8 of the oracle's reference at a 1e-10 residual."""
    from paper_1208_6387_amd import structure as ST
    p, pats, pb, f = elast
    prec = R.FP64 if form == "fp64" else R.BF16X3
    pc = R.PRECOND_NONE if precond == "none" else R.PRECOND_DIRICHLET
    meth = R.BLOCK_CG if method == "block_cg" else R.ORTHODIR
    res = R.block_krylov_solve(pb, pats, f, p.n_rhs, tol=1e-10, max_it=2000, method=meth, prec=prec,
                               inner_tol=1e-4, graph_batch=gb, precond=pc, max_blocks=24)
    assert res.stats["rel_residual"] <= 1e-10 and res.stats["graph_replays"] > 0, res.stats
    u = ST.split_u(p, res.u)
    _, u_o, _ = O.FetiOracle(p).solve("block", tol=1e-12)
    scale = max(np.abs(x).max() for x in u_o)
    err = max(np.abs(a - b).max() for a, b in zip(u, u_o)) / scale
    assert err <= 1e-8, err


def test_graph_batch_refused_negative_and_off_while_tracing(elast, R):
    from paper_1208_6387_amd import _lib
    p, pats, pb, f = elast
    R.trace_enable(True)
    try:
        res = R.block_krylov_solve(pb, pats, f, p.n_rhs, tol=1e-10, max_it=2000, method=R.ORTHODIR, graph_batch=4)
    finally:
        R.trace_enable(False)
        R.trace_read()
    assert res.stats["graph_replays"] == 0 and res.stats["rel_residual"] <= 1e-10
    with pytest.raises(R.RpfError) as e:
        R.block_krylov_solve(pb, pats, f, p.n_rhs, tol=1e-10, max_it=10, method=R.BLOCK_CG, graph_batch=-2)
    assert e.value.code == _lib.RPF_EINVAL
