"""feti_apply_noalloc: the FP64 operator on the library's fixed per-GPU workspace, through the C ABI,
against feti_apply (same kernels, so the same bits) and against the oracle's F, on consecutive
calls of decreasing size, plus its refusals."""
import ctypes as C

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


def _setup(R, p):
    from paper_1208_6387_amd import structure as ST
    pats = ST.factor_patterns(p)
    ST.condense_patterns(pats, (R.FP64,))
    return pats, ST.create_problem(p)


@pytest.mark.timeout(300)
def test_noalloc_matches_feti_apply(R):
    """Two calls in a row on the 64-occurrence structure (8 columns, then 3), then a call on a small
    structure: each equal to feti_apply's result, the small one also within 1e-12 of the oracle."""
    p = W.config(1)
    print("\n[noalloc] 64 x 12^3 bricks: 8 columns, then 3", flush=True)
    pats, pb = _setup(R, p)
    rng = np.random.default_rng(5)
    for m in (8, 3):
        X = torch.from_numpy(rng.standard_normal((p.n_lambda, m))).cuda()
        Y = torch.full_like(X, np.nan)
        R.feti_apply_noalloc(pb, pats, X, out=Y)
        ref = R.feti_apply(pb, pats, X)
        torch.cuda.synchronize()
        assert torch.equal(Y, ref), m
    q = W.small_elast((3, 3, 3), (2, 2, 2), n_rhs=1, seed=9)
    print("[noalloc] 2 x 2 x 2 small structure, 5 columns", flush=True)
    qpats, qpb = _setup(R, q)
    Xs = rng.standard_normal((q.n_lambda, 5))
    Xd = torch.from_numpy(Xs).cuda()
    Ys = torch.full_like(Xd, np.nan)
    R.feti_apply_noalloc(qpb, qpats, Xd, out=Ys)
    assert torch.equal(Ys, R.feti_apply(qpb, qpats, Xd))
    ref = O.FetiOracle(q).F(Xs)
    assert np.abs(Ys.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.timeout(300)
def test_noalloc_refusals(R):
    """A block whose workspace exceeds the fixed array, a projection flag and a low precision are
    refused with RPF_EINVAL before anything is queued; the output is left untouched."""
    from paper_1208_6387_amd import _lib
    q = W.small_elast((3, 3, 3), (2, 2, 2), n_rhs=1, seed=9)
    pats, pb = _setup(R, q)
    lib = _lib.load()
    hs = (C.c_void_p * len(pats))(*[x.handle for x in pats])
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    X = torch.ones((q.n_lambda, 4), dtype=torch.float64, device="cuda")
    Y = torch.zeros_like(X)
    args = (pb.handle, hs, 4, C.c_void_p(X.data_ptr()), 4, C.c_void_p(Y.data_ptr()), 4)
    assert lib.feti_apply_noalloc(*args, R.FP64, _lib.APPLY_PROJECT, stream) == _lib.RPF_EINVAL
    assert lib.feti_apply_noalloc(*args, R.BF16X3, 0, stream) == _lib.RPF_EINVAL
    # more columns than the workspace holds: n_b = 4^3 - 2^3 boundary nodes x 3 = 168 rows per
    # occurrence, 8 occurrences; m columns need at least 2 x 168 x 8 x m doubles
    m = int(_lib.NOALLOC_SCRATCH_BYTES // (8 * 2 * 168 * 8)) + 1
    Xb = torch.ones((q.n_lambda, m), dtype=torch.float64, device="cuda")
    Yb = torch.zeros_like(Xb)
    code = lib.feti_apply_noalloc(pb.handle, hs, m, C.c_void_p(Xb.data_ptr()), m, C.c_void_p(Yb.data_ptr()), m,
                                  R.FP64, 0, stream)
    assert code == _lib.RPF_EINVAL
    assert b"limit" in lib.rpf_last_error()
    torch.cuda.synchronize()
    assert float(Yb.abs().max()) == 0.0 and float(Y.abs().max()) == 0.0
