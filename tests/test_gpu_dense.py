"""Dense FP64 building blocks of the library (MFMA GEMM, blocked Cholesky, Jacobi eigensolver)
against NumPy, on the GPU."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def cm(a):
    """Host array -> column-major device tensor."""
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().T


@pytest.fixture(scope="module")
def R():
    import paper_1208_6387_amd as R
    R.load()
    return R


SHAPES = [(37, 129, 45), (128, 128, 64), (300, 17, 260), (16, 700, 33), (5, 3, 1000), (257, 255, 513),
          (64, 64, 0), (1, 1, 1)]


@pytest.mark.parametrize("M,N,K", SHAPES)
@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_dgemm(R, M, N, K, ta, tb):
    rng = np.random.default_rng(M * 1000 + N + K)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    Cd = cm(C0)
    out = R.dgemm(bool(ta), bool(tb), cm(A), cm(B), alpha=0.7, beta=-0.3, C_out=Cd)
    torch.cuda.synchronize()
    ref = 0.7 * ((A.T if ta else A) @ (B.T if tb else B)) - 0.3 * C0
    got = out.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()) * max(K, 1) ** 0.5


@pytest.mark.parametrize("n", [1, 63, 64, 65, 200, 700])
def test_dposv(R, n):
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, n))
    A = X @ X.T + n * np.eye(n)
    B = rng.standard_normal((n, 5))
    Ad, Bd = cm(A), cm(B)
    R.dposv(Ad, Bd)
    torch.cuda.synchronize()
    x = Bd.cpu().numpy()
    ref = np.linalg.solve(A, B)
    assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()
    L = np.tril(Ad.cpu().numpy())
    assert np.abs(L - np.linalg.cholesky(A)).max() <= 1e-12 * np.sqrt(np.abs(A).max())


def test_dposv_rejects_indefinite(R):
    A = np.diag([1.0, 2.0, -1.0, 3.0])
    with pytest.raises(R.RpfError, match="ENOTSPD"):
        R.dposv(cm(A))


@pytest.mark.parametrize("m", [1, 2, 8, 13, 16, 64])
def test_syev_small(R, m):
    rng = np.random.default_rng(m)
    X = rng.standard_normal((3, m, m))
    A = X + X.transpose(0, 2, 1)
    A[1] = X[1] @ X[1].T          # PSD member
    w, V = R.dsyev_small(torch.from_numpy(A).cuda())
    torch.cuda.synchronize()
    w, V = w.cpu().numpy(), V.cpu().numpy()
    for b in range(3):
        wr = np.linalg.eigvalsh(A[b])
        assert np.abs(w[b] - wr).max() <= 1e-12 * np.abs(wr).max()
        assert np.abs(A[b] @ V[b] - V[b] * w[b][None, :]).max() <= 1e-11 * np.abs(wr).max()
        assert np.abs(V[b].T @ V[b] - np.eye(m)).max() <= 1e-12
