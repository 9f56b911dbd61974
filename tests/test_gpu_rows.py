"""Row-block products of the multivector solver (section 3.3: orthogonalisation of a new block
against the stored blocks) through the C ABI, against NumPy in FP64, on the GPU.

The shapes reach every kernel the library picks for them: the narrow forms (a <= 64), the
wave-per-row form (few rows, long inner dimension), the MFMA row form with 16-byte and 8-byte
loads, the LDS-staged form (more than 16 columns), and every tile split of the wide Gram
(5 to 8 tiles per wave, 1 to 4 tile groups, 1, 2 or 4 tile slices per workgroup); ragged row
counts, odd widths and leading dimensions, and unaligned X."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    import paper_1208_6387_amd as R
    R.load()
    return R


def _block(rng, N, a, ld, shift=0):
    """Row-major N x a device block with leading dimension ld, starting `shift` doubles into a
    zeroed storage (shift = 1 leaves it 8-byte but not 16-byte aligned); returns (view, host copy,
    storage)."""
    host = rng.standard_normal((N, a))
    store = torch.zeros(N * ld + shift + 8, dtype=torch.float64, device="cuda")
    view = store[shift:shift + N * ld].view(N, ld)[:, :a]
    view.copy_(torch.from_numpy(host))
    return view, host, store


# (N, a, b, ldx, shift, M column-major)
ROWS_CASES = [
    (70001, 752, 16, 752, 0, False),    # all stored blocks of a 48-block restart, ragged rows
    (5000, 80, 16, 96, 0, False),
    (4099, 65, 5, 65, 0, False),        # odd a and ldx: 8-byte loads
    (3000, 80, 16, 80, 1, False),       # unaligned X: 8-byte loads
    (300, 127, 16, 130, 0, True),
    (1, 100, 3, 100, 0, False),
    (1000, 272, 1, 272, 0, True),
    (257, 64, 16, 64, 0, False),
    (20000, 33, 16, 40, 0, True),       # narrow form
    (100, 200, 20, 200, 0, True),       # more than 16 columns
    (300, 129, 16, 129, 0, False),      # few rows, long inner dimension: one wave per row
]


@pytest.mark.parametrize("N,a,b,ldx,shift,mcol", ROWS_CASES)
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (-1.0, 1.0), (0.75, -0.5)])
def test_rows_gemm(R, N, a, b, ldx, shift, mcol, alpha, beta):
    rng = np.random.default_rng(N + 7 * a + 13 * b + (1 if beta else 0))
    X, Xh, _ = _block(rng, N, a, ldx, shift)
    Y, Yh, ystore = _block(rng, N, b, b + 3)
    Mh = rng.standard_normal((a, b))
    M = torch.from_numpy(Mh).cuda()
    if mcol:
        M = torch.from_numpy(np.ascontiguousarray(Mh.T)).cuda().T
    R.rows_gemm(X, M, Y, alpha=alpha, beta=beta)
    torch.cuda.synchronize()
    want = beta * Yh + alpha * (Xh @ Mh)
    got = Y.cpu().numpy()
    scale = np.abs(Xh).max() * np.abs(Mh).max() * a + abs(beta) * np.abs(Yh).max()
    assert np.abs(got - want).max() <= 1e-13 * scale
    # nothing written outside the block: the padding columns and the storage's tail stay zero
    pad = ystore[:N * (b + 3)].view(N, b + 3)[:, b:]
    assert not pad.any() and not ystore[N * (b + 3):].any()


def test_rows_gemm_refuses(R):
    X = torch.zeros((4, 3), dtype=torch.float64, device="cuda")
    M = torch.zeros((3, 2), dtype=torch.float64, device="cuda")
    Y = torch.zeros((4, 2), dtype=torch.float64, device="cuda")
    lib = R.load()
    st = lib.rpf_rows_gemm(4, 3, 2, 1.0, R._ptr(X), 2, R._ptr(M), 0, 0.0, R._ptr(Y), 2, None)
    assert st == -1   # ldx < a
    st = lib.rpf_rows_gemm(4, 0, 2, 1.0, R._ptr(X), 3, R._ptr(M), 0, 0.0, R._ptr(Y), 2, None)
    assert st == -1   # empty inner dimension


# (N, a, b, ldx, ldy); tile counts ta = ceil(a / 16) of 47, 5, 9, 17, 32, 33, 64, 100 and 75 give
# tiles per wave 6, 5, 5, 5, 8, 5, 8, 7, 7 in 2, 1, 1, 1, 1, 2, 2, 4 and 3 tile groups
GRAM_CASES = [
    (70001, 752, 16, 752, 16),
    (5000, 80, 16, 80, 16),
    (3000, 140, 3, 141, 5),
    (100000, 272, 16, 272, 16),
    (20000, 512, 16, 512, 16),
    (20000, 528, 16, 530, 16),
    (257, 1024, 16, 1024, 16),
    (4000, 1600, 7, 1600, 9),
    (3000, 1200, 16, 1200, 16),
    (10, 300, 7, 300, 7),
    (1, 66, 1, 66, 1),
    (7777, 48, 16, 48, 16),             # narrow form
]


@pytest.mark.parametrize("N,a,b,ldx,ldy", GRAM_CASES)
def test_gram(R, N, a, b, ldx, ldy):
    rng = np.random.default_rng(3 * N + a + b)
    X, Xh, _ = _block(rng, N, a, ldx)
    Y, Yh, _ = _block(rng, N, b, ldy)
    got = R.gram(X, Y).cpu().numpy()
    want = Xh.T @ Yh
    scale = np.sqrt((Xh ** 2).sum(axis=0))[:, None] * np.sqrt((Yh ** 2).sum(axis=0))[None, :]
    assert np.all(np.abs(got - want) <= 1e-13 * scale + 1e-300)
    # fixed summation order: a second call gives the same bits
    again = R.gram(X, Y).cpu().numpy()
    assert np.array_equal(got, again)
