"""Repeated-pattern FETI hot path on MI355X: Python binding of librpfeti.so.

The functions below carry the names of the C ABI (include/rpfeti.h) and only
marshal arguments: every numerical step runs in the HIP library.  Device
memory and streams come from PyTorch (ROCm build).  Importing the package does
not load the library; the first call does, and fails loudly when it has not
been built (`python -m paper_1208_6387_amd.build`).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import (APPLY_PROJECT, BF16, BF16X3, BLOCK_CG, CLASSICAL, FP32, FP64, ORTHODIR, PRECOND_DIRICHLET,
                   PRECOND_LUMPED, PRECOND_NONE, RpfError, SolveStats, check, load)

__all__ = ["Pattern", "Problem", "pattern_factor", "pattern_condense", "pattern_export", "problem_create", "problem_set_schedule", "problem_tune",
           "feti_apply", "feti_apply_noalloc", "feti_precond", "feti_permute", "block_krylov_solve", "dgemm", "dposv", "dsyev_small",
           "load", "RpfError", "FP64", "FP32", "BF16X3", "BF16", "CLASSICAL", "BLOCK_CG", "ORTHODIR",
           "PRECOND_NONE", "PRECOND_LUMPED", "PRECOND_DIRICHLET", "APPLY_PROJECT"]


def _stream(stream=None) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t: torch.Tensor) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _host(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


class Pattern:
    """Owner of an rpf_pattern handle."""

    def __init__(self, handle: C.c_void_p, kernel_dim: int, n: int, n_b: int):
        self.handle = handle
        self.kernel_dim = kernel_dim
        self.n = n
        self.n_b = n_b

    def free(self):
        if self.handle:
            load().pattern_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Problem:
    """Owner of an rpf_problem handle (structure: assembly, permutations)."""

    def __init__(self, handle: C.c_void_p):
        self.handle = handle
        self.n_lambda = int(load().problem_n_lambda(handle))
        self.n_perm = int(load().problem_n_perm(handle))

    def free(self):
        if self.handle:
            load().problem_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def pattern_factor(rowptr, colind, val: torch.Tensor, bdofs, dofs_per_node: int, kernel_tol: float = 0.0,
                   expected_kernel_dim: int = -1, stream=None) -> Pattern:
    """Factor a pattern.  rowptr/colind/bdofs: host int32 arrays; val: device float64 tensor."""
    lib = load()
    rp, ci, bd = _host(rowptr, np.int32), _host(colind, np.int32), _host(bdofs, np.int32)
    assert val.is_cuda and val.dtype == torch.float64 and val.numel() == rp[-1]
    h, k = C.c_void_p(), C.c_int32()
    check(lib.pattern_factor(len(rp) - 1, rp.ctypes.data, ci.ctypes.data, _ptr(val), len(bd), bd.ctypes.data,
                             dofs_per_node, kernel_tol, expected_kernel_dim, _stream(stream), C.byref(h),
                             C.byref(k)))
    return Pattern(h, k.value, len(rp) - 1, len(bd))


def pattern_condense(p: Pattern, prec: int = FP64, stream=None) -> None:
    check(load().pattern_condense(p.handle, prec, _stream(stream)))


def pattern_export(p: Pattern, what: str, stream=None) -> torch.Tensor:
    """'S', 'Z' or 'Splus' as a column-major device matrix returned as a (rows, cols) tensor."""
    code = {"S": 0, "Z": 1, "Splus": 2}[what]
    cols = p.kernel_dim if what == "Z" else p.n_b
    out = torch.empty((max(cols, 1), p.n_b), dtype=torch.float64, device="cuda")
    if cols:
        check(load().pattern_export(p.handle, code, _ptr(out), p.n_b, _stream(stream)))
    return out[:cols].T


def problem_create(dofs_per_node: int, pat_n_nodes, pat_bnodes, occ_pattern, occ_rot, mult_occ, mult_node,
                   mult_sign, perm_node=None, entries=None) -> Problem:
    """Structure from host arrays: pat_bnodes is a list of per-pattern sorted boundary node arrays,
    mult_* are (n_mult, 2) arrays, occ_rot an (n_occ, 3, 3) array or None, perm_node (n_perm, n_mult).
    entries: None (signed Boolean assembly) or (entry_ptr, entry_node, entry_weight) of a
    non-Boolean one."""
    lib = load()
    nn = _host(pat_n_nodes, np.int32)
    ptr = _host(np.concatenate([[0], np.cumsum([len(b) for b in pat_bnodes])]), np.int32)
    bn = _host(np.concatenate([np.asarray(b) for b in pat_bnodes]), np.int32)
    op = _host(occ_pattern, np.int32)
    rot = None if occ_rot is None else _host(occ_rot, np.float64).reshape(-1)
    mo, mn, ms = _host(mult_occ, np.int32).reshape(-1), _host(mult_node, np.int32).reshape(-1), _host(mult_sign, np.int8).reshape(-1)
    if perm_node is None:
        n_perm, pn = 1, None
    else:
        pn = _host(perm_node, np.int32)
        n_perm = pn.shape[0]
        pn = pn.reshape(-1)
    if entries is not None:
        eptr, enode, ew = (_host(entries[0], np.int32), _host(entries[1], np.int32), _host(entries[2], np.float64))
    d = _lib.ProblemDesc(dofs_per_node, len(nn), nn.ctypes.data, ptr.ctypes.data, bn.ctypes.data, len(op),
                         op.ctypes.data, None if rot is None else rot.ctypes.data, len(mo) // 2, mo.ctypes.data,
                         mn.ctypes.data, ms.ctypes.data, n_perm, None if pn is None else pn.ctypes.data,
                         None if entries is None else eptr.ctypes.data,
                         None if entries is None else enode.ctypes.data,
                         None if entries is None else ew.ctypes.data)
    h = C.c_void_p()
    check(lib.problem_create(C.byref(d), C.byref(h)))
    return Problem(h)


def problem_set_schedule(pb: Problem, m: int, prec: int, tile: int, work: int = 1024) -> None:
    """Install the schedule of the flexibility products for block width m and arithmetic prec
    (tile 0: the size rule; 64 / 128: one grouped launch; 256: the single-pattern large tile)."""
    check(load().problem_set_schedule(pb.handle, m, prec, tile, work))


def problem_tune(pb: Problem, patterns, m: int, prec: int = FP64, reps: int = 5, stream=None) -> list:
    """Time every candidate schedule for an m-column block, install the fastest, return them all as
    dicts (tile, work, ms, chosen)."""
    arr = (_lib.ScheduleEntry * 64)()
    n = C.c_int32()
    check(load().problem_tune(pb.handle, _handles(patterns), m, prec, reps, arr, 64, C.byref(n), _stream(stream)))
    return [{"tile": arr[i].tile, "work": arr[i].work, "ms": arr[i].ms, "chosen": bool(arr[i].chosen)}
            for i in range(min(n.value, 64))]


def _handles(patterns):
    arr = (C.c_void_p * len(patterns))(*[p.handle for p in patterns])
    return arr


def feti_apply(pb: Problem, patterns, X: torch.Tensor, prec: int = FP64, project: bool = False,
               out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Y = F X (or Q^T F X) for a row-major N_lambda x m device block."""
    assert X.is_cuda and X.dtype == torch.float64 and X.dim() == 2 and X.shape[0] == pb.n_lambda
    assert X.stride(1) == 1
    m = X.shape[1]
    Y = out if out is not None else torch.empty_like(X)
    check(load().feti_apply(pb.handle, _handles(patterns), m, _ptr(X), X.stride(0), _ptr(Y), Y.stride(0), prec,
                            APPLY_PROJECT if project else 0, _stream(stream)))
    return Y


def feti_apply_noalloc(pb: Problem, patterns, X: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """Y = F X in FP64 with the library's fixed per-GPU workspace (no device allocation); out must be
    given.  Calls overlapping on one GPU share that workspace and race."""
    assert X.is_cuda and X.dtype == torch.float64 and X.dim() == 2 and X.shape[0] == pb.n_lambda
    assert X.stride(1) == 1 and out.stride(1) == 1 and out.shape == X.shape
    m = X.shape[1]
    check(load().feti_apply_noalloc(pb.handle, _handles(patterns), m, _ptr(X), X.stride(0), _ptr(out),
                                    out.stride(0), FP64, 0, _stream(stream)))
    return out


def feti_precond(pb: Problem, patterns, X: torch.Tensor, kind: int, prec: int = FP64, project: bool = False,
                 out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Y = F~^{-1} X (or Q F~^{-1} X) for a row-major N_lambda x m device block; kind is PRECOND_NONE,
    PRECOND_LUMPED or PRECOND_DIRICHLET."""
    assert X.is_cuda and X.dtype == torch.float64 and X.dim() == 2 and X.shape[0] == pb.n_lambda
    assert X.stride(1) == 1
    m = X.shape[1]
    Y = out if out is not None else torch.empty_like(X)
    hs = _handles(patterns) if patterns is not None else None
    check(load().feti_precond(pb.handle, hs, m, _ptr(X), X.stride(0), _ptr(Y), Y.stride(0), int(kind), prec,
                              APPLY_PROJECT if project else 0, _stream(stream)))
    return Y


def feti_permute(pb: Problem, Z: torch.Tensor, patterns=None, project: bool = False,
                 out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """[Pi_0 z_l, .., Pi_{n_perm-1} z_l] for every column l of a row-major N_lambda x nr block
    (column l*n_perm + k), optionally re-projected by Q (then the patterns are needed)."""
    assert Z.is_cuda and Z.dtype == torch.float64 and Z.dim() == 2 and Z.shape[0] == pb.n_lambda
    assert Z.stride(1) == 1
    nr = Z.shape[1]
    W = out if out is not None else torch.empty((pb.n_lambda, nr * pb.n_perm), dtype=torch.float64,
                                                device=Z.device)
    assert W.stride(1) == 1 and W.shape[1] >= nr * pb.n_perm
    hs = _handles(patterns) if patterns is not None else None
    check(load().feti_permute(pb.handle, hs, nr, _ptr(Z), Z.stride(0), _ptr(W), W.stride(0),
                              APPLY_PROJECT if project else 0, _stream(stream)))
    return W


@dataclass
class SolveResult:
    lam: torch.Tensor
    u: torch.Tensor
    stats: dict
    status: int


def block_krylov_solve(pb: Problem, patterns, f_local: torch.Tensor, n_rhs: int, tol: float = 1e-8,
                       max_it: int = 1000, method: int = ORTHODIR, prec: int = FP64, inner_tol: float = 0.0,
                       max_sweeps: int = 0, check_every: int = 1, max_blocks: int = 0, lam_out=None, u_out=None,
                       stream=None, raise_on_noconv: bool = True, precond: int = PRECOND_NONE,
                       periodic: bool = False, coarse: int = PRECOND_NONE, graph_batch: int = 0) -> SolveResult:
    """Solve the interface problem and recover the displacements.  f_local: flat device float64 tensor,
    occurrence blocks of n_p x n_rhs column-major, concatenated.  coarse: the preconditioner used as
    F~^{-1} in the projector and lambda_0 (PRECOND_NONE: the identity).  graph_batch: iterations per
    captured HIP graph (0: no capture; ORTHODIR: one graph per place in its restart cycle of max_blocks)."""
    assert f_local.is_cuda and f_local.dtype == torch.float64 and f_local.is_contiguous()
    lam = lam_out if lam_out is not None else torch.empty((pb.n_lambda, n_rhs), dtype=torch.float64, device="cuda")
    u = u_out if u_out is not None else torch.empty_like(f_local)
    opts = _lib.SolveOpts(tol, max_it, method, prec, inner_tol, max_sweeps, check_every, max_blocks, int(precond),
                          int(bool(periodic)), int(coarse), int(graph_batch))
    st = SolveStats()
    code = load().block_krylov_solve(pb.handle, _handles(patterns), n_rhs, _ptr(f_local), C.byref(opts), _ptr(lam),
                                     lam.stride(0), _ptr(u), C.byref(st), _stream(stream))
    if code != _lib.RPF_OK and not (code == _lib.RPF_ENOCONV and not raise_on_noconv):
        check(code)
    return SolveResult(lam, u, st.as_dict(), code)


# ------------------------------------------------------------------ dense helpers
def dgemm(ta: bool, tb: bool, A: torch.Tensor, B: torch.Tensor, alpha=1.0, beta=0.0, C_out=None, stream=None):
    """Column-major GEMM on the library's MFMA kernel; A, B given as (rows, cols) tensors stored
    column-major (i.e. their .T is contiguous)."""
    def cm(t):
        assert t.is_cuda and t.dtype == torch.float64 and t.T.is_contiguous()
        return t.shape[0], t.shape[1], t.stride(1)
    ar, ac, lda = cm(A)
    br, bc, ldb = cm(B)
    M, K = (ac, ar) if ta else (ar, ac)
    K2, N = (bc, br) if tb else (br, bc)
    assert K == K2
    if C_out is None:
        C_out = torch.zeros((N, M), dtype=torch.float64, device="cuda").T
    ldc = C_out.stride(1)
    check(load().rpf_dgemm(int(ta), int(tb), M, N, K, alpha, _ptr(A), lda, _ptr(B), ldb, beta, _ptr(C_out), ldc,
                           _stream(stream)))
    return C_out


def dposv(A: torch.Tensor, B: torch.Tensor | None = None, stream=None):
    """In-place Cholesky of a column-major SPD matrix A, then B <- A^{-1} B."""
    n = A.shape[0]
    nrhs = 0 if B is None else B.shape[1]
    check(load().rpf_dposv(n, _ptr(A), A.stride(1), nrhs, None if B is None else _ptr(B),
                           n if B is None else B.stride(1), _stream(stream)))
    return A, B


def dsyev_small(A: torch.Tensor, stream=None):
    """Eigen-decomposition of a batch (b, m, m) of symmetric matrices (column-major = any, symmetric)."""
    b, m, _ = A.shape
    A = A.contiguous()
    V = torch.empty_like(A)
    w = torch.empty((b, m), dtype=torch.float64, device="cuda")
    check(load().rpf_dsyev_small(m, b, _ptr(A), _ptr(V), _ptr(w), _stream(stream)))
    return w, V.transpose(1, 2)


def _rows(t: torch.Tensor):
    """(rows, cols, leading dimension) of a row-major FP64 device block."""
    assert t.is_cuda and t.dtype == torch.float64 and t.dim() == 2 and t.stride(1) == 1
    return t.shape[0], t.shape[1], t.stride(0)


def rows_gemm(X: torch.Tensor, M: torch.Tensor, Y: torch.Tensor, alpha=1.0, beta=0.0, stream=None) -> torch.Tensor:
    """Y <- beta Y + alpha X M for row-major blocks X (N x a), Y (N x b); M (a x b) row-major or, when
    its transpose is contiguous, column-major."""
    N, a, ldx = _rows(X)
    N2, b, ldy = _rows(Y)
    assert N2 == N and tuple(M.shape) == (a, b) and M.is_cuda and M.dtype == torch.float64
    if M.stride(1) == 1 and M.stride(0) >= b:
        mrow = M.stride(0)
    else:
        assert M.stride(0) == 1 and M.stride(1) == a, "M must be row-major or column-major with ld a"
        mrow = 0
    check(load().rpf_rows_gemm(N, a, b, alpha, _ptr(X), ldx, _ptr(M), mrow, beta, _ptr(Y), ldy, _stream(stream)))
    return Y


def gram(X: torch.Tensor, Y: torch.Tensor, stream=None) -> torch.Tensor:
    """X^T Y (a x b) for row-major blocks X (N x a), Y (N x b)."""
    N, a, ldx = _rows(X)
    N2, b, ldy = _rows(Y)
    assert N2 == N
    C_out = torch.zeros((b, a), dtype=torch.float64, device="cuda")
    check(load().rpf_gram(N, a, b, _ptr(X), ldx, _ptr(Y), ldy, _ptr(C_out), _stream(stream)))
    return C_out.T


def trace_enable(on: bool = True) -> None:
    """Bracket every flexibility product S+ W with HIP events (see rpf_trace_read)."""
    check(load().rpf_trace_enable(1 if on else 0))


def trace_read(prec: int = -1) -> dict:
    """Products launched since the last read in precision prec (FP64, FP32, BF16X3 or BF16; -1 for all): count,
    summed kernel ms, algorithmic flops.  Every recorded product is dropped by the read."""
    n, ms, fl = C.c_int64(), C.c_double(), C.c_double()
    check(load().rpf_trace_read(int(prec), C.byref(n), C.byref(ms), C.byref(fl)))
    return {"count": n.value, "ms": ms.value, "flops": fl.value}
