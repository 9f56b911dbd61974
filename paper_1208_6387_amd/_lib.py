"""ctypes declarations of the C ABI in include/rpfeti.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librpfeti.so")

RPF_OK, RPF_EINVAL, RPF_ENOTSPD, RPF_EKERNEL, RPF_EBREAKDOWN, RPF_ENOCONV, RPF_EHIP, RPF_ENOMEM = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "RPF_OK", -1: "RPF_EINVAL", -2: "RPF_ENOTSPD", -3: "RPF_EKERNEL", -4: "RPF_EBREAKDOWN",
                -5: "RPF_ENOCONV", -6: "RPF_EHIP", -7: "RPF_ENOMEM"}
FP64, FP32, BF16X3, BF16 = 0, 1, 2, 3
CLASSICAL, BLOCK_CG, ORTHODIR = 0, 1, 2
PRECOND_NONE, PRECOND_LUMPED, PRECOND_DIRICHLET = 0, 1, 2
APPLY_PROJECT = 1
NOALLOC_SCRATCH_BYTES = 128 << 20   # RPF_NOALLOC_SCRATCH_BYTES

# every symbol the header declares
EXPORTS = ["rpf_last_error", "rpf_version", "pattern_factor", "pattern_condense", "pattern_info", "pattern_export",
           "pattern_free", "problem_create", "problem_n_lambda", "problem_free", "problem_n_perm", "problem_set_schedule", "problem_tune", "feti_apply",
           "feti_apply_noalloc", "feti_precond", "feti_permute",
           "block_krylov_solve",
           "rpf_dgemm", "rpf_dposv", "rpf_dsyev_small", "rpf_rows_gemm", "rpf_gram", "rpf_trace_enable",
           "rpf_trace_read"]


class ProblemDesc(C.Structure):
    _fields_ = [("dofs_per_node", C.c_int32), ("n_patterns", C.c_int32), ("pat_n_nodes", C.c_void_p),
                ("pat_bnode_ptr", C.c_void_p), ("pat_bnodes", C.c_void_p), ("n_occ", C.c_int32),
                ("occ_pattern", C.c_void_p), ("occ_rot", C.c_void_p), ("n_mult", C.c_int32),
                ("mult_occ", C.c_void_p), ("mult_node", C.c_void_p), ("mult_sign", C.c_void_p),
                ("n_perm", C.c_int32), ("perm_node", C.c_void_p), ("entry_ptr", C.c_void_p),
                ("entry_node", C.c_void_p), ("entry_weight", C.c_void_p)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_it", C.c_int32), ("method", C.c_int32), ("prec", C.c_int32),
                ("inner_tol", C.c_double), ("max_sweeps", C.c_int32), ("check_every", C.c_int32),
                ("max_blocks", C.c_int32), ("precond", C.c_int32), ("periodic", C.c_int32),
                ("coarse", C.c_int32), ("graph_batch", C.c_int32)]


class ScheduleEntry(C.Structure):
    _fields_ = [("tile", C.c_int32), ("work", C.c_int32), ("ms", C.c_double), ("chosen", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("sweeps", C.c_int32), ("rank_drops", C.c_int32),
                ("converged", C.c_int32), ("rel_residual", C.c_double), ("ms_loads", C.c_double),
                ("ms_coarse", C.c_double), ("ms_iterate", C.c_double), ("ms_recover", C.c_double),
                ("graph_replays", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load() -> C.CDLL:
    """Load librpfeti.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1208_6387_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "rpf_last_error": (C.c_char_p, []),
        "rpf_version": (i32, []),
        "pattern_factor": (i32, [i32, vp, vp, vp, i32, vp, i32, f64, i32, vp, C.POINTER(vp), C.POINTER(i32)]),
        "pattern_condense": (i32, [vp, i32, vp]),
        "pattern_info": (i32, [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]),
        "pattern_export": (i32, [vp, i32, vp, i64, vp]),
        "pattern_free": (None, [vp]),
        "problem_create": (i32, [C.POINTER(ProblemDesc), C.POINTER(vp)]),
        "problem_n_lambda": (i64, [vp]),
        "problem_free": (None, [vp]),
        "problem_n_perm": (i32, [vp]),
        "problem_set_schedule": (i32, [vp, i32, i32, i32, i32]),
        "problem_tune": (i32, [vp, vp, i32, i32, i32, C.POINTER(ScheduleEntry), i32, C.POINTER(i32), vp]),
        "feti_apply": (i32, [vp, vp, i32, vp, i64, vp, i64, i32, C.c_uint32, vp]),
        "feti_apply_noalloc": (i32, [vp, vp, i32, vp, i64, vp, i64, i32, C.c_uint32, vp]),
        "feti_precond": (i32, [vp, vp, i32, vp, i64, vp, i64, i32, i32, C.c_uint32, vp]),
        "feti_permute": (i32, [vp, vp, i32, vp, i64, vp, i64, C.c_uint32, vp]),
        "block_krylov_solve": (i32, [vp, vp, i32, vp, C.POINTER(SolveOpts), vp, i64, vp, C.POINTER(SolveStats), vp]),
        "rpf_dgemm": (i32, [i32, i32, i64, i64, i64, f64, vp, i64, vp, i64, f64, vp, i64, vp]),
        "rpf_dposv": (i32, [i64, vp, i64, i64, vp, i64, vp]),
        "rpf_dsyev_small": (i32, [i32, i32, vp, vp, vp, vp]),
        "rpf_rows_gemm": (i32, [i64, i32, i32, f64, vp, i64, vp, i64, f64, vp, i64, vp]),
        "rpf_gram": (i32, [i64, i32, i32, vp, i64, vp, i64, vp, vp]),
        "rpf_trace_enable": (i32, [i32]),
        "rpf_trace_read": (i32, [i32, C.POINTER(i64), C.POINTER(f64), C.POINTER(f64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class RpfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code: int):
    if code != RPF_OK:
        raise RpfError(code, load().rpf_last_error().decode(errors="replace"))
