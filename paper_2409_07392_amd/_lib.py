"""ctypes declarations of the C ABI in include/firal.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfiral.so")

F64, F32, BF16X3 = 0, 1, 2
PREC = {"f64": F64, "f32": F32, "bf16x3": BF16X3}

OK = 0
WARN_NOT_CONVERGED = 1
EINVAL, EHIP, ENOMEM, ENOTSUP, EBREAKDOWN, ENOTSPD = -1, -2, -3, -4, -5, -6
PCG_PROJECT = 1
ROUND_FP32 = 1
PROF_PRODUCT, PROF_PRODUCT_T, PROF_ROUND_SCORE = 0, 1, 2

# every symbol include/firal.h declares
EXPORTS = ("firal_create", "firal_destroy", "firal_hvp", "firal_build_precond",
           "firal_pcg_solve", "firal_grad_z", "firal_probes", "firal_relax_step",
           "firal_sampled_objective", "firal_profile_begin", "firal_profile_end",
           "firal_autotune", "firal_batch_create", "firal_batch_run", "firal_batch_info",
           "firal_batch_next_t", "firal_batch_destroy", "firal_round_create", "firal_round_step",
           "firal_round_scores", "firal_round_result", "firal_round_criterion",
           "firal_round_destroy", "firal_round_eta_sweep", "firal_default_beta0",
           "firal_relax_solve", "firal_hvp_noalloc", "firal_strerror", "firal_last_error")


class Info(ctypes.Structure):
    """firal_info."""
    _fields_ = [("cg_iters", ctypes.c_int32 * 2), ("converged", ctypes.c_int32),
                ("bad_block", ctypes.c_int32), ("relres_max", ctypes.c_double),
                ("f_hat", ctypes.c_double), ("g_absmax", ctypes.c_double),
                ("beta", ctypes.c_double)]

    def as_dict(self) -> dict:
        return dict(cg_iters=(int(self.cg_iters[0]), int(self.cg_iters[1])),
                    converged=bool(self.converged), bad_block=int(self.bad_block),
                    relres_max=float(self.relres_max), f_hat=float(self.f_hat),
                    g_absmax=float(self.g_absmax), beta=float(self.beta))


class BatchProblem(ctypes.Structure):
    """firal_batch_problem."""
    _fields_ = [("ctx", ctypes.c_void_p), ("w", ctypes.c_void_p), ("b", ctypes.c_double),
                ("lam", ctypes.c_double), ("beta0", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("t0", ctypes.c_int32), ("s", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class FiralError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(what)
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load libfiral.so (built in-tree); raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2409_07392_amd.build` (needs hipcc)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                   ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double)
    pinfo = ctypes.POINTER(Info)
    sig = {
        "firal_create": [ctypes.POINTER(vp), i64, i64, i32, i32, i32, i32, vp, vp, vp],
        "firal_destroy": [vp],
        "firal_hvp": [vp, vp, i64, dbl, vp, vp, i32, vp],
        "firal_hvp_noalloc": [vp, vp, i64, i32, i32, vp, dbl, vp, vp, i32, vp],
        "firal_build_precond": [vp, vp, dbl, vp, vp, pinfo, vp],
        "firal_pcg_solve": [vp, vp, dbl, vp, vp, vp, i32, dbl, i32, u32, pinfo, vp],
        "firal_grad_z": [vp, vp, vp, i32, vp, vp],
        "firal_probes": [vp, u64, i32, i32, vp, vp],
        "firal_relax_step": [vp, vp, dbl, dbl, dbl, u64, i32, i32, dbl, i32, u32, vp, pinfo, vp],
        "firal_relax_solve": [vp, dbl, dbl, dbl, u64, i32, i32, dbl, i32, u32, dbl, vp, vp, vp,
                              ctypes.POINTER(i32), pinfo, vp],
        "firal_sampled_objective": [vp, vp, dbl, vp, i32, dbl, i32, u32, ctypes.POINTER(dbl), vp,
                                    pinfo, vp],
        "firal_autotune": [vp, i32, ctypes.POINTER(i32), vp],
        "firal_batch_create": [ctypes.POINTER(vp), i32, ctypes.POINTER(BatchProblem), vp],
        "firal_batch_run": [vp, i32, vp],
        "firal_batch_info": [vp, i32, pinfo, vp],
        "firal_batch_next_t": [vp, i32, ctypes.POINTER(i32)],
        "firal_batch_destroy": [vp],
        "firal_round_create": [ctypes.POINTER(vp), vp, vp, dbl, dbl, i32, u32, vp],
        "firal_round_step": [vp, i32, vp],
        "firal_round_scores": [vp, vp, vp],
        "firal_round_result": [vp, vp, vp, vp, ctypes.POINTER(i32), vp],
        "firal_round_criterion": [vp, ctypes.POINTER(dbl), vp],
        "firal_round_destroy": [vp],
        "firal_round_eta_sweep": [vp, vp, dbl, vp, i32, i32, u32, vp, vp, ctypes.POINTER(i32), vp],
        "firal_profile_begin": [vp, i32],
        "firal_profile_end": [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)],
        "firal_strerror": [ctypes.c_int],
        "firal_last_error": [],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.firal_default_beta0.argtypes = [i64, i32]
    lib.firal_default_beta0.restype = dbl
    lib.firal_strerror.restype = ctypes.c_char_p
    lib.firal_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(rc: int) -> int:
    """Raise FiralError for negative return codes; pass warnings through."""
    if rc < 0:
        lib = load()
        raise FiralError(rc, f"{lib.firal_strerror(rc).decode()} ({rc}): "
                             f"{lib.firal_last_error().decode()}")
    return rc
