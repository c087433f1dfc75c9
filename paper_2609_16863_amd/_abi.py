"""ctypes declarations of the C ABI in include/aao_heat.h (argument marshalling only)."""
import ctypes
import os

LIB_NAME = "libaao_heat.so"
LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), LIB_NAME)

c_int, c_double, c_void_p, c_size_t = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
c_int64 = ctypes.c_int64

AAO_OK = 0
AAO_NOT_CONVERGED = 1
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "INVALID_ARG", -2: "HIP_ERROR", -3: "NONFINITE",
                -4: "WORKSPACE_TOO_SMALL", -5: "NO_WORKSPACE"}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3, "fp16_all": 4}
SCHUR = {"sweep": 0, "mgrit": 1}
SIDES = {"right": 0, "left": 1, "split": 2}
OUTER = {"fp64": 0, "fp32": 1}
ORTH = {"cgs2": 0, "cgs1": 1, "gram": 2}


class Desc(ctypes.Structure):
    _fields_ = [("dim", c_int), ("n", c_int), ("s", c_int), ("nt", c_int), ("T", c_double),
                ("kappa", c_void_p), ("disc", c_int), ("length", c_double)]


DISCS = {"fd": 0, "q1": 1, "q2": 2}


class Opts(ctypes.Structure):
    _fields_ = [("restart", c_int), ("maxit", c_int), ("tol", c_double), ("inner_k", c_int),
                ("cycles", c_int), ("nu1", c_int), ("nu2", c_int), ("omega", c_double),
                ("precision", c_int), ("use_graph", c_int), ("mg_tail_max", c_int), ("coarse_max", c_int),
                ("inner_tol", c_double), ("schur", c_int), ("mgrit_cf", c_int), ("mgrit_iters", c_int),
                ("mgrit_fcf", c_int), ("side", c_int),
                ("outer_precision", c_int), ("mg_low_from", c_int), ("mg_coarse_fp32", c_int),
                ("relax_matvec", c_int), ("mgrit_coarse_k", c_int), ("schur_k", c_int),
                ("inner_orth", c_int), ("outer_orth", c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("outer_iterations", c_int), ("restarts", c_int), ("relres", c_double),
                ("time_ms", c_double), ("precond_ms", c_double), ("history", c_double * 128),
                ("history_len", c_int), ("inner_solves", c_int), ("inner_iterations", ctypes.c_longlong),
                ("theta_ms", c_double), ("schur_ms", c_double), ("relaxed_fp32", c_int),
                ("relaxed_bf16", c_int)]


class Tune(ctypes.Structure):
    _fields_ = [("tall_min_b", c_int), ("tail_extend", c_int), ("from_cache", c_int), ("blocks", c_int * 3),
                ("weight", c_double * 3), ("us", (c_double * 3) * 6)]


# name -> (restype, argtypes); every entry point declared in include/aao_heat.h
SIGNATURES = {
    "aao_default_opts": (None, [ctypes.POINTER(Opts)]),
    "aao_create_problem": (c_int, [ctypes.POINTER(Desc), ctypes.POINTER(Opts), ctypes.POINTER(c_void_p)]),
    "aao_workspace_size": (c_int, [c_void_p, ctypes.POINTER(c_size_t)]),
    "aao_set_workspace": (c_int, [c_void_p, c_void_p, c_size_t]),
    "aao_set_stream": (c_int, [c_void_p, c_void_p]),
    "aao_set_kappa": (c_int, [c_void_p, c_void_p, c_int]),
    "aao_destroy": (c_int, [c_void_p]),
    "aao_get_tableau": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "aao_sizes": (c_int, [c_void_p, ctypes.POINTER(c_int64), ctypes.POINTER(c_int64)]),
    "aao_apply_A": (c_int, [c_void_p, c_void_p, c_void_p]),
    "aao_apply_AT": (c_int, [c_void_p, c_void_p, c_void_p]),
    "aao_apply_P": (c_int, [c_void_p, c_void_p, c_void_p]),
    "aao_apply_P_with": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int]),
    "aao_apply_mg": (c_int, [c_void_p, c_int, c_int, c_int, c_int, c_void_p, c_void_p]),
    "aao_mg_levels": (c_int, [c_void_p, c_int, c_void_p, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
    "aao_assemble_rhs": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "aao_solve": (c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(Stats)]),
    "aao_solve_adjoint": (c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(Stats)]),
    "aao_solve_no_alloc": (c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(Stats)]),
    "aao_grad_logkappa": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "aao_last_error": (ctypes.c_char_p, [c_void_p]),
    "aao_profile_vcycle": (c_int, [c_void_p, c_int, c_int, c_int, ctypes.c_char_p, c_size_t, c_void_p, c_void_p,
                                   c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_double)]),
    "aao_autotune": (c_int, [c_void_p, c_int, ctypes.c_char_p, ctypes.POINTER(Tune)]),
    "aao_set_launch_shapes": (c_int, [c_void_p, c_int, c_int]),
    "aao_create_batch": (c_int, [ctypes.POINTER(Desc), c_int, ctypes.POINTER(Opts), c_int, ctypes.POINTER(c_void_p)]),
    "aao_batch_count": (c_int, [c_void_p]),
    "aao_batch_offsets": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "aao_batch_workspace_size": (c_int, [c_void_p, ctypes.POINTER(c_size_t)]),
    "aao_batch_set_workspace": (c_int, [c_void_p, c_void_p, c_size_t]),
    "aao_batch_set_stream": (c_int, [c_void_p, c_void_p]),
    "aao_batch_problem": (c_int, [c_void_p, c_int, ctypes.POINTER(c_void_p)]),
    "aao_batch_assemble_rhs": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "aao_batch_solve": (c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(Stats)]),
    "aao_batch_solve_adjoint": (c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(Stats)]),
    "aao_batch_grad_logkappa": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "aao_batch_last_error": (ctypes.c_char_p, [c_void_p]),
    "aao_batch_destroy": (c_int, [c_void_p]),
}

_lib = None


def load():
    """Load the in-tree HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_NAME} is not built; run paper_2609_16863_amd.build.build() "
                           "(hipcc, gfx950) first")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
