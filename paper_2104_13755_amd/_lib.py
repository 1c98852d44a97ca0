"""ctypes declarations of libsmg.so (see include/smg.h).

Loading fails loudly if the library has not been built: there is no CPU
fallback anywhere in this package.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmg.so")

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p
P_i32 = ctypes.POINTER(c_int32)
P_f64 = ctypes.POINTER(c_double)


class PreOpts(ctypes.Structure):
    _fields_ = [("n_levels", c_int32), ("min_coarse", c_int32), ("collapses", c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("mu_pre", c_int32), ("mu_post", c_int32), ("tail_rows", c_int32),
                ("lanes_per_row", c_int32 * 16), ("team_level", c_int32), ("team_size", c_int32)]


class SolveParams(ctypes.Structure):
    _fields_ = [("rtol", c_double), ("max_cycles", c_int32), ("precision", c_int32),
                ("fixed_cycles", c_int32), ("use_graph", c_int32), ("timed", c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("cycles", c_int32), ("k", c_int32), ("rel_res", c_double * 4), ("ms", c_double),
                ("ms_phase", c_double * 5)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("threads", c_int32), ("lanes_level0", c_int32), ("lanes_coarse", c_int32),
                ("team_max", c_int32), ("cache_file", ctypes.c_char_p), ("device_teams", c_int32),
                ("balance", c_int32)]


SMG_OK = 0
STATUS = {0: "OK", -1: "INVALID_ARG", -2: "OOM", -3: "HIP", -4: "NOT_SPD",
          -5: "NO_CONVERGENCE", -6: "NONFINITE", -7: "STATE", -8: "PRECOMPUTE"}
SMG_FP64 = 0
SMG_FP32_IR = 1
SMG_SMOOTH_GS = 0
SMG_SMOOTH_JACOBI = 1
SMG_COLLAPSE_ALL = 0
SMG_COLLAPSE_INTERIOR = 1
SMG_COLLAPSE_STRAIGHT = 2
PHASES = ("prepare", "relax", "transfer", "norm", "other")   # SMG_PHASE_* order
SMG_TAIL_RELAX, SMG_TAIL_RESIDUAL, SMG_TAIL_RESTRICT, SMG_TAIL_PROLONG, SMG_TAIL_COARSE = range(5)

# caller allocator of a context: void *alloc(size_t, void *user), void free(void *, size_t, void *user)
ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, ctypes.c_size_t, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, ctypes.c_size_t, c_void_p)

# name -> (restype, argtypes)
SIGNATURES = {
    "smg_ctx_create": (c_int32, [c_int32, ALLOC_FN, FREE_FN, c_void_p, ctypes.POINTER(c_void_p)]),
    "smg_ctx_destroy": (None, [c_void_p]),
    "smg_solver_create_ctx": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(Opts), ctypes.POINTER(c_void_p)]),
    "smg_pre_build": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, ctypes.POINTER(PreOpts), ctypes.POINTER(c_void_p)]),
    "smg_hier_from_prolongations": (c_int32, [c_int32, c_void_p, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p)]),
    "smg_pre_assemble": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "smg_hier_save": (c_int32, [c_void_p, ctypes.c_char_p]),
    "smg_hier_load": (c_int32, [ctypes.c_char_p, ctypes.POINTER(c_void_p)]),
    "smg_hier_num_levels": (c_int32, [c_void_p]),
    "smg_hier_level_size": (c_int32, [c_void_p, c_int32]),
    "smg_hier_get_prolongation": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "smg_hier_stats": (c_int32, [c_void_p, c_int32, c_void_p]),
    "smg_hier_free": (None, [c_void_p]),
    "smg_color_pattern": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p]),
    "smg_mesh_pattern": (c_int32, [c_int32, c_void_p, c_int32, c_void_p, c_void_p, P_i32]),
    "smg_solver_create": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p, ctypes.POINTER(Opts), ctypes.POINTER(c_void_p)]),
    "smg_solver_destroy": (None, [c_void_p]),
    "smg_solver_attach_mesh": (c_int32, [c_void_p, c_void_p, c_int32]),
    "smg_assemble": (c_int32, [c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "smg_set_values": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "smg_num_levels": (c_int32, [c_void_p]),
    "smg_level_size": (c_int32, [c_void_p, c_int32]),
    "smg_level_nnz": (c_int64, [c_void_p, c_int32]),
    "smg_level_colors": (c_int32, [c_void_p, c_int32, c_void_p]),
    "smg_get_level_matrix": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "smg_get_coarse_factor": (c_int32, [c_void_p, c_void_p]),
    "smg_residual": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "smg_smooth": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_int32, c_int32, c_void_p]),
    "smg_restrict": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_int32, c_void_p]),
    "smg_prolong_add": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_int32, c_void_p]),
    "smg_coarse_solve": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_void_p]),
    "smg_tail_first_level": (c_int32, [c_void_p, c_int32, c_int32]),
    "smg_tail_step": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                c_void_p]),
    "smg_vcycle": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_void_p]),
    "smg_solve": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, ctypes.POINTER(SolveParams), ctypes.POINTER(SolveInfo), c_void_p]),
    "smg_set_smoother": (c_int32, [c_void_p, c_int32, ctypes.c_double]),
    "smg_split_prepare": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "smg_hier_dirichlet": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(c_void_p), c_void_p, ctypes.POINTER(c_int32)]),
    "smg_dirichlet_pattern": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32)]),
    "smg_dirichlet_reduce": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "smg_split_combine": (c_int32, [c_void_p, ctypes.c_double, ctypes.c_double, c_void_p]),
    "smg_get_jacobi_omega": (c_int32, [c_void_p, c_int32, ctypes.POINTER(ctypes.c_double)]),
    "smg_pcg_solve": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, ctypes.POINTER(SolveParams), ctypes.POINTER(SolveInfo), c_void_p]),
    "smg_spmv_dot": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, P_f64, c_void_p]),
    "smg_spmv_dot_noalloc": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                       c_void_p]),
    "smg_mass_grad": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "smg_profile_enable": (c_int32, [c_void_p, c_int32, c_int32]),
    "smg_launch_floor": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, P_f64, P_f64]),
    "smg_profile_read": (c_int32, [c_void_p, P_f64, ctypes.POINTER(c_int64), P_f64]),
    "smg_batch_create": (c_int32, [ctypes.POINTER(c_void_p), c_int32, ctypes.POINTER(BatchOpts), ctypes.POINTER(c_void_p)]),
    "smg_batch_destroy": (None, [c_void_p]),
    "smg_batch_solve": (c_int32, [c_void_p, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), P_i32, ctypes.POINTER(SolveParams), ctypes.POINTER(SolveInfo), c_void_p]),
    "smg_batch_autotune": (c_int32, [c_void_p, c_int32, c_void_p]),
    "smg_batch_shape": (c_int32, [c_void_p, P_i32]),
    "smg_status_string": (ctypes.c_char_p, [c_int32]),
    "smg_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load libsmg.so; raises if it is missing (build it with
    ``python -m paper_2104_13755_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libsmg.so not built at {LIB_PATH}; run python -m paper_2104_13755_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class SmgError(RuntimeError):
    def __init__(self, status, where):
        lib = load()
        msg = lib.smg_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


def check(status, where):
    if status != SMG_OK:
        raise SmgError(status, where)
    return status
