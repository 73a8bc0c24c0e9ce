"""ctypes declarations of the C ABI in include/adafac.h (argument marshalling only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadafac.so")

OK, EINVAL, ESTATE, ENOMEM, EDEVICE, EDIVERGED, EAGAIN, EUNSUPPORTED = 0, 1, 2, 3, 4, 5, 6, 7
REQ_STATUS = {0: "queued", 1: "running", 2: "converged", 3: "diverged", 4: "capped", 5: "failed"}
TRANSFER = {"dlinear": 0, "boxmg": 1}
RTILDE = {"const": 0, "operator": 1}
STATIC_WORKSPACE_BYTES = 32 << 20   # ADAFAC_STATIC_WORKSPACE_BYTES
DAMPING = {"jac": 0, "pi": 1, "none": 2, "exp": 3}
PRECISION = {"fp64": 0, "fp32_refined": 1}
LEVEL_ARRAY = {"u": 0, "b": 1, "btilde": 2, "r": 3, "S": 4}

# every symbol the header declares
EXPORTS = [
    "adafac_default_opts", "adafac_create", "adafac_set_coefficient_blocks", "adafac_set_rhs_lattice",
    "adafac_build_operators", "adafac_workspace_bytes", "adafac_bind", "adafac_cycle", "adafac_solve",
    "adafac_residual", "adafac_cycles_run", "adafac_get_solution", "adafac_set_solution",
    "adafac_get_level", "adafac_host_operator", "adafac_dofs_per_cycle", "adafac_set_kernel_timing", "adafac_kernel_time",
    "adafac_destroy", "adafac_last_error", "adafac_set_refinement", "adafac_refine_ball", "adafac_composite_dofs",
    "adafac_regrid_prepare", "adafac_regrid", "adafac_set_rhs_gaussian",
    "adafac_server_default_cfg", "adafac_server_create", "adafac_server_submit", "adafac_server_step",
    "adafac_server_poll", "adafac_server_fetch", "adafac_server_destroy", "adafac_server_last_error",
    "adafac_stream_copy", "adafac_set_rhs_fn", "adafac_residual_normalised", "adafac_dof_coords",
    "adafac_get_composite", "adafac_set_composite", "adafac_bind_static", "adafac_set_dirichlet_lattice",
    "adafac_amr_mark", "adafac_set_solution_coarse",
]


# double f(const double* x, void* user)
RHS_FN = C.CFUNCTYPE(C.c_double, C.POINTER(C.c_double), C.c_void_p)


class Opts(C.Structure):
    _fields_ = [("transfer", C.c_int), ("damping", C.c_int), ("rtilde", C.c_int), ("precision", C.c_int),
                ("inner_k", C.c_int), ("fused", C.c_int), ("omega", C.c_double),
                ("omega_tilde", C.c_double), ("omega_hat", C.c_double)]


class ServerCfg(C.Structure):
    _fields_ = [("max_active", C.c_int), ("max_queued", C.c_int), ("cycles_per_round", C.c_int),
                ("max_streams", C.c_int), ("batch_max_vertices", C.c_size_t)]


class Request(C.Structure):
    _fields_ = [("dim", C.c_int), ("l_min", C.c_int), ("l_max", C.c_int), ("blocks_per_axis", C.c_int),
                ("eps", C.POINTER(C.c_double)), ("f", C.POINTER(C.c_double)), ("opts", Opts),
                ("rel_tol", C.c_double), ("max_cycles", C.c_int)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("cycles", C.c_int), ("batched", C.c_int), ("error", C.c_int),
                ("l2h0", C.c_double), ("l2h", C.c_double), ("linf", C.c_double),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("footprint", C.c_size_t)]


class AdafacError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"adafac error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libadafac.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} missing: run `python -m paper_1903_10367_amd.build` first")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "adafac_default_opts": (None, [C.POINTER(Opts)]),
        "adafac_create": (C.c_int, [C.POINTER(P), C.c_int, C.c_int, C.c_int]),
        "adafac_set_coefficient_blocks": (C.c_int, [P, C.c_int, C.POINTER(C.c_double)]),
        "adafac_set_rhs_lattice": (C.c_int, [P, C.POINTER(C.c_double), C.c_size_t]),
        "adafac_build_operators": (C.c_int, [P, C.POINTER(Opts)]),
        "adafac_workspace_bytes": (C.c_int, [P, C.POINTER(C.c_size_t)]),
        "adafac_bind": (C.c_int, [P, P, C.c_size_t, P]),
        "adafac_bind_static": (C.c_int, [P, P]),
        "adafac_set_dirichlet_lattice": (C.c_int, [P, C.POINTER(C.c_double), C.c_size_t]),
        "adafac_cycle": (C.c_int, [P, C.c_int]),
        "adafac_solve": (C.c_int, [P, C.c_double, C.c_int, C.POINTER(C.c_int)]),
        "adafac_residual": (C.c_int, [P, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "adafac_cycles_run": (C.c_int, [P]),
        "adafac_get_solution": (C.c_int, [P, C.POINTER(C.c_double), C.c_size_t]),
        "adafac_set_solution": (C.c_int, [P, C.POINTER(C.c_double), C.c_size_t]),
        "adafac_get_level": (C.c_int, [P, C.c_int, C.c_int, C.POINTER(C.c_double), C.c_size_t]),
        "adafac_host_operator": (C.c_int, [P, C.c_int, C.c_int, C.POINTER(C.c_double), C.c_size_t]),
        "adafac_dofs_per_cycle": (C.c_int64, [P]),
        "adafac_set_kernel_timing": (C.c_int, [P, C.c_int]),
        "adafac_kernel_time": (C.c_int, [P, C.POINTER(C.c_double), C.POINTER(C.c_int)]),
        "adafac_destroy": (None, [P]),
        "adafac_set_refinement": (C.c_int, [P, C.c_int, C.POINTER(C.c_uint8), C.c_size_t]),
        "adafac_refine_ball": (C.c_int, [P, C.POINTER(C.c_double), C.c_double, C.c_int]),
        "adafac_composite_dofs": (C.c_int64, [P]),
        "adafac_regrid_prepare": (C.c_int, [P, C.POINTER(C.c_double), C.c_double, C.c_int, C.POINTER(C.c_double),
                                            C.c_size_t, C.POINTER(C.c_size_t)]),
        "adafac_regrid": (C.c_int, [P, P, C.c_size_t]),
        "adafac_set_rhs_gaussian": (C.c_int, [P, C.POINTER(C.c_double), C.c_double, C.c_double]),
        "adafac_last_error": (C.c_char_p, [P]),
        "adafac_server_default_cfg": (None, [C.POINTER(ServerCfg)]),
        "adafac_server_create": (C.c_int, [C.POINTER(ServerCfg), P, C.c_size_t, P, C.POINTER(P)]),
        "adafac_server_submit": (C.c_int, [P, C.POINTER(Request), C.POINTER(C.c_uint64)]),
        "adafac_server_step": (C.c_int, [P, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "adafac_server_poll": (C.c_int, [P, C.c_uint64, C.POINTER(Result)]),
        "adafac_server_fetch": (C.c_int, [P, C.c_uint64, C.POINTER(C.c_double), C.c_size_t]),
        "adafac_server_destroy": (None, [P]),
        "adafac_server_last_error": (C.c_char_p, [P]),
        "adafac_stream_copy": (C.c_int, [P, P, C.c_size_t, P]),
        "adafac_set_rhs_fn": (C.c_int, [P, RHS_FN, P]),
        "adafac_residual_normalised": (C.c_int, [P, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "adafac_dof_coords": (C.c_int, [P, C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_size_t]),
        "adafac_get_composite": (C.c_int, [P, C.POINTER(C.c_double), C.c_size_t]),
        "adafac_set_composite": (C.c_int, [P, C.POINTER(C.c_double), C.c_size_t]),
        "adafac_amr_mark": (C.c_int, [P, C.c_double, C.c_int, C.c_int, C.POINTER(C.c_uint8), C.c_size_t,
                                      C.POINTER(C.c_int)]),
        "adafac_set_solution_coarse": (C.c_int, [P, C.POINTER(C.c_double), C.c_size_t, C.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype, f.argtypes = res, args
    _lib = L
    return L
