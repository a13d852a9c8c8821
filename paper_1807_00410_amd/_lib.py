"""ctypes declarations of the C ABI in include/pn.h (argument marshalling only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpn.so")

PN_MAX_COEFF = 64
PN_MAX_HISTORY = 64
PN_PHASES = 5
PHASES = ("setup", "residual", "krylov", "learned", "finish")

PN_OK = 0
PN_ERR_ARG = 1
PN_ERR_ALLOC = 2
PN_ERR_HIP = 3
PN_ERR_NONFINITE = 4
PN_ERR_NOT_CONVERGED = 5
PN_ERR_BREAKDOWN = 6

PN_BC_VACUUM = 0
PN_BC_PERIODIC = 1
PN_BC_NEUMANN = 2
PN_BC_PER_AXIS = 3
PN_FP32_IR = 0
PN_FP64 = 1


class PnGrid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("h", C.c_double), ("bc", C.c_int),
                ("bc_axis", C.c_int * 3)]


class PnMedium(C.Structure):
    _fields_ = [("sigma_t", C.c_void_p), ("albedo", C.c_void_p), ("g", C.c_float), ("sigma_t_min", C.c_float)]


class PnLayout(C.Structure):
    _fields_ = [("order", C.c_int), ("ncoeff", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("bc", C.c_int), ("bc_axis", C.c_int * 3), ("n_unknowns", C.c_longlong),
                ("cls", (C.c_int * 3) * PN_MAX_COEFF), ("ext", (C.c_int * 3) * PN_MAX_COEFF),
                ("offset", C.c_longlong * (PN_MAX_COEFF + 1))]


class PnSolveOpts(C.Structure):
    _fields_ = [("precision", C.c_int), ("max_iter", C.c_int), ("max_refine", C.c_int),
                ("inner_tol", C.c_double), ("use_guess", C.c_int), ("graph_iters", C.c_int),
                ("variant", C.c_int), ("learned", C.c_int)]


class PnSolveInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("outer_iters", C.c_int), ("inner_iters", C.c_int),
                ("rel_residual", C.c_double), ("bnorm", C.c_double), ("seconds", C.c_double),
                ("nhistory", C.c_int), ("history", C.c_double * PN_MAX_HISTORY),
                ("learned_steps", C.c_int), ("learned_ratio", C.c_double),
                ("t_ms", C.c_double * PN_PHASES), ("bytes", C.c_double), ("achieved_gbs", C.c_double)]


class PnProblem(C.Structure):
    _fields_ = [("order", C.c_int), ("grid", PnGrid), ("medium", PnMedium)]


# (name, restype, argtypes) of every exported symbol declared in include/pn.h
SIGNATURES = [
    ("pn_abi_version", C.c_int, []),
    ("pn_status_string", C.c_char_p, [C.c_int]),
    ("pn_default_opts", None, [C.POINTER(PnSolveOpts)]),
    ("pn_setup", C.c_int, [C.c_int, C.POINTER(PnGrid), C.POINTER(PnMedium), C.c_void_p, C.POINTER(C.c_void_p)]),
    ("pn_layout_query", C.c_int, [C.c_void_p, C.POINTER(PnLayout)]),
    ("pn_apply", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    ("pn_apply64", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    ("pn_residual64", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    ("pn_solve", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.POINTER(PnSolveOpts),
                           C.POINTER(PnSolveInfo)]),
    ("pn_destroy", None, [C.c_void_p]),
    ("pn_last_error", C.c_char_p, [C.c_void_p]),
    ("pn_bench_apply", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_double)]),
    ("pn_set_zchunk", C.c_int, [C.c_void_p, C.c_int]),
    ("pn_get_zchunk", C.c_int, [C.c_void_p]),
    ("pn_bench_kernel", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_double)]),
    ("pn_row_weights", C.c_int, [C.c_void_p, C.c_void_p]),
    ("pn_apply_schur", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pn_apply_precond", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    ("pn_single_scatter", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_double, C.c_void_p]),
    ("pn_unstagger", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pn_set_tiles", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int]),
    ("pn_get_tiles", C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    ("pn_coupling_table", C.c_int, [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                    C.POINTER(C.c_double), C.c_int]),
    ("pn_autotune", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    ("pn_tune_cache_save", C.c_int, [C.c_char_p]),
    ("pn_tune_cache_load", C.c_int, [C.c_char_p]),
    ("pn_tune_cache_size", C.c_int, []),
    ("pn_tune_cache_clear", None, []),
    ("pn_batch_setup", C.c_int, [C.c_int, C.POINTER(PnProblem), C.c_int, C.c_int, C.c_void_p,
                                 C.POINTER(C.c_void_p)]),
    ("pn_batch_layout", C.c_int, [C.c_void_p, C.c_int, C.POINTER(PnLayout)]),
    ("pn_batch_zchunk", C.c_int, [C.c_void_p, C.c_int]),
    ("pn_batch_unknowns", C.c_longlong, [C.c_void_p]),
    ("pn_batch_solve", C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_double,
                                 C.POINTER(PnSolveOpts), C.POINTER(PnSolveInfo)]),
    ("pn_batch_bench_apply", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_double)]),
    ("pn_batch_destroy", None, [C.c_void_p]),
    ("pn_batch_last_error", C.c_char_p, [C.c_void_p]),
    ("pn_batch_problem", C.c_void_p, [C.c_void_p, C.c_int]),
]

_V = C.c_void_p
_I = C.c_int
# (name, restype, argtypes) of every exported symbol declared in include/pn_nn.h
NN_SIGNATURES = [
    ("pn_nn_conv3d", _I, [_I, _I, _I, _I, _V, _V, _V, _I, _I, _V, _V]),
    ("pn_nn_conv3d_dgrad", _I, [_I, _I, _I, _I, _V, _V, _V, _V]),
    ("pn_nn_conv3d_wgrad", _I, [_I, _I, _I, _I, _V, _V, _V, _V, _V]),
    ("pn_nn_conv3d_wgrad_noalloc", _I, [_I, _I, _I, _I, _V, _V, _V, _V, _V]),
    ("pn_nn_pool2", _I, [_I, _I, _I, _I, _V, _V, _V]),
    ("pn_nn_pool2_bwd_add", _I, [_I, _I, _I, _I, _V, _V, _V, _V]),
    ("pn_nn_up2_add", _I, [_I, _I, _I, _I, _V, _V, _V, _V]),
    ("pn_nn_up2_bwd", _I, [_I, _I, _I, _I, _V, _V, _V]),
    ("pn_nn_adam", _I, [_V, _V, _V, _V, C.c_longlong, C.c_longlong, C.c_float, C.c_double, C.c_double, C.c_float,
                        _V]),
    ("pn_nn_last_error", C.c_char_p, []),
    ("pn_net_nparams", _I, []),
    ("pn_net_create", _I, [C.c_ulonglong, _V, C.POINTER(_V)]),
    ("pn_net_destroy", None, [_V]),
    ("pn_net_last_error", C.c_char_p, [_V]),
    ("pn_net_get_params", _I, [_V, _V, _V]),
    ("pn_net_set_params", _I, [_V, _V]),
    ("pn_net_save", _I, [_V, C.c_char_p]),
    ("pn_net_load", _I, [_V, C.c_char_p]),
    ("pn_net_forward", _I, [_V, _I, _I, _I, _I, _V, _V]),
    ("pn_net_train_step", _I, [_V, _I, _I, _I, _I, _V, _V, _I, C.c_float, C.POINTER(C.c_double)]),
    ("pn_net_set_stream", _I, [_V, _V]),
    ("pn_net_train", _I, [_V, _I, _I, _I, _I, C.POINTER(_V), C.POINTER(_V), _I, _I, _I, C.c_float,
                          C.c_ulonglong, C.POINTER(C.c_double)]),
    ("pn_net_get_stream", _V, [_V]),
    ("pn_net_grid", _I, [_V, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I)]),
    ("pn_net_features", _I, [_V, _V, _V]),
    ("pn_net_targets", _I, [_V, _V, _V]),
    ("pn_net_targets_diff", _I, [_V, _V, _V, _V]),
    ("pn_attach_net", _I, [_V, _V]),
]

_lib = None


def load(path=None):
    """Loads libpn.so (built by paper_1807_00410_amd.build); raises if absent."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError("libpn.so not found at %s: run `python -m paper_1807_00410_amd.build` "
                           "(there is no CPU fallback)" % p)
    lib = C.CDLL(p)
    for name, res, args in SIGNATURES + NN_SIGNATURES:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib
