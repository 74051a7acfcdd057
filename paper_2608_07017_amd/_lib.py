"""ctypes binding of libwos.so (argument marshalling only).

Device buffers are torch tensors on the current HIP device; the stream is
torch's current stream.  Every computation happens in the library's
kernels; nothing here falls back to a CPU path: if the library is missing
the import fails.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwos.so")

WOS_OK = 0
STATUS = {0: "WOS_OK", -1: "WOS_EINVAL", -2: "WOS_EDOMAIN", -3: "WOS_ENOMEM", -4: "WOS_EDEVICE",
          -5: "WOS_ENOTCONV", -6: "WOS_EBUSY", -7: "WOS_ENOTIMPL"}
KINDS = {"ball": 1, "box": 2, "polygon": 3, "box_minus_ball": 4}
PRECISION = {"f32": 0, "f64": 1}
EXPORTS = {"A": 0, "B": 1, "H": 2, "K": 3, "Hcount": 4, "lambda": 5, "vcount": 6, "lambda_v": 7, "site_steps": 8,
           "moments": 9, "shadow_v": 10, "shadow_g": 11}


class WosDomain(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dim", ctypes.c_int32),
                ("center", ctypes.c_double * 3), ("radius", ctypes.c_double),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("nvert", ctypes.c_int32), ("verts", ctypes.POINTER(ctypes.c_double))]


class WosBuildOpts(ctypes.Structure):
    _fields_ = [("walks_per_site", ctypes.c_int64), ("eps", ctypes.c_double),
                ("max_steps", ctypes.c_int32), ("fixed_M", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("precision", ctypes.c_int32),
                ("volume_samples", ctypes.c_int64), ("walks_per_item", ctypes.c_int32),
                ("regen_threshold", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("tally_mode", ctypes.c_int32), ("sampler", ctypes.c_int32),
                ("walker_block", ctypes.c_int32), ("tally_acc", ctypes.c_int32),
                ("window_pages", ctypes.c_int32), ("window_bpages", ctypes.c_int32),
                ("test_phi", ctypes.POINTER(ctypes.c_double)), ("test_psi", ctypes.POINTER(ctypes.c_double))]


class WosBuildPlan(ctypes.Structure):
    _fields_ = [("tally_mode", ctypes.c_int32), ("tally_acc", ctypes.c_int32),
                ("walks_per_item", ctypes.c_int32), ("items_per_site", ctypes.c_int32),
                ("window_pages", ctypes.c_int32), ("window_bpages", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int64), ("fixed_bound", ctypes.c_double)]


TALLY_MODES = {"auto": 0, "lds_rows": 1, "window": 2, "hbm": 3}
TALLY_ACC = {"auto": 0, "fixed": 1, "f64": 2}


class WosToolboxInfo(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("p", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("walks_per_site", ctypes.c_int64), ("walk_steps", ctypes.c_uint64),
                ("walks", ctypes.c_uint64), ("capped_walks", ctypes.c_uint64),
                ("max_walk_steps", ctypes.c_uint64), ("volume_inside", ctypes.c_uint64),
                ("device_bytes", ctypes.c_size_t)]


class WosCoeffs(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("A", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("c", ctypes.c_void_p), ("kappa", ctypes.c_double), ("rcond", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("solver", ctypes.c_int32), ("precision", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("refine_tol", ctypes.c_double)]


class WosServerOpts(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("mem_budget", ctypes.c_size_t), ("max_batch", ctypes.c_int32)]


class WosOperatorOpts(ctypes.Structure):
    _fields_ = [("want_grad", ctypes.c_int32), ("storage", ctypes.c_int32)]


class WosOperatorInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("p", ctypes.c_int32), ("dim", ctypes.c_int32),
                ("want_grad", ctypes.c_int32), ("storage", ctypes.c_int32), ("reg", ctypes.c_double),
                ("device_bytes", ctypes.c_size_t), ("prep_ms", ctypes.c_double)]


class WosSolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("rank", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("sigma_max", ctypes.c_double), ("sigma_threshold", ctypes.c_double),
                ("grad_norm", ctypes.c_double), ("grad_norm0", ctypes.c_double),
                ("update_norm", ctypes.c_double), ("reg", ctypes.c_double), ("refine_iters", ctypes.c_int32),
                ("fallback", ctypes.c_int32), ("refine_residual", ctypes.c_double),
                ("refine_converged", ctypes.c_int32)]


class WosAdamOpts(ctypes.Structure):
    _fields_ = [("energy", ctypes.c_int32), ("p_exp", ctypes.c_double), ("alpha", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double), ("check_every", ctypes.c_int32),
                ("coef_A", ctypes.c_void_p), ("coef_c", ctypes.c_void_p), ("coef_w", ctypes.c_void_p),
                ("graph", ctypes.c_int32)]


class WosAdamInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("J", ctypes.c_double), ("grad_norm", ctypes.c_double),
                ("grad_norm0", ctypes.c_double), ("seconds", ctypes.c_double)]


class WosHisdOpts(ctypes.Structure):
    _fields_ = [("energy", ctypes.c_int32), ("p_exp", ctypes.c_double), ("k", ctypes.c_int32),
                ("eta", ctypes.c_double), ("tau", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("tol", ctypes.c_double), ("check_every", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("init", ctypes.c_int32), ("graph", ctypes.c_int32)]


class WosHisdInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("J", ctypes.c_double), ("grad_norm", ctypes.c_double),
                ("grad_norm0", ctypes.c_double), ("seconds", ctypes.c_double), ("ns_iters", ctypes.c_int32),
                ("ns_residual", ctypes.c_double)]


ENERGIES = {"plaplace": 0, "minimal_surface": 1, "semilinear": 2, "elliptic": 3}
HISD_PRECOND = {"identity": 0, "A": 1}
HISD_INIT = {"given": 0, "hessian": 1}
PROBLEMS = {"linear": 0, "semilinear_cubic": 1, "quasilinear": 2}
SOLVERS = {"tsvd": 0, "tikhonov": 1}
SOLVE_PRECISION = {"f64": 0, "mixed": 1, "bf16": 2}

# every symbol include/wos.h declares, with its ctypes signature
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "wos_toolbox_create": (ctypes.c_int, [ctypes.POINTER(WosDomain), _D, ctypes.c_int32, _D, ctypes.c_int32,
                                          ctypes.POINTER(WosBuildOpts), ctypes.POINTER(_P)]),
    "wos_toolbox_create_wv": (ctypes.c_int, [ctypes.POINTER(WosDomain), _D, ctypes.c_int32, _D, ctypes.c_int32, _D,
                                             ctypes.c_int32, ctypes.POINTER(WosBuildOpts), ctypes.POINTER(_P)]),
    "wos_toolbox_plan": (ctypes.c_int, [ctypes.POINTER(WosDomain), _D, ctypes.c_int32, _D, ctypes.c_int32, _D,
                                        ctypes.c_int32, ctypes.POINTER(WosBuildOpts), ctypes.POINTER(WosBuildPlan)]),
    "wos_toolbox_build": (ctypes.c_int, [_P, ctypes.c_uint64, _P]),
    "wos_build_toolbox": (ctypes.c_int, [ctypes.POINTER(WosDomain), _D, ctypes.c_int32, _D, ctypes.c_int32,
                                         ctypes.POINTER(WosBuildOpts), _P, ctypes.POINTER(_P)]),
    "wos_toolbox_get_info": (ctypes.c_int, [_P, ctypes.POINTER(WosToolboxInfo)]),
    "wos_toolbox_export": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_size_t, ctypes.c_int32, _P]),
    "wos_apply": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "wos_toolbox_make_bf16": (ctypes.c_int, [_P, _P]),
    "wos_apply_bf16": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "wos_gemm_bf16_nt": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, _P,
                                        ctypes.c_int64, _P, ctypes.c_int64, ctypes.c_float, _P, ctypes.c_int64, _P]),
    "wos_solve": (ctypes.c_int, [_P, ctypes.POINTER(WosCoeffs), _P, _P, _P, _P, _P,
                                 ctypes.POINTER(WosSolveInfo), _P]),
    "wos_solve_noalloc": (ctypes.c_int, [_P, ctypes.POINTER(WosCoeffs), _P, _P, _P, _P, _P,
                                         ctypes.POINTER(WosSolveInfo), _P]),
    "wos_interpolate": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int64, _P, _P, _P]),
    "wos_toolbox_take": (ctypes.c_int, [_P, _P, ctypes.c_uint32, _P]),
    "wos_minimize": (ctypes.c_int, [_P, ctypes.POINTER(WosAdamOpts), _P, _P, _P, _P, _P,
                                    ctypes.POINTER(WosAdamInfo), _P]),
    "wos_saddle": (ctypes.c_int, [_P, ctypes.POINTER(WosHisdOpts), _P, _P, _P, _P, _P, _P,
                                  ctypes.POINTER(WosHisdInfo), _P]),
    "wos_toolbox_set_timing": (ctypes.c_int, [_P, ctypes.c_int32]),
    "wos_toolbox_get_timings": (ctypes.c_int, [_P, _D, _D, _D]),
    "wos_toolbox_free": (None, [_P]),
    "wos_toolbox_save": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "wos_toolbox_load": (ctypes.c_int, [ctypes.c_char_p, _P, ctypes.POINTER(_P)]),
    "wos_last_error": (ctypes.c_char_p, []),
    "wos_version": (ctypes.c_char_p, []),
    "wos_server_create": (ctypes.c_int, [ctypes.POINTER(WosServerOpts), ctypes.POINTER(_P)]),
    "wos_server_submit": (ctypes.c_int, [_P, _P, ctypes.POINTER(WosCoeffs), _P, _P, _P, _P,
                                         ctypes.POINTER(ctypes.c_uint64)]),
    "wos_operator_create": (ctypes.c_int, [_P, ctypes.POINTER(WosCoeffs), ctypes.POINTER(WosOperatorOpts), _P,
                                           ctypes.POINTER(_P)]),
    "wos_operator_apply": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                          ctypes.POINTER(_P), ctypes.POINTER(_P), _P]),
    "wos_operator_get_info": (ctypes.c_int, [_P, ctypes.POINTER(WosOperatorInfo)]),
    "wos_operator_free": (None, [_P]),
    "wos_server_submit_op": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_uint64)]),
    "wos_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(WosSolveInfo), _D]),
    "wos_server_pending": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "wos_server_destroy": (None, [_P]),
    "wos_probe_valu": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _D, _P]),
}


class WosError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


_lib = None


def lib():
    """The loaded library (raises if libwos.so has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libwos.so not built: run `python -m paper_2608_07017_amd.build` "
                              "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != WOS_OK:
        raise WosError(status, lib().wos_last_error().decode())
