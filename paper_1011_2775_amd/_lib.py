"""ctypes binding of libwcmg.so (argument marshalling only).

torch is imported first so that the HIP runtime it ships is the one the
library binds to (both carry the soname libamdhip64.so.7).  Loading fails
loudly when the library has not been built: there is no fallback path.
"""
import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime before libwcmg)

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "lib", "libwcmg.so")

OK, EINVAL, EDIM, ESTATE, ENOCONV, EBREAKDOWN, ENAN, ECLOVER_NOT_PD, ERANK, ENOMEM, EHIP, ENODEV = range(12)
F64, F32, F16 = 0, 1, 2
OP_FULL, OP_SCHUR, OP_DP, OP_SCHUR_X = 0, 1, 2, 3
MG_GCR, GCR, BICGSTAB, MP_BICGSTAB, CGNR = 0, 1, 2, 3, 4
MAX_LEVELS = 4

ERROR_NAMES = {0: "OK", 1: "EINVAL", 2: "EDIM", 3: "ESTATE", 4: "ENOCONV", 5: "EBREAKDOWN", 6: "ENAN",
               7: "ECLOVER_NOT_PD", 8: "ERANK", 9: "ENOMEM", 10: "EHIP", 11: "ENODEV"}


class Lattice(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("t_bc", ctypes.c_int)]


class MGParams(ctypes.Structure):
    _fields_ = [("nlevels", ctypes.c_int),
                ("block", (ctypes.c_int * 4) * MAX_LEVELS),
                ("nvec", ctypes.c_int * MAX_LEVELS),
                ("tol", ctypes.c_double * MAX_LEVELS),
                ("max_iter", ctypes.c_int * MAX_LEVELS),
                ("restart", ctypes.c_int * MAX_LEVELS),
                ("nu_post", ctypes.c_int),
                ("outer_restart", ctypes.c_int),
                ("outer_max_iter", ctypes.c_int),
                ("smoother_prec", ctypes.c_int),
                ("setup_relax", ctypes.c_int),
                ("setup_max_steps", ctypes.c_int),
                ("setup_rq_tol", ctypes.c_double),
                ("seed", ctypes.c_uint64),
                ("coarsest", ctypes.c_int),
                ("cycle_mode", ctypes.c_int),
                ("setup_prec", ctypes.c_int),
                ("coarse_launch", ctypes.c_int),
                ("plain_max_iter", ctypes.c_int),
                ("mp_inner_tol", ctypes.c_double),
                ("coarse_fp16", ctypes.c_int),
                ("transfer_fp16", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int),
                ("inner_iters", ctypes.c_double * MAX_LEVELS),
                ("true_rel_res", ctypes.c_double),
                ("t_solve_s", ctypes.c_double),
                ("status", ctypes.c_int),
                ("inner_status", ctypes.c_int)]

    def as_dict(self):
        return dict(iters=self.iters, inner_iters=list(self.inner_iters), true_rel_res=self.true_rel_res,
                    t_solve_s=self.t_solve_s, status=ERROR_NAMES.get(self.status, self.status),
                    inner_status=ERROR_NAMES.get(self.inner_status, self.inner_status))


_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double

SIGNATURES = {
    "wcmg_mg_params_default": [ctypes.POINTER(MGParams)],
    "wcmg_create": [ctypes.POINTER(Lattice), _i, _vp, ctypes.POINTER(_vp)],
    "wcmg_destroy": [_vp],
    "wcmg_set_gauge": [_vp, _i, _vp, _i],
    "wcmg_set_clover": [_vp, _i, _d, _d, _vp, _i],
    "wcmg_set_clover_aniso": [_vp, _i, _d, _d, _d, _d],
    "wcmg_set_mg_params": [_vp, _i, ctypes.POINTER(MGParams)],
    "wcmg_build_null_vectors": [_vp, _i, _i],
    "wcmg_set_null_vectors": [_vp, _i, _i, _vp, _i, _i],
    "wcmg_get_null_vectors": [_vp, _i, _i, _vp, _i],
    "wcmg_build_coarse": [_vp, _i, _i],
    "wcmg_refine_null_vectors": [_vp, _i, _i, _i],
    "wcmg_setup_start_vectors": [_vp, _i, _i, ctypes.c_uint64, _i, _i, _vp],
    "wcmg_get_coarse": [_vp, _i, _i, _vp, _i],
    "wcmg_apply_D": [_vp, _i, _i, _i, _vp, _vp, _i],
    "wcmg_apply_Ddag": [_vp, _i, _i, _i, _vp, _vp, _i],
    "wcmg_restrict": [_vp, _i, _i, _i, _vp, _vp, _i],
    "wcmg_prolong": [_vp, _i, _i, _i, _vp, _vp, _i],
    "wcmg_apply_coarse": [_vp, _i, _i, _i, _i, _vp, _vp, _i],
    "wcmg_coarse_solve": [_vp, _i, _i, _i, _vp, _vp, _d, _i, _i, _i, _vp],
    "wcmg_coarse_solve_noalloc": [_vp, _i, _i, _i, _vp, _vp, _d, _i, _i, _vp],
    "wcmg_solve": [_vp, _i, _i, _vp, _vp, _i, _d, ctypes.POINTER(Stats)],
    "wcmg_solve_dag": [_vp, _i, _i, _vp, _vp, _i, _d, ctypes.POINTER(Stats)],
    "wcmg_force": [_vp, _i, _vp, _vp, _vp, _i, _i],
    "wcmg_autotune": [_vp, _i],
    "wcmg_autotune_report": [_vp, ctypes.c_char_p, _i],
    "wcmg_dot": [_vp, _i, _vp, _vp, ctypes.c_long, ctypes.POINTER(_d)],
    "wcmg_timer_enable": [_vp, _i],
    "wcmg_timer_read": [_vp, _i, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(_d)],
}


def load():
    if not os.path.exists(LIBPATH):
        raise ImportError("libwcmg.so is not built (%s); run python -m paper_1011_2775_amd.build" % LIBPATH)
    lib = ctypes.CDLL(LIBPATH)
    for name, args in SIGNATURES.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.wcmg_last_error.argtypes = []
    lib.wcmg_last_error.restype = ctypes.c_char_p
    return lib


_LIB = None


def get():
    """The loaded library (loaded on first use, so the package imports without it)."""
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


def __getattr__(name):
    if name == "LIB":
        return get()
    raise AttributeError(name)


class WcmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERROR_NAMES.get(code, code), msg))
        self.code = code


def check(rc):
    if rc != OK:
        raise WcmgError(rc, get().wcmg_last_error().decode())
    return rc
