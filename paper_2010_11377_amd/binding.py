"""ctypes binding of libirk (include/irk.h): structures, prototypes and the
library loader.  Argument marshalling only; every step of the solve runs in
the HIP library.  Loading fails loudly when the library has not been built.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libirk.so")

IRK_OK = 0
IRK_E_INVALID = -1
IRK_E_SINGULAR_PIVOT = -2
IRK_E_NOT_CONVERGED = -3
IRK_E_BREAKDOWN = -4
IRK_E_NONFINITE = -5
IRK_E_HIP = -6
IRK_E_OOM = -7

KERNEL_CLASSES = ["spmm_dots", "spmm_update", "vec_dots", "vec_update", "couple", "vdown_l0",
                  "vup_l0", "vmid_down", "vtail", "vmid_up"]

IRK_FP64 = 0
IRK_MIXED = 1
IRK_RIGHT = 0
IRK_LEFT = 1
IRK_INTERP_LINEAR = 0
IRK_INTERP_CONSTANT = 1
SMOOTHER = {"rbgs": 0, "jacobi": 1}
PRECOND = {"LD": 0, "DU": 1, "GSL": 2, "J": 3}


class Butcher(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int), ("A", ctypes.POINTER(ctypes.c_double)),
                ("b", ctypes.POINTER(ctypes.c_double)), ("c", ctypes.POINTER(ctypes.c_double))]


class CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("nnz", ctypes.c_int),
                ("rowptr", ctypes.POINTER(ctypes.c_int)), ("colind", ctypes.POINTER(ctypes.c_int)),
                ("val", ctypes.POINTER(ctypes.c_double))]


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("precond", ctypes.c_int), ("restart", ctypes.c_int),
                ("max_iter", ctypes.c_int), ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int),
                ("coarse_max", ctypes.c_int), ("vcycles", ctypes.c_int),
                ("true_resid", ctypes.c_int), ("reorth", ctypes.c_int), ("rtol", ctypes.c_double),
                ("side", ctypes.c_int),
                ("interp", ctypes.c_int), ("graphs", ctypes.c_int),
                ("coarse_ratio", ctypes.c_double), ("smoother", ctypes.c_int),
                ("jacobi_omega", ctypes.c_double), ("fuse_levels", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int),
                ("rel_resid_est", ctypes.c_double), ("rel_resid_true", ctypes.c_double),
                ("seconds", ctypes.c_double)]


class IRKError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (status_string(status), message))
        self.status = status


_lib = None

_PD = ctypes.POINTER(ctypes.c_double)
_VP = ctypes.c_void_p

_PROTOS = {
    "irk_default_options": (None, [ctypes.POINTER(Options)]),
    "irk_ldu": (ctypes.c_int, [ctypes.c_int, _PD, _PD, _PD, _PD]),
    "irk_setup": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.POINTER(Butcher), ctypes.POINTER(CSR),
                                 ctypes.POINTER(CSR), ctypes.c_double, ctypes.POINTER(Grid),
                                 ctypes.POINTER(Options), _VP]),
    "irk_set_source": (ctypes.c_int, [_VP, _VP]),
    "irk_update_operator": (ctypes.c_int, [_VP, ctypes.POINTER(CSR)]),
    "irk_step": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(Stats)]),
    "irk_step_stages": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.POINTER(Stats)]),
    "irk_step_noalloc": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(Stats)]),
    "irk_adjoint_step": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, ctypes.POINTER(Stats)]),
    "irk_grad_diffusion_nodes": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_double, _VP]),
    "irk_grad_diffusion_faces": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_double, _VP]),
    "irk_apply_operator": (ctypes.c_int, [_VP, _VP, _VP]),
    "irk_apply_preconditioner": (ctypes.c_int, [_VP, _VP, _VP]),
    "irk_destroy": (None, [_VP]),
    "irk_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "irk_last_error": (ctypes.c_char_p, [_VP]),
    "irk_profile_select": (ctypes.c_int, [_VP, ctypes.c_int]),
    "irk_profile_read": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_longlong),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "irk_info": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "irk_graph_stats": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_longlong)]),
}


def lib():
    """The loaded libirk (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libirk.so is not built (%s); run __graft_entry__.build() or "
                               "python -m paper_2010_11377_amd.build" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(st):
    return lib().irk_status_string(int(st)).decode()


def check(status, handle=None):
    if status != IRK_OK:
        msg = lib().irk_last_error(handle).decode() if True else ""
        raise IRKError(status, msg)


def default_options():
    o = Options()
    lib().irk_default_options(ctypes.byref(o))
    return o


def dptr(arr):
    """ctypes double pointer of a contiguous float64 numpy array."""
    return arr.ctypes.data_as(_PD)
