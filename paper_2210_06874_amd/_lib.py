"""ctypes declarations of the C ABI in include/hub.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhubhip.so")

HUB_OK, HUB_ERR_ARG, HUB_ERR_DEVICE, HUB_ERR_NOMEM, HUB_ERR_NOCONV, HUB_ERR_NONFINITE = range(6)
STATUS_NAMES = {0: "HUB_OK", 1: "HUB_ERR_ARG", 2: "HUB_ERR_DEVICE", 3: "HUB_ERR_NOMEM",
                4: "HUB_ERR_NOCONV", 5: "HUB_ERR_NONFINITE"}
HUB_PREC_FP64, HUB_PREC_MIXED = 0, 1
HUB_PATH_AUTO, HUB_PATH_FUSED, HUB_PATH_SPLIT = 0, 1, 2
HUB_FORM_EXP, HUB_FORM_LINEAR = 0, 1
HUB_MD_LEAPFROG, HUB_MD_OMELYAN = 0, 1


class HubParams(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("Nt", ctypes.c_int32), ("beta", ctypes.c_double),
                ("kappa", ctypes.c_double), ("nrhs_max", ctypes.c_int32), ("path", ctypes.c_int32),
                ("mu", ctypes.c_double), ("form", ctypes.c_int32)]


class HubCgOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("reliable_every", ctypes.c_int32), ("prec", ctypes.c_int32), ("use_x0", ctypes.c_int32),
                ("stall_updates", ctypes.c_int32), ("history_host", ctypes.c_void_p),
                ("history_len", ctypes.c_int32)]


class HubCgInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("reliable_updates", ctypes.c_int32),
                ("true_rel_res", ctypes.c_double), ("recursive_rel_res", ctypes.c_double),
                ("persistent_launches", ctypes.c_int32)]


class HubTrajOpts(ctypes.Structure):
    _fields_ = [("U", ctypes.c_double), ("eps", ctypes.c_double), ("n_md", ctypes.c_int32),
                ("integrator", ctypes.c_int32), ("cg", HubCgOpts)]


class HubTrajInfo(ctypes.Structure):
    _fields_ = [("accepted", ctypes.c_int32), ("n_forces", ctypes.c_int32), ("cg_iters", ctypes.c_int32),
                ("H0", ctypes.c_double), ("H1", ctypes.c_double), ("dH", ctypes.c_double)]


_P = ctypes.c_void_p
_I = ctypes.c_int32
SIGNATURES = {
    "hub_create": (ctypes.POINTER(HubParams), _P, ctypes.POINTER(_P)),
    "hub_destroy": (_P,),
    "hub_apply_M": (_P, _P, _P, _P, _I, _P),
    "hub_apply_Mdag": (_P, _P, _P, _P, _I, _P),
    "hub_apply_M_c64": (_P, _P, _P, _P, _I, _P),
    "hub_apply_Mdag_c64": (_P, _P, _P, _P, _I, _P),
    "hub_cg_solve": (_P, _P, _P, _P, _I, ctypes.POINTER(HubCgOpts), ctypes.POINTER(HubCgInfo), _P),
    "hub_force": (_P, _P, _P, _P, _I, _P),
    "hub_force_noalloc": (_P, _P, _P, _P, _I, _P),
    "hub_log_det": (_P, _P, _P, _P),
    "hub_apply_M_slab": (_P, _I, _I, _P, _P, _P, _P, _P, _I, _P),
    "hub_apply_Mdag_slab": (_P, _I, _I, _P, _P, _P, _P, _I, _P),
    "hub_apply_M_slab_c64": (_P, _I, _I, _P, _P, _P, _P, _P, _I, _P),
    "hub_apply_Mdag_slab_c64": (_P, _I, _I, _P, _P, _P, _P, _I, _P),
    "hub_force_slab": (_P, _I, _I, _P, _P, _P, _P, _I, _P),
    "hub_action": (_P, _P, _P, _I, _P, _P),
    "hub_md_update": (_P, _P, _P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _P),
    "hub_boson_energy": (_P, _P, _P, ctypes.c_double, _P, _P),
    "hub_trajectory": (_P, _P, _P, _P, _I, ctypes.c_double, ctypes.POINTER(HubTrajOpts),
                       ctypes.POINTER(HubTrajInfo), _P),
    "hub_query": (_P, ctypes.POINTER(_I), ctypes.POINTER(_I)),
    "hub_set_cg_launch": (_P, _I, ctypes.c_int64),
    "hub_last_error": (),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libhubhip.so; raise if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2210_06874_amd/build.py "
                           "(or __graft_entry__.build()); there is no non-HIP fallback")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = list(args)
        fn.restype = ctypes.c_char_p if name == "hub_last_error" else (None if name == "hub_destroy" else ctypes.c_int)
    _lib = lib
    return lib


class HubError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def check(status: int) -> None:
    if status != HUB_OK:
        msg = load().hub_last_error()
        raise HubError(status, msg.decode() if msg else "")
