"""ctypes binding of libqme.so (argument marshalling only).

Every computation of the solver runs inside the library; this module only
declares the C structures and signatures of ``include/qme.h``.  Loading fails
loudly when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libqme.so")

QME_OK, QME_E_ARG, QME_E_SIZE, QME_E_DEVICE, QME_E_NUMERIC, QME_E_STATE, QME_E_UNSUPPORTED = range(7)
STATUS_NAMES = ["QME_OK", "QME_E_ARG", "QME_E_SIZE", "QME_E_DEVICE", "QME_E_NUMERIC",
                "QME_E_STATE", "QME_E_UNSUPPORTED"]
FP64, FP32, BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}


class System(ctypes.Structure):
    _fields_ = [("n_cavities", c_int32), ("atoms", POINTER(c_int32)),
                ("photon_cap", POINTER(c_int32)), ("exc_min", c_int32), ("exc_max", c_int32)]


class Hop(ctypes.Structure):
    _fields_ = [("a", c_int32), ("b", c_int32), ("mu", c_double)]


class Jump(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("cavity", c_int32), ("atom", c_int32), ("gamma", c_double)]


class GeneralJump(ctypes.Structure):
    _fields_ = [("gamma", c_double), ("n_moves", c_int64), ("source", POINTER(c_int32)),
                ("target", POINTER(c_int32)), ("coef", POINTER(c_double))]


class Params(ctypes.Structure):
    _fields_ = [("omega_c", POINTER(c_double)), ("omega_a", POINTER(c_double)),
                ("g", POINTER(c_double)), ("n_hops", c_int32), ("hops", POINTER(Hop)),
                ("n_jumps", c_int32), ("jumps", POINTER(Jump)), ("dt", c_double)]


# name -> (restype, argtypes); mirrors include/qme.h
SIGNATURES = {
    "qme_basis": (c_int32, [POINTER(System), POINTER(c_int64), POINTER(c_int32), c_int64]),
    "qme_hamiltonian_coo": (c_int32, [POINTER(System), POINTER(Params), POINTER(c_int64),
                                      POINTER(c_int32), POINTER(c_int32), POINTER(c_double),
                                      c_int64]),
    "qme_propagator_host": (c_int32, [POINTER(System), POINTER(Params), POINTER(c_double),
                                      POINTER(c_double), c_int64]),
    "qme_hamiltonian": (c_int32, [POINTER(System), POINTER(Params), c_int32, c_void_p,
                                  POINTER(c_void_p)]),
    "qme_state_layout": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int64),
                                   POINTER(c_int64), POINTER(c_size_t)]),
    "qme_workspace_size": (c_int32, [c_void_p, POINTER(c_size_t)]),
    "qme_set_state": (c_int32, [c_void_p, c_void_p, POINTER(c_double), POINTER(c_double),
                                c_double, c_void_p]),
    "qme_get_state": (c_int32, [c_void_p, c_void_p, POINTER(c_double), POINTER(c_double),
                                POINTER(c_double), c_void_p]),
    "qme_step": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
    "qme_step_noalloc": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p]),
    "qme_observe": (c_int32, [c_void_p, c_void_p, POINTER(c_double), POINTER(c_double),
                              POINTER(c_double), c_void_p]),
    "qme_observe_weighted": (c_int32, [c_void_p, c_void_p, POINTER(c_double), POINTER(c_double),
                                       c_void_p]),
    "qme_cgemm": (c_int32, [c_int32, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                            c_void_p, c_void_p, c_void_p, c_double, c_double, c_int32, c_int32,
                            c_int32, c_int32, c_int32, c_void_p]),
    "qme_adjoint": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, POINTER(c_double),
                              POINTER(c_double), POINTER(c_double), c_void_p, c_size_t, c_void_p]),
    "qme_gradient_size": (c_int32, [c_void_p, POINTER(c_int64)]),
    "qme_adjoint_workspace_size": (c_int32, [c_void_p, c_int64, c_int32, POINTER(c_size_t)]),
    "qme_batch_create": (c_int32, [POINTER(c_void_p), POINTER(c_void_p), c_int32,
                                   POINTER(c_void_p)]),
    "qme_batch_workspace_size": (c_int32, [c_void_p, POINTER(c_size_t)]),
    "qme_batch_config": (c_int32, [c_void_p, c_int32, c_int32]),
    "qme_batch_persistent": (c_int32, [c_void_p, c_int32]),
    "qme_batch_step": (c_int32, [c_void_p, c_int64, c_void_p, c_size_t, c_void_p]),
    "qme_batch_destroy": (None, [c_void_p]),
    "qme_set_tiles": (c_int32, [c_void_p, c_int32, c_int32]),
    "qme_get_tiles": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32)]),
    "qme_set_split": (c_int32, [c_void_p, c_int32]),
    "qme_set_fused": (c_int32, [c_void_p, c_int32]),
    "qme_set_fold": (c_int32, [c_void_p, c_int32]),
    "qme_set_direct_loads": (c_int32, [c_void_p, c_int32]),
    "qme_set_graph": (c_int32, [c_void_p, c_int32]),
    "qme_hamiltonian_general": (c_int32, [c_int64, c_int64, POINTER(c_int32), POINTER(c_int32),
                                          POINTER(c_double), c_int32, POINTER(GeneralJump), c_double,
                                          c_int32, c_void_p, POINTER(c_void_p)]),
    "qme_select_states": (c_int32, [c_int64, POINTER(c_double), POINTER(c_double), c_double,
                                    c_double, POINTER(c_int32), POINTER(c_int64)]),
    "qme_select_device": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_double,
                                    c_void_p, c_void_p, c_void_p]),
    "qme_select_workspace_size": (c_int32, [c_void_p, POINTER(c_size_t)]),
    "qme_select_run": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_int64, c_double,
                                 c_int32, POINTER(c_int64), POINTER(c_int64), POINTER(c_int32),
                                 c_void_p]),
    "qme_subspace": (c_int32, [c_void_p, POINTER(c_int32), c_int64, c_void_p, POINTER(c_void_p)]),
    "qme_compact_state": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "qme_profile_enable": (c_int32, [c_void_p, c_int32]),
    "qme_profile_read": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_int64)]),
    "qme_pure_layout": (c_int32, [c_void_p, c_int32, POINTER(c_size_t), POINTER(c_size_t)]),
    "qme_pure_set": (c_int32, [c_void_p, c_void_p, c_int32, POINTER(c_double), POINTER(c_double),
                               c_void_p]),
    "qme_pure_get": (c_int32, [c_void_p, c_void_p, c_int32, POINTER(c_double), POINTER(c_double),
                               c_void_p]),
    "qme_pure_step": (c_int32, [c_void_p, c_void_p, c_int32, c_int64, c_void_p, c_void_p]),
    "qme_destroy": (None, [c_void_p]),
    "qme_last_error": (c_char_p, []),
    "qme_version": (c_char_p, []),
}

_lib = None


class QmeError(RuntimeError):
    def __init__(self, status, msg):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {msg}")


def load():
    """Load libqme.so once.  Raises if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2403_07042_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status):
    if status != QME_OK:
        msg = load().qme_last_error().decode(errors="replace")
        raise QmeError(status, msg)
