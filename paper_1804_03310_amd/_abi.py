"""ctypes declarations of the C ABI in include/afqmc.h (marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libafqmc.so")

c_int32 = ctypes.c_int32
c_int = ctypes.c_int
c_void_p = ctypes.c_void_p
c_double = ctypes.c_double
c_size_t = ctypes.c_size_t
c_uint64 = ctypes.c_uint64

AFQMC_OK = 0
STATUS_NAMES = {0: "AFQMC_OK", -1: "AFQMC_ERR_ARG", -2: "AFQMC_ERR_OOM", -3: "AFQMC_ERR_DEVICE",
                -4: "AFQMC_ERR_STATE", -5: "AFQMC_ERR_SINGULAR", -6: "AFQMC_ERR_NONFINITE",
                -7: "AFQMC_ERR_UNSUPPORTED"}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3}
MAX_EXC = 4
QROUTE_FP32_MAX_K = 4096  # AFQMC_QROUTE_FP32_MAX_K
NOALLOC_SCRATCH_BYTES = 32 << 20  # AFQMC_NOALLOC_SCRATCH_BYTES

# Every symbol include/afqmc.h declares.
EXPORTED = ["afqmc_init_hamiltonian", "afqmc_init_trial", "afqmc_walker_workspace_bytes",
            "afqmc_walkers_from_trial", "afqmc_propagate", "afqmc_local_energy",
            "afqmc_orthonormalize", "afqmc_reconfigure", "afqmc_fields",
            "afqmc_timing_enable", "afqmc_timing_read", "afqmc_footprint_bytes",
            "afqmc_trial_exchange_route", "afqmc_trial_set_exchange_route",
            "afqmc_reblock", "afqmc_cs_difference", "afqmc_reconfigure_noalloc",
            "afqmc_resident_supported", "afqmc_group_create", "afqmc_group_propagate",
            "afqmc_group_tune", "afqmc_group_config", "afqmc_group_set_config",
            "afqmc_free_group", "afqmc_tune_cache_path", "afqmc_group_timing",
            "afqmc_group_timing_read",
            "afqmc_free_hamiltonian", "afqmc_free_trial", "afqmc_last_error"]
KERNEL_CLASSES = ["exchange", "propagator_build", "taylor_b1", "overlap_theta", "mgs", "comb",
                  "other", "force_bias"]


class WalkersStruct(ctypes.Structure):
    _fields_ = [("n_walkers", c_int32), ("system_id", c_int32),
                ("phi_re", c_void_p), ("phi_im", c_void_p), ("weight", c_void_p),
                ("logovlp_re", c_void_p), ("logovlp_im", c_void_p),
                ("eloc_re", c_void_p), ("eloc_im", c_void_p),
                ("workspace", c_void_p), ("workspace_bytes", c_size_t)]


class OptionsStruct(ctypes.Structure):
    _fields_ = [("taylor_order", c_int32), ("ortho_every", c_int32), ("pc_every", c_int32),
                ("e_trial", c_double), ("chol_prec", c_int), ("taylor_prec", c_int),
                ("weight_mode", c_int32), ("meas_every", c_int32)]


WEIGHT_MODES = {"local": 0, "hybrid": 1}


class GroupMemberStruct(ctypes.Structure):
    _fields_ = [("ham", c_void_p), ("trial", c_void_p), ("walkers", ctypes.POINTER(WalkersStruct)),
                ("dt", c_double), ("seed", c_uint64), ("opt", OptionsStruct)]


class AfqmcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libafqmc.so, building it first (hipcc, gfx950) when it is missing
    or was built from other sources.  There is no fallback: if the library
    cannot be built or loaded this raises ImportError."""
    global _lib
    if _lib is not None:
        return _lib
    if path == LIB_PATH:
        from . import build as _build
        try:
            _build.ensure_built()
        except Exception as e:  # no hipcc, compile error
            raise ImportError(f"HIP library {path} could not be built: {e}") from e
    if not os.path.exists(path):
        raise ImportError(f"HIP library {path} is missing")
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7).
    # Loaded first, it is the one the dynamic linker hands this library, so
    # the library's kernels and torch's allocations and streams live in one
    # runtime.  Loaded the other way round, the process holds two runtimes and
    # the library's sees no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = c_void_p
    sig = {
        "afqmc_init_hamiltonian": (c_int, [ctypes.POINTER(P), c_int, P, c_int, c_int, P, P, c_double]),
        "afqmc_init_trial": (c_int, [ctypes.POINTER(P), P, c_int, c_int, P, P, c_int, P, P, c_int]),
        "afqmc_walker_workspace_bytes": (c_int, [P, c_int, ctypes.POINTER(c_size_t)]),
        "afqmc_walkers_from_trial": (c_int, [P, P, ctypes.POINTER(WalkersStruct), P]),
        "afqmc_propagate": (c_int, [P, P, ctypes.POINTER(WalkersStruct), c_int, c_double, c_uint64,
                                    c_uint64, ctypes.POINTER(OptionsStruct), P, P]),
        "afqmc_local_energy": (c_int, [P, P, ctypes.POINTER(WalkersStruct), P, P]),
        "afqmc_orthonormalize": (c_int, [P, P, ctypes.POINTER(WalkersStruct), P]),
        "afqmc_reconfigure": (c_int, [P, ctypes.POINTER(WalkersStruct), c_uint64, c_uint64, P, P]),
        "afqmc_reconfigure_noalloc": (c_int, [P, ctypes.POINTER(WalkersStruct), c_uint64, c_uint64,
                                              P, P]),
        "afqmc_fields": (c_int, [c_uint64, c_uint64, c_int, c_int, c_int, P, P]),
        "afqmc_timing_enable": (c_int, [P, c_int]),
        "afqmc_footprint_bytes": (c_int, [c_int, c_int, c_int, c_int, c_int, c_int,
                                          ctypes.POINTER(c_size_t)]),
        "afqmc_trial_exchange_route": (c_int, [P, ctypes.POINTER(c_int)]),
        "afqmc_trial_set_exchange_route": (c_int, [P, c_int]),
        "afqmc_reblock": (c_int, [P, c_int, c_int, P, P, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
        "afqmc_cs_difference": (c_int, [P, P, c_int, c_int, c_int, P, P]),
        "afqmc_timing_read": (c_int, [P, c_int, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(c_double)]),
        "afqmc_resident_supported": (c_int, [P, ctypes.POINTER(c_int)]),
        "afqmc_group_create": (c_int, [ctypes.POINTER(P), c_int, ctypes.POINTER(GroupMemberStruct), P]),
        "afqmc_group_propagate": (c_int, [P, c_int, c_uint64, ctypes.POINTER(P), P]),
        "afqmc_group_tune": (c_int, [P, c_int, ctypes.POINTER(c_double), P]),
        "afqmc_group_config": (c_int, [P, ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                                       ctypes.POINTER(c_int)]),
        "afqmc_group_set_config": (c_int, [P, c_int, c_int]),
        "afqmc_free_group": (None, [P]),
        "afqmc_group_timing": (c_int, [P, c_int]),
        "afqmc_group_timing_read": (c_int, [P, ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(c_double)]),
        "afqmc_tune_cache_path": (c_int, [ctypes.c_char_p]),
        "afqmc_free_hamiltonian": (None, [P]),
        "afqmc_free_trial": (None, [P]),
        "afqmc_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != AFQMC_OK:
        msg = load().afqmc_last_error()
        raise AfqmcError(status, msg.decode() if msg else "")
