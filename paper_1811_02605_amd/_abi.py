"""ctypes binding of the C ABI declared in include/mas.h (argument marshalling only).

Every function keeps the C name.  Pointers are plain integers (device
addresses from ``tensor.data_ptr()``, host addresses from ctypes/numpy);
``hip_stream`` is a hipStream_t handle as an integer (0 = null stream).
Loading fails loudly if the HIP library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libmas_hip.so")

MAS_OK = 0
MAS_ENOTCONV = 1
MAS_EINVAL = -1
MAS_EBREAKDOWN = -2
MAS_EHIP = -3
MAS_ENOMEM = -4

MAS_BC_DIRICHLET0 = 0
MAS_BC_NEUMANN0 = 1

MAS_FP64 = 0
MAS_FP32_REFINED = 1

MAS_REFINE_RESTART = 0
MAS_REFINE_RELIABLE = 1

MAS_PC1 = 0
MAS_PC2 = 1

MAS_LAUNCH_AUTO = 0
MAS_LAUNCH_PER_ITERATION = 1
MAS_LAUNCH_PERSISTENT = 2

# workspace of the allocation-free solve (a static device array in the library)
MAS_NOALLOC_WORK_BYTES = 64 * 1024 * 1024


class mas_grid(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int32), ("nt", ctypes.c_int32), ("np", ctypes.c_int32),
                ("r_faces", ctypes.POINTER(ctypes.c_double)),
                ("t_faces", ctypes.POINTER(ctypes.c_double)),
                ("bc_inner", ctypes.c_int32), ("bc_outer", ctypes.c_int32)]


class mas_pcg_opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_iters", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("inner_rtol", ctypes.c_double),
                ("max_outer", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("use_x0", ctypes.c_int32), ("max_restarts", ctypes.c_int32),
                ("sample_timing", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("chunk_planes", ctypes.c_int32),
                ("launch", ctypes.c_int32)]


class mas_pcg_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("outer_iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("rel_resid_true", ctypes.c_double), ("rel_resid_recursive", ctypes.c_double),
                ("bnorm", ctypes.c_double), ("seconds", ctypes.c_double),
                ("iter_kernel_us", ctypes.c_double), ("iter_kernel_samples", ctypes.c_int32),
                ("launch", ctypes.c_int32), ("grad_kernel_us", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class mas_sts_opts(ctypes.Structure):
    _fields_ = [("stages", ctypes.c_int32), ("sample_timing", ctypes.c_int32),
                ("single_stage_kernels", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class mas_sts_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("stages", ctypes.c_int32),
                ("z_max", ctypes.c_double), ("step_us", ctypes.c_double),
                ("stage_kernel_us", ctypes.c_double), ("stage_kernel_samples", ctypes.c_int32),
                ("stages_per_kernel", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# name -> (restype, argtypes), in the order of include/mas.h
_VP = ctypes.c_void_p
_SIGS = {
    "mas_pcg_default_opts": (None, [ctypes.POINTER(mas_pcg_opts)]),
    "mas_op_storage_bytes": (ctypes.c_int64, [ctypes.POINTER(mas_grid), ctypes.c_int32]),
    "mas_op_build": (ctypes.c_int, [ctypes.POINTER(mas_grid), _VP, ctypes.c_double, ctypes.c_int32,
                                    _VP, ctypes.c_int64, _VP, ctypes.POINTER(_VP)]),
    "mas_op_destroy": (None, [_VP]),
    "mas_op_apply": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "mas_op_export": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "mas_pcg_workspace_bytes": (ctypes.c_int64, [_VP, ctypes.POINTER(mas_pcg_opts)]),
    "mas_pcg_solve": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(mas_pcg_opts), _VP,
                                     ctypes.c_int64, _VP, ctypes.POINTER(mas_pcg_info)]),
    "mas_pcg_solve_adjoint": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP,
                                             ctypes.POINTER(mas_pcg_opts), _VP, ctypes.c_int64,
                                             _VP, ctypes.POINTER(mas_pcg_info)]),
    "mas_pcg_multi_workspace_bytes": (ctypes.c_int64, [_VP, ctypes.c_int32]),
    "mas_pcg_solve_multi": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, _VP,
                                           ctypes.POINTER(mas_pcg_opts), _VP, ctypes.c_int64, _VP,
                                           ctypes.POINTER(mas_pcg_info)]),
    "mas_sts_default_opts": (None, [ctypes.POINTER(mas_sts_opts)]),
    "mas_sts_stages": (ctypes.c_int32, [_VP]),
    "mas_sts_workspace_bytes": (ctypes.c_int64, [_VP]),
    "mas_sts_step": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(mas_sts_opts), _VP,
                                    ctypes.c_int64, _VP, ctypes.POINTER(mas_sts_info)]),
    "mas_pcg_solve_noalloc": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(mas_pcg_opts), _VP,
                                             ctypes.POINTER(mas_pcg_info)]),
    "mas_probe_copy": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, _VP]),
    "mas_probe_stream_bytes": (ctypes.c_int64, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]),
    "mas_probe_stream": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.c_int32, _VP]),
    "mas_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "mas_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library not built: {LIB_PATH} is missing "
                "(run `python -m paper_1811_02605_amd.build`)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_names():
    return list(_SIGS)


def last_error() -> str:
    return load().mas_last_error().decode()


def status_string(status: int) -> str:
    return load().mas_status_string(int(status)).decode()


def default_opts() -> mas_pcg_opts:
    o = mas_pcg_opts()
    load().mas_pcg_default_opts(ctypes.byref(o))
    return o


class MasError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_string(status)}: {last_error()}")


def check(status: int, where: str, allow_notconv: bool = False) -> int:
    if status == MAS_OK or (allow_notconv and status == MAS_ENOTCONV):
        return status
    raise MasError(status, where)
