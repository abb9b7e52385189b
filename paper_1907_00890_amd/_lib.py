"""ctypes view of libvofpoisson.so (the C ABI declared in include/vofpoisson.h).

Argument marshalling only: every step of the solve, projection and
extension runs in the library's HIP kernels.  There is no fallback: if the
shared library is missing or does not load, importing this module fails.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("VOFPOISSON_LIB", os.path.join(HERE, "libvofpoisson.so"))

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libvofpoisson.so not found at {LIB_PATH}; build it first "
        "(python paper_1907_00890_amd/build.py or __graft_entry__.build())")

# torch first: the library's HIP runtime dependency then resolves to the
# runtime torch has already loaded, so the process holds one HIP / HSA runtime.
# Loaded first, the library would bring in the system runtime next to torch's
# own copy, and the second of the two to initialise cannot open the device.
import torch  # noqa: E402,F401

lib = ctypes.CDLL(LIB_PATH)

_p = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double


class ExtendFields(ctypes.Structure):
    """vp_extend_fields: device pointers of one extension."""
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("u", "v", "w", "src", "qx", "qy", "qz", "ue", "ve", "we", "ug", "vg", "wg",
                 "phi")]


class LowerFaces(ctypes.Structure):
    """vp_lower_faces: device planes of the faces at -1/2 of lower outflow ends."""
    _fields_ = [(n, ctypes.c_void_p) for n in ("u", "v", "w")]


_lf = ctypes.POINTER(LowerFaces)

# name -> (restype, argtypes)
SIGNATURES = {
    "poisson_plan_create": (_p, [_i, _i, _i, _d, _d, ctypes.POINTER(_d), ctypes.c_char_p, _i, _i,
                                 ctypes.POINTER(_i)]),
    "poisson_plan_check": (_i, [_i, _i, _i, _d, _d, ctypes.POINTER(_d), ctypes.c_char_p, _i, _i]),
    "poisson_plan_destroy": (None, [_p]),
    "poisson_solve": (_i, [_p, _p, _p, _p]),
    "poisson_solve_batched": (_i, [_p, _i, ctypes.POINTER(_p), ctypes.POINTER(_p), _p]),
    "poisson_solve_noalloc": (_i, [_p, _p, _p, _p]),
    "project": (_i, [_p, _p, _p, _p, _p, _p, _d, _p, _d, _p, _p]),
    "extend_liquid_velocity": (_i, [_p] + [_p] * 14 + [_p]),
    "extend_liquid_velocity_batched": (_i, [_p, _i, ctypes.POINTER(ExtendFields), _p]),
    "vof_step": (_i, [_p, _p, _p, _p, _p, _p, _d, _p, _d, _p] + [_p] * 11 + [_p]),
    "interface_terms": (_i, [_p, _p, _p, _d, _d, _i, _p, _p, _p, _p, _p]),
    "vof_step_interface": (_i, [_p, _p, _p, _p, _p, _p, _d, _p, _p, _d, _d, _i, _d, _p, _p]
                           + [_p] * 7 + [_p]),
    "vof_advect": (_i, [_p, _p, _p, _p, _p, _lf, _d, _d, _i, _p, _p]),
    "project_lf": (_i, [_p, _p, _p, _p, _lf, _p, _p, _d, _p, _d, _p, _p]),
    "extend_liquid_velocity_lf": (_i, [_p, _p, _p, _p, _lf, _p, _p, _p, _p, _p, _p, _p, _lf,
                                       _p, _p, _p, _p, _p]),
    "vof_step_lf": (_i, [_p, _p, _p, _p, _lf, _p, _p, _d, _p, _d, _p, _p, _p, _p, _p, _p, _p, _p,
                         _lf, _p, _p, _p, _p, _p]),
    "poisson_plan_set_mixed": (_i, [_p, _i]),
    "poisson_plan_set_mixed_tol": (_i, [_p, _d]),
    "poisson_plan_mixed_report": (_i, [_p, _i, ctypes.POINTER(_i), ctypes.POINTER(_d), _p]),
    "poisson_plan_last_mean": (_i, [_p, ctypes.POINTER(_d), _p]),
    "poisson_plan_footprint": (ctypes.c_longlong, [_i, _i, _i, _i, _i]),
    "poisson_plan_device_bytes": (ctypes.c_longlong, [_p]),
    "poisson_plan_tune": (_i, [_p, ctypes.c_char_p, _i]),
    "poisson_plan_get_tuning": (_i, [_p, ctypes.c_char_p, ctypes.POINTER(_i)]),
    "poisson_plan_autotune": (_i, [_p, _i, _p, ctypes.POINTER(_i)]),
    "poisson_plan_set_profiling": (_i, [_p, _i]),
    "poisson_plan_kernel_times": (_i, [_p, ctypes.POINTER(_d), ctypes.POINTER(_i), _i]),
    "poisson_kernel_class_name": (ctypes.c_char_p, [_i]),
    "poisson_strerror": (ctypes.c_char_p, [_i]),
    "vofpoisson_version": (ctypes.c_char_p, []),
}

for _name, (_res, _args) in SIGNATURES.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

VP_OK, VP_EINVAL, VP_EUNSUPPORTED, VP_ENOMEM, VP_EHIP = 0, -1, -2, -3, -4
NUM_KERNEL_CLASSES = 19
MAX_BATCH = 16
PRECISION = {"fp64": 0, "mixed": 1}
NOALLOC_MAX_POINTS = 1 << 23


class VofPoissonError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib.poisson_strerror(status).decode(errors="replace")
        super().__init__(f"{where}: status {status} ({msg})")


def check(status: int, where: str) -> None:
    if status != VP_OK:
        raise VofPoissonError(status, where)
