"""ctypes loader for libtnlm.so (the HIP library built from csrc/).

Argument marshalling only. The library is loaded on first use of `lib`
(so that the build script can be imported from a checkout that has no
built library yet); if it has not been built, that first use raises
ImportError: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtnlm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "tnlm.h")

# values of the enums in include/tnlm.h
F32, BF16, F16 = 0, 1, 2
GRAD_EQ6, GRAD_EXACT = 0, 1
OP_WEIGHTS, OP_JACOBI, OP_ENERGY, OP_GRAD_EQ6, OP_GRAD_EXACT = 0, 1, 2, 3, 4
OK, EINVAL, ENULL, EALIAS, ERANGE, EWORKSPACE, EHIP = 0, -1, -2, -3, -4, -5, -6


class Geom(ctypes.Structure):
    """struct tnlm_geom."""
    _fields_ = [("np", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("patch_r", ctypes.c_int32), ("search_r", ctypes.c_int32),
                ("h", ctypes.c_float)]


class CTGeom(ctypes.Structure):
    """struct tnlm_ct_geom."""
    _fields_ = [("np", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("nu", ctypes.c_int32), ("nv", ctypes.c_int32),
                ("na", ctypes.c_int32), ("sid", ctypes.c_float),
                ("sdd", ctypes.c_float), ("du", ctypes.c_float),
                ("dv", ctypes.c_float), ("angles", ctypes.c_void_p)]


class TNLMError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: tnlm status {code} "
                         f"({strerror(code)})")


def _load():
    # PyTorch first: its ROCm runtime is the one libtnlm.so must bind to
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libtnlm.so not found at {LIB_PATH}: build it first with "
            "`python -m paper_1201_2450_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, fp = ctypes.c_void_p, ctypes.c_void_p
    gp = ctypes.POINTER(Geom)
    i, sz = ctypes.c_int, ctypes.c_size_t
    lib.tnlm_weights.argtypes = [gp, i, vp, fp, fp, vp]
    lib.tnlm_jacobi_step.argtypes = [gp, i, vp, vp, vp, ctypes.c_float, vp,
                                     vp]
    lib.tnlm_energy.argtypes = [gp, i, vp, vp, fp, fp, vp, sz, vp]
    lib.tnlm_energy_noalloc.argtypes = [gp, i, vp, vp, fp, fp, vp]
    lib.tnlm_grad.argtypes = [gp, i, vp, vp, i, fp, fp, fp, vp, sz, vp]
    cp = ctypes.POINTER(CTGeom)
    lib.tnlm_ct_project.argtypes = [cp, fp, fp, vp]
    lib.tnlm_ct_backproject.argtypes = [cp, fp, fp, vp]
    lib.tnlm_ct_workspace_bytes.argtypes = [cp]
    lib.tnlm_ct_workspace_bytes.restype = sz
    lib.tnlm_cgls_init.argtypes = [cp, fp, fp, vp, sz, vp]
    lib.tnlm_cgls_step.argtypes = [cp, fp, i, vp, sz, vp]
    lib.tnlm_clamp_nonneg.argtypes = [fp, ctypes.c_int64, vp]
    lib.tnlm_workspace_bytes.argtypes = [gp, i]
    lib.tnlm_workspace_bytes.restype = sz
    lib.tnlm_strerror.argtypes = [i]
    lib.tnlm_strerror.restype = ctypes.c_char_p
    lib.tnlm_version.argtypes = []
    lib.tnlm_version.restype = ctypes.c_char_p
    for name in ("tnlm_weights", "tnlm_jacobi_step", "tnlm_energy",
                 "tnlm_energy_noalloc", "tnlm_grad", "tnlm_ct_project",
                 "tnlm_ct_backproject", "tnlm_cgls_init", "tnlm_cgls_step",
                 "tnlm_clamp_nonneg"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


_handle = None


def get():
    """The loaded libtnlm.so (loaded on the first call)."""
    global _handle
    if _handle is None:
        _handle = _load()
    return _handle


def __getattr__(name):
    # module attribute `lib`: the library, loaded on first access
    if name == "lib":
        return get()
    raise AttributeError(f"module {__name__!r} has no attribute {name!r}")


def strerror(code: int) -> str:
    return get().tnlm_strerror(int(code)).decode()


def check(code: int, what: str):
    if code != OK:
        raise TNLMError(code, what)


def header_functions():
    """Names of the functions include/tnlm.h declares."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tnlm_[a-z_0-9]+)\s*\(", text)))
