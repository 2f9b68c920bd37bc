"""FP64 oracle of the reconstruction model's data-fidelity part: the
cone-beam projector P and its transpose (ct_oracle.c), CGLS for the (P1)
sub-problem of Eq. (5), and the TNLM-R algorithm (Sec. 2.3).

TEST INFRASTRUCTURE ONLY: imported by the tests and the smoke check, never
by the product library. Volumes are float64 (Np, Nx, Ny, Nz), projections
float64 (Np, Na, Nu, Nv), angles (Np, Na) radians; the geometry is the one
described at the top of ct_oracle.c.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ct_oracle.c")
_LIB = os.path.join(_HERE, "libct_oracle.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=c99", "-O3", "-fopenmp", "-fPIC",
                               "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


@dataclasses.dataclass(frozen=True)
class CTGeom:
    """Circular cone-beam geometry (lengths in voxel units)."""
    np_: int
    nx: int
    ny: int
    nz: int
    nu: int
    nv: int
    na: int
    sid: float
    sdd: float
    du: float
    dv: float

    @property
    def vol_shape(self):
        return (self.np_, self.nx, self.ny, self.nz)

    @property
    def proj_shape(self):
        return (self.np_, self.na, self.nu, self.nv)


class _G(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("np", "nx", "ny", "nz", "nu", "nv", "na")] + \
               [(k, ctypes.c_double) for k in ("sid", "sdd", "du", "dv")]


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        g = ctypes.POINTER(_G)
        lib.ctor_project.argtypes = [g, dp, dp, dp, dp, dp]
        lib.ctor_backproject.argtypes = [g, dp, dp, dp, dp, dp]
        lib.ctor_error_model.argtypes = [g, dp, dp, dp, dp, dp]
        i64 = ctypes.c_int64
        lib.ctor_pair_error.argtypes = [g, ctypes.c_double, i64, i64, i64, i64, i64,
                                        ctypes.POINTER(ctypes.c_double)]
        lib.ctor_pair_error.restype = ctypes.c_double
        lib.ctor_box_chord.argtypes = [g, ctypes.c_double, ctypes.c_int64,
                                       ctypes.c_int64, dp, dp]
        lib.ctor_box_chord.restype = ctypes.c_double
        _lib = lib
    return _lib


def _g(geo: CTGeom):
    return _G(geo.np_, geo.nx, geo.ny, geo.nz, geo.nu, geo.nv, geo.na,
              float(geo.sid), float(geo.sdd), float(geo.du), float(geo.dv))


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def project(geo: CTGeom, angles, vol, want_stats=False):
    """P vol (per phase); with want_stats also, per ray, the number of voxels
    it crosses and the sum of |vol| over them."""
    angles, vol = _c(angles), _c(vol)
    assert angles.shape == (geo.np_, geo.na) and vol.shape == geo.vol_shape
    out = np.empty(geo.proj_shape)
    cnt = np.empty(geo.proj_shape) if want_stats else None
    sab = np.empty(geo.proj_shape) if want_stats else None
    _L().ctor_project(ctypes.byref(_g(geo)), _dp(angles), _dp(vol), _dp(out),
                      _dp(cnt), _dp(sab))
    return (out, cnt, sab) if want_stats else out


def backproject(geo: CTGeom, angles, proj, want_stats=False):
    """P^T proj (per phase); with want_stats also, per voxel, the number of
    rays through it and the sum of |proj| over them."""
    angles, proj = _c(angles), _c(proj)
    assert angles.shape == (geo.np_, geo.na) and proj.shape == geo.proj_shape
    out = np.empty(geo.vol_shape)
    cnt = np.empty(geo.vol_shape) if want_stats else None
    sab = np.empty(geo.vol_shape) if want_stats else None
    _L().ctor_backproject(ctypes.byref(_g(geo)), _dp(angles), _dp(proj),
                          _dp(out), _dp(cnt), _dp(sab))
    return (out, cnt, sab) if want_stats else out


def error_model(geo: CTGeom, angles, xabs=None, yabs=None):
    """First-order rounding-error bounds of an FP32 evaluation of P and P^T
    (see ct_oracle.c): per ray for P applied to a volume of magnitudes xabs,
    per voxel for P^T applied to projections of magnitudes yabs. Returns
    (eproj or None, evol or None)."""
    angles = _c(angles)
    assert angles.shape == (geo.np_, geo.na)
    xa = _c(xabs) if xabs is not None else None
    ya = _c(yabs) if yabs is not None else None
    ep = np.empty(geo.proj_shape) if xa is not None else None
    ev = np.empty(geo.vol_shape) if ya is not None else None
    _L().ctor_error_model(ctypes.byref(_g(geo)), _dp(angles), _dp(xa), _dp(ya), _dp(ep), _dp(ev))
    return ep, ev


def pair_error(geo: CTGeom, theta, iu, iv, voxel):
    """(exact length of ray (theta, iu, iv) in voxel (ix, iy, iz), its FP32
    error bound under error_model's model)."""
    ln = ctypes.c_double()
    b = _L().ctor_pair_error(ctypes.byref(_g(geo)), float(theta), int(iu), int(iv),
                             *[int(k) for k in voxel], ctypes.byref(ln))
    return ln.value, b


def box_chord(geo: CTGeom, theta, iu, iv, lo, hi):
    """Length of a ray inside the box [lo, hi] (voxel units, isocentre at
    the origin)."""
    lo, hi = _c(lo), _c(hi)
    return _L().ctor_box_chord(ctypes.byref(_g(geo)), float(theta), int(iu),
                               int(iv), _dp(lo), _dp(hi))


# ---------------------------------------------------------------------------
# CGLS for (P1) of Eq. (5): min_g sum_i ||P_i g_i - y_i||^2, each phase its
# own least-squares problem (the phases are uncoupled in (P1), Sec. 2.3),
# started from a given volume. Conjugate gradients on the normal equations
# in the least-squares form (CGLS): r = y - P x, s = P^T r, p = s,
# gamma = ||s||^2; per iteration q = P p, alpha = gamma / ||q||^2,
# x += alpha p, r -= alpha q, s = P^T r, gamma' = ||s||^2,
# p = s + (gamma'/gamma) p. Dot products and scalars are per phase.
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class CGLSState:
    x: np.ndarray       # (Np, Nx, Ny, Nz)
    r: np.ndarray       # (Np, Na, Nu, Nv)
    p: np.ndarray       # (Np, Nx, Ny, Nz)
    gamma: np.ndarray   # (Np,)


def _pdot(a, b):
    """Per-phase dot products of two (Np, ...) arrays."""
    return np.sum((a * b).reshape(a.shape[0], -1), axis=1)


def cgls_init(geo, angles, y, x0):
    x = _c(x0).copy()
    r = _c(y) - project(geo, angles, x)
    s = backproject(geo, angles, r)
    return CGLSState(x=x, r=r, p=s.copy(), gamma=_pdot(s, s))


def cgls_step(geo, angles, st: CGLSState) -> CGLSState:
    q = project(geo, angles, st.p)
    qq = _pdot(q, q)
    bshape = (-1,) + (1,) * 3
    alpha = np.where(qq > 0, st.gamma / np.where(qq > 0, qq, 1.0), 0.0)
    x = st.x + alpha.reshape(bshape) * st.p
    r = st.r - alpha.reshape(bshape) * q
    s = backproject(geo, angles, r)
    g2 = _pdot(s, s)
    beta = np.where(st.gamma > 0, g2 / np.where(st.gamma > 0, st.gamma, 1.0), 0.0)
    p = s + beta.reshape(bshape) * st.p
    return CGLSState(x=x, r=r, p=p, gamma=g2)


def cgls(geo, angles, y, x0, iters):
    st = cgls_init(geo, angles, y, x0)
    for _ in range(iters):
        st = cgls_step(geo, angles, st)
    return st.x


def tnlm_r(geo, angles, y, f0, mu, d, M, h, outer, cg_iters):
    """The TNLM-R algorithm (Sec. 2.3): for k = 1..outer, (P1) by cg_iters
    CGLS iterations from f^(k-1) -> g^(k); one Gauss-Jacobi step of Eq. (8)
    with the weights and the fidelity target from g^(k), started from
    g^(k); positivity: negative voxels set to zero. Returns f^(outer)."""
    from oracle import oracle as O
    f = _c(f0)
    for _ in range(outer):
        gk = cgls(geo, angles, y, f, cg_iters)
        f = np.maximum(O.jacobi(gk, gk, gk, mu, d, M, h), 0.0)
    return f
