"""ctypes shim over the FP64 C oracle (tnlm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the product library. Every function
takes float64 numpy arrays of shape (Np, Nx, Ny, Nz) (z fastest) and returns
float64 results; see tnlm_oracle.c for the definitions and the readings of
the paper they follow.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tnlm_oracle.c")
_LIB = os.path.join(_HERE, "libtnlm_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O3, OpenMP, baseline x86-64)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=c99", "-O3", "-fopenmp", "-fPIC",
                               "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [("np", ctypes.c_int64), ("nx", ctypes.c_int64),
                ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("d", ctypes.c_int64), ("M", ctypes.c_int64),
                ("h", ctypes.c_double)]


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        ip = P(ctypes.c_int64)
        g = P(_Geom)
        lib.tnlmo_weights.argtypes = [g, dp, dp, dp]
        lib.tnlmo_jacobi.argtypes = [g, dp, dp, dp, ctypes.c_double, ip,
                                     ctypes.c_int64, dp]
        lib.tnlmo_grad_eq6.argtypes = [g, dp, dp, ip, ctypes.c_int64, dp]
        lib.tnlmo_stats.argtypes = [g, dp, dp, ip, ctypes.c_int64, dp]
        lib.tnlmo_energy.argtypes = [g, dp, dp, dp]
        lib.tnlmo_energy.restype = ctypes.c_double
        lib.tnlmo_grad_exact_scatter.argtypes = [g, dp, dp, dp, dp]
        lib.tnlmo_grad_exact_at.argtypes = [g, dp, dp, ip, ctypes.c_int64, dp,
                                            dp]
        lib.tnlmo_local_energy.argtypes = [g, dp, dp, ctypes.c_int64,
                                           ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_int64]
        lib.tnlmo_local_energy.restype = ctypes.c_double
        lib.tnlmo_error_model.argtypes = [g, dp, dp] + [ctypes.c_double] * 4 \
            + [dp] * 11
        lib.tnlmo_error_model_at.argtypes = [g, dp, dp] \
            + [ctypes.c_double] * 4 + [ip, ctypes.c_int64] + [dp] * 7
        _lib = lib
    return _lib


def _geom(shape, d, M, h):
    np_, nx, ny, nz = shape
    if np_ < 2:
        raise ValueError("Np >= 2 required")
    return _Geom(np_, nx, ny, nz, d, M, float(h))


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    if a is None:
        return None
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _vol(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _idx(idx):
    return None if idx is None else np.ascontiguousarray(idx, dtype=np.int64)


def n_offsets(M):
    return (2 * M + 1) ** 3


def weights(u, d, M, h, want_w=True):
    """(w, lse): w [Np, 2, W, Nx*Ny*Nz] (or None), lse [Np, 2, Nx*Ny*Nz]."""
    u = _vol(u)
    g = _geom(u.shape, d, M, h)
    N = int(np.prod(u.shape[1:]))
    lse = np.empty((u.shape[0], 2, N))
    w = np.empty((u.shape[0], 2, n_offsets(M), N)) if want_w else None
    _L().tnlmo_weights(ctypes.byref(g), _dp(u), _dp(w), _dp(lse))
    return w, lse


def jacobi(u, f, gin, mu, d, M, h, idx=None):
    """Eq. (8) step; full volume, or the values at flat indices idx."""
    u, f, gin = _vol(u), _vol(f), _vol(gin)
    g = _geom(u.shape, d, M, h)
    idx = _idx(idx)
    out = np.empty(u.shape if idx is None else idx.shape[0])
    _L().tnlmo_jacobi(ctypes.byref(g), _dp(u), _dp(f), _dp(gin), float(mu),
                      _ip(idx), 0 if idx is None else idx.shape[0], _dp(out))
    return out


def grad_eq6(u, f, d, M, h, idx=None):
    u, f = _vol(u), _vol(f)
    g = _geom(u.shape, d, M, h)
    idx = _idx(idx)
    out = np.empty(u.shape if idx is None else idx.shape[0])
    _L().tnlmo_grad_eq6(ctypes.byref(g), _dp(u), _dp(f), _ip(idx),
                        0 if idx is None else idx.shape[0], _dp(out))
    return out


def stats(u, f, d, M, h, idx=None):
    """Full: [Np, 2, 2, N] (lse, e); at idx: [n, 2, 2]."""
    u, f = _vol(u), _vol(f)
    g = _geom(u.shape, d, M, h)
    idx = _idx(idx)
    N = int(np.prod(u.shape[1:]))
    out = (np.empty((u.shape[0], 2, 2, N)) if idx is None
           else np.empty((idx.shape[0], 2, 2)))
    _L().tnlmo_stats(ctypes.byref(g), _dp(u), _dp(f), _ip(idx),
                     0 if idx is None else idx.shape[0], _dp(out))
    return out


def energy(u, f, d, M, h, want_stats=False):
    u, f = _vol(u), _vol(f)
    g = _geom(u.shape, d, M, h)
    N = int(np.prod(u.shape[1:]))
    st = np.empty((u.shape[0], 2, 2, N)) if want_stats else None
    E = _L().tnlmo_energy(ctypes.byref(g), _dp(u), _dp(f), _dp(st))
    return (E, st) if want_stats else E


def grad_exact_scatter(u, f, d, M, h):
    """(dE/df, dE/du), full volumes; single-threaded, small grids only."""
    u, f = _vol(u), _vol(f)
    g = _geom(u.shape, d, M, h)
    gf = np.empty(u.shape)
    gu = np.empty(u.shape)
    _L().tnlmo_grad_exact_scatter(ctypes.byref(g), _dp(u), _dp(f), _dp(gf),
                                  _dp(gu))
    return gf, gu


def grad_exact_at(u, f, d, M, h, idx):
    """(dE/df, dE/du) at flat indices idx (gather form)."""
    u, f = _vol(u), _vol(f)
    g = _geom(u.shape, d, M, h)
    idx = _idx(idx)
    gf = np.empty(idx.shape[0])
    gu = np.empty(idx.shape[0])
    _L().tnlmo_grad_exact_at(ctypes.byref(g), _dp(u), _dp(f), _ip(idx),
                             idx.shape[0], _dp(gf), _dp(gu))
    return gf, gu


def local_energy(u, f, d, M, h, k, x, y, z):
    u, f = _vol(u), _vol(f)
    g = _geom(u.shape, d, M, h)
    return _L().tnlmo_local_energy(ctypes.byref(g), _dp(u), _dp(f), k, x, y, z)



def error_model(u, f, d, M, h, depth, ulp, lam, corr, grad=False):
    """First-order rounding-error model of an FP32 evaluation whose distance
    sums pass every term through at most `depth` roundings of unit roundoff
    `ulp` (see tnlm_oracle.c): for each output the variance proxy V of the independent
    roundings and the coefficient sum D of the correlated one, so that the
    error is at most lam*sqrt(V) + corr*|D| (corr = bound of the relative
    error of 1/(2h^2)). Returns a dict of float64 arrays: lse_v, lse_d,
    nb_v, nb_d, e_v, e_d ([Np, 2, N]), w_b ([Np, 2, N], already combined) and,
    with grad=True, gf_v, gf_d, gu_v, gu_d ([Np, Nx, Ny, Nz]; a
    single-threaded scatter, small grids only)."""
    u, f = _vol(u), _vol(f)
    g = _geom(u.shape, d, M, h)
    N = int(np.prod(u.shape[1:]))
    keys = ("lse_v", "lse_d", "w_b", "nb_v", "nb_d", "e_v", "e_d")
    out = {k: np.empty((u.shape[0], 2, N)) for k in keys}
    gkeys = ("gf_v", "gf_d", "gu_v", "gu_d")
    if grad:
        out.update({k: np.empty(u.shape) for k in gkeys})
    _L().tnlmo_error_model(ctypes.byref(g), _dp(u), _dp(f), float(depth),
                           float(ulp), float(lam), float(corr),
                           *[_dp(out[k]) for k in keys],
                           *[_dp(out.get(k)) for k in gkeys])
    return out


def error_model_at(u, f, d, M, h, depth, ulp, lam, corr, idx):
    """The per-voxel outputs of error_model at flat indices idx: lse_v,
    lse_d, w_b, nb_v, nb_d, e_v, e_d, each [len(idx), 2]."""
    u, f = _vol(u), _vol(f)
    g = _geom(u.shape, d, M, h)
    idx = _idx(idx)
    keys = ("lse_v", "lse_d", "w_b", "nb_v", "nb_d", "e_v", "e_d")
    out = {k: np.empty((idx.shape[0], 2)) for k in keys}
    _L().tnlmo_error_model_at(ctypes.byref(g), _dp(u), _dp(f), float(depth),
                              float(ulp), float(lam), float(corr), _ip(idx),
                              idx.shape[0], *[_dp(out[k]) for k in keys])
    return out
