"""Tensor-level entry points over the C ABI (include/tnlm.h).

Volumes are torch tensors of shape (Np, Nx, Ny, Nz), contiguous, on a ROCm
device, in float32, bfloat16 or float16 (the storage dtype). Every call runs
on the current torch stream of the tensors' device; nothing is computed in
Python.

Names follow the paper: u is the weight source of Eq. (9), f the current
images, g the input images of Eq. (4), mu the fidelity weight, h the
similarity scale of Eq. (3), d the patch radius and M the search radius of
Sec. 2.4.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import check

_DT = {torch.float32: _lib.F32, torch.bfloat16: _lib.BF16,
       torch.float16: _lib.F16}


def _geom(t: torch.Tensor, d: int, M: int, h: float) -> _lib.Geom:
    if t.dim() != 4:
        raise ValueError("volumes are (Np, Nx, Ny, Nz) tensors")
    np_, nx, ny, nz = t.shape
    return _lib.Geom(int(np_), int(nx), int(ny), int(nz), int(d), int(M),
                     float(h))


def _vol(t: torch.Tensor, ref: torch.Tensor | None = None) -> int:
    if not t.is_cuda:
        raise ValueError("tnlm operates on GPU tensors only (no CPU path)")
    if not t.is_contiguous():
        raise ValueError("volumes must be contiguous (z fastest)")
    if t.dtype not in _DT:
        raise TypeError(f"unsupported storage dtype {t.dtype}")
    if ref is not None and (t.shape != ref.shape or t.dtype != ref.dtype
                            or t.device != ref.device):
        raise ValueError("volumes must share shape, dtype and device")
    return t.data_ptr()


def _f32(t: torch.Tensor | None, shape=None, device=None) -> int | None:
    if t is None:
        return None
    if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError("float32 contiguous GPU tensor expected")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"float32 tensor of shape {tuple(shape)} expected, "
                         f"got {tuple(t.shape)}")
    if device is not None and t.device != device:
        raise ValueError("tensor on another device")
    return t.data_ptr()


def _stats_shape(f: torch.Tensor):
    """Shape of the per-voxel statistics of volumes shaped like f."""
    return (f.shape[0], 2, 2, f.shape[1] * f.shape[2] * f.shape[3])


def _ws_bytes(ws: torch.Tensor, f: torch.Tensor) -> int:
    if not ws.is_cuda or ws.device != f.device or not ws.is_contiguous():
        raise ValueError("workspace must be a contiguous tensor on the "
                         "volumes' device")
    return ws.numel() * ws.element_size()


def _stream(t: torch.Tensor) -> int:
    return torch.cuda.current_stream(t.device).cuda_stream


def n_offsets(M: int) -> int:
    return (2 * M + 1) ** 3


def workspace_bytes(shape, d, M, h, op) -> int:
    g = _lib.Geom(*[int(s) for s in shape], int(d), int(M), float(h))
    n = _lib.lib.tnlm_workspace_bytes(ctypes.byref(g), int(op))
    if n == ctypes.c_size_t(-1).value:
        # the library's answer for a geometry it rejects (or an unknown op)
        raise _lib.TNLMError(_lib.EINVAL, "tnlm_workspace_bytes")
    return n


def _workspace(t: torch.Tensor, nbytes: int) -> torch.Tensor:
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=t.device)


def weights(u, *, d, M, h, want_w=False, want_lse=True):
    """Weights of Eq. (3) from u: (w [Np,2,W,N] or None, lse [Np,2,N] or
    None), float32."""
    g = _geom(u, d, M, h)
    _vol(u)
    N = u.shape[1] * u.shape[2] * u.shape[3]
    w = (torch.empty((u.shape[0], 2, n_offsets(M), N), dtype=torch.float32,
                     device=u.device) if want_w else None)
    lse = (torch.empty((u.shape[0], 2, N), dtype=torch.float32,
                       device=u.device) if want_lse else None)
    check(_lib.lib.tnlm_weights(ctypes.byref(g), _DT[u.dtype], u.data_ptr(),
                                _f32(w), _f32(lse), _stream(u)),
          "tnlm_weights")
    return w, lse


def jacobi_step(u, f, g, mu, *, d, M, h, out=None):
    """One Gauss-Jacobi step of Eq. (8) with weights from u; returns f_out
    (same dtype as f)."""
    geo = _geom(f, d, M, h)
    _vol(f)
    _vol(u, f)
    _vol(g, f)
    if out is None:
        out = torch.empty_like(f)
    _vol(out, f)
    check(_lib.lib.tnlm_jacobi_step(ctypes.byref(geo), _DT[f.dtype],
                                    u.data_ptr(), f.data_ptr(), g.data_ptr(),
                                    float(mu), out.data_ptr(), _stream(f)),
          "tnlm_jacobi_step")
    return out


def energy(f, *, d, M, h, u=None, want_stats=False, ws=None):
    """TNLM energy E(f; u) (u defaults to f).

    Returns (e, stats): e is a float32[2] device tensor with E = e[0] + e[1];
    stats is [Np,2,2,N] float32 (log-normaliser, e) or None."""
    if u is None:
        u = f
    geo = _geom(f, d, M, h)
    _vol(f)
    _vol(u, f)
    N = f.shape[1] * f.shape[2] * f.shape[3]
    e = torch.empty(2, dtype=torch.float32, device=f.device)
    stats = (torch.empty((f.shape[0], 2, 2, N), dtype=torch.float32,
                         device=f.device) if want_stats else None)
    need = workspace_bytes(f.shape, d, M, h, _lib.OP_ENERGY)
    if ws is None:
        ws = _workspace(f, need)
    check(_lib.lib.tnlm_energy(ctypes.byref(geo), _DT[f.dtype], u.data_ptr(),
                               f.data_ptr(), e.data_ptr(), _f32(stats),
                               ws.data_ptr(), _ws_bytes(ws, f), _stream(f)),
          "tnlm_energy")
    return e, stats


def energy_noalloc(f, *, d, M, h, u=None, e=None, stats=None):
    """TNLM energy through tnlm_energy_noalloc: no workspace; the library's
    fixed per-GPU scratch holds the partial sums. e (float32[2]) and stats
    ([Np,2,2,N] float32 or None) are written in place when given; returns
    (e, stats)."""
    if u is None:
        u = f
    geo = _geom(f, d, M, h)
    _vol(f)
    _vol(u, f)
    if e is None:
        e = torch.empty(2, dtype=torch.float32, device=f.device)
    _f32(e, (2,), f.device)
    _f32(stats, _stats_shape(f), f.device)
    check(_lib.lib.tnlm_energy_noalloc(ctypes.byref(geo), _DT[f.dtype],
                                       u.data_ptr(), f.data_ptr(),
                                       e.data_ptr(), _f32(stats), _stream(f)),
          "tnlm_energy_noalloc")
    return e, stats


def grad(f, *, d, M, h, u=None, mode="exact", stats=None, want_f=True,
         want_u=True, total=False):
    """Gradient of the TNLM term.

    mode='eq6': returns 2 f - sum w f_{i+-1} (TNLM part of Eq. (6), weights
    frozen from u).
    mode='exact': returns (dE/df, dE/du) of E(f; u); with total=True (needs
    u is f) returns dE/df + dE/du as one tensor."""
    if u is None:
        u = f
    geo = _geom(f, d, M, h)
    _vol(f)
    _vol(u, f)
    mk = lambda: torch.empty(f.shape, dtype=torch.float32, device=f.device)
    if mode == "eq6":
        out = mk()
        check(_lib.lib.tnlm_grad(ctypes.byref(geo), _DT[f.dtype],
                                 u.data_ptr(), f.data_ptr(), _lib.GRAD_EQ6,
                                 None, out.data_ptr(), None, None, 0,
                                 _stream(f)), "tnlm_grad(eq6)")
        return out
    if mode != "exact":
        raise ValueError(mode)
    # the C ABI cannot see the statistics' extent: check it here
    _f32(stats, _stats_shape(f), f.device)
    need = workspace_bytes(f.shape, d, M, h, _lib.OP_GRAD_EXACT)
    if stats is None:
        need += 16 * f.numel()
    ws = _workspace(f, need)
    if total:
        if u.data_ptr() != f.data_ptr():
            raise ValueError("total gradient needs u is f")
        gt = mk()
        check(_lib.lib.tnlm_grad(ctypes.byref(geo), _DT[f.dtype],
                                 u.data_ptr(), f.data_ptr(), _lib.GRAD_EXACT,
                                 _f32(stats), gt.data_ptr(), gt.data_ptr(),
                                 ws.data_ptr(), _ws_bytes(ws, f), _stream(f)),
              "tnlm_grad(exact, total)")
        return gt
    gf = mk() if want_f else None
    gu = mk() if want_u else None
    check(_lib.lib.tnlm_grad(ctypes.byref(geo), _DT[f.dtype], u.data_ptr(),
                             f.data_ptr(), _lib.GRAD_EXACT, _f32(stats),
                             _f32(gf), _f32(gu), ws.data_ptr(),
                             _ws_bytes(ws, f), _stream(f)), "tnlm_grad(exact)")
    return gf, gu
