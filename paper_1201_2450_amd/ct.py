"""Reconstruction model over the C ABI: the cone-beam projector P of every
phase and its transpose (Eq. (1)), CGLS for the (P1) sub-problem of Eq. (5)
and the TNLM-R algorithm (Sec. 2.3). Argument marshalling only: every step
runs in the library's kernels on the current torch stream.

Volumes are float32 (Np, Nx, Ny, Nz) and projections float32 (Np, Na, Nu, Nv)
GPU tensors; angles a float32 (Np, Na) GPU tensor in radians. Geometry in
voxel units, as described in include/tnlm.h.
"""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _lib, ops
from ._lib import check


@dataclasses.dataclass(frozen=True)
class Geometry:
    """Circular cone-beam geometry: detector nu x nv pixels of pitch du x dv,
    na angles per phase, source-isocentre distance sid and source-detector
    distance sdd (voxel units)."""
    nu: int
    nv: int
    sid: float
    sdd: float
    du: float
    dv: float


def _g(geo: Geometry, vol_shape, angles: torch.Tensor, device) -> _lib.CTGeom:
    if angles.dtype != torch.float32 or not angles.is_cuda or not angles.is_contiguous():
        raise ValueError("angles: contiguous float32 GPU tensor (Np, Na)")
    if angles.device != device:
        raise ValueError("angles on a different device")
    np_, nx, ny, nz = vol_shape
    if angles.dim() != 2 or angles.shape[0] != np_:
        raise ValueError("angles must be (Np, Na)")
    return _lib.CTGeom(int(np_), int(nx), int(ny), int(nz), int(geo.nu), int(geo.nv),
                       int(angles.shape[1]), float(geo.sid), float(geo.sdd),
                       float(geo.du), float(geo.dv), angles.data_ptr())


def _f32(t, shape, device):
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("contiguous float32 GPU tensor expected")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"shape {tuple(shape)} expected, got {tuple(t.shape)}")
    if t.device != device:
        raise ValueError("tensors on different devices")
    return t.data_ptr()


def proj_shape(geo: Geometry, vol_shape, na):
    return (vol_shape[0], na, geo.nu, geo.nv)


def _stream(t):
    return torch.cuda.current_stream(t.device).cuda_stream


def project(vol, geo: Geometry, angles, out=None):
    """P vol for every phase: (Np, Na, Nu, Nv) float32."""
    g = _g(geo, vol.shape, angles, vol.device)
    shp = proj_shape(geo, vol.shape, angles.shape[1])
    if out is None:
        out = torch.empty(shp, dtype=torch.float32, device=vol.device)
    check(_lib.lib.tnlm_ct_project(ctypes.byref(g), _f32(vol, vol.shape, vol.device),
                                   _f32(out, shp, vol.device), _stream(vol)), "tnlm_ct_project")
    return out


def backproject(proj, geo: Geometry, angles, vol_shape, out=None):
    """P^T proj for every phase: (Np, Nx, Ny, Nz) float32."""
    g = _g(geo, vol_shape, angles, proj.device)
    if out is None:
        out = torch.empty(vol_shape, dtype=torch.float32, device=proj.device)
    check(_lib.lib.tnlm_ct_backproject(
        ctypes.byref(g), _f32(proj, proj_shape(geo, vol_shape, angles.shape[1]), proj.device),
        _f32(out, vol_shape, proj.device), _stream(proj)), "tnlm_ct_backproject")
    return out


class CGLS:
    """CGLS for min sum_i ||P_i x_i - y_i||^2 ((P1) of Eq. (5)), state in a
    device workspace: CGLS(y, x, geo, angles) starts from x (updated in
    place by step()). Views of the state (r, p, gamma) follow the workspace
    layout of include/tnlm.h."""

    def __init__(self, y, x, geo: Geometry, angles):
        self.g = _g(geo, x.shape, angles, x.device)
        self.x, self.geo, self.angles = x, geo, angles
        n = _lib.lib.tnlm_ct_workspace_bytes(ctypes.byref(self.g))
        if n == ctypes.c_size_t(-1).value:
            raise _lib.TNLMError(_lib.EINVAL, "tnlm_ct_workspace_bytes")
        self.ws = torch.empty(n, dtype=torch.uint8, device=x.device)
        pshape = proj_shape(geo, x.shape, angles.shape[1])
        check(_lib.lib.tnlm_cgls_init(ctypes.byref(self.g), _f32(y, pshape, x.device),
                                      _f32(x, x.shape, x.device), self.ws.data_ptr(), n,
                                      _stream(x)), "tnlm_cgls_init")

    def step(self, iters=1):
        check(_lib.lib.tnlm_cgls_step(ctypes.byref(self.g), self.x.data_ptr(), int(iters),
                                      self.ws.data_ptr(), self.ws.numel(), _stream(self.x)),
              "tnlm_cgls_step")
        return self.x

    def state(self):
        """(r, p, gamma): views of the workspace for r and p; gamma a float64
        copy (hi + lo) of its current value."""
        np_ = self.x.shape[0]
        R = self.angles.shape[1] * self.geo.nu * self.geo.nv
        N = self.x[0].numel()
        f = self.ws.view(torch.float32)
        r = f[:np_ * R].view(np_, self.angles.shape[1], self.geo.nu, self.geo.nv)
        p = f[2 * np_ * R:2 * np_ * R + np_ * N].view(self.x.shape)
        base = 2 * np_ * R + 2 * np_ * N
        gam = f[base:base + 2 * np_].view(np_, 2).double().sum(dim=1)
        return r, p, gam


def clamp_nonneg(x):
    """x = max(x, 0) in place (positivity step of TNLM-R)."""
    if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
        raise ValueError("contiguous float32 GPU tensor expected")
    check(_lib.lib.tnlm_clamp_nonneg(x.data_ptr(), x.numel(), _stream(x)), "tnlm_clamp_nonneg")
    return x


def reconstruct(y, geo: Geometry, angles, f0, *, mu, d, M, h, outer, cg_iters,
                step_hook=None):
    """The TNLM-R algorithm (Sec. 2.3): f = f0; for k = 1..outer:
    g = (P1) by cg_iters CGLS iterations from f; f = one Gauss-Jacobi step of
    Eq. (8) with the weights and the fidelity target from g, started from g;
    f = max(f, 0). Returns f (float32)."""
    f = f0.clone()
    for k in range(outer):
        gk = f.clone()
        CGLS(y, gk, geo, angles).step(cg_iters)
        f = ops.jacobi_step(gk, gk, gk, mu, d=d, M=M, h=h)
        clamp_nonneg(f)
        if step_hook is not None:
            step_hook(k, gk, f)
    return f
