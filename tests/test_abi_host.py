"""Host-side checks of the C ABI: the library loads, exports every function
include/tnlm.h declares, and rejects bad arguments before launching anything.

Every call here fails validation, so no kernel is launched and no device is
touched: the pointers are never dereferenced on the host.
"""
import ctypes

import pytest

from paper_1201_2450_amd import _lib
from paper_1201_2450_amd._lib import Geom, lib

FAKE = 0x10000          # never dereferenced: validation fails first
FAKE2 = 0x20000000
FAKE3 = 0x40000000


def geom(np_=3, nx=8, ny=8, nz=8, d=1, M=2, h=0.05):
    return Geom(np_, nx, ny, nz, d, M, h)


def test_every_declared_function_is_exported():
    names = _lib.header_functions()
    assert set(names) >= {"tnlm_weights", "tnlm_jacobi_step", "tnlm_energy",
                          "tnlm_grad", "tnlm_workspace_bytes",
                          "tnlm_strerror", "tnlm_version"}
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_strerror():
    assert lib.tnlm_version().startswith(b"tnlm")
    for code in (0, -1, -2, -3, -4, -5, -6, -99):
        assert isinstance(lib.tnlm_strerror(code), bytes)


@pytest.mark.parametrize("g", [
    geom(np_=1), geom(np_=0), geom(nx=0), geom(nz=-3), geom(d=-1), geom(M=-1),
    geom(d=9), geom(M=17), geom(h=0.0), geom(h=-1.0), geom(h=float("nan")),
    geom(h=float("inf")), geom(h=1e-30),
])
def test_bad_geometry_is_einval(g):
    rc = lib.tnlm_jacobi_step(ctypes.byref(g), 0, FAKE, FAKE, FAKE, 1.0,
                              FAKE2, None)
    assert rc == _lib.EINVAL
    assert lib.tnlm_workspace_bytes(ctypes.byref(g), _lib.OP_ENERGY) == \
        ctypes.c_size_t(-1).value


def test_null_geometry():
    assert lib.tnlm_jacobi_step(None, 0, FAKE, FAKE, FAKE, 1.0, FAKE2,
                                None) == _lib.ENULL


def test_size_overflow_is_erange():
    g = geom(nx=2048, ny=2048, nz=1024)  # 2^32 voxels per phase
    assert lib.tnlm_jacobi_step(ctypes.byref(g), 0, FAKE, FAKE, FAKE, 1.0,
                                FAKE2, None) == _lib.ERANGE


def test_total_voxel_count_overflow_is_erange():
    g = geom(np_=2048, nx=1024, ny=1024, nz=1024)  # 2^41 voxels in all
    assert lib.tnlm_weights(ctypes.byref(g), 0, FAKE, FAKE2, None,
                            None) == _lib.ERANGE


def test_jacobi_argument_checks():
    g = geom()
    call = lambda dt=0, u=FAKE, f=FAKE, gg=FAKE, mu=1.0, out=FAKE2: \
        lib.tnlm_jacobi_step(ctypes.byref(g), dt, u, f, gg, mu, out, None)
    assert call(dt=3) == _lib.EINVAL
    assert call(dt=-1) == _lib.EINVAL
    assert call(mu=0.0) == _lib.EINVAL
    assert call(mu=-1.0) == _lib.EINVAL
    assert call(mu=float("nan")) == _lib.EINVAL
    assert call(u=None) == _lib.ENULL
    assert call(f=None) == _lib.ENULL
    assert call(gg=None) == _lib.ENULL
    assert call(out=None) == _lib.ENULL
    # output overlapping an input: same pointer, or a partial overlap
    assert call(out=FAKE) == _lib.EALIAS
    assert call(out=FAKE + 64) == _lib.EALIAS
    assert call(f=FAKE3, out=FAKE3 - 16) == _lib.EALIAS


def test_weights_argument_checks():
    g = geom()
    assert lib.tnlm_weights(ctypes.byref(g), 0, FAKE, None, None, None) == \
        _lib.ENULL
    assert lib.tnlm_weights(ctypes.byref(g), 0, None, FAKE2, None, None) == \
        _lib.ENULL
    assert lib.tnlm_weights(ctypes.byref(g), 5, FAKE, FAKE2, None, None) == \
        _lib.EINVAL
    assert lib.tnlm_weights(ctypes.byref(g), 0, FAKE, FAKE, None, None) == \
        _lib.EALIAS
    assert lib.tnlm_weights(ctypes.byref(g), 0, FAKE, FAKE2, FAKE2 + 4,
                            None) == _lib.EALIAS


def test_energy_argument_checks():
    g = geom()
    need = lib.tnlm_workspace_bytes(ctypes.byref(g), _lib.OP_ENERGY)
    assert need > 0
    e = lambda u=FAKE, f=FAKE, eo=FAKE2, st=None, ws=FAKE3, n=need: \
        lib.tnlm_energy(ctypes.byref(g), 0, u, f, eo, st, ws, n, None)
    assert e(eo=None) == _lib.ENULL
    assert e(u=None) == _lib.ENULL
    assert e(ws=None) == _lib.EWORKSPACE
    assert e(n=need - 1) == _lib.EWORKSPACE
    assert e(eo=FAKE) == _lib.EALIAS
    assert e(ws=FAKE2) == _lib.EALIAS


def test_grad_argument_checks():
    g = geom()
    need = lib.tnlm_workspace_bytes(ctypes.byref(g), _lib.OP_GRAD_EXACT)
    stats_bytes = 16 * 3 * 512
    G = lambda u=FAKE, f=FAKE, mode=1, st=None, gf=FAKE2, gu=None, ws=FAKE3, \
        n=need + stats_bytes: lib.tnlm_grad(ctypes.byref(g), 0, u, f, mode,
                                            st, gf, gu, ws, n, None)
    assert G(mode=2) == _lib.EINVAL
    assert G(mode=0, gu=FAKE2 + 1 << 20) == _lib.EINVAL   # grad_u with EQ6
    assert G(gf=None, gu=None) == _lib.ENULL
    assert G(f=None) == _lib.ENULL
    # total gradient (grad_u == grad_f) needs u == f
    assert G(u=FAKE, f=FAKE + 4096 * 16, gu=FAKE2) == _lib.EINVAL
    # recomputing the statistics needs the larger workspace
    assert G(n=need) == _lib.EWORKSPACE
    assert G(ws=None) == _lib.EWORKSPACE
    assert G(gf=FAKE) == _lib.EALIAS
    assert G(ws=FAKE2) == _lib.EALIAS
    assert G(gf=FAKE2, gu=FAKE2 + 8) == _lib.EALIAS


def test_workspace_sizes():
    g = geom()
    assert lib.tnlm_workspace_bytes(ctypes.byref(g), _lib.OP_JACOBI) == 0
    assert lib.tnlm_workspace_bytes(ctypes.byref(g), _lib.OP_WEIGHTS) == 0
    assert lib.tnlm_workspace_bytes(ctypes.byref(g), _lib.OP_GRAD_EQ6) == 0
    assert lib.tnlm_workspace_bytes(ctypes.byref(g), 99) == \
        ctypes.c_size_t(-1).value
    a = lib.tnlm_workspace_bytes(ctypes.byref(g), _lib.OP_ENERGY)
    assert a % 256 == 0 and a >= 8


def test_package_has_no_cpu_path():
    import torch

    import paper_1201_2450_amd as tnlm
    x = torch.zeros((2, 4, 4, 4))
    with pytest.raises(ValueError, match="GPU"):
        tnlm.jacobi_step(x, x, x, 1.0, d=1, M=1, h=0.1)


def test_binding_raises_library_error_for_rejected_geometry():
    """The binding reports a geometry the library rejects (empty grid, one
    phase) as the library's status, before any device call."""
    from paper_1201_2450_amd import ops
    for shape in ((2, 0, 4, 4), (1, 4, 4, 4)):
        with pytest.raises(_lib.TNLMError) as ei:
            ops.workspace_bytes(shape, 1, 1, 0.1, _lib.OP_ENERGY)
        assert ei.value.code == _lib.EINVAL


def test_energy_noalloc_argument_checks():
    g = geom()
    call = lambda gg=g, dt=0, u=FAKE, f=FAKE, e=FAKE2: \
        lib.tnlm_energy_noalloc(ctypes.byref(gg), dt, u, f, e, None, None)
    assert call(dt=5) == _lib.EINVAL
    assert call(u=None) == _lib.ENULL
    assert call(e=None) == _lib.ENULL
    assert call(e=FAKE) == _lib.EALIAS
    # a problem whose partial sums exceed the fixed 4 MiB scratch
    big = geom(np_=64, nx=1024, ny=1024, nz=512, M=3)
    assert lib.tnlm_workspace_bytes(ctypes.byref(big), _lib.OP_ENERGY) > (4 << 20)
    assert call(gg=big) == _lib.EWORKSPACE


def _ctg(**kw):
    d = dict(np=2, nx=8, ny=8, nz=8, nu=16, nv=12, na=4, sid=40.0, sdd=64.0, du=1.0,
             dv=1.0, angles=FAKE3)
    d.update(kw)
    return _lib.CTGeom(d["np"], d["nx"], d["ny"], d["nz"], d["nu"], d["nv"], d["na"],
                       d["sid"], d["sdd"], d["du"], d["dv"], d["angles"])


@pytest.mark.parametrize("kw", [dict(np=0), dict(nx=0), dict(nu=0), dict(na=0),
                                dict(sid=0.0), dict(du=-1.0), dict(dv=float("nan")),
                                dict(sid=4.0),           # source inside the volume
                                dict(sdd=42.0)])         # detector inside the volume
def test_ct_bad_geometry_is_einval(kw):
    g = _ctg(**kw)
    assert lib.tnlm_ct_project(ctypes.byref(g), FAKE, FAKE2, None) == _lib.EINVAL
    assert lib.tnlm_ct_workspace_bytes(ctypes.byref(g)) == ctypes.c_size_t(-1).value


def test_ct_argument_checks():
    g = _ctg()
    assert lib.tnlm_ct_project(None, FAKE, FAKE2, None) == _lib.ENULL
    assert lib.tnlm_ct_project(ctypes.byref(g), None, FAKE2, None) == _lib.ENULL
    assert lib.tnlm_ct_project(ctypes.byref(g), FAKE, FAKE, None) == _lib.EALIAS
    assert lib.tnlm_ct_backproject(ctypes.byref(g), FAKE, FAKE, None) == _lib.EALIAS
    assert lib.tnlm_ct_project(ctypes.byref(_ctg(angles=None)), FAKE, FAKE2, None) == _lib.ENULL
    big = _ctg(np=64, nx=1024, ny=1024, nz=1024, sid=2000.0, sdd=4000.0)
    assert lib.tnlm_ct_project(ctypes.byref(big), FAKE, FAKE2, None) == _lib.ERANGE
    need = lib.tnlm_ct_workspace_bytes(ctypes.byref(g))
    assert need > 0
    assert lib.tnlm_cgls_init(ctypes.byref(g), FAKE, FAKE2, None, need, None) == _lib.EWORKSPACE
    assert lib.tnlm_cgls_init(ctypes.byref(g), FAKE, FAKE2, 0x60000000, need - 1,
                              None) == _lib.EWORKSPACE
    assert lib.tnlm_cgls_step(ctypes.byref(g), FAKE2, -1, 0x60000000, need, None) == _lib.EINVAL
    assert lib.tnlm_cgls_step(ctypes.byref(g), FAKE2, 0, 0x60000000, need, None) == _lib.OK
    assert lib.tnlm_clamp_nonneg(None, 5, None) == _lib.ENULL
    assert lib.tnlm_clamp_nonneg(FAKE, -1, None) == _lib.EINVAL
    assert lib.tnlm_clamp_nonneg(None, 0, None) == _lib.OK
