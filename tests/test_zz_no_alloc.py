"""tnlm_energy_noalloc (the energy with the library's fixed per-GPU scratch
instead of a caller workspace) against tnlm_energy, both called through the
C ABI with ctypes: two calls in a row, the second on a smaller input, so the
second reads scratch that the first left behind. The two entry points run
the same kernels in the same order, so energy and statistics agree bit for
bit."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1201_2450_amd import _lib
from tests.gpu_util import device, say, to_dev
from phantom import scaled_phantom

pytestmark = pytest.mark.gpu


def _energy_both(shape, d, M, h, seed):
    lib = _lib.lib
    x64 = scaled_phantom(shape, seed)
    _, f = to_dev(x64, "f32")
    g = _lib.Geom(*shape, d, M, h)
    N = shape[1] * shape[2] * shape[3]
    stream = torch.cuda.current_stream().cuda_stream
    e_ws = torch.empty(2, dtype=torch.float32, device=device())
    st_ws = torch.empty((shape[0], 2, 2, N), dtype=torch.float32, device=device())
    need = lib.tnlm_workspace_bytes(ctypes.byref(g), _lib.OP_ENERGY)
    ws = torch.empty(need, dtype=torch.uint8, device=device())
    rc = lib.tnlm_energy(ctypes.byref(g), _lib.F32, f.data_ptr(), f.data_ptr(),
                         e_ws.data_ptr(), st_ws.data_ptr(), ws.data_ptr(), need, stream)
    assert rc == 0, _lib.strerror(rc)
    # poison the outputs of the no-allocation call: every value must be rewritten
    e_na = torch.full((2,), float("nan"), dtype=torch.float32, device=device())
    st_na = torch.full_like(st_ws, float("nan"))
    rc = lib.tnlm_energy_noalloc(ctypes.byref(g), _lib.F32, f.data_ptr(), f.data_ptr(),
                                 e_na.data_ptr(), st_na.data_ptr(), stream)
    assert rc == 0, _lib.strerror(rc)
    # without statistics
    e_na2 = torch.full((2,), float("nan"), dtype=torch.float32, device=device())
    rc = lib.tnlm_energy_noalloc(ctypes.byref(g), _lib.F32, f.data_ptr(), f.data_ptr(),
                                 e_na2.data_ptr(), None, stream)
    assert rc == 0, _lib.strerror(rc)
    torch.cuda.synchronize()
    return e_ws.cpu(), st_ws.cpu(), e_na.cpu(), st_na.cpu(), e_na2.cpu()


@pytest.mark.parametrize("first,second", [
    # tiled kernels (d = 1, M <= 5): a large grid, then a smaller one
    (((4, 40, 64, 48), 1, 2, 0.05), ((3, 12, 10, 20), 1, 2, 0.05)),
    # generic kernels (d = 0), large then small
    (((3, 20, 24, 16), 0, 2, 0.05), ((2, 6, 5, 7), 0, 1, 0.05)),
])
def test_noalloc_energy_matches_workspace_energy(first, second):
    for case, (shape, d, M, h) in (("first", first), ("second", second)):
        say(f"noalloc energy {case}: shape {shape} d={d} M={M}")
        e_ws, st_ws, e_na, st_na, e_na2 = _energy_both(shape, d, M, h, 1201)
        assert torch.equal(e_ws, e_na), (e_ws, e_na)
        assert torch.equal(e_ws, e_na2), (e_ws, e_na2)
        assert torch.equal(st_ws, st_na)
        say(f"  E = {float(e_na[0]) + float(e_na[1]):.9g} (bitwise equal)")


def test_noalloc_energy_rejects_problems_beyond_its_scratch():
    lib = _lib.lib
    # 64 phases of 1024 x 1024 x 512 voxels: far more partial sums than 4 MiB
    g = _lib.Geom(64, 1024, 1024, 512, 1, 3, 0.04)
    assert lib.tnlm_workspace_bytes(ctypes.byref(g), _lib.OP_ENERGY) > (4 << 20)
    rc = lib.tnlm_energy_noalloc(ctypes.byref(g), _lib.F32, 0x10000, 0x10000,
                                 0x20000000, None, None)
    assert rc == _lib.EWORKSPACE
