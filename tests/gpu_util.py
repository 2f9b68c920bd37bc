"""Helpers shared by the GPU parity tests (inputs, tolerances, comparisons)."""
import sys

import numpy as np
import torch

from phantom import quantise, random_volumes, scaled_phantom

TORCH_DT = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}
# half a unit in the last place, relative, of each storage format
STORE_EPS = {"f32": 0.0, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}
FP32_TOL = 1e-5  # normwise relative tolerance of FP32 outputs vs the oracle
# Stress inputs (uniform noise with h far below the data range) push the
# weight exponent c2*D = D*log2(e)/(2h^2) to ~300 for the candidates that
# matter; FP32 rounding of the 27-term distance D (about sqrt(27)*2^-24
# relative) then moves each exponent by ~1e-5, so weights and everything
# built from them carry ~1e-5..1e-4 relative error before any kernel error.
STRESS_TOL = 1e-4


def tol_for(kind):
    return STRESS_TOL if kind == "uniform" else FP32_TOL


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def device():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda", 0)


def to_dev(x64, storage="f32"):
    """(float64 values the oracle sees, device tensor in storage dtype)."""
    q, raw = quantise(x64, storage)
    if storage == "bf16":
        t = torch.from_numpy(raw.view(np.int16).copy()).view(torch.bfloat16)
    else:
        t = torch.from_numpy(np.ascontiguousarray(raw))
    return q, t.to(device())


def host(t):
    return t.float().cpu().numpy().astype(np.float64)


def normwise(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max()
    return err / scale if scale > 0 else err


def with_peaks(idx, *fields):
    """Sampled checks normalise by the largest reference value among the
    samples; adding each output field's largest-magnitude voxel (from the
    device result, then checked against the oracle like every other sample)
    makes that scale the field's own, as in the full-volume comparisons.
    Without it a few dozen random voxels can miss the field's peaks by 10x
    and turn 1e-6 errors into 1e-5."""
    def peak(f):
        if isinstance(f, torch.Tensor):
            return int(torch.argmax(f.detach().reshape(-1).float().abs()).item())
        return int(np.argmax(np.abs(np.asarray(f)).ravel()))
    extra = {peak(f) for f in fields}
    return np.array(sorted(set(int(i) for i in idx) | extra), dtype=np.int64)


def assert_close(got, ref, tol, what):
    e = normwise(got, ref)
    say(f"  {what}: normwise rel err {e:.3e} (tol {tol:.1e})")
    assert np.isfinite(np.asarray(got)).all(), f"{what}: non-finite output"
    assert e <= tol, f"{what}: normwise rel err {e:.3e} > {tol:.1e}"


def assert_close_faces(got, ref, idx, shape, what):
    """The weight part of the exact gradient, dE/du, at flat indices idx:
    FP32_TOL inside the grid and 2 FP32_TOL on its faces, where the
    derivatives of the clamped copies of a face voxel are added (chain rule
    through clamp-to-edge: large terms of both signs). Both relative to the
    largest reference value among the samples."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    pos = np.unravel_index(np.asarray(idx), shape)
    face = np.zeros(len(idx), dtype=bool)
    for ax in (1, 2, 3):
        face |= (pos[ax] == 0) | (pos[ax] == shape[ax] - 1)
    scale = np.abs(ref).max()
    err = np.abs(got - ref)
    e_in = err[~face].max() / scale if (~face).any() else 0.0
    e_face = err[face].max() / scale if face.any() else 0.0
    say(f"  {what}: inside {e_in:.3e} (tol {FP32_TOL:.1e}), faces {e_face:.3e} "
        f"(tol {2 * FP32_TOL:.1e})")
    assert np.isfinite(got).all(), f"{what}: non-finite output"
    assert e_in <= FP32_TOL and e_face <= 2 * FP32_TOL, (what, e_in, e_face)


def inputs(shape, kind, seed):
    """Seeded float64 volumes of a given flavour."""
    if kind == "phantom":
        return scaled_phantom(shape, seed)
    if kind == "uniform":
        return random_volumes(shape, seed, scale=0.3)
    if kind == "smooth":  # mild contrast: a well-conditioned case
        return 0.2 + random_volumes(shape, seed, scale=0.02)
    raise ValueError(kind)
