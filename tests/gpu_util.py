"""Helpers shared by the GPU parity tests (inputs, tolerances, comparisons)."""
import sys

import numpy as np
import torch

from oracle import oracle
from phantom import quantise, random_volumes, scaled_phantom

TORCH_DT = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}
# half a unit in the last place, relative, of each storage format
STORE_EPS = {"f32": 0.0, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}
# Tolerances. Every FP32 output is compared normwise (max |x - ref| / max
# |ref|) with the FP64 oracle on identical inputs, at
#   tol = max(FP32_TOL, max(bound) / max|ref|),
# where bound is the first-order rounding-error bound of oracle.error_model
# for that case and output (the patch distances' rounding amplified by the
# weight exponents, which reach c2*D ~ 300 on steep inputs): FP32_TOL is the
# target wherever the conditioning allows it, the derived bound where it
# does not.
FP32_TOL = 1e-5
U32 = 2.0 ** -24   # unit roundoff of FP32
LAM = 6.0          # Hoeffding factor: each bound fails with prob <= 2 e^-18
CORR = 3 * U32     # relative error of 1/(2h^2): h rounded to FP32, then the constant


def tiled(d, M):
    """Geometries the LDS-tiled kernels take (patch 3^3, window up to 11^3)."""
    return d == 1 and 1 <= M <= 5


def depth(d, M, generic=False):
    """Roundings a squared difference passes through in the kernels'
    distance sums: the tiled kernels take three separable 3-tap sums (the
    z sum with the squares fused, 3; x, 2; y, 2), the one-thread kernels a
    running sum over the (2d+1)^3 patch."""
    return 7 if tiled(d, M) and not generic else (2 * d + 1) ** 3


class Bounds:
    """Per-element FP32 error bounds of one case (oracle.error_model). With
    idx, only the per-voxel outputs at those flat indices (error_model_at)."""

    def __init__(self, u64, f64, d, M, h, grad=False, idx=None):
        self.args = (u64, f64, d, M, h)
        self.shape = u64.shape
        self.N = int(np.prod(self.shape[1:]))
        self.idx = idx
        if idx is None:
            self.m = oracle.error_model(u64, f64, d, M, h, depth(d, M), U32,
                                        LAM, CORR, grad=grad)
        else:
            self.m = oracle.error_model_at(u64, f64, d, M, h, depth(d, M),
                                           U32, LAM, CORR, idx)

    def _b(self, v, dd):
        return LAM * np.sqrt(v) + CORR * np.abs(dd)

    def _dirs(self, key):
        # [Np, 2, N] whole grid, or [n, 2] sampled
        return self.m[key + "_v"], self.m[key + "_d"]

    def lse(self):
        return self._b(*self._dirs("lse"))

    def e(self):
        return self._b(*self._dirs("e"))

    def stats(self):
        # [Np, 2, 2, N] whole grid, [n, 2, 2] sampled (as the oracle's stats)
        return np.stack([self.lse(), self.e()], axis=2)

    def _both(self, key):
        v, dd = self._dirs(key)
        b = self._b(v.sum(axis=1), dd.sum(axis=1))
        return b.reshape(self.shape) if self.idx is None else b

    def jacobi(self, mu):
        return self._both("nb") / (2.0 + mu)

    def eq6(self):
        return self._both("nb")

    def energy(self):
        return LAM * np.sqrt(self.m["e_v"].sum() / 16.0) + \
            CORR * abs(self.m["e_d"].sum() / 4.0)

    def w(self):
        """Bound of every weight of a voxel and direction, [Np, 2, 1, N]
        (the full weight tensor comes from the one-thread kernels)."""
        u64, f64, d, M, h = self.args
        m = oracle.error_model(u64, f64, d, M, h, depth(d, M, generic=True),
                               U32, LAM, CORR)
        return m["w_b"][:, :, None, :]

    def gf(self):
        return self._b(self.m["gf_v"], self.m["gf_d"])

    def gu(self):
        return self._b(self.m["gu_v"], self.m["gu_d"])

    def total(self):
        return self.gf() + self.gu()


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


def assert_close(got, ref, what, bound=None, extra=0.0, floor=FP32_TOL):
    """Normwise comparison at tol = max(floor, max(bound) / max|ref|) +
    extra (extra: storage rounding of 16-bit outputs). bound is an array of
    per-element error bounds shaped like ref (or None: the floor alone)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    e = normwise(got, ref)
    scale = np.abs(ref).max()
    b = float(np.max(bound)) / scale if bound is not None and scale > 0 else 0.0
    tol = max(floor, b) + extra
    say(f"  {what}: normwise rel err {e:.3e} (bound {b:.2e}, tol {tol:.2e})")
    say(f"TOL|{what}|{e:.3e}|{b:.3e}|{tol:.3e}")
    assert np.isfinite(got).all(), f"{what}: non-finite output"
    assert e <= tol, f"{what}: normwise rel err {e:.3e} > {tol:.2e}"


def assert_close_scalar(got, ref, what, bound=None, floor=FP32_TOL):
    e = abs(got - ref) / abs(ref)
    b = bound / abs(ref) if bound is not None else 0.0
    tol = max(floor, b)
    say(f"  {what}: rel err {e:.3e} (bound {b:.2e}, tol {tol:.2e}); gpu {got!r} oracle {ref!r}")
    say(f"TOL|{what}|{e:.3e}|{b:.3e}|{tol:.3e}")
    assert e <= tol, f"{what}: rel err {e:.3e} > {tol:.2e}"


def inputs(shape, kind, seed):
    """Seeded float64 volumes of a given flavour."""
    if kind == "phantom":
        return scaled_phantom(shape, seed)
    if kind == "uniform":
        return random_volumes(shape, seed, scale=0.3)
    if kind == "smooth":  # mild contrast: a well-conditioned case
        return 0.2 + random_volumes(shape, seed, scale=0.02)
    raise ValueError(kind)
