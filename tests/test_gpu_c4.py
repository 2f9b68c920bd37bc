"""Mixed-precision storage at clinical size: the 10x256x256x128 enhancement
workload (patch 3^3, window 7^3, h = 0.04, mu = 0.5, 20 Gauss-Jacobi steps
with the weights refreshed from the iterate every 5 steps, then the energy
and its exact gradient) with the volumes stored in FP32, BF16 and FP16,
arithmetic in FP32.

Asserted (kernel error, the library against the oracle run on the very
values the library read): Gauss-Jacobi steps 0, 5 and 19 and the final
log-normalisers, statistics and gradient at sampled voxels, within the FP32
tolerance (max(1e-5, derived bound)), stored volumes within half a storage
ulp more; the energy equals the compensated sum of its own statistics.
Reported (end-to-end error, what 16-bit storage costs): every output of the
16-bit runs against the FP32 run at every voxel, and on a reduced grid of
the same phantom family, every run after 20 steps against 20 oracle steps on
the FP32 input.
"""
import numpy as np
import pytest
import torch

import paper_1201_2450_amd as tnlm
from oracle import oracle
from phantom import WORKLOADS, breathing_phantom, quantise, workload_inputs
from tests.gpu_util import (STORE_EPS, Bounds, assert_close, host, normwise, say, to_dev,
                            with_peaks)
from tests.test_gpu_workloads import sample_idx

pytestmark = pytest.mark.gpu

CHECK_STEPS = (0, 5, 19)


def _run(g, w, keep):
    """20 steps (weights from f every 5), keeping the outputs of the steps
    in `keep`; then log-normalisers, energy + statistics and the total
    gradient of E(f; f) at the final iterate."""
    outs = {}

    def hook(k, f):
        if k in keep:
            outs[k] = f.clone()

    f = tnlm.enhance(g, w.mu, d=w.d, M=w.M, h=w.h, iters=w.iters,
                     recompute_every=w.recompute_every, step_hook=hook)
    _, lse = tnlm.weights(f, d=w.d, M=w.M, h=w.h)
    e, st = tnlm.energy(f, d=w.d, M=w.M, h=w.h, want_stats=True)
    gt = tnlm.grad(f, d=w.d, M=w.M, h=w.h, mode="exact", stats=st, total=True)
    torch.cuda.synchronize()
    return f, outs, lse, e, st, gt


def test_c4_enh256_16bit_storage_20_steps_energy_gradient():
    w = WORKLOADS["enh256_bf16"]
    say(f"c4 {w.shape}: generating the phantom")
    g32 = workload_inputs(w, out_dtype=np.float32)[0]
    N = w.nx * w.ny * w.nz
    # steps whose outputs the kernel checks need: the step itself, the
    # iterate before it and the weight source of its block of 5
    keep = set()
    for k in CHECK_STEPS:
        keep |= {k, k - 1, 5 * (k // 5) - 1}
    keep.discard(-1)
    runs = {}
    for storage in ("f32", "bf16", "f16"):
        say(f"c4 {storage}: 20 steps + energy + gradient")
        gq64, g = to_dev(g32.astype(np.float64), storage)
        f, outs, lse, e, st, gt = _run(g, w, keep)
        it = lambda k: g if k < 0 else outs[k]
        idx = with_peaks(sample_idx(w.shape, 150, 40), f)
        for k in CHECK_STEPS:
            u_t, f_prev = it(5 * (k // 5) - 1), it(k - 1)
            u64, fp64 = host(u_t), host(f_prev)
            ref = oracle.jacobi(u64, fp64, gq64, w.mu, w.d, w.M, w.h, idx=idx)
            B = Bounds(u64, fp64, w.d, w.M, w.h, idx=idx)
            assert_close(host(outs[k]).ravel()[idx], ref, f"c4 {storage} step {k}",
                         B.jacobi(w.mu), extra=STORE_EPS[storage])
            del u64, fp64
        f64 = host(f)
        B = Bounds(f64, f64, w.d, w.M, w.h, idx=idx)
        st_ref = oracle.stats(f64, f64, w.d, w.M, w.h, idx=idx)
        assert_close(host(lse)[idx // N, :, idx % N], st_ref[:, :, 0],
                     f"c4 {storage} lse", B.lse())
        sth = st.double().cpu().numpy()
        assert_close(sth[idx // N, :, :, idx % N], st_ref, f"c4 {storage} stats", B.stats())
        E = float(e[0]) + float(e[1])
        E_sum = 0.25 * float(np.sum(sth[:, :, 1, :]))
        assert abs(E - E_sum) <= 1e-9 * abs(E_sum), (E, E_sum)
        gidx = with_peaks(idx[::5], gt)
        rf, ru = oracle.grad_exact_at(f64, f64, w.d, w.M, w.h, gidx)
        # floor only: the gradient's bound needs the whole-grid scatter model
        assert_close(host(gt).ravel()[gidx], rf + ru, f"c4 {storage} grad", None)
        runs[storage] = dict(f=f, lse=lse, E=E, gt=gt)
        del f64, sth, outs
    # end-to-end: 16-bit runs against the FP32 run, every voxel
    ref = runs["f32"]

    def rel(a, b):
        # (largest error, rms error) relative to the largest / rms reference
        d = a.double() - b.double()
        return (float(d.abs().max() / b.double().abs().max()),
                float(d.square().mean().sqrt() / b.double().square().mean().sqrt()))

    for storage in ("bf16", "f16"):
        r = runs[storage]
        errs = {}
        for k, key in (("f20", "f"), ("lse", "lse"), ("grad", "gt")):
            errs[k + "_max"], errs[k + "_rms"] = rel(r[key], ref[key])
        errs["E"] = abs(r["E"] - ref["E"]) / abs(ref["E"])
        say(f"  c4 {storage} vs FP32 run (every voxel): "
            + "  ".join(f"{k} {v:.2e}" for k, v in errs.items()))
        say("E2E|" + storage + "|" + "|".join(f"{k}={v:.3e}" for k, v in errs.items()))
        assert all(np.isfinite(v) for v in errs.values())


def test_c4_reduced_grid_20_steps_against_20_oracle_steps():
    """The c4 run on a 10x32x32x16 grid of the same phantom family and
    parameters, where 20 oracle steps finish in about a minute: every
    storage format's 20-step result against the oracle's 20 steps on the
    FP32 input (end-to-end: kernel rounding, storage rounding and the
    weights' response to both), reported per output."""
    w = WORKLOADS["enh256_bf16"]
    shape = (10, 32, 32, 16)
    g64 = quantise(breathing_phantom(*shape, lesion_r=3.0, amp=2.0, sigma=w.sigma,
                                     streaks=True, seed=w.seed)[0], "f32")[0]
    say(f"c4 reduced {shape}: 20 oracle steps")
    f = g64.copy()
    for k in range(w.iters):
        if k % w.recompute_every == 0:
            u = f.copy()
        f = oracle.jacobi(u, f, g64, w.mu, w.d, w.M, w.h)
    E_ref, st_ref = oracle.energy(f, f, w.d, w.M, w.h, want_stats=True)
    for storage in ("f32", "bf16", "f16"):
        _, g = to_dev(g64, storage)
        fd, _, lse, e, st, gt = _run(g, w, set())
        E = float(e[0]) + float(e[1])
        rms = lambda a, b: float(np.sqrt(np.mean((a - b) ** 2) / np.mean(b ** 2)))
        errs = {"f20_max": normwise(host(fd), f), "f20_rms": rms(host(fd), f),
                "lse_max": normwise(host(lse), st_ref[:, :, 0]),
                "e_max": normwise(host(st)[:, :, 1], st_ref[:, :, 1]),
                "E": abs(E - E_ref) / abs(E_ref)}
        say(f"  c4 reduced {storage} vs 20 oracle steps: "
            + "  ".join(f"{k} {v:.2e}" for k, v in errs.items()))
        say("E2E-ORACLE|" + storage + "|" + "|".join(f"{k}={v:.3e}" for k, v in errs.items()))
        assert all(np.isfinite(v) for v in errs.values())
