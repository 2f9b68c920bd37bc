"""Storage precision (BF16 / FP16 volumes, FP32 arithmetic) and the remaining
workloads: the small enhancement run end to end, the large FP16 regulariser
gradient, and the descent driver.

Two errors are reported for 16-bit storage:
  * kernel error: the library against the oracle run on the dequantised
    inputs (what the kernel itself adds): FP32 outputs within the FP32
    tolerance, stored volumes within half a storage ulp more;
  * end-to-end error: against the oracle on the FP32 inputs (what storing the
    volumes in 16 bits costs); reported, not asserted: it depends on how
    strongly the weights react to the rounded inputs.
"""
import numpy as np
import pytest
import torch

import paper_1201_2450_amd as tnlm
from oracle import oracle
from phantom import WORKLOADS, quantise, workload_inputs
from tests.gpu_util import (FP32_TOL, STORE_EPS, U32, Bounds, assert_close,
                            assert_close_scalar, device, host, inputs, normwise, say,
                            to_dev, with_peaks)
from tests.test_gpu_workloads import sample_idx

pytestmark = pytest.mark.gpu


def test_enh32_five_steps_full_volume():
    """Small enhancement workload: weights from the input g for all five
    Gauss-Jacobi steps, whole-volume comparison after every step. Each step
    is checked against the oracle's step from the GPU's previous iterate (the
    one-step bound); the five-step result against five oracle steps, where
    the one-step errors add up at most as sum_k L^k tau_k: with the weights
    frozen, Eq. (8) is a contraction of modulus L = 2/(2+mu) in the maximum
    norm (every output is mu/(2+mu) g plus 1/(2+mu) times two convex
    combinations of f)."""
    w = WORKLOADS["enh32"]
    say(f"enh32 {w.shape}")
    g64, g = to_dev(workload_inputs(w)[0])
    steps = []
    out = tnlm.enhance(g, w.mu, d=w.d, M=w.M, h=w.h, iters=w.iters,
                       weights_from="g", step_hook=lambda k, f: steps.append(f.clone()))
    torch.cuda.synchronize()
    assert torch.equal(out, steps[-1])
    prev = [g] + steps[:-1]
    taus = []
    for k in range(w.iters):
        f64 = host(prev[k])
        ref = oracle.jacobi(g64, f64, g64, w.mu, w.d, w.M, w.h)
        b = Bounds(g64, f64, w.d, w.M, w.h).jacobi(w.mu)
        assert_close(host(steps[k]), ref, f"enh32 step {k}", b)
        taus.append(max(FP32_TOL * np.abs(ref).max(), float(b.max())))
    f = g64.copy()
    for _ in range(w.iters):
        f = oracle.jacobi(g64, f, g64, w.mu, w.d, w.M, w.h)
    L = 2.0 / (2.0 + w.mu)
    acc = sum(L ** (w.iters - 1 - k) * t for k, t in enumerate(taus))
    err = np.abs(host(out) - f).max()
    say(f"  five steps: max abs err {err:.3e}, accumulated bound {acc:.3e}")
    assert err <= acc
    # the full weight tensor of this workload (164 MB) at sampled voxels
    wt, lse = tnlm.weights(g, d=w.d, M=w.M, h=w.h, want_w=True)
    torch.cuda.synchronize()
    N = w.nx * w.ny * w.nz
    idx = sample_idx(w.shape, 200, 8)
    wr, lr = oracle.weights(g64, w.d, w.M, w.h)
    i, v = idx // N, idx % N
    B = Bounds(g64, g64, w.d, w.M, w.h)
    assert_close(host(wt)[i, :, :, v], wr[i, :, :, v], "w (sampled)", B.w()[i, :, :, v])
    assert_close(host(lse), lr, "lse", B.lse())


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_storage_error_tables(storage):
    """enh256-like parameters (patch 3^3, window 7^3, h = 0.04, mu = 0.5) on
    a 6x40x40x24 phantom: every output in 16-bit storage against the oracle
    (kernel and end-to-end errors)."""
    shape, d, M, h, mu = (6, 40, 40, 24), 1, 3, 0.04, 0.5
    say(f"storage {storage} {shape}")
    x64 = inputs(shape, "phantom", 31)
    xq64, xq = to_dev(x64, storage)
    x32_64 = quantise(x64, "f32")[0]
    idx = sample_idx(shape, 300, 9)
    N = int(np.prod(shape[1:]))
    rows = []
    # one Gauss-Jacobi step (u = f = g)
    out = tnlm.jacobi_step(xq, xq, xq, mu, d=d, M=M, h=h)
    _, lse = tnlm.weights(xq, d=d, M=M, h=h)
    e, st = tnlm.energy(xq, d=d, M=M, h=h, want_stats=True)
    gt = tnlm.grad(xq, d=d, M=M, h=h, mode="exact", stats=st, total=True)
    torch.cuda.synchronize()
    gidx = with_peaks(idx[:40], gt)
    idx = with_peaks(idx, out)
    got = {"jacobi": host(out).ravel()[idx],
           "lse": host(lse)[idx // N, :, idx % N],
           "grad": host(gt).ravel()[gidx]}
    E = float(e[0]) + float(e[1])
    for name, src in (("kernel", xq64), ("end-to-end", x32_64)):
        ref = {"jacobi": oracle.jacobi(src, src, src, mu, d, M, h, idx=idx),
               "lse": oracle.stats(src, src, d, M, h, idx=idx)[:, :, 0]}
        rf, ru = oracle.grad_exact_at(src, src, d, M, h, gidx)
        ref["grad"] = rf + ru
        Er = oracle.energy(src, src, d, M, h)
        errs = {k: normwise(got[k], ref[k]) for k in got}
        errs["energy"] = abs(E - Er) / abs(Er)
        rows.append((name, errs))
        say(f"  {storage} {name:10s} " + "  ".join(f"{k} {v:.2e}"
                                                  for k, v in errs.items()))
    # kernel error: the derived bounds of the dequantised case; the sampled
    # gradient takes the floor (its bound needs the whole-grid scatter model)
    B = Bounds(xq64, xq64, d, M, h, idx=idx)
    tol = lambda bnd, ref: max(FP32_TOL, float(np.max(bnd)) / np.abs(ref).max())
    kref = oracle.jacobi(xq64, xq64, xq64, mu, d, M, h, idx=idx)
    kern = rows[0][1]
    assert kern["jacobi"] <= tol(B.jacobi(mu), kref) + STORE_EPS[storage]
    lref = oracle.stats(xq64, xq64, d, M, h, idx=idx)[:, :, 0]
    assert kern["lse"] <= tol(B.lse(), lref), kern["lse"]
    assert kern["grad"] <= FP32_TOL, kern["grad"]
    Bw = Bounds(xq64, xq64, d, M, h)
    assert kern["energy"] <= max(FP32_TOL, Bw.energy() / abs(oracle.energy(xq64, xq64, d, M, h)))


def test_fbs512_fp16_gradient_sampled():
    """Large regulariser workload, FP16 storage: the exact gradient of
    E(f; f) at sampled voxels against the oracle on the dequantised volume,
    then one descent step f <- f - 0.1 grad checked at those voxels."""
    w = WORKLOADS["fbs512"]
    say(f"fbs512 {w.shape} (FP16)")
    f16 = workload_inputs(w, out_dtype=np.float16)[0]
    f = torch.from_numpy(f16).to(device())
    gt = tnlm.grad(f, d=w.d, M=w.M, h=w.h, mode="exact", total=True)
    torch.cuda.synchronize()
    idx = with_peaks(sample_idx(w.shape, 8, 10), gt)
    f64 = f16.astype(np.float64)
    rf, ru = oracle.grad_exact_at(f64, f64, w.d, w.M, w.h, idx)
    g32 = gt.cpu().numpy().ravel()[idx]
    # floor only: the gradient's bound needs the whole-grid scatter model
    assert_close(g32, rf + ru, "dE/df total (sampled)", None)
    step = tnlm.descend(f, d=w.d, M=w.M, h=w.h, tau=0.1, iters=1)
    torch.cuda.synchronize()
    # the update is float32 arithmetic rounded to FP16, as in the driver
    want = (f16.ravel()[idx].astype(np.float32)
            - np.float32(0.1) * g32).astype(np.float16)
    got = step.cpu().numpy().ravel()[idx]
    assert np.array_equal(got.view(np.uint16), want.view(np.uint16))


def test_descent_driver_matches_oracle_steps():
    """Three descent steps f <- f - tau dE(f; f)/df. The driver's result is
    bitwise three one-step calls; each step matches the oracle's step from
    the GPU's previous iterate within tau times the gradient's bound plus the
    FP32 rounding of the update (u (|f| + tau |grad|) per voxel)."""
    shape, d, M, h, tau = (3, 8, 9, 10), 1, 2, 0.08, 0.05
    say(f"descent {shape}")
    f64, f = to_dev(inputs(shape, "phantom", 32))
    out = tnlm.descend(f, d=d, M=M, h=h, tau=tau, iters=3)
    x = f
    for k in range(3):
        x64 = host(x)
        nxt = tnlm.descend(x, d=d, M=M, h=h, tau=tau, iters=1)
        torch.cuda.synchronize()
        a, b = oracle.grad_exact_scatter(x64, x64, d, M, h)
        ref = x64 - tau * (a + b)
        bound = tau * Bounds(x64, x64, d, M, h, grad=True).total() + \
            U32 * (np.abs(x64) + tau * np.abs(a + b))
        assert_close(host(nxt), ref, f"descent step {k}", bound)
        x = nxt
    assert torch.equal(out, x)


def _lesion_regions(shape, clean, lesion_r_roi, bg_in, bg_out, amp):
    """Per phase: the lesion ROI (a ball around the lesion centre) and a
    background shell of lung tissue around it, from the known ground truth."""
    np_, nx, ny, nz = shape
    X = np.arange(nx)[:, None, None]
    Y = np.arange(ny)[None, :, None]
    Z = np.arange(nz)[None, None, :]
    cx, cy, cz = (nx - 1) / 2, (ny - 1) / 2, (nz - 1) / 2
    out = []
    for i in range(np_):
        lz = cz + amp * np.sin(2 * np.pi * i / np_)
        r2 = (X - cx - 0.2 * nx) ** 2 + (Y - cy) ** 2 + (Z - lz) ** 2
        roi = r2 <= lesion_r_roi ** 2
        bg = (r2 >= bg_in ** 2) & (r2 <= bg_out ** 2) & (clean[i] == 0.02)
        out.append((roi, bg))
    return out


def test_enhancement_removes_streaks_and_raises_lesion_cnr():
    """TNLM-E (Sec. 2.3) on a streaked breathing phantom with known ground
    truth: the streak-reduction ratio of Eq. (10) is positive and the
    lesion's contrast-to-noise ratio grows, as the paper reports (Table 1)."""
    from phantom import breathing_phantom
    shape = (10, 64, 64, 32)
    noisy, clean = breathing_phantom(*shape, lesion_r=6.0, amp=3.0,
                                     sigma=0.02, streaks=True, seed=77)
    say(f"enhancement quality {shape}")
    g = torch.from_numpy(noisy.astype(np.float32)).to(device())
    f = tnlm.enhance(g, 0.5, d=1, M=3, h=0.04, iters=10)
    truth = torch.from_numpy(clean).to(device())
    s = tnlm.metrics.srr(g.double(), f.double(), truth)
    c_in, c_out = [], []
    for i, (roi, bg) in enumerate(_lesion_regions(shape, clean, 4.0, 8.0, 11.0, 3.0)):
        roi, bg = torch.from_numpy(roi).to(device()), torch.from_numpy(bg).to(device())
        c_in.append(tnlm.metrics.cnr(g[i], roi, bg))
        c_out.append(tnlm.metrics.cnr(f[i], roi, bg))
    say(f"  SRR {s:.3f}  CNR {np.mean(c_in):.2f} -> {np.mean(c_out):.2f}")
    say(f"QUALITY|{shape}|SRR={s:.4f}|CNR_in={np.mean(c_in):.3f}|CNR_out={np.mean(c_out):.3f}")
    assert s > 0.3
    assert np.mean(c_out) > 1.5 * np.mean(c_in)


def test_tnlm_e_metrics_match_the_oracles_tnlm_e():
    """TNLM-E (weights from the current iterate at every step, Sec. 2.3) for
    10 iterations on a 10x32x32x16 streaked phantom, on the GPU and in the
    oracle. Every GPU step is held to the one-step bound against the oracle's
    step from the GPU's previous iterate; SRR (Eq. (10)) and the lesion CNR
    of the two 10-step results differ by no more than the difference of the
    two volumes allows. Per phase, |dSRR| <= TV(f_gpu - f_oracle) / TV(g - f*)
    (TV is a semi-norm), and with A = 2|mean_roi - mean_bg|, S the sum of
    the two regions' standard deviations (also semi-norms) and dl the volume
    difference, |dCNR| <= (2(|mean_roi dl| + |mean_bg dl|) + CNR s(dl)) /
    (S - s(dl)), s(dl) = std_roi dl + std_bg dl; the phase means obey the
    means of these bounds. The metrics are evaluated in FP64 (1e-12 relative
    slack)."""
    from oracle import metrics_ref
    from phantom import breathing_phantom
    shape, d, M, h, mu, iters = (10, 32, 32, 16), 1, 2, 0.05, 0.5, 10
    noisy, clean = breathing_phantom(*shape, lesion_r=3.0, amp=2.0, sigma=0.02,
                                     streaks=True, seed=78)
    g64, g = to_dev(noisy)
    say(f"TNLM-E metrics {shape}, {iters} iterations")
    steps = []
    f = tnlm.enhance(g, mu, d=d, M=M, h=h, iters=iters,
                     step_hook=lambda k, x: steps.append(x.clone()))
    torch.cuda.synchronize()
    prev = [g] + steps[:-1]
    for k in range(iters):
        x64 = host(prev[k])
        ref = oracle.jacobi(x64, x64, g64, mu, d, M, h)
        assert_close(host(steps[k]), ref, f"TNLM-E step {k}",
                     Bounds(x64, x64, d, M, h).jacobi(mu))
    fo = g64.copy()
    for _ in range(iters):
        fo = oracle.jacobi(fo, fo, g64, mu, d, M, h)
    fg = host(f)
    srr_g = np.mean([metrics_ref.srr(g64[i], fg[i], clean[i]) for i in range(shape[0])])
    srr_o = np.mean([metrics_ref.srr(g64[i], fo[i], clean[i]) for i in range(shape[0])])
    srr_b = np.mean([metrics_ref.tv(fg[i] - fo[i]) / metrics_ref.tv(g64[i] - clean[i])
                     for i in range(shape[0])])
    c_g, c_o, c_b = [], [], []
    for i, (roi, bg) in enumerate(_lesion_regions(shape, clean, 2.0, 4.0, 6.0, 2.0)):
        c_g.append(metrics_ref.cnr(fg[i], roi, bg))
        c_o.append(metrics_ref.cnr(fo[i], roi, bg))
        dl = fg[i] - fo[i]
        num = 2 * (abs(dl[roi].mean()) + abs(dl[bg].mean()))
        den = fo[i][roi].std() + fo[i][bg].std()
        dsd = dl[roi].std() + dl[bg].std()
        c_b.append((num + c_o[-1] * dsd) / max(den - dsd, 1e-300))
    cg, co = np.mean(c_g), np.mean(c_o)
    say(f"  SRR gpu {srr_g:.6f} oracle {srr_o:.6f} (|d| {abs(srr_g - srr_o):.2e}, "
        f"Lipschitz bound {srr_b:.2e})")
    say(f"  CNR gpu {cg:.6f} oracle {co:.6f} (|d| {abs(cg - co):.2e}, "
        f"bound {np.mean(c_b):.2e}); input CNR "
        f"{np.mean([metrics_ref.cnr(g64[i], *r) for i, r in enumerate(_lesion_regions(shape, clean, 2.0, 4.0, 6.0, 2.0))]):.3f}")
    say(f"QUALITY-PARITY|{shape}|SRR_gpu={srr_g:.6f}|SRR_oracle={srr_o:.6f}|"
        f"CNR_gpu={cg:.5f}|CNR_oracle={co:.5f}")
    assert abs(srr_g - srr_o) <= srr_b + 1e-12 * abs(srr_o)
    assert abs(cg - co) <= np.mean(c_b) + 1e-12 * co
