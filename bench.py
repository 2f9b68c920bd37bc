"""Benchmark of the TNLM hot path on one MI355X.

One step = one pass of the whole hot path over the clinical-size
enhancement workload (10 phases of 256x256x128 voxels, patch 3^3, window
7^3, h = 0.04, mu = 0.5):
  * 20 Gauss-Jacobi steps (Eq. (8)), weight source u <- f every 5 steps,
  * log-normalisers of the final iterate (weights, Eq. (3)),
  * the TNLM energy forward with its per-voxel statistics,
  * the Eq. (6) operator,
  * the exact adjoint (dE/df + dE/du of E(f; f)) from the saved statistics.
`value` counts the 20 Jacobi sweeps as voxel-updates (20 * 10*256*256*128)
and divides by the wall time of the whole step, so the energy and gradient
passes count against it. Inputs are resident on the GPU before timing.

`--workload fbs512` (not the default) times the forward-backward splitting
regulariser instead: one step is f <- f - 0.1 dE(f; f)/df on 20 phases of
512x512x128 voxels in FP16 (window 9^3), and `value` counts its voxels.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("TNLM voxel-updates/s + fwd/adjoint ms, 10×256²×128, "
          "FP32 vs BF16, % VALU peak")
# MI355X FP32 vector peak: 256 CUs x 4 SIMDs x 64 lanes x 2 (FMA) / 2 cycles
# x 2.4 GHz; plain (non-packed) FMAs whose operands are all vector registers
# issue at that rate (one wave64 instruction per SIMD every ~2.1 cycles,
# measured), FMAs reading a scalar register at half of it
PEAK_FP32_TFLOPS = 157.3
# algorithmic flops per Jacobi voxel-update and search offset, patch 3^3:
# squared difference 2 + separable 3-tap box sums 6 (once per link), then per
# direction: exponent 2, numerator FMA 2, normaliser add 1 (x2 directions)
FLOP_PER_UPDATE_PER_OFFSET = 18
FLOP_PER_VOXEL_OFFSET_ADJOINT = 35
# algorithmic flops per (ray, voxel) pair of the cone-beam projector and of
# its transpose (the same pairs): the stepped axis's next crossing (one
# multiply-add, 2), the least of the three crossings (2 comparisons), the
# length inside the voxel (difference times the ray's length scale, 2) and
# the accumulation (one fused multiply-add, 2)
FLOP_PER_RAY_VOXEL = 8


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def profile_figures(name="jacobi_enh256_traffic.txt", source="tiled_fwd.hip"):
    """HBM bytes (and, where recorded, counter FP32 flop) per launch of a
    kernel from a committed rocprofv3 counter summary, or {} when the
    kernel's source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    src = os.path.join(ROOT, "paper_1201_2450_amd", "csrc", source)
    key = "source_sha256_" + source.replace(".", "_")
    try:
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if kv.get(key) != sha:
            return {}
        out = {"traffic": float(kv["traffic_bytes"])}
        if "counter_flop_per_launch" in kv:
            out["counter_flop"] = float(kv["counter_flop_per_launch"])
        return out
    except (OSError, KeyError, ValueError):
        return {}


def cpu_model():
    """The host CPU's model name (first 'model name' of /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(w, target_s):
    """Time the FP64 oracle on a bounded sample of the same workload: one
    Jacobi step (u = f = g) at a random sample of voxels."""
    import numpy as np

    from oracle import oracle
    from phantom import workload_inputs
    g64 = workload_inputs(w, out_dtype=np.float32)[0].astype(np.float64)
    rng = np.random.default_rng(7)
    total = g64.size
    # batches of random voxels until target_s of oracle time has been spent,
    # each batch sized from the rate so far (at most ~5 s)
    n_all, t_all, n = 0, 0.0, 4096
    while t_all < target_s:
        idx = rng.choice(total, size=n, replace=False)
        t0 = time.perf_counter()
        oracle.jacobi(g64, g64, g64, w.mu, w.d, w.M, w.h, idx=idx)
        t_all += time.perf_counter() - t0
        n_all += n
        rate = n_all / t_all
        n = int(min(total, max(4096, rate * min(max(target_s - t_all, 0.0), 5.0))))
    n2, dt = n_all, t_all
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n2 / dt, "unit": "voxel-updates/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"one Gauss-Jacobi step of the 10x256x256x128 "
                      f"workload (u=f=g) at {n2} random voxels, FP64, "
                      f"{dt:.1f} s on {threads} OpenMP threads"}


def cpu_baseline_gradient(f64, w, target_s):
    """The FP64 oracle's exact gradient of E(f; f) (gather form, the part
    that dominates the regulariser step) at random voxels of the same
    volume, in batches until target_s of oracle time has been spent."""
    import numpy as np

    from oracle import oracle
    rng = np.random.default_rng(8)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n_all, t_all, n = 0, 0.0, threads
    while t_all < target_s:
        idx = rng.choice(f64.size, size=n, replace=False)
        t0 = time.perf_counter()
        oracle.grad_exact_at(f64, f64, w.d, w.M, w.h, idx)
        t_all += time.perf_counter() - t0
        n_all += n
        rate = n_all / t_all
        n = int(max(threads, rate * min(max(target_s - t_all, 0.0), 5.0)))
    return {"value": n_all / t_all, "unit": "voxel-updates/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"exact gradient of E(f; f) of the {w.name} volume "
                      f"(FP16 values) at {n_all} random voxels, FP64 gather form, "
                      f"{t_all:.1f} s on {threads} OpenMP threads"}


def regulariser(args, w, dev):
    """Non-default mode for the workloads without a fidelity weight (the
    forward-backward splitting regulariser, e.g. --workload fbs512): one
    step is f <- f - tau * dE(f; f)/df with tau = 0.1, i.e. the energy with
    statistics, the exact adjoint and the update, in the workload's storage
    format (FP16 for fbs512)."""
    import numpy as np
    import torch

    import paper_1201_2450_amd as tnlm
    from phantom import workload_inputs

    dt = np.float16 if w.name == "fbs512" else np.float32
    log(f"generating {w.name} {w.shape} ({np.dtype(dt).name}) ...")
    f = torch.from_numpy(workload_inputs(w, out_dtype=dt)[0]).to(dev)
    d, M, h, tau = w.d, w.M, w.h, 0.1
    EV = lambda: torch.cuda.Event(enable_timing=True)
    names = ["energy_fwd", "adjoint", "update"]

    def step(x):
        ev = {}
        e = [EV() for _ in range(4)]
        e[0].record()
        _, st = tnlm.energy(x, d=d, M=M, h=h, want_stats=True)
        e[1].record()
        gt = tnlm.grad(x, d=d, M=M, h=h, mode="exact", stats=st, total=True)
        e[2].record()
        x = (x.float() - tau * gt).to(x.dtype)
        e[3].record()
        for k, n in enumerate(names):
            ev[n] = (e[k], e[k + 1])
        return x, ev

    x = f
    for _ in range(args.warmup):
        x, _ = step(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = []
    for _ in range(args.steps):
        x, ev = step(x)
        evs.append(ev)
    torch.cuda.synchronize()
    ms_step = 1e3 * (time.perf_counter() - t0) / args.steps
    ms = {n: float(np.mean([e[n][0].elapsed_time(e[n][1]) for e in evs])) for n in names}
    log(f"step {ms_step:.1f} ms; per-op ms {ms}")
    # dominant kernel: the exact adjoint. Algorithmic flop per voxel and
    # offset, patch 3^3: distance 8 (once per link), two weights 2 x 2,
    # centred terms 8, box sum back 6, times Delta 3, image part 3 = 32,
    # rounded up to 35 (plus two exponentials)
    W = (2 * M + 1) ** 3
    alg = FLOP_PER_VOXEL_OFFSET_ADJOINT * W * w.nvox
    ach = alg / (ms["adjoint"] / 1e3) / 1e12
    roofline = {"bound": "alu", "achieved": ach, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / PEAK_FP32_TFLOPS, "traffic": None,
                "kernel": "tnlm_grad (exact adjoint)",
                "algorithmic_flop_per_launch": alg}
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle gradient on a sample ...")
        cpu = cpu_baseline_gradient(f.float().cpu().numpy().astype(np.float64), w,
                                    args.cpu_seconds)
    print(json.dumps({
        "metric": METRIC, "value": w.nvox / (ms_step / 1e3), "unit": "voxel-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"float16": "f16", "float32": "f32"}[np.dtype(dt).name],
        "data": "synthetic",
        "config": {"workload": w.name, "phases": w.np_, "grid": [w.nx, w.ny, w.nz],
                   "patch": 2 * d + 1, "window": 2 * M + 1, "h": h, "tau": tau,
                   "step": "energy + exact adjoint + descent update"},
        "breakdown_ms": ms, "roofline": roofline, "cpu_baseline": cpu}), flush=True)


def recon_cpu_sample(name, target_s, cg_iters=10):
    """The FP64 oracle on a bounded sample of the reconstruction workload:
    the projector and its transpose for a few of phase 0's angles (every
    detector pixel; the angles spread over the circle) and one Gauss-Jacobi
    step at random voxels, each scaled to the whole workload and combined as
    one TNLM-R outer iteration ((cg_iters + 1) projector/transpose pairs plus
    the Eq. (8) step). Also returns the mean number of voxels a ray crosses
    (positive lengths), from the same projector sample."""
    import numpy as np

    from oracle import ct as OCT
    from oracle import oracle
    from phantom.breathing import CT_WORKLOADS, ct_angles

    w = CT_WORKLOADS[name]
    ang = ct_angles(w.np_, w.na)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rng = np.random.default_rng(9)
    vol = rng.random((1, w.nx, w.ny, w.nz))

    def geom(k):
        return OCT.CTGeom(1, w.nx, w.ny, w.nz, w.nu, w.nv, k, w.sid, w.sdd, w.du, w.dv)

    # projector: angles 0, s, 2s, ... of phase 0 until a third of the budget
    order = list(range(0, w.na, max(1, w.na // 6))) + list(range(w.na))
    seen, cnt_sum, rays, tp = [], 0.0, 0, 0.0
    for a in order:
        if a in seen:
            continue
        seen.append(a)
        sel = np.array([[ang[0, a]]])
        t0 = time.perf_counter()
        _, cnt, _ = OCT.project(geom(1), sel, vol, want_stats=True)
        tp += time.perf_counter() - t0
        cnt_sum += float(cnt.sum())
        rays += cnt.size
        if tp >= target_s / 3 or len(seen) == w.na:
            break
    n_p = len(seen)
    # transpose: the same angles, one at a time, until another third
    tb, n_b = 0.0, 0
    for a in seen:
        sel = np.array([[ang[0, a]]])
        yv = rng.random((1, 1, w.nu, w.nv))
        t0 = time.perf_counter()
        OCT.backproject(geom(1), sel, yv)
        tb += time.perf_counter() - t0
        n_b += 1
        if tb >= target_s / 3:
            break
    # Eq. (8) step (window 5^3, patch 3^3) at random voxels
    x = rng.random((w.np_, w.nx, w.ny, w.nz))
    tj, n_j, n = 0.0, 0, 4096
    while tj < target_s / 3:
        idx = rng.choice(x.size, size=n, replace=False)
        t0 = time.perf_counter()
        oracle.jacobi(x, x, x, 0.5, 1, 2, 0.05, idx=idx)
        tj += time.perf_counter() - t0
        n_j += n
        n = int(min(x.size, max(4096, n_j / tj * min(max(target_s / 3 - tj, 0.0), 5.0))))
    total_angles = w.np_ * w.na
    p_full = tp / n_p * total_angles
    b_full = tb / n_b * total_angles
    j_full = tj / n_j * x.size
    outer_s = (cg_iters + 1) * (p_full + b_full) + j_full
    return {"value": outer_s * 1e3, "unit": "ms", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"FP64 oracle on {n_p} (projector) and {n_b} (transpose) of "
                      f"{total_angles} projections of the {name} workload (all "
                      f"{w.nu}x{w.nv} pixels each) and one Eq. (8) step at {n_j} random "
                      f"voxels, {tp + tb + tj:.1f} s on {threads} OpenMP threads, scaled to "
                      f"one TNLM-R outer iteration ({cg_iters + 1} projector/transpose "
                      f"pairs + the Eq. (8) step)"}, cnt_sum / rays


def reconstruction(name, dev, cg_iters=10, reps=2):
    """One outer iteration of the TNLM-R algorithm on a cone-beam workload:
    cg_iters CGLS iterations of (P1) for all phases, one Gauss-Jacobi step
    (weights from the CGLS result, window 5^3, patch 3^3) and positivity;
    plus the projector and its transpose alone. Returns the timings (ms)."""
    import numpy as np
    import torch

    import paper_1201_2450_amd as tnlm
    from phantom.breathing import CT_WORKLOADS, analytic_projections, ct_angles

    w = CT_WORKLOADS[name]
    geo = tnlm.ct.Geometry(w.nu, w.nv, w.sid, w.sdd, w.du, w.dv)
    ang = np.ascontiguousarray(ct_angles(w.np_, w.na), dtype=np.float32)
    at = torch.from_numpy(ang).to(dev)
    log(f"{name}: analytic projections {(w.np_, w.na, w.nu, w.nv)} ...")
    y = torch.from_numpy(analytic_projections(w, ang.astype(np.float64)).astype(np.float32)).to(dev)
    shape = (w.np_, w.nx, w.ny, w.nz)
    f = torch.zeros(shape, dtype=torch.float32, device=dev)
    EV = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = EV(), EV()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    q = tnlm.ct.project(f + 0.1, geo, at)
    proj_ms = timed(lambda: tnlm.ct.project(f, geo, at, out=q))
    bp = torch.empty_like(f)
    back_ms = timed(lambda: tnlm.ct.backproject(y, geo, at, shape, out=bp))
    outer_ms = timed(lambda: tnlm.ct.reconstruct(y, geo, at, f, mu=0.5, d=1, M=2, h=0.05,
                                                 outer=1, cg_iters=cg_iters))
    return {"workload": name, "phases": w.np_, "grid": [w.nx, w.ny, w.nz],
            "detector": [w.nu, w.nv], "angles_per_phase": w.na,
            "project_ms": proj_ms, "backproject_ms": back_ms,
            "tnlm_r_outer_iteration_ms": outer_ms, "cg_iterations": cg_iters,
            "rays_per_s_project": w.np_ * w.na * w.nu * w.nv / (proj_ms / 1e3)}


def recon_main(args, dev):
    """Prints the JSON line of the reconstruction workload: one TNLM-R outer
    iteration, with the roofline of its dominant kernel (the transpose of the
    projector) and the oracle's time on a bounded sample."""
    r = reconstruction(args.workload, dev)
    cpu, pairs_per_ray = None, None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a sample ...")
        cpu, pairs_per_ray = recon_cpu_sample(args.workload, args.cpu_seconds)
    roof = None
    if pairs_per_ray is not None:
        rays = r["phases"] * r["angles_per_phase"] * r["detector"][0] * r["detector"][1]
        flop = rays * pairs_per_ray * FLOP_PER_RAY_VOXEL
        ach = flop / (r["backproject_ms"] / 1e3) / 1e12
        roof = {"bound": "alu", "achieved": ach, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / PEAK_FP32_TFLOPS,
                "traffic": profile_figures("ct_recon128_traffic.txt", "ct.hip").get("traffic")
                if args.workload == "recon128" else None,
                "kernel": "tnlm_ct_backproject",
                "algorithmic_flop_per_launch": flop,
                "ray_voxel_pairs_per_launch": rays * pairs_per_ray,
                "projector_achieved": flop / (r["project_ms"] / 1e3) / 1e12,
                "note": ("gather-bound, not ALU- or HBM-bound: every (ray, voxel) pair of "
                         "the projector is one 64-lane gather (texture addressers 87 % busy "
                         "in the committed counters); the transpose reads four detector rows "
                         "per gather (49 % busy) and sits between that and its instruction "
                         "issue")}
        r["ray_voxel_pairs_per_ray"] = pairs_per_ray
    print(json.dumps({"metric": "TNLM-R outer iteration ms (CGLS + Eq. 8 + positivity)",
                      "value": r["tnlm_r_outer_iteration_ms"], "unit": "ms",
                      "higher_is_better": False, "n_gpus": 1, "dtype": "f32",
                      "data": "synthetic", "config": {"workload": args.workload},
                      "breakdown": r, "roofline": roof, "cpu_baseline": cpu,
                      "vs_baseline": None}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="enh256")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dtypes", action="store_true",
                    help="skip the BF16/FP16 storage and autograd comparisons")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the TNLM path here is a "
              "single-GPU build (no multi-GPU sharding); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1201_2450_amd as tnlm
    from phantom import WORKLOADS, workload_inputs

    dev = torch.device("cuda", 0)
    if args.workload.startswith("recon"):
        # the reconstruction model alone (not the default)
        return recon_main(args, dev)
    w = WORKLOADS[args.workload]
    if w.mu is None:
        return regulariser(args, w, dev)
    log(f"generating {w.name} {w.shape} ...")
    g_host = workload_inputs(w, out_dtype=np.float32)[0]
    g = torch.from_numpy(g_host).to(dev)
    del g_host
    d, M, h, mu = w.d, w.M, w.h, w.mu
    nvox = w.nvox
    W = (2 * M + 1) ** 3
    iters, every = w.iters, w.recompute_every or 1

    f_a = torch.empty_like(g)
    f_b = torch.empty_like(g)
    u_snap = torch.empty_like(g)

    EV = lambda: torch.cuda.Event(enable_timing=True)
    names = ["jacobi", "weights_lse", "energy_fwd", "grad_eq6", "adjoint"]

    def step(timing):
        ev = {k: [] for k in names}
        f, nxt = f_a, f_b
        f.copy_(g)
        for k in range(iters):
            if k % every == 0:
                u_snap.copy_(f)
            e0, e1 = EV(), EV()
            e0.record()
            tnlm.jacobi_step(u_snap, f, g, mu, d=d, M=M, h=h, out=nxt)
            e1.record()
            ev["jacobi"].append((e0, e1))
            f, nxt = nxt, f

        def timed(name, fn):
            e0, e1 = EV(), EV()
            e0.record()
            r = fn()
            e1.record()
            ev[name].append((e0, e1))
            return r

        timed("weights_lse", lambda: tnlm.weights(f, d=d, M=M, h=h))
        e, est = timed("energy_fwd",
                       lambda: tnlm.energy(f, d=d, M=M, h=h, want_stats=True))
        timed("grad_eq6", lambda: tnlm.grad(f, d=d, M=M, h=h, mode="eq6"))
        timed("adjoint", lambda: tnlm.grad(f, d=d, M=M, h=h, mode="exact",
                                           stats=est, total=True))
        return ev, e

    log(f"warmup x{args.warmup} ...")
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    log(f"timing x{args.steps} ...")
    all_ev = {k: [] for k in names}
    t0 = time.perf_counter()
    for s in range(args.steps):
        ev, e = step(True)
        for k in names:
            all_ev[k].extend(ev[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    ms = {k: float(np.mean([a.elapsed_time(b) for a, b in all_ev[k]]))
          for k in names}
    E = float(e[0]) + float(e[1])
    value = iters * nvox / (ms_step / 1e3)
    log(f"step {ms_step:.2f} ms; per-op ms {ms}; E = {E}")

    # dominant kernel: the Gauss-Jacobi step
    alg_flop = FLOP_PER_UPDATE_PER_OFFSET * W * nvox
    achieved = alg_flop / (ms["jacobi"] / 1e3) / 1e12
    prof = profile_figures()
    roofline = {"bound": "alu", "achieved": achieved,
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS,
                "traffic": prof.get("traffic"),
                "kernel": "tnlm_jacobi_step",
                "algorithmic_flop_per_launch": alg_flop}
    if "counter_flop" in prof:
        # the hardware's count of FP32 operations (64 x (ADD + MUL + TRANS +
        # 2 FMA) wave instructions) over the same measured launch time
        c = prof["counter_flop"] / (ms["jacobi"] / 1e3) / 1e12
        roofline["counter_achieved"] = c
        roofline["counter_frac"] = c / PEAK_FP32_TFLOPS
        roofline["counter_flop_per_launch"] = prof["counter_flop"]
        roofline["counter_note"] = ("hardware FP32 operation count: includes work the "
                                    "algorithmic count leaves out (each distance once per "
                                    "direction, lane-block halos, reference distances); "
                                    "frac is the algorithmic figure")

    def time_ms(fn, reps=2):
        fn()
        torch.cuda.synchronize()
        e0, e1 = EV(), EV()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    # storage formats compared on one call pattern: a Jacobi step with
    # u = f = g (the noisy input) and energy + adjoint of g, in each format;
    # then the whole mixed-precision workload (20 steps, weights every 5,
    # log-normalisers, energy, exact gradient) in each format, timed, and its
    # outputs compared with the FP32 run's at every voxel
    def rel(a, b):
        dd = a.double() - b.double()
        return {"max": float(dd.abs().max() / b.double().abs().max()),
                "rms": float(dd.square().mean().sqrt() / b.double().square().mean().sqrt())}

    def c4_run(gq):
        fq = tnlm.enhance(gq, mu, d=d, M=M, h=h, iters=iters, recompute_every=every)
        _, lq = tnlm.weights(fq, d=d, M=M, h=h)
        eq, sq = tnlm.energy(fq, d=d, M=M, h=h, want_stats=True)
        gtq = tnlm.grad(fq, d=d, M=M, h=h, mode="exact", stats=sq, total=True)
        return fq, lq, eq, gtq

    dtypes = {}
    ref = {}
    if not args.no_dtypes:
        for name, dt in (("f32", torch.float32), ("bf16", torch.bfloat16),
                         ("f16", torch.float16)):
            log(f"storage format {name} ...")
            gq = g.to(dt)
            outq = torch.empty_like(gq)
            tnlm.jacobi_step(gq, gq, gq, mu, d=d, M=M, h=h, out=outq)
            torch.cuda.synchronize()
            reps = 3
            e0, e1 = EV(), EV()
            e0.record()
            for _ in range(reps):
                tnlm.jacobi_step(gq, gq, gq, mu, d=d, M=M, h=h, out=outq)
            e1.record()
            torch.cuda.synchronize()
            jms = e0.elapsed_time(e1) / reps

            def energy_adjoint():
                ee, st = tnlm.energy(gq, d=d, M=M, h=h, want_stats=True)
                return ee, tnlm.grad(gq, d=d, M=M, h=h, mode="exact", stats=st, total=True)

            eams = time_ms(energy_adjoint)
            e1q, gr1 = energy_adjoint()
            c4_run(gq)
            torch.cuda.synchronize()
            e0, e1 = EV(), EV()
            e0.record()
            fq, lq, eq, gtq = c4_run(gq)
            e1.record()
            torch.cuda.synchronize()
            res = {"jacobi_ms": jms,
                   "jacobi_voxel_updates_per_s": nvox / (jms / 1e3),
                   "energy_plus_adjoint_ms": eams,
                   "workload_ms": e0.elapsed_time(e1),
                   "workload": "20 Jacobi (weights every 5) + lse + energy + exact gradient"}
            one = {"jacobi": outq, "E": float(e1q[0]) + float(e1q[1]), "grad": gr1}
            run = {"f20": fq, "lse": lq, "E": float(eq[0]) + float(eq[1]), "grad20": gtq}
            if name == "f32":
                ref = {"one": one, "run": run}
            else:
                # errors against the FP32 form: largest and rms, relative
                res["err_jacobi_one_step_vs_f32"] = rel(one["jacobi"], ref["one"]["jacobi"])
                res["err_energy_vs_f32"] = abs(one["E"] - ref["one"]["E"]) / abs(ref["one"]["E"])
                res["err_grad_vs_f32"] = rel(one["grad"], ref["one"]["grad"])
                res["err_workload_f20_vs_f32"] = rel(run["f20"], ref["run"]["f20"])
                res["err_workload_lse_vs_f32"] = rel(run["lse"], ref["run"]["lse"])
                res["err_workload_energy_vs_f32"] = \
                    abs(run["E"] - ref["run"]["E"]) / abs(ref["run"]["E"])
                res["err_workload_grad_vs_f32"] = rel(run["grad20"], ref["run"]["grad20"])
            dtypes[name] = res
            del gq, outq, one, run, fq, lq, gtq, gr1
        del ref
        torch.cuda.empty_cache()

    # the differentiable form against the plain calls it wraps: energy with
    # statistics + exact adjoint, vs autograd forward + backward of E(f; f)
    def autograd_vs_plain(x, dd, MM, hh):
        def plain():
            _, st = tnlm.energy(x, d=dd, M=MM, h=hh, want_stats=True)
            return tnlm.grad(x, d=dd, M=MM, h=hh, mode="exact", stats=st, total=True)

        def differentiable():
            fr = x.detach().requires_grad_(True)
            tnlm.tnlm_energy(fr, dd, MM, hh).backward()
            return fr.grad

        return {"plain_energy_plus_adjoint_ms": time_ms(plain),
                "autograd_forward_backward_ms": time_ms(differentiable)}

    autograd = None
    if not args.no_dtypes:
        log("timing the autograd form against the plain calls ...")
        autograd = {w.name: autograd_vs_plain(f_a, d, M, h)}
        we = WORKLOADS["energy128"]
        fe = torch.from_numpy(workload_inputs(we, out_dtype=np.float32)[0]).to(dev)
        autograd[we.name] = dict(autograd_vs_plain(fe, we.d, we.M, we.h),
                                 shape=list(we.shape), window=2 * we.M + 1)
        del fe

    recon = None
    if not args.no_dtypes:
        log("timing one TNLM-R outer iteration (reconstruction model) ...")
        recon = reconstruction("recon64", dev)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a sample ...")
        cpu = cpu_baseline(w, args.cpu_seconds)

    out = {
        "metric": METRIC, "value": value, "unit": "voxel-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "phases": w.np_,
                   "grid": [w.nx, w.ny, w.nz], "patch": 2 * d + 1,
                   "window": 2 * M + 1, "h": h, "mu": mu,
                   "jacobi_steps": iters, "weights_every": every,
                   "step": "20 Jacobi + lse + energy fwd + Eq.6 + adjoint"},
        "breakdown_ms": ms,
        "energy": E,
        "jacobi_voxel_updates_per_s": nvox / (ms["jacobi"] / 1e3),
        "storage_dtypes": dtypes,
        "autograd": autograd,
        "reconstruction": recon,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "paper_context": {"tnlm_e_per_iteration_s": 55.07,
                          "hardware": "NVIDIA Tesla C1060",
                          "workload": "10 x 128^3, window and patch unstated",
                          "derived_voxel_updates_per_s": 3.8e5},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
