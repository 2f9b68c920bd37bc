"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Each case draws seeded inputs, rounds them to the storage dtype, runs the
oracle on exactly those values and the library on the device, and compares
element by element (normwise relative error), at sizes the oracle finishes in
seconds that still span several tiles and ragged tails. Tolerances: FP32
outputs max(1e-5, the case's derived rounding-error bound) (tests/gpu_util.py);
volumes stored in BF16/FP16 additionally half a storage ulp.
"""
import itertools
import math

import numpy as np
import pytest
import torch

import paper_1201_2450_amd as tnlm
from oracle import oracle
from tests.test_gpu_workloads import sample_idx
from tests.gpu_util import (STORE_EPS, Bounds, assert_close, assert_close_scalar, device,
                            host, inputs, say, to_dev, with_peaks)

pytestmark = pytest.mark.gpu

# (shape, d, M, h, kind): ragged shapes, borders on every side, d/M spread
CASES = [
    ((3, 13, 11, 37), 1, 2, 0.05, "phantom"),
    ((2, 9, 10, 70), 1, 3, 0.04, "phantom"),
    ((4, 7, 6, 5), 0, 1, 0.1, "smooth"),
    ((3, 6, 17, 9), 2, 2, 0.08, "phantom"),
    ((2, 5, 5, 5), 1, 4, 0.3, "uniform"),
    ((5, 8, 3, 129), 1, 1, 0.05, "phantom"),
    ((3, 1, 9, 33), 1, 2, 0.05, "phantom"),    # nx = 1
    ((2, 4, 4, 1), 1, 2, 0.2, "uniform"),      # nz = 1
    ((3, 12, 10, 20), 1, 2, 0.03, "uniform"),  # deep-underflow / overflow path
    ((2, 6, 7, 8), 1, 0, 0.05, "phantom"),     # M = 0: single candidate
    ((3, 6, 1, 12), 1, 2, 0.05, "phantom"),    # ny = 1
    ((2, 7, 8, 9), 1, 5, 0.05, "phantom"),     # M = 5: largest tiled window
    ((2, 6, 7, 8), 1, 6, 0.05, "phantom"),     # M = 6: generic kernels
]


def ids(c):
    return "np{}x{}x{}x{}-d{}M{}-{}".format(*c[0], c[1], c[2], c[4])


@pytest.mark.parametrize("case", CASES, ids=[ids(c) for c in CASES])
def test_weights_and_lse(case):
    shape, d, M, h, kind = case
    say(f"weights {shape} d={d} M={M} h={h} {kind}")
    u64, u = to_dev(inputs(shape, kind, 1), "f32")
    w_ref, lse_ref = oracle.weights(u64, d, M, h)
    w, lse = tnlm.weights(u, d=d, M=M, h=h, want_w=True)
    torch.cuda.synchronize()
    B = Bounds(u64, u64, d, M, h)
    assert_close(host(w), w_ref, "w", B.w())
    assert_close(host(lse), lse_ref, "lse", B.lse())
    assert np.abs(host(w).sum(axis=2) - 1).max() <= 1e-5


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("case", CASES, ids=[ids(c) for c in CASES])
def test_jacobi_step(case, storage):
    shape, d, M, h, kind = case
    say(f"jacobi {shape} d={d} M={M} h={h} {kind} {storage}")
    u64, u = to_dev(inputs(shape, kind, 2), storage)
    f64, f = to_dev(inputs(shape, kind, 3), storage)
    g64, g = to_dev(inputs(shape, kind, 4), storage)
    mu = 0.7
    ref = oracle.jacobi(u64, f64, g64, mu, d, M, h)
    out = tnlm.jacobi_step(u, f, g, mu, d=d, M=M, h=h)
    torch.cuda.synchronize()
    assert out.dtype == f.dtype
    assert_close(host(out), ref, "f_out", Bounds(u64, f64, d, M, h).jacobi(mu),
                 extra=STORE_EPS[storage])


@pytest.mark.parametrize("case", CASES, ids=[ids(c) for c in CASES])
def test_eq6_operator(case):
    shape, d, M, h, kind = case
    say(f"eq6 {shape} d={d} M={M} h={h} {kind}")
    u64, u = to_dev(inputs(shape, kind, 5), "f32")
    f64, f = to_dev(inputs(shape, kind, 6), "f32")
    ref = oracle.grad_eq6(u64, f64, d, M, h)
    out = tnlm.grad(f, u=u, d=d, M=M, h=h, mode="eq6")
    torch.cuda.synchronize()
    assert_close(host(out), ref, "G6", Bounds(u64, f64, d, M, h).eq6())


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("case", CASES, ids=[ids(c) for c in CASES])
def test_energy_and_stats(case, storage):
    shape, d, M, h, kind = case
    say(f"energy {shape} d={d} M={M} h={h} {kind} {storage}")
    u64, u = to_dev(inputs(shape, kind, 7), storage)
    f64, f = to_dev(inputs(shape, kind, 8), storage)
    E_ref, st_ref = oracle.energy(u64, f64, d, M, h, want_stats=True)
    e, st = tnlm.energy(f, u=u, d=d, M=M, h=h, want_stats=True)
    torch.cuda.synchronize()
    E = float(e[0].item()) + float(e[1].item())
    B = Bounds(u64, f64, d, M, h)
    assert_close_scalar(E, E_ref, "E", B.energy())
    N = int(np.prod(shape[1:]))
    st_ref = st_ref.reshape(shape[0], 2, 2, N)
    assert_close(host(st)[:, :, 0], st_ref[:, :, 0], "stats.lse", B.lse())
    assert_close(host(st)[:, :, 1], st_ref[:, :, 1], "stats.e", B.e())


GRAD_CASES = [c for c in CASES if np.prod(c[0]) <= 6000]


@pytest.mark.parametrize("case", GRAD_CASES, ids=[ids(c) for c in GRAD_CASES])
def test_exact_gradient(case):
    shape, d, M, h, kind = case
    say(f"grad exact {shape} d={d} M={M} h={h} {kind}")
    u64, u = to_dev(inputs(shape, kind, 9), "f32")
    f64, f = to_dev(inputs(shape, kind, 10), "f32")
    gf_ref, gu_ref = oracle.grad_exact_scatter(u64, f64, d, M, h)
    gf, gu = tnlm.grad(f, u=u, d=d, M=M, h=h, mode="exact")
    torch.cuda.synchronize()
    B = Bounds(u64, f64, d, M, h, grad=True)
    assert_close(host(gf), gf_ref, "dE/df", B.gf())
    assert_close(host(gu), gu_ref, "dE/du", B.gu())
    # total gradient of E(f; f), with saved statistics
    e, st = tnlm.energy(f, d=d, M=M, h=h, want_stats=True)
    gt = tnlm.grad(f, d=d, M=M, h=h, mode="exact", stats=st, total=True)
    a, b = oracle.grad_exact_scatter(f64, f64, d, M, h)
    torch.cuda.synchronize()
    assert_close(host(gt), a + b, "dE/df+dE/du (u=f)",
                 Bounds(f64, f64, d, M, h, grad=True).total())


def test_results_are_bitwise_deterministic():
    """Every entry point twice on the same input: bitwise the same outputs
    (fixed-order sums, no atomics), on the tiled kernels and, with M = 6, on
    the generic ones (the full weight tensor too)."""
    shape, d, h = (3, 16, 12, 40), 1, 0.05
    say(f"determinism {shape}")
    _, u = to_dev(inputs(shape, "phantom", 11))
    for M in (2, 6):
        outs = []
        for _ in range(2):
            w, lse = tnlm.weights(u, d=d, M=M, h=h, want_w=(M == 6))
            j = tnlm.jacobi_step(u, u, u, 0.5, d=d, M=M, h=h)
            e, st = tnlm.energy(u, d=d, M=M, h=h, want_stats=True)
            g6 = tnlm.grad(u, d=d, M=M, h=h, mode="eq6")
            gt = tnlm.grad(u, d=d, M=M, h=h, mode="exact", stats=st, total=True)
            torch.cuda.synchronize()
            res = [t for t in (w, lse, j, e, st, g6, gt) if t is not None]
            outs.append([t.cpu().numpy().copy() for t in res])
        for a, b in zip(*outs):
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), f"M = {M}"


@pytest.mark.parametrize("M", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_adjoint_image_equal_to_weight_source_instance(M, storage):
    """The adjoint has an instance for u and f being one buffer (f_j read
    from the staged u_j, residual from the centre difference). Handing it a
    copy of f as u takes the general instance; on interior and border tiles
    both must give the same gradient, and both match the oracle. The grid
    holds interior (unmasked) tiles for every M."""
    shape, d, h = (2, 16, 120, 30), 1, 0.05
    say(f"adjoint u=f instance M={M} {storage} {shape}")
    f64, f = to_dev(inputs(shape, "phantom", 40 + M), storage)
    u = f.clone()
    gs_f, gs_u = tnlm.grad(f, d=d, M=M, h=h, mode="exact")           # u is f
    gg_f, gg_u = tnlm.grad(f, u=u, d=d, M=M, h=h, mode="exact")      # u a copy
    torch.cuda.synchronize()
    B = Bounds(f64, f64, d, M, h, grad=True)
    # two FP32 evaluations, each within its bound of the exact value
    assert_close(host(gs_f), host(gg_f), "dE/df: u = f vs copy", 2 * B.gf())
    assert_close(host(gs_u), host(gg_u), "dE/du: u = f vs copy", 2 * B.gu())
    idx = with_peaks(sample_idx(shape, 60, M), gs_f, gs_u)
    rf, ru = oracle.grad_exact_at(f64, f64, d, M, h, idx)
    assert_close(host(gs_f).ravel()[idx], rf, "dE/df vs oracle", B.gf().ravel()[idx])
    assert_close(host(gs_u).ravel()[idx], ru, "dE/du vs oracle", B.gu().ravel()[idx])


def test_exact_gradient_whole_field_interior_and_border_planes():
    """Whole-field check of the exact gradient on the phantom where the
    weight exponents are steepest (moving edges, c2*D_min up to ~310,
    log-normalisers down to -216): every voxel against the oracle's scatter
    form. A voxel on a face of the grid also collects the derivatives of the
    clamped copies of itself that patches reaching past the face use (the
    chain rule through clamp-to-edge): large terms of both signs whose
    rounding errors add while their sum shrinks. The derived bound covers
    both; the worst error inside the grid and on the faces is printed."""
    shape, d, M, h = (2, 16, 120, 30), 1, 2, 0.05
    say(f"whole-field gradient {shape} M={M}")
    f64, f = to_dev(inputs(shape, "phantom", 42), "f32")
    gf, gu = tnlm.grad(f, d=d, M=M, h=h, mode="exact")
    torch.cuda.synchronize()
    a, b = oracle.grad_exact_scatter(f64, f64, d, M, h)
    B = Bounds(f64, f64, d, M, h, grad=True)
    assert_close(host(gf), a, "dE/df (whole field)", B.gf())
    inner = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    eu = np.abs(host(gu) - b)
    scale = np.abs(b).max()
    say(f"  dE/du: inside {eu[inner].max() / scale:.3e}, whole field {eu.max() / scale:.3e}")
    assert_close(host(gu), b, "dE/du (whole field)", B.gu())


def test_empty_and_too_few_phases_are_rejected_before_any_launch():
    """Empty volumes and a single phase are invalid geometries: the library
    returns EINVAL (no kernel runs) and the binding raises."""
    for shape in ((2, 0, 4, 4), (2, 4, 0, 4), (2, 4, 4, 0), (1, 4, 4, 4)):
        say(f"rejected {shape}")
        x = torch.zeros(shape, device=device())
        with pytest.raises(tnlm.TNLMError):
            tnlm.jacobi_step(x, x, x, 0.5, d=1, M=1, h=0.1)
        with pytest.raises(tnlm.TNLMError):
            tnlm.energy(x, d=1, M=1, h=0.1)
    torch.cuda.synchronize()


def test_calls_run_on_the_callers_stream_and_share_no_state():
    """Each call is enqueued on the caller's current stream and keeps no
    state: the same calls issued on two side streams at once (default
    priority) give bitwise the results of the default stream."""
    shape, d, M, h = (3, 16, 31, 40), 1, 3, 0.05
    say(f"streams {shape}")
    _, u = to_dev(inputs(shape, "phantom", 50))
    _, v = to_dev(inputs(shape, "phantom", 51))

    def work(x):
        j = tnlm.jacobi_step(x, x, x, 0.5, d=d, M=M, h=h)
        e, st = tnlm.energy(x, d=d, M=M, h=h, want_stats=True)
        g = tnlm.grad(x, d=d, M=M, h=h, mode="exact", stats=st, total=True)
        return j, e, g

    ref = [work(u), work(v)]
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s1):
        out1 = work(u)
    with torch.cuda.stream(s2):
        out2 = work(v)
    s1.synchronize()
    s2.synchronize()
    for got, want in zip(out1 + out2, ref[0] + ref[1]):
        assert torch.equal(got.view(torch.int32) if got.dtype == torch.float32 else got,
                           want.view(torch.int32) if want.dtype == torch.float32 else want)


def test_graph_capture_and_replay():
    """The library allocates, clears and synchronises nothing, so a sequence
    of calls can be captured in a HIP graph: two Gauss-Jacobi steps, the
    energy and the exact gradient, replayed three times on new inputs (with
    eager work between the replays), each replay bitwise equal to the same
    calls run eagerly."""
    shape, d, M, h, mu = (3, 12, 31, 36), 1, 2, 0.05, 0.5
    say(f"graph capture {shape}")
    g0 = to_dev(inputs(shape, "phantom", 60))[1]
    x = torch.empty_like(g0)
    b1, b2 = torch.empty_like(g0), torch.empty_like(g0)

    def calls(src, o1, o2):
        tnlm.jacobi_step(g0, src, g0, mu, d=d, M=M, h=h, out=o1)
        tnlm.jacobi_step(g0, o1, g0, mu, d=d, M=M, h=h, out=o2)
        e, st = tnlm.energy(o2, d=d, M=M, h=h, want_stats=True)
        gt = tnlm.grad(o2, d=d, M=M, h=h, mode="exact", stats=st, total=True)
        return e, gt

    x.copy_(g0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        calls(x, b1, b2)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        e_cap, g_cap = calls(x, b1, b2)
    for r in range(3):
        x.copy_(to_dev(inputs(shape, "phantom", 61 + r))[1])
        graph.replay()
        torch.cuda.synchronize()
        got = (b2.clone(), e_cap.clone(), g_cap.clone())
        # the same calls eagerly, on separate buffers
        c1, c2 = torch.empty_like(g0), torch.empty_like(g0)
        e_ref, g_ref = calls(x, c1, c2)
        torch.cuda.synchronize()
        for a, b in zip(got, (c2, e_ref, g_ref)):
            assert torch.equal(a.view(torch.int32), b.view(torch.int32)), f"replay {r}"
    del graph


def test_constant_volume_is_a_fixed_point_on_gpu():
    shape = (3, 20, 9, 33)
    say(f"constant fixed point {shape}")
    c = torch.full(shape, 0.3125, device=device())
    out = tnlm.jacobi_step(c, c, c, 0.5, d=1, M=3, h=0.04)
    e, _ = tnlm.energy(c, d=1, M=3, h=0.04)
    torch.cuda.synchronize()
    assert torch.all(out == c)
    assert float(e[0]) == 0.0 and float(e[1]) == 0.0


def test_autograd_energy_matches_exact_gradient():
    shape, d, M, h = (3, 6, 5, 7), 1, 2, 0.08
    say(f"autograd {shape}")
    f64, f = to_dev(inputs(shape, "phantom", 12))
    x = f.clone().requires_grad_(True)
    E = tnlm.tnlm_energy(x, d, M, h)
    E.backward()
    a, b = oracle.grad_exact_scatter(f64, f64, d, M, h)
    B = Bounds(f64, f64, d, M, h, grad=True)
    assert_close_scalar(float(E.detach()), oracle.energy(f64, f64, d, M, h), "autograd E",
                        B.energy())
    assert_close(host(x.grad), a + b, "autograd grad", B.total())


def test_enhance_driver_matches_repeated_oracle_steps():
    """The enhancement driver with the weights refreshed every second step:
    each step against the oracle's Eq.-(8) step from the driver's own
    previous iterate and weight snapshot (so every step is held to the
    one-step bound), and the whole run bitwise equal to the same library
    calls made by hand."""
    shape, d, M, h, mu = (3, 10, 9, 12), 1, 2, 0.05, 1.0
    say(f"enhance driver {shape}")
    g64, g = to_dev(inputs(shape, "phantom", 13))
    steps = []
    out = tnlm.enhance(g, mu, d=d, M=M, h=h, iters=3, recompute_every=2,
                       step_hook=lambda k, f: steps.append(f.clone()))
    torch.cuda.synchronize()
    assert torch.equal(out, steps[-1])
    prev = [g] + steps[:-1]
    for k in range(3):
        u_t = prev[2 * (k // 2)]  # weights from the iterate at the last snapshot
        u64, f64 = host(u_t), host(prev[k])
        ref = oracle.jacobi(u64, f64, g64, mu, d, M, h)
        assert_close(host(steps[k]), ref, f"enhance step {k}",
                     Bounds(u64, f64, d, M, h).jacobi(mu))
        by_hand = tnlm.jacobi_step(u_t, prev[k], g, mu, d=d, M=M, h=h)
        torch.cuda.synchronize()
        assert torch.equal(by_hand, steps[k]), k


@pytest.mark.parametrize("k_stop", [2, 3])
def test_enhance_checkpoint_resume_is_bitwise(k_stop):
    """Stopping the enhancement driver after k_stop steps, saving its state
    (f, u, k) through torch.save and resuming from the reloaded state gives
    bit for bit the uninterrupted run (weights refreshed every third step;
    k_stop = 2 resumes between refreshes, with the saved snapshot u)."""
    import io
    shape, d, M, h, mu = (3, 10, 9, 12), 1, 2, 0.05, 1.0
    say(f"enhance checkpoint/resume {shape} at k={k_stop}")
    _, g = to_dev(inputs(shape, "phantom", 17))
    full = tnlm.enhance(g, mu, d=d, M=M, h=h, iters=7, recompute_every=3)
    saved = {}

    def keep(state):
        if state["k"] == k_stop:
            buf = io.BytesIO()
            torch.save({"f": state["f"].cpu(), "u": state["u"].cpu(), "k": state["k"]}, buf)
            saved["blob"] = buf.getvalue()

    tnlm.enhance(g, mu, d=d, M=M, h=h, iters=k_stop, recompute_every=3, checkpoint=keep)
    state = torch.load(io.BytesIO(saved["blob"]), weights_only=True)
    state = {"f": state["f"].to(g.device), "u": state["u"].to(g.device), "k": state["k"]}
    resumed = tnlm.enhance(g, mu, d=d, M=M, h=h, iters=7, recompute_every=3, resume=state)
    torch.cuda.synchronize()
    assert torch.equal(resumed, full)


@pytest.mark.parametrize("d,M", [(1, 1), (1, 3), (2, 1)])
def test_nan_in_the_data_reaches_the_same_outputs_as_the_oracle(d, M):
    """NaN in the volumes is not checked but propagated: one NaN voxel of
    phase 1 (in u, f and g) makes exactly the oracle's NaN set of the
    Gauss-Jacobi output NaN (the tiled kernel for d = 1, the generic one for
    d = 2), every other output matches the oracle, and the energy is NaN."""
    shape, h, mu = (3, 12, 40, 20), 0.1, 0.5
    say(f"NaN propagation {shape} d={d} M={M}")
    u64 = inputs(shape, "phantom", 23)
    u64[1, 6, 20, 10] = np.nan
    _, u = to_dev(u64)
    out = host(tnlm.jacobi_step(u, u, u, mu, d=d, M=M, h=h))
    ref = oracle.jacobi(u64, u64, u64, mu, d, M, h)
    assert np.array_equal(np.isnan(out), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.isfinite(out[ok]).all()
    err = np.max(np.abs(out[ok] - ref[ok])) / np.max(np.abs(ref[ok]))
    assert err <= 1e-5, err
    e, _ = tnlm.energy(u, d=d, M=M, h=h)
    torch.cuda.synchronize()
    assert math.isnan(float(e[0]) + float(e[1]))
