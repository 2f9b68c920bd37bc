"""GPU parity of the reconstruction model (Eq. (1), (P1) of Eq. (5), TNLM-R
of Sec. 2.3): the cone-beam projector, its transpose, CGLS and the TNLM-R
driver against the FP64 oracle (oracle/ct.py), through the C ABI.

Tolerances come from a first-order model of the kernels' FP32 arithmetic
(oracle.ct.error_model): the ray's source and direction carry the rounding
of sin, cos and their products, every plane crossing t = (p - S_k) / d_k
inherits it amplified by 1/|d_k| (a crossing nearly parallel to its planes is
ill-conditioned), and each ray-voxel length (t_out - t_in) |d| the errors of
its two crossings; the n-term sums add n u sum |a x|. Per ray for P, per
voxel for P^T. Comparisons are normwise at max(1e-5, max bound / max|ref|),
and every element must also lie within its own bound.
"""
import numpy as np
import pytest
import torch

import paper_1201_2450_amd as tnlm
from oracle import ct as OCT
from oracle import oracle as O
from phantom.breathing import CTWorkload, analytic_projections, ct_angles, ct_clean_volumes
from tests.gpu_util import Bounds, U32, assert_close, device, host, say

pytestmark = pytest.mark.gpu


def setup(nx, ny, nz, nu, nv, na, np_, sid, sdd, du, dv, seed=0, angles=None):
    geo = tnlm.ct.Geometry(nu, nv, sid, sdd, du, dv)
    og = OCT.CTGeom(np_, nx, ny, nz, nu, nv, na, sid, sdd, du, dv)
    if angles is None:
        angles = np.random.default_rng(seed).uniform(0, 2 * np.pi, size=(np_, na))
    a32 = np.ascontiguousarray(angles, dtype=np.float32)
    return geo, og, a32.astype(np.float64), torch.from_numpy(a32).to(device())


def fwd_bound(og, ang, x):
    return OCT.error_model(og, ang, xabs=np.abs(x))[0]


def bwd_bound(og, ang, y):
    return OCT.error_model(og, ang, yabs=np.abs(y))[1]


def assert_within(got, ref, bound, what):
    """Every element within its own first-order bound."""
    r = np.abs(np.asarray(got, dtype=np.float64) - ref) / np.maximum(bound, 1e-300)
    say(f"  {what}: largest error / element bound {r.max():.3f}")
    assert r.max() <= 1.0, f"{what}: error exceeds its element bound ({r.max():.3f})"


GEOMS = [
    # nx, ny, nz, nu, nv, na, np, sid, sdd, du, dv
    (16, 16, 16, 32, 24, 6, 2, 60.0, 96.0, 1.1, 1.1),
    (13, 17, 9, 27, 19, 5, 3, 50.0, 80.0, 1.3, 0.9),   # odd, ragged, anisotropic pixels
    (24, 20, 12, 40, 20, 4, 1, 90.0, 140.0, 1.0, 1.2),
    # 2 x 2100 angles: the transpose's per-block angle table no longer fits
    # its LDS budget, so it takes its sines and cosines from sincosf
    (6, 5, 4, 8, 7, 2100, 2, 30.0, 50.0, 1.5, 1.5),
    # even ny and nz, odd nu and nv: the centre row's rays run in the plane
    # z = 0 between two voxel layers, and at angle 0 the centre column's in
    # y = 0 (each counted in one layer)
    (8, 6, 4, 9, 7, 5, 2, 30.0, 50.0, 1.5, 1.5),
    # detector columns of 64 and 128 rows (a wave's rays share one column):
    # a moderate cone, a steep one (several z crossings per x-y cell) and a
    # shallow volume that steep rays cross in a few z layers
    (16, 16, 16, 12, 64, 5, 2, 60.0, 96.0, 1.1, 0.5),
    (12, 10, 24, 8, 128, 4, 2, 30.0, 50.0, 1.5, 0.9),
    (8, 8, 6, 8, 64, 3, 1, 30.0, 50.0, 1.5, 1.0),
]


@pytest.mark.parametrize("gm", GEOMS, ids=[f"{g[0]}x{g[1]}x{g[2]}-{g[3]}x{g[4]}" for g in GEOMS])
def test_projector_and_transpose_match_the_oracle(gm):
    nx, ny, nz, nu, nv, na, np_, sid, sdd, du, dv = gm
    angles = np.random.default_rng(1).uniform(0, 2 * np.pi, size=(np_, na))
    angles[0, 0], angles[0, 1] = 0.0, np.pi / 2    # rays along the grid axes
    geo, og, ang, at = setup(nx, ny, nz, nu, nv, na, np_, sid, sdd, du, dv, angles=angles)
    say(f"projector {gm}")
    rng = np.random.default_rng(2)
    x = rng.uniform(0.0, 1.0, size=og.vol_shape).astype(np.float32).astype(np.float64)
    y = rng.normal(0.0, 1.0, size=og.proj_shape).astype(np.float32).astype(np.float64)
    xt = torch.from_numpy(x.astype(np.float32)).to(device())
    yt = torch.from_numpy(y.astype(np.float32)).to(device())
    p = tnlm.ct.project(xt, geo, at)
    b = tnlm.ct.backproject(yt, geo, at, og.vol_shape)
    torch.cuda.synchronize()
    bp = fwd_bound(og, ang, x)
    bb = bwd_bound(og, ang, y)
    pr, br = OCT.project(og, ang, x), OCT.backproject(og, ang, y)
    assert_close(host(p), pr, "P x", bp)
    assert_close(host(b), br, "P^T y", bb)
    assert_within(host(p), pr, bp, "P x")
    assert_within(host(b), br, bb, "P^T y")
    # adjointness of the two GPU operators, within what their bounds allow
    lhs = float(np.vdot(host(p), y))
    rhs = float(np.vdot(x, host(b)))
    allow = float(np.sum(bp * np.abs(y)) + np.sum(bb * np.abs(x)))
    say(f"  <Px,y> {lhs:.9g}  <x,P^T y> {rhs:.9g}  (allowed {allow:.2e})")
    assert abs(lhs - rhs) <= allow



@pytest.mark.parametrize("gm", [GEOMS[4], GEOMS[3], GEOMS[5]],
                         ids=["angle-tables", "sincosf", "whole-columns"])
def test_non_finite_angles_give_nan_for_their_rays_and_phase_only(gm):
    """A NaN or infinite angle defines no ray: its projections are NaN, the
    transpose puts NaN on every voxel of its phase, and every other ray and
    phase is bitwise what the same call gives with finite angles (both
    transpose paths: per-block angle tables and per-thread sincosf; waves
    that hold whole detector columns)."""
    nx, ny, nz, nu, nv, na, np_, sid, sdd, du, dv = gm
    angles = np.random.default_rng(3).uniform(0, 2 * np.pi, size=(np_, na))
    bad = angles.copy()
    bad[0, 1], bad[0, na - 1] = np.nan, np.inf
    geo, og, _, at = setup(nx, ny, nz, nu, nv, na, np_, sid, sdd, du, dv, angles=angles)
    _, _, _, atb = setup(nx, ny, nz, nu, nv, na, np_, sid, sdd, du, dv, angles=bad)
    say(f"non-finite angles {gm[:7]}")
    rng = np.random.default_rng(4)
    xt = torch.from_numpy(rng.uniform(0.0, 1.0, size=og.vol_shape).astype(np.float32)).to(device())
    yt = torch.from_numpy(rng.normal(0.0, 1.0, size=og.proj_shape).astype(np.float32)).to(device())
    p, pb = tnlm.ct.project(xt, geo, at), tnlm.ct.project(xt, geo, atb)
    b = tnlm.ct.backproject(yt, geo, at, og.vol_shape)
    bb = tnlm.ct.backproject(yt, geo, atb, og.vol_shape)
    torch.cuda.synchronize()
    p, pb, b, bb = host(p), host(pb), host(b), host(bb)
    assert np.isnan(pb[0, 1]).all() and np.isnan(pb[0, na - 1]).all()
    keep = np.ones((np_, na), dtype=bool)
    keep[0, 1] = keep[0, na - 1] = False
    assert np.isfinite(p).all() and np.array_equal(pb[keep], p[keep])
    assert np.isnan(bb[0]).all()
    assert np.isfinite(b).all() and np.array_equal(bb[1:], b[1:])

def test_analytic_phantom_projections_and_empty_rays():
    """The phantom's voxelised projections on the GPU track the analytic
    line integrals of its ellipsoids (discretisation error only, as on the
    oracle) and rays that miss the volume give exactly zero."""
    w = CTWorkload("t", 2, 32, 32, 32, 80, 48, 6, 125.0, 192.0, 1.2, 1.2, 3.0, 1.5, 0.0, 7)
    geo, og, ang, at = setup(32, 32, 32, 80, 48, 6, 2, w.sid, w.sdd, w.du, w.dv,
                             angles=ct_angles(2, 6))
    vol = ct_clean_volumes(w)
    p = host(tnlm.ct.project(torch.from_numpy(vol.astype(np.float32)).to(device()), geo, at))
    y = analytic_projections(w, ang)
    o = OCT.project(og, ang, vol.astype(np.float32).astype(np.float64))
    rel = lambda a, b: np.sqrt(np.mean((a - b) ** 2) / np.mean(b ** 2))
    say(f"  rms vs analytic: gpu {rel(p, y):.4f} oracle {rel(o, y):.4f}")
    assert abs(rel(p, y) - rel(o, y)) <= 1e-5
    miss = o == 0.0
    assert miss.sum() > 0 and np.all(p[miss] == 0.0)


def _cgls_bounds(og, ang, st, p_next_gpu=None):
    """Element bounds of one CGLS step taken in FP32 from state st, for x and
    r: the projection q = P p carries its bound bq, alpha = gamma/|q|^2 a
    relative error of at most 2 sum |q| bq / |q|^2 + 4u, and each update a
    rounding of u times its operands."""
    q = OCT.project(og, ang, st.p)
    bq = fwd_bound(og, ang, st.p)
    qq = OCT._pdot(q, q)
    alpha = st.gamma / qq
    ra = 2 * OCT._pdot(np.abs(q), bq) / qq + 4 * U32
    ex = lambda a: a.reshape((-1,) + (1,) * 3)
    bx = ex(ra * alpha) * np.abs(st.p) + U32 * (np.abs(st.x) + ex(alpha) * np.abs(st.p))
    br = ex(ra * alpha) * np.abs(q) + ex(alpha) * bq + U32 * (np.abs(st.r) + ex(alpha) * np.abs(q))
    return bx, br


def test_cgls_steps_match_the_oracle_step_by_step():
    """CGLS (P1) on the GPU: after the initialisation and each of four
    iterations, x and r against the oracle's iteration from the GPU's
    previous state, gamma against |P^T r|^2 of the GPU's r."""
    nx = ny = nz = 16
    geo, og, ang, at = setup(nx, ny, nz, 32, 24, 6, 2, 60.0, 96.0, 1.1, 1.1, seed=3)
    rng = np.random.default_rng(4)
    y = rng.uniform(0.0, 10.0, size=og.proj_shape).astype(np.float32).astype(np.float64)
    x0 = rng.uniform(0.0, 0.1, size=og.vol_shape).astype(np.float32).astype(np.float64)
    yt = torch.from_numpy(y.astype(np.float32)).to(device())
    xt = torch.from_numpy(x0.astype(np.float32)).to(device())
    cg = tnlm.ct.CGLS(yt, xt, geo, at)
    r, p, gam = cg.state()
    torch.cuda.synchronize()
    # initialisation: r = y - P x0, p = P^T r, gamma = |p|^2
    ref = OCT.cgls_init(og, ang, y, x0)
    assert_close(host(r), ref.r, "cgls r0", fwd_bound(og, ang, x0) + U32 * np.abs(y))
    for k in range(4):
        st = OCT.CGLSState(x=host(xt).copy(), r=host(r).copy(), p=host(p).copy(),
                           gamma=gam.cpu().numpy().copy())
        say(f"cgls step {k}")
        cg.step(1)
        r, p, gam = cg.state()  # gamma is read out as a copy
        torch.cuda.synchronize()
        nxt = OCT.cgls_step(og, ang, st)
        bx, br = _cgls_bounds(og, ang, st)
        assert_close(host(xt), nxt.x, f"cgls x{k + 1}", bx)
        assert_close(host(r), nxt.r, f"cgls r{k + 1}", br)
        s = OCT.backproject(og, ang, host(r))
        g2 = OCT._pdot(s, s)
        bs = bwd_bound(og, ang, host(r))
        gtol = 2 * OCT._pdot(np.abs(s), bs) / g2 + 4 * U32
        got = gam.cpu().numpy()
        say(f"  gamma rel err {np.abs(got - g2) / g2} (tol {gtol})")
        assert np.all(np.abs(got - g2) <= gtol * g2)


def test_tnlm_r_driver_composes_cgls_jacobi_and_positivity():
    """TNLM-R on a 4-phase 24^3 breathing phantom from analytic projections:
    each outer iteration's g is the CGLS result from the previous f (bitwise
    the same calls made by hand), its Eq.-(8) step matches the oracle's from
    that g within the Jacobi bound, positivity holds, and the reconstruction
    error against the ground truth falls."""
    w = CTWorkload("t", 4, 24, 24, 24, 48, 36, 8, 100.0, 154.0, 1.2, 1.2, 2.5, 1.2, 0.0, 8)
    geo, og, ang, at = setup(24, 24, 24, 48, 36, 8, 4, w.sid, w.sdd, w.du, w.dv,
                             angles=ct_angles(4, 8))
    y32 = analytic_projections(w, ang).astype(np.float32)
    yt = torch.from_numpy(y32).to(device())
    truth = ct_clean_volumes(w)
    f0 = torch.zeros(og.vol_shape, dtype=torch.float32, device=device())
    mu, d, M, h = 0.5, 1, 1, 0.05
    stages = []
    f = tnlm.ct.reconstruct(yt, geo, at, f0, mu=mu, d=d, M=M, h=h, outer=3, cg_iters=4,
                            step_hook=lambda k, g, ff: stages.append((g.clone(), ff.clone())))
    torch.cuda.synchronize()
    prev = f0
    errs = []
    for k, (g, ff) in enumerate(stages):
        again = prev.clone()
        tnlm.ct.CGLS(yt, again, geo, at).step(4)
        torch.cuda.synchronize()
        assert torch.equal(again, g), k
        g64 = host(g)
        ref = np.maximum(O.jacobi(g64, g64, g64, mu, d, M, h), 0.0)
        assert_close(host(ff), ref, f"TNLM-R f{k + 1}", Bounds(g64, g64, d, M, h).jacobi(mu))
        assert float(ff.min()) >= 0.0
        errs.append(float(np.sqrt(np.mean((host(ff) - truth) ** 2))))
        prev = ff
    say(f"  rms error against the truth per outer iteration: {errs}")
    assert errs[-1] < errs[0]
    assert torch.equal(f, stages[-1][1])


def test_recon128_at_full_size_on_sampled_projections():
    """The recon128 workload at full size, in the launch configuration the
    benchmark times (10 x 128^3 voxels, 10 x 30 projections of 512 x 512):
    every ray of two of the 300 projections against the oracle, and the
    transpose of a projection stack that is zero except at those two
    projections against the oracle's transpose of them over every voxel of
    their phases (the other phases must come out exactly zero)."""
    from phantom.breathing import CT_WORKLOADS
    w = CT_WORKLOADS["recon128"]
    a32 = np.ascontiguousarray(ct_angles(w.np_, w.na), dtype=np.float32)
    at = torch.from_numpy(a32).to(device())
    geo = tnlm.ct.Geometry(w.nu, w.nv, w.sid, w.sdd, w.du, w.dv)
    og = OCT.CTGeom(1, w.nx, w.ny, w.nz, w.nu, w.nv, 1, w.sid, w.sdd, w.du, w.dv)
    shape = (w.np_, w.nx, w.ny, w.nz)
    rng = np.random.default_rng(11)
    x = rng.uniform(0.0, 1.0, size=shape).astype(np.float32)
    say("recon128 projector, full size")
    p = tnlm.ct.project(torch.from_numpy(x).to(device()), geo, at)
    picks = [(0, 7), (6, 22)]  # (phase, angle index within the phase)
    for i, a in picks:
        sel = a32[i:i + 1, a:a + 1].astype(np.float64)
        xi = x[i:i + 1].astype(np.float64)
        ref, bnd = OCT.project(og, sel, xi), fwd_bound(og, sel, xi)
        got = host(p[i:i + 1, a:a + 1])
        assert_close(got, ref, f"recon128 P x, phase {i} angle {a}", bnd)
        assert_within(got, ref, bnd, f"recon128 P x, phase {i} angle {a}")
    say("recon128 transpose, full size")
    y = torch.zeros((w.np_, w.na, w.nu, w.nv), dtype=torch.float32, device=device())
    ys = {}
    for i, a in picks:
        ys[i] = rng.normal(0.0, 1.0, size=(1, 1, w.nu, w.nv)).astype(np.float32)
        y[i, a] = torch.from_numpy(ys[i][0, 0]).to(device())
    b = host(tnlm.ct.backproject(y, geo, at, shape))
    for i, a in picks:
        sel = a32[i:i + 1, a:a + 1].astype(np.float64)
        yi = ys[i].astype(np.float64)
        ref, bnd = OCT.backproject(og, sel, yi), bwd_bound(og, sel, yi)
        assert_close(b[i:i + 1], ref, f"recon128 P^T y, phase {i} angle {a}", bnd)
        assert_within(b[i:i + 1], ref, bnd, f"recon128 P^T y, phase {i} angle {a}")
    others = [k for k in range(w.np_) if k not in dict(picks)]
    assert np.all(b[others] == 0.0)


def test_tnlm_r_outer_iteration_replays_bitwise_from_a_hip_graph():
    """The reconstruction calls allocate, clear and synchronise nothing
    either (CGLS keeps its scalars on the device), so a whole TNLM-R outer
    iteration (CGLS initialisation, three CGLS iterations, the Eq. (8) step,
    positivity) can be captured in a HIP graph: three replays on new
    projections, with eager runs between them, are each bitwise equal to the
    same calls run eagerly."""
    nx, ny, nz, nu, nv, na, np_, sid, sdd, du, dv = GEOMS[1]
    geo, og, _, at = setup(nx, ny, nz, nu, nv, na, np_, sid, sdd, du, dv, seed=5)
    say(f"TNLM-R graph capture {GEOMS[1][:7]}")
    rng = np.random.default_rng(6)
    new_y = lambda: torch.from_numpy(
        rng.uniform(0.0, 1.0, size=og.proj_shape).astype(np.float32)).to(device())
    y = new_y()
    f0 = torch.from_numpy(rng.uniform(0.0, 0.5, size=og.vol_shape).astype(np.float32)).to(device())
    kw = dict(mu=0.5, d=1, M=1, h=0.1, outer=1, cg_iters=3)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        tnlm.ct.reconstruct(y, geo, at, f0, **kw)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        f_cap = tnlm.ct.reconstruct(y, geo, at, f0, **kw)
    for r in range(3):
        y.copy_(new_y())
        graph.replay()
        torch.cuda.synchronize()
        got = f_cap.clone()
        ref = tnlm.ct.reconstruct(y, geo, at, f0, **kw)
        torch.cuda.synchronize()
        assert torch.isfinite(ref).all()
        assert torch.equal(got.view(torch.int32), ref.view(torch.int32)), f"replay {r}"
    del graph
