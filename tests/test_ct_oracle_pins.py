"""Pins of the reconstruction oracle (oracle/ct.py, ct_oracle.c), CPU.

  * a voxel-aligned, off-centre box projects to its exact chord lengths,
    computed independently from the geometry's definition (slab clipping in
    phantom.box_projections): pins the source side, the detector axes, the
    angle sense, the candidate enumeration and every length;
  * rays lying in a plane between two voxel layers are counted once: their
    lengths add up to the chord, like every other ray's;
  * <P x, y> = <x, P^T y> for random x, y: pins the transpose's indexing;
  * the voxelised breathing phantom's projections approach the analytic line
    integrals of its ellipsoids as the voxels shrink (first order);
  * CGLS iterate k is the minimiser of ||P x - y|| over x0 + the Krylov space
    K_k(P^T P, P^T r0), computed densely; its residual never grows;
  * TNLM-R keeps a positive constant volume with consistent data fixed, and
    its output is never negative.
"""
import numpy as np
import pytest

from oracle import ct
from phantom.breathing import (CTWorkload, analytic_projections, box_projections,
                               ct_angles, ct_clean_volumes)


def small(n=12, nu=20, nv=16, na=5, np_=2):
    s = n / 32
    w = CTWorkload("t", np_, n, n, n, nu, nv, na, 125.0 * s, 192.0 * s, 1.3 * s, 1.3 * s,
                   2.0 * s, 1.0 * s, 0.0, 7)
    g = ct.CTGeom(np_, n, n, n, nu, nv, na, w.sid, w.sdd, w.du, w.dv)
    return w, g


@pytest.mark.parametrize("shape", [(12, 12, 12), (9, 14, 7)])
def test_voxel_aligned_box_projects_to_its_chords(shape):
    nx, ny, nz = shape
    w = CTWorkload("t", 2, nx, ny, nz, 24, 18, 7, 40.0, 64.0, 1.1, 0.9, 1.0, 1.0, 0.0, 7)
    g = ct.CTGeom(2, nx, ny, nz, w.nu, w.nv, w.na, w.sid, w.sdd, w.du, w.dv)
    rng = np.random.default_rng(3)
    ang = rng.uniform(0, 2 * np.pi, size=(2, w.na))
    ang[0, 0], ang[0, 1], ang[1, 0] = 0.0, np.pi / 2, np.pi  # axis-aligned rays too
    c = np.array([(nx - 1) / 2, (ny - 1) / 2, (nz - 1) / 2])
    ix, iy, iz = (2, nx - 3), (1, 4), (nz - 4, nz - 2)   # voxel index ranges
    vol = np.zeros((2, nx, ny, nz))
    vol[:, ix[0]:ix[1] + 1, iy[0]:iy[1] + 1, iz[0]:iz[1] + 1] = 0.7
    lo = np.array([ix[0], iy[0], iz[0]]) - c - 0.5
    hi = np.array([ix[1], iy[1], iz[1]]) - c + 0.5
    want = box_projections(w, ang, lo, hi, 0.7)
    got = ct.project(g, ang, vol)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    assert (want > 0).sum() > 100  # the box is seen by many rays


def test_rays_in_voxel_face_planes_are_counted_once():
    """Rays parallel to an axis that run exactly in a plane between two
    voxel layers (the centre detector row of an even-nz grid lies in z = 0;
    at angle 0 the centre column of an even-ny grid lies in y = 0): the
    lengths of such a ray, like those of every other ray, add up to its
    chord through the volume, so a uniform volume projects to the chord
    lengths of the volume's box (a ray in a face plane is counted in one of
    the two voxel layers, not in both)."""
    nx, ny, nz, nu, nv = 8, 6, 4, 9, 7
    w = CTWorkload("t", 1, nx, ny, nz, nu, nv, 3, 30.0, 50.0, 1.5, 1.5, 1.0, 1.0, 0.0, 7)
    g = ct.CTGeom(1, nx, ny, nz, nu, nv, 3, w.sid, w.sdd, w.du, w.dv)
    ang = np.array([[0.0, 1.0, 2.5]])
    c = np.array([(nx - 1) / 2, (ny - 1) / 2, (nz - 1) / 2])
    want = box_projections(w, ang, -c - 0.5, c + 0.5, 1.0)
    got = ct.project(g, ang, np.ones(g.vol_shape))
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    # the degenerate rays are there: the centre row of every angle, the
    # centre column at angle 0
    assert (want[0, :, :, nv // 2] > 0).sum() >= 15 and want[0, 0, nu // 2, nv // 2] > 0


def test_transpose_is_the_adjoint():
    w, g = small(10, 18, 14, 6, 3)
    rng = np.random.default_rng(4)
    ang = rng.uniform(0, 2 * np.pi, size=(3, 6))
    x = rng.normal(size=g.vol_shape)
    y = rng.normal(size=g.proj_shape)
    lhs = np.vdot(ct.project(g, ang, x), y)
    rhs = np.vdot(x, ct.backproject(g, ang, y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_voxelised_phantom_converges_to_the_analytic_projections():
    errs = []
    for n in (16, 32, 64):
        s = n / 32
        w = CTWorkload("t", 1, n, n, n, 48, 36, 3, 125.0 * s, 192.0 * s, 1.6 * s,
                       1.6 * s, 3.0 * s, 1.5 * s, 0.0, 7)
        g = ct.CTGeom(1, n, n, n, w.nu, w.nv, w.na, w.sid, w.sdd, w.du, w.dv)
        ang = ct_angles(1, w.na)
        y = analytic_projections(w, ang)
        p = ct.project(g, ang, ct_clean_volumes(w))
        errs.append(np.sqrt(np.mean((p - y) ** 2) / np.mean(y ** 2)))
    # voxelising sharp edges: an error of first order in the voxel size
    assert errs[1] < 0.65 * errs[0] and errs[2] < 0.65 * errs[1], errs
    assert errs[2] < 0.05


def _dense(g, ang):
    """P as a dense matrix per phase, column by column from unit volumes."""
    N = g.nx * g.ny * g.nz
    R = g.na * g.nu * g.nv
    A = np.zeros((g.np_, R, N))
    for v in range(N):
        e = np.zeros(g.vol_shape)
        e[:, v // (g.ny * g.nz), (v // g.nz) % g.ny, v % g.nz] = 1.0
        A[:, :, v] = ct.project(g, ang, e).reshape(g.np_, R)
    return A


def test_cgls_iterates_are_the_krylov_least_squares_minimisers():
    w, g = small(5, 10, 8, 4, 2)
    ang = ct_angles(2, 4)
    rng = np.random.default_rng(5)
    y = rng.uniform(0.5, 1.5, size=g.proj_shape)
    x0 = rng.uniform(0.0, 0.2, size=g.vol_shape)
    A = _dense(g, ang)
    st = ct.cgls_init(g, ang, y, x0)
    res = [np.linalg.norm((A @ st.x.reshape(2, -1, 1))[..., 0] - y.reshape(2, -1), axis=1)]
    for k in range(1, 6):
        st = ct.cgls_step(g, ang, st)
        for i in range(2):
            Ai, bi, xi0 = A[i], y[i].ravel(), x0[i].ravel()
            r0 = bi - Ai @ xi0
            # Krylov basis of A^T A started at A^T r0, orthonormalised
            K = [Ai.T @ r0]
            for _ in range(k - 1):
                K.append(Ai.T @ (Ai @ K[-1]))
            Q, _ = np.linalg.qr(np.stack(K, axis=1))
            c, *_ = np.linalg.lstsq(Ai @ Q, r0, rcond=None)
            want = xi0 + Q @ c
            got = st.x[i].ravel()
            assert np.abs(got - want).max() <= 1e-8 * np.abs(want).max(), (k, i)
        res.append(np.linalg.norm((A @ st.x.reshape(2, -1, 1))[..., 0] - y.reshape(2, -1), axis=1))
    res = np.array(res)
    assert np.all(np.diff(res, axis=0) <= 1e-12 * res[0])


def test_tnlm_r_fixed_point_and_positivity():
    w, g = small(8, 16, 12, 4, 3)
    ang = ct_angles(3, 4)
    c = np.full(g.vol_shape, 0.3)
    y = ct.project(g, ang, c)
    f = ct.tnlm_r(g, ang, y, c, 0.5, 1, 1, 0.05, outer=2, cg_iters=3)
    assert np.abs(f - 0.3).max() <= 1e-12
    rng = np.random.default_rng(6)
    y2 = y + rng.normal(0, 0.5, size=y.shape)
    f2 = ct.tnlm_r(g, ang, y2, np.zeros(g.vol_shape), 0.5, 1, 1, 0.05, outer=2, cg_iters=3)
    assert f2.min() >= 0.0 and f2.max() > 0.0


def _f32_length(g, th, iu, iv, voxel):
    """The length of ray (th, iu, iv) in a voxel's cube evaluated with float32
    operations, the geometry formed from float32 sin and cos as a
    single-precision kernel forms it."""
    f = np.float32
    th = f(th)
    s, c = f(np.sin(np.float64(th))), f(np.cos(np.float64(th)))
    ou = f(f(iu - 0.5 * (g.nu - 1)) * f(g.du))
    ov = f(f(iv - 0.5 * (g.nv - 1)) * f(g.dv))
    S = (f(g.sid) * c, f(g.sid) * s, f(0))
    d = (f(-f(g.sdd) * c - ou * s), f(-f(g.sdd) * s + ou * c), ov)
    n = (g.nx, g.ny, g.nz)
    tin, tout = f(-np.inf), f(np.inf)
    for k in range(3):
        cen = f(voxel[k] - 0.5 * (n[k] - 1))
        if d[k] == 0:
            if not (cen - f(0.5) <= S[k] < cen + f(0.5)):
                return 0.0
            continue
        inv = f(1) / d[k]
        t0, t1 = ((cen - f(0.5)) - S[k]) * inv, ((cen + f(0.5)) - S[k]) * inv
        tin, tout = max(tin, min(t0, t1)), min(tout, max(t0, t1))
    L = f(np.sqrt(f(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])))
    return float((tout - tin) * L) if tout > tin else 0.0


def test_fp32_error_model_bounds_float32_lengths_at_shallow_crossings():
    """The per-pair FP32 error model (ct.pair_error, behind ct.error_model)
    bounds the error of a float32 evaluation of each ray-voxel length, also
    where a ray leaves a voxel through a face it is nearly parallel to: in
    the recon128 scan geometry (source 500 voxels from the isocentre) the
    rays of detector columns 49-53 at 84 degrees run almost parallel to the
    x faces near x = 52, and a float32 position error of one ulp moves their
    crossing far along the ray: errors of ~1e-3 of the length, thousands of
    times a length's own rounding, which the model's 1/|d_k| amplification
    must (and does) cover."""
    from phantom.breathing import CT_WORKLOADS
    w = CT_WORKLOADS["recon128"]
    g = ct.CTGeom(1, w.nx, w.ny, w.nz, w.nu, w.nv, 1, w.sid, w.sdd, w.du, w.dv)
    th = float(np.float32(ct_angles(w.np_, w.na)[0, 7]))
    worst_ratio, worst_rel = 0.0, 0.0
    for iu in range(49, 54):
        for iv in (300, 303, 306):
            for voxel in ((116, 32, 77), (115, 32, 77), (116, 33, 77), (117, 31, 77)):
                ln, b = ct.pair_error(g, th, iu, iv, voxel)
                if ln == 0.0:
                    continue
                err = abs(_f32_length(g, th, iu, iv, voxel) - ln)
                worst_ratio = max(worst_ratio, err / b)
                worst_rel = max(worst_rel, err / ln)
    print("largest error / bound", worst_ratio, "largest relative error", worst_rel)
    assert worst_ratio <= 1.0
    assert worst_rel >= 1e-3  # the amplified regime is reached


def test_fp32_error_model_bounds_a_float32_evaluation():
    """The first-order FP32 error model of the projector (ct.error_model)
    bounds the error of an actual float32 evaluation of the same lengths:
    every ray's sum over all voxels of (t_out - t_in) |d| |x_v|, each length
    clipped against the voxel's cube with float32 operations (geometry from
    float32 sin and cos, as a single-precision kernel forms it), against the
    FP64 oracle, element by element; a long source distance makes the
    near-parallel crossings (the model's 1/|d_k| amplification) matter."""
    n, nu, nv = 24, 40, 30
    g = ct.CTGeom(1, n, n, n, nu, nv, 3, 300.0, 460.0, 0.9, 0.9)
    # near 90 degrees the x component of the central rays' directions
    # changes sign on the detector: near-parallel x crossings
    ang = np.array([[0.3, 1.55, 1.5625]])
    x = np.random.default_rng(5).uniform(0.0, 1.0, size=g.vol_shape)
    ref = ct.project(g, ang, x)
    bound = ct.error_model(g, ang, xabs=np.abs(x))[0]
    f = np.float32
    c0 = (np.arange(n, dtype=f) - f(0.5 * (n - 1)))
    X, Y, Z = np.meshgrid(c0, c0, c0, indexing="ij")
    xv = x[0].astype(f)
    worst = 0.0
    for a in range(g.na):
        th = f(ang[0, a])
        s, c = f(np.sin(np.float64(th))), f(np.cos(np.float64(th)))
        S = (f(g.sid) * c, f(g.sid) * s, f(0))
        for iu in range(nu):
            ou = f(f(iu - 0.5 * (nu - 1)) * f(g.du))
            for iv in range(0, nv, 3):
                ov = f(f(iv - 0.5 * (nv - 1)) * f(g.dv))
                d = (f(-f(g.sdd) * c - ou * s), f(-f(g.sdd) * s + ou * c), ov)
                tin = np.full(X.shape, -np.inf, dtype=f)
                tout = np.full(X.shape, np.inf, dtype=f)
                ok = np.ones(X.shape, dtype=bool)
                for C, Sk, dk in ((X, S[0], d[0]), (Y, S[1], d[1]), (Z, S[2], d[2])):
                    if dk == 0:
                        ok &= (Sk >= C - f(0.5)) & (Sk < C + f(0.5))
                        continue
                    inv = f(1) / dk
                    t0 = ((C - f(0.5)) - Sk) * inv
                    t1 = ((C + f(0.5)) - Sk) * inv
                    tin = np.maximum(tin, np.minimum(t0, t1))
                    tout = np.minimum(tout, np.maximum(t0, t1))
                L = np.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], dtype=f)
                ln = np.where(ok & (tout > tin), (tout - tin) * L, f(0))
                got = float(np.sum(ln.astype(np.float64) * xv))
                r = abs(got - ref[0, a, iu, iv]) / bound[0, a, iu, iv]
                worst = max(worst, r)
    print("largest error / bound", worst)
    assert 0.0 < worst <= 1.0, worst
