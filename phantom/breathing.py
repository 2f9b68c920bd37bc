"""Seeded synthetic 4D breathing phantoms and random test volumes.

This module only draws inputs. It holds none of the TNLM arithmetic (no patch
distances, weights, updates, energies or gradients), so that the FP64 oracle
and the HIP path can both take their inputs from it without sharing any of the
method's code.

The paper evaluates on an NCAT digital phantom and on one patient scan
(Sec. 2.5), neither of which is available. The phantoms below stand in for
them: a cyclic stack of `Np` respiratory phases (Sec. 2.1, periodic in phase),
with a lesion that moves along z from phase to phase, plus i.i.d. Gaussian
noise and phase-dependent radial streaks that mimic FDK under-sampling
artefacts, which do not repeat across phases (Sec. 2.2).

Layout everywhere: float64 array of shape (Np, Nx, Ny, Nz), z fastest.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ----------------------------------------------------------------------------
# Workload presets: phantom shape + TNLM parameters for each benchmark workload.
# d is the patch radius (patch (2d+1)^3), M the search radius (window
# (2M+1)^3), h the similarity scale and mu the fidelity weight.
# ----------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    np_: int
    nx: int
    ny: int
    nz: int
    d: int
    M: int
    h: float
    mu: float | None
    lesion_r: float
    amp: float
    sigma: float
    streaks: bool
    iters: int
    recompute_every: int | None
    seed: int
    storage: str
    what: str

    @property
    def shape(self):
        return (self.np_, self.nx, self.ny, self.nz)

    @property
    def nvox(self):
        return self.np_ * self.nx * self.ny * self.nz


WORKLOADS = {
    # small enhancement case: weights from the input volume g for every step
    "enh32": Workload("enh32", 10, 32, 32, 16, 1, 2, 0.05, 1.0, 3.0, 2.0, 0.02,
                      False, 5, None, 1201 + 0, "f32",
                      "TNLM enhancement, 10x32x32x16, patch 3^3, window 5^3, "
                      "h=0.05, mu=1, weights from g, 5 Gauss-Jacobi steps"),
    # clinical-size enhancement: weight source u <- f every 5 steps
    "enh256": Workload("enh256", 10, 256, 256, 128, 1, 3, 0.04, 0.5, 12.0, 6.0,
                       0.02, True, 20, 5, 1201 + 1, "f32",
                       "TNLM enhancement, 10x256x256x128, patch 3^3, window "
                       "7^3, h=0.04, mu=0.5, 20 Gauss-Jacobi steps, weights "
                       "recomputed every 5"),
    # differentiable energy case
    "energy128": Workload("energy128", 10, 128, 128, 64, 1, 2, 0.05, None, 12.0,
                          6.0, 0.02, True, 1, None, 1201 + 2, "f32",
                          "TNLM energy + exact adjoint, 10x128x128x64, patch "
                          "3^3, window 5^3, h=0.05"),
    # clinical size in 16-bit storage
    "enh256_bf16": Workload("enh256_bf16", 10, 256, 256, 128, 1, 3, 0.04, 0.5,
                            12.0, 6.0, 0.02, True, 20, 5, 1201 + 3, "bf16",
                            "enh256 volumes stored in BF16 (and FP16), FP32 "
                            "arithmetic, 20 steps + energy + gradient"),
    # large regulariser descent
    "fbs512": Workload("fbs512", 20, 512, 512, 128, 1, 4, 0.04, None, 20.0,
                       10.0, 0.03, True, 10, None, 1201 + 4, "f16",
                       "forward-backward regulariser, 20x512x512x128, FP16 "
                       "storage, patch 3^3, window 9^3, h=0.04, 10 steps of "
                       "f <- f - 0.1 grad E"),
}


def _axis(n):
    return np.arange(n, dtype=np.float64)


def clean_phase(nx, ny, nz, i, np_, lesion_r, amp):
    """Noise-free phase i: torso, two lungs and a lesion moving along z.

    Voxel centres sit at integer coordinates; the body is centred at
    c = (N-1)/2 on each axis. Priority when shapes overlap: lesion > lung >
    torso. Background is 0.
    """
    cx, cy, cz = (nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0
    X = _axis(nx)[:, None, None]
    Y = _axis(ny)[None, :, None]
    Z = _axis(nz)[None, None, :]
    vol = np.zeros((nx, ny, nz), dtype=np.float64)

    def ellipsoid(ox, oy, oz, ax, ay, az):
        return (((X - ox) / ax) ** 2 + ((Y - oy) / ay) ** 2
                + ((Z - oz) / az) ** 2) <= 1.0

    torso = ellipsoid(cx, cy, cz, 0.45 * nx, 0.35 * ny, 0.45 * nz)
    vol[torso] = 0.2
    for sgn in (+1.0, -1.0):
        lung = ellipsoid(cx + sgn * 0.2 * nx, cy, cz, 0.14 * nx, 0.2 * ny,
                         0.35 * nz)
        vol[lung] = 0.02
    lz = cz + amp * math.sin(2.0 * math.pi * i / np_)
    lesion = ellipsoid(cx + 0.2 * nx, cy, lz, lesion_r, lesion_r, lesion_r)
    vol[lesion] = 0.25
    return vol


def streak_field(nx, ny, rng, n_angles=60, amplitude=0.03, width=0.75,
                 ramp=8.0):
    """Radial streaks through the axial centre, constant along z.

    n_angles lines through the in-plane centre at angles theta_k ~ U[0, pi),
    each with a random sign; a Gaussian profile of std `width` voxels across
    the line, damped within `ramp` voxels of the centre.
    """
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    X = _axis(nx)[:, None] - cx
    Y = _axis(ny)[None, :] - cy
    rho = np.sqrt(X * X + Y * Y)
    theta = rng.uniform(0.0, math.pi, size=n_angles)
    signs = rng.choice(np.array([-1.0, 1.0]), size=n_angles)
    field = np.zeros((nx, ny), dtype=np.float64)
    for t, s in zip(theta, signs):
        # distance to the line through the centre with direction (cos t, sin t)
        dist = np.abs(-math.sin(t) * X + math.cos(t) * Y)
        field += amplitude * s * np.exp(-dist * dist / (2.0 * width * width))
    field *= np.minimum(1.0, rho / ramp)
    return field


def breathing_phantom(np_, nx, ny, nz, lesion_r=3.0, amp=2.0, sigma=0.02,
                      streaks=False, seed=1201, out_dtype=np.float64):
    """FDK-like noisy input g and its clean ground truth.

    Draw order (phase by phase, one PCG64 stream): Gaussian noise of the
    whole phase volume, then (if streaks) 60 angles and 60 signs.
    Returns (noisy, clean), both (Np, Nx, Ny, Nz) in `out_dtype`, rounded
    to nearest from float64.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    noisy = np.empty((np_, nx, ny, nz), dtype=out_dtype)
    clean = np.empty((np_, nx, ny, nz), dtype=out_dtype)
    for i in range(np_):
        c = clean_phase(nx, ny, nz, i, np_, lesion_r, amp)
        g = c + rng.normal(0.0, sigma, size=c.shape)
        if streaks:
            g += streak_field(nx, ny, rng)[:, :, None]
        noisy[i] = g
        clean[i] = c
    return noisy, clean


def workload_inputs(w: Workload, out_dtype=np.float64):
    """(noisy, clean) volumes of a workload preset."""
    return breathing_phantom(w.np_, w.nx, w.ny, w.nz, lesion_r=w.lesion_r,
                             amp=w.amp, sigma=w.sigma, streaks=w.streaks,
                             seed=w.seed, out_dtype=out_dtype)


def scaled_phantom(shape, seed, sigma=0.02, streaks=True):
    """Phantom of an arbitrary shape, lesion and motion scaled to the grid."""
    np_, nx, ny, nz = shape
    r = max(1.0, 0.1 * min(nx, ny, nz))
    amp = max(1.0, 0.05 * nz)
    return breathing_phantom(np_, nx, ny, nz, lesion_r=r, amp=amp,
                             sigma=sigma, streaks=streaks, seed=seed)[0]


def random_volumes(shape, seed, kind="uniform", scale=1.0):
    """Seeded random test volumes (float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if kind == "uniform":
        return rng.uniform(0.0, scale, size=shape)
    if kind == "normal":
        return rng.normal(0.0, scale, size=shape)
    raise ValueError(kind)


# ----------------------------------------------------------------------------
# Storage casts (round to nearest even), kept here so both sides see the same
# quantised values. These are plain number-format conversions.
# ----------------------------------------------------------------------------


def to_bf16_bits(x):
    """float -> bfloat16 bit patterns (uint16), round to nearest even."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16).astype(np.uint16)
    r[nan] = 0x7FC0
    return r


def bf16_bits_to_f32(bits):
    b = np.ascontiguousarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32)


def quantise(x, storage):
    """Values of x after storage in `storage` ('f32', 'bf16', 'f16'), as
    float64, plus the raw storage array."""
    if storage == "f32":
        raw = np.ascontiguousarray(x, dtype=np.float32)
        return raw.astype(np.float64), raw
    if storage == "f16":
        raw = np.ascontiguousarray(np.asarray(x, dtype=np.float32),
                                   dtype=np.float16)
        return raw.astype(np.float64), raw
    if storage == "bf16":
        raw = to_bf16_bits(x)
        return bf16_bits_to_f32(raw).astype(np.float64), raw
    raise ValueError(storage)


# ----------------------------------------------------------------------------
# Cone-beam data for the reconstruction workload (Sec. 2.5, scaled): the
# breathing phantom's projections taken analytically from its ellipsoids, so
# the data are not produced by the discrete projector that reconstructs them.
# Geometry: voxel units, isocentre at the volume centre; for gantry angle t
# the source is at sid (cos t, sin t, 0), the flat detector perpendicular to
# the central ray at sdd from the source, pixel (iu, iv) centred at
# (iu - (nu-1)/2) du along (-sin t, cos t, 0) and (iv - (nv-1)/2) dv along z.
# ----------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class CTWorkload:
    name: str
    np_: int
    nx: int
    ny: int
    nz: int
    nu: int
    nv: int
    na: int          # angles per phase
    sid: float
    sdd: float
    du: float
    dv: float
    lesion_r: float
    amp: float
    noise: float     # relative Gaussian noise of the projections
    seed: int


CT_WORKLOADS = {
    # 10 phases of 64^3 voxels; 300 projections over 360 degrees binned into
    # 10 phases (30 each, interleaved); source-isocentre and source-detector
    # distances in the ratio 100 : 153.6 of the paper's geometry
    "recon64": CTWorkload("recon64", 10, 64, 64, 64, 128, 96, 30, 250.0, 384.0,
                          1.2, 1.2, 6.0, 3.0, 0.0, 1201 + 5),
    # the paper's scan at 2 mm voxels: 10 phases of 128^3, 300 projections of
    # 512 x 512 pixels (0.8 mm = 0.4 voxel pitch) over 360 degrees, source at
    # 100 cm (500 voxels) from the isocentre and 153.6 cm (768) from the
    # detector
    "recon128": CTWorkload("recon128", 10, 128, 128, 128, 512, 512, 30, 500.0, 768.0,
                           0.4, 0.4, 12.0, 6.0, 0.0, 1201 + 6),
}


def ct_angles(np_, na, total=None):
    """Gantry angles (np_, na): `total` = np_ * na projections equally spaced
    over 360 degrees, projection k going to phase k mod np_ (a regular
    breathing pattern sampled at a constant rate)."""
    total = np_ * na if total is None else total
    k = np.arange(np_ * na).reshape(na, np_).T  # phase i: k = i, i + np_, ...
    return 2.0 * math.pi * k / total


def _ray_ellipsoid_chord(S, D, centre, axes):
    """Chord length of the lines S + t D (arrays (..., 3)) through an
    ellipsoid."""
    q = (S - centre) / axes
    e = D / axes
    A = np.sum(e * e, axis=-1)
    B = 2.0 * np.sum(q * e, axis=-1)
    C = np.sum(q * q, axis=-1) - 1.0
    disc = B * B - 4.0 * A * C
    dt = np.sqrt(np.maximum(disc, 0.0)) / A
    return np.where(disc > 0.0, dt * np.linalg.norm(D, axis=-1), 0.0)


def analytic_projections(w: CTWorkload, angles=None):
    """Line integrals of the clean phantom of every phase along every ray,
    from the ellipsoids themselves: torso 0.2, lungs 0.02 inside it, lesion
    0.25 inside the +x lung, so the image is 0.2 T - 0.18 (L1 + L2) +
    0.23 S. Returns (np_, na, nu, nv) float64."""
    angles = ct_angles(w.np_, w.na) if angles is None else angles
    nx, ny, nz = w.nx, w.ny, w.nz
    out = np.empty((w.np_, w.na, w.nu, w.nv))
    ou = (np.arange(w.nu) - 0.5 * (w.nu - 1)) * w.du
    ov = (np.arange(w.nv) - 0.5 * (w.nv - 1)) * w.dv
    for i in range(w.np_):
        lz = w.amp * math.sin(2.0 * math.pi * i / w.np_)
        shapes = [((0.0, 0.0, 0.0), (0.45 * nx, 0.35 * ny, 0.45 * nz), 0.2),
                  ((0.2 * nx, 0.0, 0.0), (0.14 * nx, 0.2 * ny, 0.35 * nz), -0.18),
                  ((-0.2 * nx, 0.0, 0.0), (0.14 * nx, 0.2 * ny, 0.35 * nz), -0.18),
                  ((0.2 * nx, 0.0, lz), (w.lesion_r,) * 3, 0.23)]
        for a in range(w.na):
            t = angles[i, a]
            c, s = math.cos(t), math.sin(t)
            S = np.array([w.sid * c, w.sid * s, 0.0])
            P = np.empty((w.nu, w.nv, 3))
            P[..., 0] = S[0] - w.sdd * c - ou[:, None] * s
            P[..., 1] = S[1] - w.sdd * s + ou[:, None] * c
            P[..., 2] = ov[None, :]
            D = P - S
            acc = np.zeros((w.nu, w.nv))
            for centre, axes, val in shapes:
                acc += val * _ray_ellipsoid_chord(S, D, np.array(centre), np.array(axes))
            out[i, a] = acc
    if w.noise > 0:
        rng = np.random.Generator(np.random.PCG64(w.seed))
        out = out + rng.normal(0.0, w.noise, size=out.shape) * np.abs(out)
    return out


def ct_clean_volumes(w: CTWorkload):
    """The voxelised clean phantom of every phase (the reconstruction's
    ground truth), float64 (np_, nx, ny, nz)."""
    return np.stack([clean_phase(w.nx, w.ny, w.nz, i, w.np_, w.lesion_r, w.amp)
                     for i in range(w.np_)])


def ray_geometry(w, angles):
    """Source points S (np_, na, 3) and ray directions D (np_, na, nu, nv, 3)
    from the source to every pixel centre (the geometry above)."""
    ou = (np.arange(w.nu) - 0.5 * (w.nu - 1)) * w.du
    ov = (np.arange(w.nv) - 0.5 * (w.nv - 1)) * w.dv
    c, s = np.cos(angles), np.sin(angles)
    S = np.stack([w.sid * c, w.sid * s, np.zeros_like(c)], axis=-1)
    D = np.empty(angles.shape + (w.nu, w.nv, 3))
    D[..., 0] = (-w.sdd * c)[..., None, None] - ou[None, None, :, None] * s[..., None, None]
    D[..., 1] = (-w.sdd * s)[..., None, None] + ou[None, None, :, None] * c[..., None, None]
    D[..., 2] = np.broadcast_to(ov, D.shape[:-1])
    return S, D


def box_projections(w, angles, lo, hi, value=1.0):
    """value x the length of every ray inside the axis-aligned box [lo, hi]
    (voxel units, isocentre at the origin), by slab clipping."""
    S, D = ray_geometry(w, angles)
    S = S[:, :, None, None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        t0 = (np.asarray(lo) - S) / D
        t1 = (np.asarray(hi) - S) / D
    inside = (S >= np.asarray(lo)) & (S <= np.asarray(hi))
    tmin = np.where(D == 0, np.where(inside, -np.inf, np.inf), np.minimum(t0, t1))
    tmax = np.where(D == 0, np.where(inside, np.inf, -np.inf), np.maximum(t0, t1))
    tin, tout = tmin.max(axis=-1), tmax.min(axis=-1)
    return value * np.maximum(tout - tin, 0.0) * np.linalg.norm(D, axis=-1)
