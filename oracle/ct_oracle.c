/*
 * FP64 CPU oracle for the cone-beam projector of the reconstruction model.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, links or
 * loads this file; only the tests and the smoke check do. It shares no code
 * with the HIP implementation.
 *
 * The projection matrix P_i of phase i (Sec. 2.1, Eq. (1)) maps a volume to
 * line integrals along the x-ray paths of that phase's gantry angles:
 *   (P f)_r = sum_v a_{r,v} f_v,   a_{r,v} = length of ray r inside voxel v,
 * i.e. the exact line integral of the voxelised image (piecewise constant
 * over unit voxel cubes). Its transpose is
 *   (P^T y)_v = sum_r a_{r,v} y_r.
 *
 * Geometry (circular cone beam, Sec. 2.5; all lengths in voxel units).
 * Voxel (x, y, z) is the unit cube centred at (x - cx, y - cy, z - cz),
 * c = ((nx-1)/2, (ny-1)/2, (nz-1)/2), so the isocentre is the volume centre.
 * For gantry angle t the source sits at S = sid (cos t, sin t, 0) and the
 * flat detector is perpendicular to the central ray at distance sdd from the
 * source; pixel (iu, iv) is centred at
 *   S + sdd (-cos t, -sin t, 0) + (iu - (nu-1)/2) du e_u + (iv - (nv-1)/2) dv e_v,
 * e_u = (-sin t, cos t, 0), e_v = (0, 0, 1). Ray r of (phase, angle, iu, iv)
 * is the line through S and that pixel centre. Projections are laid out
 * [np][na][nu][nv] (v fastest), angles [np][na] in radians.
 *
 * Here every a_{r,v} is evaluated by clipping the ray against the cube of
 * voxel v (entry and exit parameters along each axis): for each x-slab the
 * ray crosses, the voxels of that slab its y and z ranges touch are
 * candidates, and each candidate's length is computed from its own cube.
 *
 * A ray parallel to an axis and lying exactly in a plane between two voxel
 * layers touches both closed cubes; it is counted in one of them, so that
 * the lengths of every ray partition its chord through the volume: along
 * such an axis a voxel's cube is taken half-open, [lo, hi), except that the
 * last voxel keeps its outer face (the grid's own box is closed).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t np, nx, ny, nz, nu, nv, na;
    double sid, sdd, du, dv;
} ctgeom;

typedef struct {
    double S[3], d[3]; /* ray: X(t) = S + t d, t in [0, 1] reaches the pixel */
} ray3;

static ray3 make_ray(const ctgeom *g, double th, int64_t iu, int64_t iv)
{
    ray3 r;
    const double c = cos(th), s = sin(th);
    r.S[0] = g->sid * c;
    r.S[1] = g->sid * s;
    r.S[2] = 0.0;
    const double ou = (iu - 0.5 * (g->nu - 1)) * g->du;
    const double ov = (iv - 0.5 * (g->nv - 1)) * g->dv;
    const double P[3] = {r.S[0] - g->sdd * c - ou * s, r.S[1] - g->sdd * s + ou * c, ov};
    for (int k = 0; k < 3; ++k)
        r.d[k] = P[k] - r.S[k];
    return r;
}

/* Parameter interval where the ray lies inside [lo, hi] along axis k. */
static int axis_interval(const ray3 *r, int k, double lo, double hi, double *t0, double *t1)
{
    if (r->d[k] == 0.0) {
        if (r->S[k] < lo || r->S[k] > hi)
            return 0;
        *t0 = -INFINITY;
        *t1 = INFINITY;
        return 1;
    }
    double a = (lo - r->S[k]) / r->d[k], b = (hi - r->S[k]) / r->d[k];
    *t0 = a < b ? a : b;
    *t1 = a < b ? b : a;
    return 1;
}

/* Length of the ray inside the unit cube of voxel (ix, iy, iz). */
static double voxel_length(const ctgeom *g, const ray3 *r, int64_t ix, int64_t iy, int64_t iz)
{
    const double cen[3] = {ix - 0.5 * (g->nx - 1), iy - 0.5 * (g->ny - 1), iz - 0.5 * (g->nz - 1)};
    const int64_t idx[3] = {ix, iy, iz}, n[3] = {g->nx, g->ny, g->nz};
    /* a ray in the face plane between two voxels belongs to the upper one */
    for (int k = 0; k < 3; ++k)
        if (r->d[k] == 0.0 && r->S[k] == cen[k] + 0.5 && idx[k] < n[k] - 1)
            return 0.0;
    double tin = -INFINITY, tout = INFINITY;
    for (int k = 0; k < 3; ++k) {
        double a, b;
        if (!axis_interval(r, k, cen[k] - 0.5, cen[k] + 0.5, &a, &b))
            return 0.0;
        if (a > tin)
            tin = a;
        if (b < tout)
            tout = b;
    }
    if (tout <= tin)
        return 0.0;
    const double L = sqrt(r->d[0] * r->d[0] + r->d[1] * r->d[1] + r->d[2] * r->d[2]);
    return (tout - tin) * L;
}

static int64_t clampl(int64_t a, int64_t lo, int64_t hi)
{
    return a < lo ? lo : (a > hi ? hi : a);
}

/* Calls fn(ctx, voxel flat index within the phase, length) for every voxel
 * the ray passes through with a positive length, in x-slab order. */
typedef void (*visit_fn)(void *ctx, int64_t v, double len);

static void ray_voxels(const ctgeom *g, const ray3 *r, visit_fn fn, void *ctx)
{
    const double cx = 0.5 * (g->nx - 1), cy = 0.5 * (g->ny - 1), cz = 0.5 * (g->nz - 1);
    double t0 = -INFINITY, t1 = INFINITY;
    const double lo[3] = {-cx - 0.5, -cy - 0.5, -cz - 0.5};
    const double hi[3] = {cx + 0.5, cy + 0.5, cz + 0.5};
    for (int k = 0; k < 3; ++k) {
        double a, b;
        if (!axis_interval(r, k, lo[k], hi[k], &a, &b))
            return;
        if (a > t0)
            t0 = a;
        if (b < t1)
            t1 = b;
    }
    if (t1 <= t0)
        return;
    for (int64_t ix = 0; ix < g->nx; ++ix) {
        double a, b;
        if (!axis_interval(r, 0, ix - cx - 0.5, ix - cx + 0.5, &a, &b))
            continue;
        if (a < t0)
            a = t0;
        if (b > t1)
            b = t1;
        if (b <= a)
            continue;
        /* y and z ranges of the ray over this slab (linear in t) */
        const double ya = r->S[1] + a * r->d[1], yb = r->S[1] + b * r->d[1];
        const double za = r->S[2] + a * r->d[2], zb = r->S[2] + b * r->d[2];
        const int64_t y0 = clampl((int64_t)floor((ya < yb ? ya : yb) + cy + 0.5) - 1, 0, g->ny - 1);
        const int64_t y1 = clampl((int64_t)floor((ya < yb ? yb : ya) + cy + 0.5) + 1, 0, g->ny - 1);
        const int64_t z0 = clampl((int64_t)floor((za < zb ? za : zb) + cz + 0.5) - 1, 0, g->nz - 1);
        const int64_t z1 = clampl((int64_t)floor((za < zb ? zb : za) + cz + 0.5) + 1, 0, g->nz - 1);
        for (int64_t iy = y0; iy <= y1; ++iy)
            for (int64_t iz = z0; iz <= z1; ++iz) {
                const double len = voxel_length(g, r, ix, iy, iz);
                if (len > 0.0)
                    fn(ctx, (ix * g->ny + iy) * g->nz + iz, len);
            }
    }
}

typedef struct {
    const double *vol;
    double sum, sabs;
    int64_t count;
} fwd_ctx;

static void fwd_visit(void *c, int64_t v, double len)
{
    fwd_ctx *f = (fwd_ctx *)c;
    f->sum += len * f->vol[v];
    f->sabs += fabs(f->vol[v]);
    f->count += 1;
}

/* proj = P vol for every phase; optionally, per ray, the number of voxels
 * it passes through (cnt) and the sum of |vol| over them (sabs). */
void ctor_project(const ctgeom *g, const double *angles, const double *vol, double *proj,
                  double *cnt, double *sabs)
{
    const int64_t N = g->nx * g->ny * g->nz;
    const int64_t R = g->na * g->nu * g->nv;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < g->np * R; ++t) {
        const int64_t i = t / R, rr = t - i * R;
        const int64_t a = rr / (g->nu * g->nv), iu = (rr / g->nv) % g->nu, iv = rr % g->nv;
        const ray3 r = make_ray(g, angles[i * g->na + a], iu, iv);
        fwd_ctx c = {vol + i * N, 0.0, 0.0, 0};
        ray_voxels(g, &r, fwd_visit, &c);
        proj[t] = c.sum;
        if (cnt)
            cnt[t] = (double)c.count;
        if (sabs)
            sabs[t] = c.sabs;
    }
}

typedef struct {
    double *vol, *cnt, *sabs;
    double y;
} bwd_ctx;

static void bwd_visit(void *c, int64_t v, double len)
{
    bwd_ctx *b = (bwd_ctx *)c;
    b->vol[v] += len * b->y;
    if (b->cnt)
        b->cnt[v] += 1.0;
    if (b->sabs)
        b->sabs[v] += fabs(b->y);
}

/* vol = P^T proj for every phase (each phase's rays scatter into its own
 * volume, phases in parallel); optionally, per voxel, the number of rays
 * through it (cnt) and the sum of |proj| over them (sabs). */
void ctor_backproject(const ctgeom *g, const double *angles, const double *proj, double *vol,
                      double *cnt, double *sabs)
{
    const int64_t N = g->nx * g->ny * g->nz;
    const int64_t R = g->na * g->nu * g->nv;
    memset(vol, 0, sizeof(double) * g->np * N);
    if (cnt)
        memset(cnt, 0, sizeof(double) * g->np * N);
    if (sabs)
        memset(sabs, 0, sizeof(double) * g->np * N);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < g->np; ++i)
        for (int64_t rr = 0; rr < R; ++rr) {
            const int64_t a = rr / (g->nu * g->nv), iu = (rr / g->nv) % g->nu, iv = rr % g->nv;
            const ray3 r = make_ray(g, angles[i * g->na + a], iu, iv);
            bwd_ctx c = {vol + i * N, cnt ? cnt + i * N : NULL, sabs ? sabs + i * N : NULL,
                         proj[i * R + rr]};
            ray_voxels(g, &r, bwd_visit, &c);
        }
}

/* Length of ray (phase angle th, pixel iu, iv) inside the axis-aligned box
 * [lo, hi] (voxel units, isocentre at the origin): a closed form used by
 * the pins (a uniform box projects to value x this length). */
double ctor_box_chord(const ctgeom *g, double th, int64_t iu, int64_t iv, const double *lo,
                      const double *hi)
{
    const ray3 r = make_ray(g, th, iu, iv);
    double tin = -INFINITY, tout = INFINITY;
    for (int k = 0; k < 3; ++k) {
        double a, b;
        if (!axis_interval(&r, k, lo[k], hi[k], &a, &b))
            return 0.0;
        if (a > tin)
            tin = a;
        if (b < tout)
            tout = b;
    }
    if (tout <= tin)
        return 0.0;
    return (tout - tin) * sqrt(r.d[0] * r.d[0] + r.d[1] * r.d[1] + r.d[2] * r.d[2]);
}
