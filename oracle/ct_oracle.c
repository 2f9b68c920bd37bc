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
    double c, s, ou;   /* cos, sin of the angle; lateral pixel offset */
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
    r.c = c;
    r.s = s;
    r.ou = ou;
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

/* Length of the ray inside the unit cube of voxel (ix, iy, iz); with
 * tio/kio non-NULL also the entry and exit parameters and the axes that set
 * them. */
static double voxel_clip(const ctgeom *g, const ray3 *r, int64_t ix, int64_t iy, int64_t iz,
                         double *tio, int *kio)
{
    const double cen[3] = {ix - 0.5 * (g->nx - 1), iy - 0.5 * (g->ny - 1), iz - 0.5 * (g->nz - 1)};
    const int64_t idx[3] = {ix, iy, iz}, n[3] = {g->nx, g->ny, g->nz};
    /* a ray in the face plane between two voxels belongs to the upper one */
    for (int k = 0; k < 3; ++k)
        if (r->d[k] == 0.0 && r->S[k] == cen[k] + 0.5 && idx[k] < n[k] - 1)
            return 0.0;
    double tin = -INFINITY, tout = INFINITY;
    int kin = -1, kout = -1;
    for (int k = 0; k < 3; ++k) {
        double a, b;
        if (!axis_interval(r, k, cen[k] - 0.5, cen[k] + 0.5, &a, &b))
            return 0.0;
        if (a > tin) {
            tin = a;
            kin = k;
        }
        if (b < tout) {
            tout = b;
            kout = k;
        }
    }
    if (tout <= tin)
        return 0.0;
    if (tio) {
        tio[0] = tin;
        tio[1] = tout;
        kio[0] = kin;
        kio[1] = kout;
    }
    const double L = sqrt(r->d[0] * r->d[0] + r->d[1] * r->d[1] + r->d[2] * r->d[2]);
    return (tout - tin) * L;
}

static int64_t clampl(int64_t a, int64_t lo, int64_t hi)
{
    return a < lo ? lo : (a > hi ? hi : a);
}

/* Calls fn(ctx, voxel flat index within the phase, length, entry and exit
 * parameters, their axes) for every voxel the ray passes through with a
 * positive length, in x-slab order. */
typedef void (*visit_fn)(void *ctx, int64_t v, double len, const double *tio, const int *kio);

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
                double tio[2];
                int kio[2];
                const double len = voxel_clip(g, r, ix, iy, iz, tio, kio);
                if (len > 0.0)
                    fn(ctx, (ix * g->ny + iy) * g->nz + iz, len, tio, kio);
            }
    }
}

typedef struct {
    const double *vol;
    double sum, sabs;
    int64_t count;
} fwd_ctx;

static void fwd_visit(void *c, int64_t v, double len, const double *tio, const int *kio)
{
    (void)tio;
    (void)kio;
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

static void bwd_visit(void *c, int64_t v, double len, const double *tio, const int *kio)
{
    (void)tio;
    (void)kio;
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

/* ---- First-order rounding-error model of an FP32 evaluation --------------
 * For test tolerances only. An FP32 evaluation of the same operator (unit
 * roundoff u = 2^-24) forms a ray's geometry and every ray-voxel length in
 * single precision:
 *   S = sid (cos t, sin t, 0),
 *   d = (-sdd cos t - ou sin t, -sdd sin t + ou cos t, ov),
 *   a plane crossing t_k = (p - S_k) / d_k, a length (t_out - t_in) |d|.
 * With sin and cos within 2 ulp (4u), the absolute errors are at most
 *   e_S = 5u sid |cos t| (x), 5u sid |sin t| (y), 0 (z),
 *   e_d = 5u sdd |cos t| + 6u |ou| |sin t| + u |d_x| (x; sin and cos
 *         swapped for y), u |ov| (z),
 * so a crossing along axis k is off by at most
 *   dt_k = (e_S_k + |t_k| e_d_k) / |d_k| + 4u |t_k|
 * (first order: dt/dS = -1/d, dt/dd = -t/d; then the subtraction, a
 * reciprocal within one ulp and the product), |d| by dL = sum_k |d_k| e_d_k / |d| + 4u |d|
 * (the sum of squares, then a square root within 1 ulp),
 * and a length by
 *   dlen = |d| (dt_in + dt_out) + (t_out - t_in) dL + 2u len.
 * A crossing nearly parallel to its planes (small |d_k|) is ill-conditioned:
 * a position error moves it far along the ray. Per ray the bound is the sum
 * over its voxels of dlen |x_v| plus n_r u sum_v len |x_v| (the n_r-term
 * sum); per voxel of the transpose the same with the rays through it.
 * xabs [np][nx][ny][nz] and yabs [np][na][nu][nv] are |x| and |y|; eproj
 * (per ray) and evol (per voxel) receive the bounds; either may be NULL. */
static double pair_error(const ctgeom *g, const ray3 *r, double len, const double *tio,
                         const int *kio)
{
    const double u = 0x1.0p-24;
    const double ac = fabs(r->c), as = fabs(r->s), aou = fabs(r->ou);
    const double eS[3] = {5 * u * g->sid * ac, 5 * u * g->sid * as, 0.0};
    const double ed[3] = {5 * u * g->sdd * ac + 6 * u * aou * as + u * fabs(r->d[0]),
                          5 * u * g->sdd * as + 6 * u * aou * ac + u * fabs(r->d[1]),
                          u * fabs(r->d[2])};
    const double L = sqrt(r->d[0] * r->d[0] + r->d[1] * r->d[1] + r->d[2] * r->d[2]);
    double dt = 0.0;
    for (int j = 0; j < 2; ++j) {
        const int k = kio[j];
        const double t = fabs(tio[j]);
        dt += (eS[k] + t * ed[k]) / fabs(r->d[k]) + 4 * u * t;
    }
    const double dL = (fabs(r->d[0]) * ed[0] + fabs(r->d[1]) * ed[1] + fabs(r->d[2]) * ed[2]) / L +
                      4 * u * L;
    return L * dt + (tio[1] - tio[0]) * dL + 2 * u * len;
}

typedef struct {
    const ctgeom *g;
    ray3 r;
    const double *xabs;
    double e, slx, n;
} efwd_ctx;

static void efwd_visit(void *c, int64_t v, double len, const double *tio, const int *kio)
{
    efwd_ctx *f = (efwd_ctx *)c;
    f->e += f->xabs[v] * pair_error(f->g, &f->r, len, tio, kio);
    f->slx += len * f->xabs[v];
    f->n += 1.0;
}

typedef struct {
    const ctgeom *g;
    ray3 r;
    double *e, *sly, *n;
    double yabs;
} ebwd_ctx;

static void ebwd_visit(void *c, int64_t v, double len, const double *tio, const int *kio)
{
    ebwd_ctx *b = (ebwd_ctx *)c;
    b->e[v] += b->yabs * pair_error(b->g, &b->r, len, tio, kio);
    b->sly[v] += len * b->yabs;
    b->n[v] += 1.0;
}

void ctor_error_model(const ctgeom *g, const double *angles, const double *xabs,
                      const double *yabs, double *eproj, double *evol)
{
    const double u = 0x1.0p-24;
    const int64_t N = g->nx * g->ny * g->nz;
    const int64_t R = g->na * g->nu * g->nv;
    if (eproj) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t t = 0; t < g->np * R; ++t) {
            const int64_t i = t / R, rr = t - i * R;
            const int64_t a = rr / (g->nu * g->nv), iu = (rr / g->nv) % g->nu, iv = rr % g->nv;
            efwd_ctx c;
            c.g = g;
            c.r = make_ray(g, angles[i * g->na + a], iu, iv);
            c.xabs = xabs + i * N;
            c.e = c.slx = c.n = 0.0;
            ray_voxels(g, &c.r, efwd_visit, &c);
            eproj[t] = c.e + c.n * u * c.slx;
        }
    }
    if (evol) {
        double *sly = (double *)calloc((size_t)(g->np * N), sizeof(double));
        double *cnt = (double *)calloc((size_t)(g->np * N), sizeof(double));
        memset(evol, 0, sizeof(double) * g->np * N);
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t i = 0; i < g->np; ++i)
            for (int64_t rr = 0; rr < R; ++rr) {
                const int64_t a = rr / (g->nu * g->nv), iu = (rr / g->nv) % g->nu, iv = rr % g->nv;
                ebwd_ctx c;
                c.g = g;
                c.e = evol + i * N;
                c.sly = sly + i * N;
                c.n = cnt + i * N;
                c.yabs = yabs[i * R + rr];
                c.r = make_ray(g, angles[i * g->na + a], iu, iv);
                ray_voxels(g, &c.r, ebwd_visit, &c);
            }
        for (int64_t v = 0; v < g->np * N; ++v)
            evol[v] += cnt[v] * u * sly[v];
        free(sly);
        free(cnt);
    }
}

/* One pair of the model: the exact length of ray (th, iu, iv) in voxel
 * (ix, iy, iz) in *len, and its FP32 error bound dlen as the return value
 * (0 where the length is 0). */
double ctor_pair_error(const ctgeom *g, double th, int64_t iu, int64_t iv, int64_t ix,
                       int64_t iy, int64_t iz, double *len)
{
    const ray3 r = make_ray(g, th, iu, iv);
    double tio[2];
    int kio[2];
    *len = voxel_clip(g, &r, ix, iy, iz, tio, kio);
    return *len > 0.0 ? pair_error(g, &r, *len, tio, kio) : 0.0;
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
