/*
 * FP64 CPU oracle for the temporal non-local means (TNLM) operator.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the CPU baseline leg
 * of the benchmark do. It shares no code, header, table or constant with the
 * HIP implementation.
 *
 * Everything is the plain definition, evaluated in double precision with
 * direct loops: the (2d+1)^3 patch sum is summed term by term (no box sums),
 * normalisers are taken in two passes (maximum, then sum of shifted
 * exponentials), and nothing is tiled, fused or reordered.
 *
 * Notation (paper Sec. 2): Np cyclic phases f_i (Sec. 2.1, f_{Np+1} = f_1);
 * weights of Eq. (3) estimated from the latest images u (Eq. (9)); patch
 * radius d and search radius M (Sec. 2.4); similarity scale h (Eq. (3));
 * fidelity weight mu (Eqs. (1), (4)).
 *
 * Readings taken where the paper is silent or ambiguous (each is listed in
 * the design notes of the repository):
 *   - The normaliser Z of Eq. (3) is taken per voxel x over its search
 *     window, separately for the neighbour phases i+1 and i-1, so that the
 *     bracket of Eq. (8) is a weighted average (Sec. 2.3, Eqs. (7)-(8)).
 *   - The patch distance is the unweighted sum of squared differences over
 *     the (2d+1)^3 cube (Eq. (3)), with exponent -D/(2h^2).
 *   - The window is the (2M+1)^3 cube of offsets around the same
 *     coordinates in the neighbour phase (Sec. 2.4); candidates outside the
 *     grid are dropped (window truncated at the borders); patch voxels
 *     outside the grid take the value of the nearest voxel of the same phase
 *     (clamp to edge, per axis).
 *   - The energy is the symmetrised TNLM energy
 *       E(f; u) = 1/4 sum_i sum_{s=+-1} sum_v sum_{delta in V(v)}
 *                 w_{i->i+s}(v, delta; u) (f_i(v) - f_{i+s}(v+delta))^2,
 *     i.e. 1/2 sum_i J[f_i, f_{i+1}] of Eqs. (1)/(4) with the two
 *     direction-normalised weights of each link averaged.
 *   - Phase indices are taken modulo Np; Np >= 2 (no intra-phase term,
 *     Sec. 2.2).
 *
 * Layout: vol[i][x][y][z], index ((i*nx + x)*ny + y)*nz + z, z fastest.
 * Direction slot 0 is the neighbour i+1, slot 1 the neighbour i-1.
 * Offset index k = ((dx+M)*(2M+1) + (dy+M))*(2M+1) + (dz+M).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t np, nx, ny, nz; /* phases and grid */
    int64_t d, M;           /* patch radius, search radius */
    double h;               /* similarity scale */
} ogeom;

static int64_t clampi(int64_t a, int64_t lo, int64_t hi)
{
    return a < lo ? lo : (a > hi ? hi : a);
}

static int64_t phase_of(const ogeom *g, int64_t i)
{
    return ((i % g->np) + g->np) % g->np;
}

static int64_t nvox_phase(const ogeom *g)
{
    return g->nx * g->ny * g->nz;
}

static int64_t vidx(const ogeom *g, int64_t i, int64_t x, int64_t y, int64_t z)
{
    return ((i * g->nx + x) * g->ny + y) * g->nz + z;
}

/* Value of phase i at a possibly out-of-grid position: clamp to edge. */
static double ext(const ogeom *g, const double *u, int64_t i, int64_t x,
                  int64_t y, int64_t z)
{
    x = clampi(x, 0, g->nx - 1);
    y = clampi(y, 0, g->ny - 1);
    z = clampi(z, 0, g->nz - 1);
    return u[vidx(g, i, x, y, z)];
}

static int inside(const ogeom *g, int64_t x, int64_t y, int64_t z)
{
    return x >= 0 && x < g->nx && y >= 0 && y < g->ny && z >= 0 && z < g->nz;
}

/* Patch distance of Eq. (3): squared l2 distance between the (2d+1)^3 cube
 * of phase i around (x,y,z) and that of phase j around (x,y,z)+(ox,oy,oz). */
static double patch_dist(const ogeom *g, const double *u, int64_t i, int64_t j,
                         int64_t x, int64_t y, int64_t z, int64_t ox,
                         int64_t oy, int64_t oz)
{
    double s = 0.0;
    for (int64_t px = -g->d; px <= g->d; ++px)
        for (int64_t py = -g->d; py <= g->d; ++py)
            for (int64_t pz = -g->d; pz <= g->d; ++pz) {
                double a = ext(g, u, i, x + px, y + py, z + pz);
                double b = ext(g, u, j, x + ox + px, y + oy + py, z + oz + pz);
                s += (a - b) * (a - b);
            }
    return s;
}

/* Normaliser of voxel (i, x, y, z) towards neighbour phase j (Eq. (3) with
 * the per-voxel reading): returns log sum_{delta valid} exp(-D/(2h^2)),
 * taken in two passes (maximum exponent first). */
static double log_normaliser(const ogeom *g, const double *u, int64_t i,
                             int64_t j, int64_t x, int64_t y, int64_t z)
{
    const double inv2h2 = 1.0 / (2.0 * g->h * g->h);
    double amax = -INFINITY;
    for (int64_t ox = -g->M; ox <= g->M; ++ox)
        for (int64_t oy = -g->M; oy <= g->M; ++oy)
            for (int64_t oz = -g->M; oz <= g->M; ++oz) {
                if (!inside(g, x + ox, y + oy, z + oz))
                    continue;
                double a = -patch_dist(g, u, i, j, x, y, z, ox, oy, oz) * inv2h2;
                if (a > amax)
                    amax = a;
            }
    double Z = 0.0;
    for (int64_t ox = -g->M; ox <= g->M; ++ox)
        for (int64_t oy = -g->M; oy <= g->M; ++oy)
            for (int64_t oz = -g->M; oz <= g->M; ++oz) {
                if (!inside(g, x + ox, y + oy, z + oz))
                    continue;
                double a = -patch_dist(g, u, i, j, x, y, z, ox, oy, oz) * inv2h2;
                Z += exp(a - amax);
            }
    return amax + log(Z);
}

/* Weight w_{i->j}((x,y,z), delta) given the log-normaliser of that voxel. */
static double weight(const ogeom *g, const double *u, int64_t i, int64_t j,
                     int64_t x, int64_t y, int64_t z, int64_t ox, int64_t oy,
                     int64_t oz, double lse)
{
    const double inv2h2 = 1.0 / (2.0 * g->h * g->h);
    double a = -patch_dist(g, u, i, j, x, y, z, ox, oy, oz) * inv2h2;
    return exp(a - lse);
}

static int64_t neighbour(const ogeom *g, int64_t i, int slot)
{
    return phase_of(g, slot == 0 ? i + 1 : i - 1);
}

static void unflatten(const ogeom *g, int64_t flat, int64_t *i, int64_t *x,
                      int64_t *y, int64_t *z)
{
    *z = flat % g->nz;
    flat /= g->nz;
    *y = flat % g->ny;
    flat /= g->ny;
    *x = flat % g->nx;
    *i = flat / g->nx;
}

/* Per-voxel local sums for direction slot s at (i,x,y,z):
 *   lse = log Z,  nb = sum_delta w f_j(v+delta),  e = sum_delta w r^2. */
static void local_sums(const ogeom *g, const double *u, const double *f,
                       int64_t i, int slot, int64_t x, int64_t y, int64_t z,
                       double *lse_out, double *nb_out, double *e_out)
{
    int64_t j = neighbour(g, i, slot);
    double lse = log_normaliser(g, u, i, j, x, y, z);
    double nb = 0.0, e = 0.0;
    double fi = f ? f[vidx(g, i, x, y, z)] : 0.0;
    for (int64_t ox = -g->M; ox <= g->M; ++ox)
        for (int64_t oy = -g->M; oy <= g->M; ++oy)
            for (int64_t oz = -g->M; oz <= g->M; ++oz) {
                if (!inside(g, x + ox, y + oy, z + oz))
                    continue;
                double w = weight(g, u, i, j, x, y, z, ox, oy, oz, lse);
                if (f) {
                    double fj = f[vidx(g, j, x + ox, y + oy, z + oz)];
                    nb += w * fj;
                    e += w * (fi - fj) * (fi - fj);
                }
            }
    if (lse_out)
        *lse_out = lse;
    if (nb_out)
        *nb_out = nb;
    if (e_out)
        *e_out = e;
}

/* ------------------------------------------------------------------------ */
/* Weights (Eqs. (3), (9)) and per-voxel log-normalisers.                  */
/* w: [np][2][W][N] (nullable), lse: [np][2][N] (nullable).                 */
/* ------------------------------------------------------------------------ */
void tnlmo_weights(const ogeom *g, const double *u, double *w, double *lse)
{
    const int64_t N = nvox_phase(g);
    const int64_t S = 2 * g->M + 1, W = S * S * S;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t flat = 0; flat < g->np * N; ++flat) {
        int64_t i, x, y, z;
        unflatten(g, flat, &i, &x, &y, &z);
        int64_t v = flat - i * N;
        for (int slot = 0; slot < 2; ++slot) {
            int64_t j = neighbour(g, i, slot);
            double l = log_normaliser(g, u, i, j, x, y, z);
            if (lse)
                lse[(i * 2 + slot) * N + v] = l;
            if (!w)
                continue;
            for (int64_t ox = -g->M; ox <= g->M; ++ox)
                for (int64_t oy = -g->M; oy <= g->M; ++oy)
                    for (int64_t oz = -g->M; oz <= g->M; ++oz) {
                        int64_t k = ((ox + g->M) * S + (oy + g->M)) * S + (oz + g->M);
                        double val = 0.0;
                        if (inside(g, x + ox, y + oy, z + oz))
                            val = weight(g, u, i, j, x, y, z, ox, oy, oz, l);
                        w[((i * 2 + slot) * W + k) * N + v] = val;
                    }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Gauss-Jacobi step, Eq. (8):                                              */
/*   out_i(v) = mu/(2+mu) g_i(v)                                            */
/*            + 1/(2+mu) [sum_d w_{i->i+1} f_{i+1} + sum_d w_{i->i-1} f_{i-1}]*/
/* idx == NULL: every voxel, out is [np][N]. Otherwise out[k] is the value  */
/* at flat index idx[k].                                                    */
/* ------------------------------------------------------------------------ */
void tnlmo_jacobi(const ogeom *g, const double *u, const double *f,
                  const double *gin, double mu, const int64_t *idx,
                  int64_t nidx, double *out)
{
    const int64_t total = idx ? nidx : g->np * nvox_phase(g);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < total; ++k) {
        int64_t flat = idx ? idx[k] : k;
        int64_t i, x, y, z;
        unflatten(g, flat, &i, &x, &y, &z);
        double nbp, nbm;
        local_sums(g, u, f, i, 0, x, y, z, NULL, &nbp, NULL);
        local_sums(g, u, f, i, 1, x, y, z, NULL, &nbm, NULL);
        out[k] = mu / (2.0 + mu) * gin[flat] + (nbp + nbm) / (2.0 + mu);
    }
}

/* ------------------------------------------------------------------------ */
/* Eq. (6) without its fidelity term (weights frozen from u):              */
/*   G6_i(v) = 2 f_i(v) - sum_d w_{i->i+1} f_{i+1} - sum_d w_{i->i-1} f_{i-1}*/
/* ------------------------------------------------------------------------ */
void tnlmo_grad_eq6(const ogeom *g, const double *u, const double *f,
                    const int64_t *idx, int64_t nidx, double *out)
{
    const int64_t total = idx ? nidx : g->np * nvox_phase(g);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < total; ++k) {
        int64_t flat = idx ? idx[k] : k;
        int64_t i, x, y, z;
        unflatten(g, flat, &i, &x, &y, &z);
        double nbp, nbm;
        local_sums(g, u, f, i, 0, x, y, z, NULL, &nbp, NULL);
        local_sums(g, u, f, i, 1, x, y, z, NULL, &nbm, NULL);
        out[k] = 2.0 * f[flat] - nbp - nbm;
    }
}

/* ------------------------------------------------------------------------ */
/* Per-voxel statistics at flat indices: stats[k][slot][0] = log-normaliser,*/
/* stats[k][slot][1] = e = sum_d w r^2. idx == NULL: every voxel, laid out  */
/* [np][2][2][N] instead.                                                   */
/* ------------------------------------------------------------------------ */
void tnlmo_stats(const ogeom *g, const double *u, const double *f,
                 const int64_t *idx, int64_t nidx, double *stats)
{
    const int64_t N = nvox_phase(g);
    const int64_t total = idx ? nidx : g->np * N;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < total; ++k) {
        int64_t flat = idx ? idx[k] : k;
        int64_t i, x, y, z;
        unflatten(g, flat, &i, &x, &y, &z);
        for (int slot = 0; slot < 2; ++slot) {
            double l, e;
            local_sums(g, u, f, i, slot, x, y, z, &l, NULL, &e);
            if (idx) {
                stats[(k * 2 + slot) * 2 + 0] = l;
                stats[(k * 2 + slot) * 2 + 1] = e;
            } else {
                int64_t v = flat - i * N;
                stats[((i * 2 + slot) * 2 + 0) * N + v] = l;
                stats[((i * 2 + slot) * 2 + 1) * N + v] = e;
            }
        }
    }
}

/* Neumaier-compensated sum of a sequence, in the given order. */
static double neumaier(const double *a, int64_t n, int64_t stride)
{
    double s = 0.0, c = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double x = a[k * stride];
        double t = s + x;
        if (fabs(s) >= fabs(x))
            c += (s - t) + x;
        else
            c += (x - t) + s;
        s = t;
    }
    return s + c;
}

/* ------------------------------------------------------------------------ */
/* TNLM energy E(f; u) = 1/4 sum_i sum_slot sum_v e_{i,slot}(v).            */
/* stats (nullable) receives [np][2][2][N] (log-normaliser, e).             */
/* ------------------------------------------------------------------------ */
double tnlmo_energy(const ogeom *g, const double *u, const double *f,
                    double *stats)
{
    const int64_t N = nvox_phase(g);
    double *st = stats ? stats : (double *)malloc(sizeof(double) * g->np * 4 * N);
    if (!st)
        return NAN;
    tnlmo_stats(g, u, f, NULL, 0, st);
    /* gather the e entries in (i, slot, v) order, then one compensated sum */
    double *e = (double *)malloc(sizeof(double) * g->np * 2 * N);
    if (!e) {
        if (!stats)
            free(st);
        return NAN;
    }
    for (int64_t i = 0; i < g->np; ++i)
        for (int slot = 0; slot < 2; ++slot)
            memcpy(e + (i * 2 + slot) * N, st + ((i * 2 + slot) * 2 + 1) * N,
                   sizeof(double) * N);
    double E = 0.25 * neumaier(e, g->np * 2 * N, 1);
    free(e);
    if (!stats)
        free(st);
    return E;
}

/* ------------------------------------------------------------------------ */
/* Exact gradient of E(f; u), scatter form (the chain rule term by term).  */
/* For every (i, slot, v, delta) with weight w and residual                 */
/* r = f_i(v) - f_j(v+delta):                                               */
/*   dE/df_i(v) += w r / 2,  dE/df_j(v+delta) -= w r / 2;                   */
/*   Dbar = dE/dD = -(1/(8h^2)) w (r^2 - e_{i,slot}(v))   (softmax Jacobian)*/
/*   for each patch offset p, with Delta = U_i(v+p) - U_j(v+delta+p):       */
/*     dE/du_i(clamp(v+p)) += 2 Dbar Delta,                                 */
/*     dE/du_j(clamp(v+delta+p)) -= 2 Dbar Delta.                           */
/* Single-threaded (the scatter would race); meant for small grids.         */
/* gf, gu: [np][N], both nullable.                                          */
/* ------------------------------------------------------------------------ */
void tnlmo_grad_exact_scatter(const ogeom *g, const double *u, const double *f,
                              double *gf, double *gu)
{
    const int64_t N = nvox_phase(g);
    if (gf)
        memset(gf, 0, sizeof(double) * g->np * N);
    if (gu)
        memset(gu, 0, sizeof(double) * g->np * N);
    const double inv8h2 = 1.0 / (8.0 * g->h * g->h);
    for (int64_t i = 0; i < g->np; ++i)
        for (int slot = 0; slot < 2; ++slot) {
            int64_t j = neighbour(g, i, slot);
            for (int64_t x = 0; x < g->nx; ++x)
                for (int64_t y = 0; y < g->ny; ++y)
                    for (int64_t z = 0; z < g->nz; ++z) {
                        double lse, e;
                        local_sums(g, u, f, i, slot, x, y, z, &lse, NULL, &e);
                        double fi = f[vidx(g, i, x, y, z)];
                        for (int64_t ox = -g->M; ox <= g->M; ++ox)
                            for (int64_t oy = -g->M; oy <= g->M; ++oy)
                                for (int64_t oz = -g->M; oz <= g->M; ++oz) {
                                    if (!inside(g, x + ox, y + oy, z + oz))
                                        continue;
                                    double w = weight(g, u, i, j, x, y, z, ox, oy, oz, lse);
                                    int64_t q = vidx(g, j, x + ox, y + oy, z + oz);
                                    double r = fi - f[q];
                                    if (gf) {
                                        gf[vidx(g, i, x, y, z)] += 0.5 * w * r;
                                        gf[q] -= 0.5 * w * r;
                                    }
                                    if (!gu)
                                        continue;
                                    double Dbar = -inv8h2 * w * (r * r - e);
                                    for (int64_t px = -g->d; px <= g->d; ++px)
                                        for (int64_t py = -g->d; py <= g->d; ++py)
                                            for (int64_t pz = -g->d; pz <= g->d; ++pz) {
                                                int64_t ax = x + px, ay = y + py, az = z + pz;
                                                int64_t bx = ax + ox, by = ay + oy, bz = az + oz;
                                                double Delta = ext(g, u, i, ax, ay, az) - ext(g, u, j, bx, by, bz);
                                                gu[vidx(g, i, clampi(ax, 0, g->nx - 1), clampi(ay, 0, g->ny - 1), clampi(az, 0, g->nz - 1))] += 2.0 * Dbar * Delta;
                                                gu[vidx(g, j, clampi(bx, 0, g->nx - 1), clampi(by, 0, g->ny - 1), clampi(bz, 0, g->nz - 1))] -= 2.0 * Dbar * Delta;
                                            }
                                }
                    }
        }
}

/* ------------------------------------------------------------------------ */
/* Exact gradient at chosen voxels, gather form (same quantity as the       */
/* scatter form, regrouped by the output voxel; parallel over samples).     */
/*                                                                          */
/* Image part at (k, q):                                                    */
/*   1/2 sum_s sum_{delta: q+delta in grid}                                 */
/*       [w_{k->k+s}(q, delta) + w_{k+s->k}(q+delta, -delta)]               */
/*       (f_k(q) - f_{k+s}(q+delta)).                                       */
/* Weight part at (k, q): every padded position q' that clamps to q gets    */
/*   2 sum_s sum_delta (U_k(q') - U_{k+s}(q'+delta))                        */
/*       sum_p [Dbar_{k,s}(q'-p, delta) + Dbar_{k+s,-s}(q'-p+delta, -delta)]*/
/* where Dbar vanishes unless both q'-p and q'-p+delta are in the grid.     */
/* ------------------------------------------------------------------------ */
/* Per-sample cache of per-voxel statistics (log-normaliser, e) for the
 * phases and voxels one gathered gradient value touches; filled on first use
 * by local_sums, so every value equals the uncached definition. */
typedef struct {
    int64_t ph[3], nph;        /* phases covered */
    int64_t x0, y0, z0, ex, ey, ez;  /* voxel box covered */
    double *lse, *e;           /* [nph][2][box] */
    unsigned char *done;
} statcache;

static void cache_init(statcache *c, const ogeom *g, int64_t k, int64_t x, int64_t y, int64_t z)
{
    int64_t ph[3] = {phase_of(g, k - 1), phase_of(g, k), phase_of(g, k + 1)};
    c->nph = 0;
    for (int a = 0; a < 3; ++a) {
        int dup = 0;
        for (int b = 0; b < c->nph; ++b)
            if (c->ph[b] == ph[a])
                dup = 1;
        if (!dup)
            c->ph[c->nph++] = ph[a];
    }
    const int64_t R = g->M + 2 * g->d;
    c->x0 = clampi(x - R, 0, g->nx - 1);
    c->y0 = clampi(y - R, 0, g->ny - 1);
    c->z0 = clampi(z - R, 0, g->nz - 1);
    c->ex = clampi(x + R, 0, g->nx - 1) - c->x0 + 1;
    c->ey = clampi(y + R, 0, g->ny - 1) - c->y0 + 1;
    c->ez = clampi(z + R, 0, g->nz - 1) - c->z0 + 1;
    int64_t n = c->nph * 2 * c->ex * c->ey * c->ez;
    c->lse = (double *)malloc(sizeof(double) * n);
    c->e = (double *)malloc(sizeof(double) * n);
    c->done = (unsigned char *)calloc((size_t)n, 1);
}

static void cache_free(statcache *c)
{
    free(c->lse);
    free(c->e);
    free(c->done);
}

/* lse and e of voxel (i; x,y,z) towards slot, through the cache when the
 * voxel lies in it (always the case for the gathered gradient). */
static void cached_stats(statcache *c, const ogeom *g, const double *u, const double *f,
                         int64_t i, int slot, int64_t x, int64_t y, int64_t z, double *lse,
                         double *e)
{
    int64_t a = -1;
    for (int64_t b = 0; b < c->nph; ++b)
        if (c->ph[b] == i)
            a = b;
    int64_t lx = x - c->x0, ly = y - c->y0, lz = z - c->z0;
    if (a < 0 || !c->lse || lx < 0 || lx >= c->ex || ly < 0 || ly >= c->ey || lz < 0 || lz >= c->ez) {
        local_sums(g, u, f, i, slot, x, y, z, lse, NULL, e);
        return;
    }
    int64_t t = ((a * 2 + slot) * c->ex + lx) * c->ey * c->ez + ly * c->ez + lz;
    if (!c->done[t]) {
        local_sums(g, u, f, i, slot, x, y, z, &c->lse[t], NULL, &c->e[t]);
        c->done[t] = 1;
    }
    *lse = c->lse[t];
    *e = c->e[t];
}

static double dbar(statcache *c, const ogeom *g, const double *u, const double *f, int64_t i,
                   int slot, int64_t x, int64_t y, int64_t z, int64_t ox, int64_t oy, int64_t oz)
{
    /* dE/dD_{i,slot}(v, delta) for v=(x,y,z); zero when not a valid pair */
    if (!inside(g, x, y, z) || !inside(g, x + ox, y + oy, z + oz))
        return 0.0;
    int64_t j = neighbour(g, i, slot);
    double lse, e;
    cached_stats(c, g, u, f, i, slot, x, y, z, &lse, &e);
    double w = weight(g, u, i, j, x, y, z, ox, oy, oz, lse);
    double r = f[vidx(g, i, x, y, z)] - f[vidx(g, j, x + ox, y + oy, z + oz)];
    return -w * (r * r - e) / (8.0 * g->h * g->h);
}

void tnlmo_grad_exact_at(const ogeom *g, const double *u, const double *f,
                         const int64_t *idx, int64_t nidx, double *gf,
                         double *gu)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nidx; ++k) {
        int64_t c, x, y, z;
        unflatten(g, idx[k], &c, &x, &y, &z);
        statcache cache;
        cache_init(&cache, g, c, x, y, z);
        /* image part */
        if (gf) {
            double acc = 0.0;
            double fc = f[idx[k]];
            for (int slot = 0; slot < 2; ++slot) {
                int64_t j = neighbour(g, c, slot);
                int back = 1 - slot; /* direction from j back to c */
                double lse_c;
                local_sums(g, u, f, c, slot, x, y, z, &lse_c, NULL, NULL);
                for (int64_t ox = -g->M; ox <= g->M; ++ox)
                    for (int64_t oy = -g->M; oy <= g->M; ++oy)
                        for (int64_t oz = -g->M; oz <= g->M; ++oz) {
                            if (!inside(g, x + ox, y + oy, z + oz))
                                continue;
                            double lse_j;
                            local_sums(g, u, f, j, back, x + ox, y + oy, z + oz, &lse_j, NULL, NULL);
                            double w1 = weight(g, u, c, j, x, y, z, ox, oy, oz, lse_c);
                            double w2 = weight(g, u, j, c, x + ox, y + oy, z + oz, -ox, -oy, -oz, lse_j);
                            acc += 0.5 * (w1 + w2) * (fc - f[vidx(g, j, x + ox, y + oy, z + oz)]);
                        }
            }
            gf[k] = acc;
        }
        if (!gu) {
            cache_free(&cache);
            continue;
        }
        /* weight part: loop over padded positions q' with clamp(q') = q */
        double acc = 0.0;
        int64_t lo[3], hi[3], q[3] = {x, y, z}, n[3] = {g->nx, g->ny, g->nz};
        for (int a = 0; a < 3; ++a) {
            lo[a] = q[a] == 0 ? -g->d : q[a];
            hi[a] = q[a] == n[a] - 1 ? n[a] - 1 + g->d : q[a];
        }
        for (int64_t qx = lo[0]; qx <= hi[0]; ++qx)
            for (int64_t qy = lo[1]; qy <= hi[1]; ++qy)
                for (int64_t qz = lo[2]; qz <= hi[2]; ++qz)
                    for (int slot = 0; slot < 2; ++slot) {
                        int64_t j = neighbour(g, c, slot);
                        int back = 1 - slot;
                        for (int64_t ox = -g->M; ox <= g->M; ++ox)
                            for (int64_t oy = -g->M; oy <= g->M; ++oy)
                                for (int64_t oz = -g->M; oz <= g->M; ++oz) {
                                    double Gs = 0.0;
                                    for (int64_t px = -g->d; px <= g->d; ++px)
                                        for (int64_t py = -g->d; py <= g->d; ++py)
                                            for (int64_t pz = -g->d; pz <= g->d; ++pz) {
                                                int64_t vx = qx - px, vy = qy - py, vz = qz - pz;
                                                Gs += dbar(&cache, g, u, f, c, slot, vx, vy, vz, ox, oy, oz);
                                                Gs += dbar(&cache, g, u, f, j, back, vx + ox, vy + oy, vz + oz, -ox, -oy, -oz);
                                            }
                                    if (Gs == 0.0)
                                        continue;
                                    double Delta = ext(g, u, c, qx, qy, qz) - ext(g, u, j, qx + ox, qy + oy, qz + oz);
                                    acc += 2.0 * Delta * Gs;
                                }
                    }
        gu[k] = acc;
        cache_free(&cache);
    }
}

/* ------------------------------------------------------------------------ */
/* Local energy around voxel (k, x, y, z): 1/4 of the e terms of every      */
/* voxel within M+d (per axis) of it, in the distinct phases among          */
/* k-1, k, k+1, both directions. Every term of E that depends on f_k or u_k */
/* at that voxel is included, so finite differences of this sum equal       */
/* finite differences of E there.                                           */
/* ------------------------------------------------------------------------ */
double tnlmo_local_energy(const ogeom *g, const double *u, const double *f,
                          int64_t k, int64_t x, int64_t y, int64_t z)
{
    int64_t phases[3] = {phase_of(g, k - 1), phase_of(g, k), phase_of(g, k + 1)};
    int64_t np_distinct = 0, list[3];
    for (int a = 0; a < 3; ++a) {
        int dup = 0;
        for (int b = 0; b < np_distinct; ++b)
            if (list[b] == phases[a])
                dup = 1;
        if (!dup)
            list[np_distinct++] = phases[a];
    }
    const int64_t R = g->M + g->d;
    int64_t x0 = clampi(x - R, 0, g->nx - 1), x1 = clampi(x + R, 0, g->nx - 1);
    int64_t y0 = clampi(y - R, 0, g->ny - 1), y1 = clampi(y + R, 0, g->ny - 1);
    int64_t z0 = clampi(z - R, 0, g->nz - 1), z1 = clampi(z + R, 0, g->nz - 1);
    int64_t cnt = np_distinct * 2 * (x1 - x0 + 1) * (y1 - y0 + 1) * (z1 - z0 + 1);
    double *terms = (double *)malloc(sizeof(double) * cnt);
    if (!terms)
        return NAN;
    int64_t t = 0;
    for (int64_t a = 0; a < np_distinct; ++a)
        for (int slot = 0; slot < 2; ++slot)
            for (int64_t vx = x0; vx <= x1; ++vx)
                for (int64_t vy = y0; vy <= y1; ++vy)
                    for (int64_t vz = z0; vz <= z1; ++vz) {
                        double e;
                        local_sums(g, u, f, list[a], slot, vx, vy, vz, NULL, NULL, &e);
                        terms[t++] = e;
                    }
    double E = 0.25 * neumaier(terms, cnt, 1);
    free(terms);
    return E;
}
