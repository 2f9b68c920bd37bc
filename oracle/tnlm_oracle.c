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

/* ------------------------------------------------------------------------ */
/* First-order rounding-error model of a single-precision evaluation.       */
/*                                                                          */
/* Tolerance infrastructure for the parity tests (how far an FP32           */
/* evaluation of the definitions above can be expected to land from them),  */
/* not part of the method.                                                  */
/*                                                                          */
/* Sources. The exponent a_k = D_k/(2h^2) of candidate k of one voxel and   */
/* direction (a "block") is computed with an error da_k = eta * a_k + t_k.  */
/* eta, the relative error of the constant 1/(2h^2), is one value for the   */
/* whole evaluation (fully correlated). t_k collects roundings modelled as  */
/* independent, mean zero and bounded (the probabilistic rounding model of  */
/* Higham and Mary, 2019), each of at most one unit roundoff ulp of the     */
/* value it rounds:                                                         */
/*   - the distance, a sum of positive terms: a rounding of partial sum s   */
/*     moves D by at most ulp*s; with every term passing through at most    */
/*     `depth` roundings, sum_r s_r^2 <= depth * D^2, and the rounding of   */
/*     each difference adds at most (2 ulp)^2 D^2 in all;                   */
/*   - the shifted exponent, one rounding of at most a_k + a_0 + 70 (shifts */
/*     start from a_0, the exponent of the zero offset, or from the         */
/*     log-normaliser, lowered by at most 69.3 = 100 ln 2);                 */
/*   - the exponential, about two units of its result.                      */
/* So t_k is a sum of independent bounded terms whose bounds have the       */
/* square sum tb_k^2 = ulp^2 [(depth + 4) a_k^2 + (a_k + a_0 + 70)^2 + 4].  */
/* There is one such set for each kernel that recomputes the distances:     */
/* the forward kernels (F) and the adjoint (A), which reads the forward     */
/* pass's log-normalisers and e.                                            */
/*                                                                          */
/* Propagation. Every output is, to first order, X = sum_src c_src da_src   */
/* (plus, for dE/du, eta times the output itself: its terms carry the       */
/* factor 1/(8h^2), which scales with 1/(2h^2)).                            */
/* This returns for each output the variance proxy V = sum c^2 tb^2 of the  */
/* independent part and the coefficient sum D = sum c a of the correlated   */
/* one, so that |X| <= lam sqrt(V) + |eta| |D| except with probability at   */
/* most 2 exp(-lam^2/2) (Hoeffding's inequality over the elementary         */
/* roundings).                                                              */
/*                                                                          */
/* Coefficients, with w_k the normalised weights, cbar = sum w c:           */
/*   forward averages sum_k w_k c_k:  c_k = -w_k (c_k - cbar)                */
/*   log-normaliser:                  c_k = -w_k                             */
/*   weight w_k:                      c_m = w_k (w_m - [m = k])              */
/* The adjoint evaluates w_k = exp(-a_k - L) with the forward L and e, so   */
/* dw_k = w_k (-dA_k + sum_m w_m dF_m) and, for Dbar_k = -(w_k/(8h^2))      */
/* (r_k^2 - e), dDbar_k = -(w_k/(8h^2)) [-dA_k (r_k^2 - e)                   */
/*                        + sum_m w_m dF_m (r_k^2 + r_m^2 - 2e)].            */
/*                                                                          */
/* Outputs (each nullable):                                                 */
/*   lse_v, lse_d [np][2][N]  log-normaliser (V, D)                         */
/*   w_b          [np][2][N]  max over offsets of lam sqrt(V) + corr |D| of  */
/*                            the weights of the voxel                      */
/*   nb_v, nb_d   [np][2][N]  sum_delta w f_j (neighbour average, Eq. (8))  */
/*   e_v, e_d     [np][2][N]  e = sum_delta w r^2                           */
/*   gf_v, gf_d, gu_v, gu_d [np][N]  the two parts of the exact gradient    */
/*                            (scatter form over blocks, single-threaded)   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n;          /* valid candidates */
    double a0, ebar, rbar;
    double *a, *tb, *w, *c; /* [W] in offset order over valid candidates */
} oblock;

static void block_eval(const ogeom *g, const double *u, const double *f, double depth, double ulp,
                       int64_t i, int slot, int64_t x, int64_t y, int64_t z, oblock *b)
{
    const int64_t j = neighbour(g, i, slot);
    const double inv2h2 = 1.0 / (2.0 * g->h * g->h);
    const double fi = f ? f[vidx(g, i, x, y, z)] : 0.0;
    b->a0 = patch_dist(g, u, i, j, x, y, z, 0, 0, 0) * inv2h2;
    int64_t n = 0;
    double amin = INFINITY;
    for (int64_t ox = -g->M; ox <= g->M; ++ox)
        for (int64_t oy = -g->M; oy <= g->M; ++oy)
            for (int64_t oz = -g->M; oz <= g->M; ++oz) {
                if (!inside(g, x + ox, y + oy, z + oz))
                    continue;
                b->a[n] = patch_dist(g, u, i, j, x, y, z, ox, oy, oz) * inv2h2;
                b->c[n] = f ? f[vidx(g, j, x + ox, y + oy, z + oz)] : 0.0;
                if (b->a[n] < amin)
                    amin = b->a[n];
                ++n;
            }
    double Z = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        b->w[k] = exp(-(b->a[k] - amin));
        Z += b->w[k];
    }
    double eb = 0.0, rb = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        b->w[k] /= Z;
        const double t = b->a[k] + b->a0 + 70.0;
        b->tb[k] = ulp * sqrt((depth + 4.0) * b->a[k] * b->a[k] + t * t + 4.0);
        const double r = fi - b->c[k];
        eb += b->w[k] * r * r;
        rb += b->w[k] * r;
    }
    b->n = n;
    b->ebar = eb;
    b->rbar = rb;
}

/* V and D of a forward average sum_k w_k c_k (c = the block's f_j values, or
 * r^2 with fi given). */
static void fwd_avg(const oblock *b, int r2mode, double fi, double *V, double *D)
{
    double cb = 0.0;
    for (int64_t k = 0; k < b->n; ++k) {
        const double c = r2mode ? (fi - b->c[k]) * (fi - b->c[k]) : b->c[k];
        cb += b->w[k] * c;
    }
    double v = 0.0, d = 0.0;
    for (int64_t k = 0; k < b->n; ++k) {
        const double c = r2mode ? (fi - b->c[k]) * (fi - b->c[k]) : b->c[k];
        const double co = -b->w[k] * (c - cb);
        v += co * co * b->tb[k] * b->tb[k];
        d += co * b->a[k];
    }
    *V = v;
    *D = d;
}

/* Per-voxel outputs of the model for one voxel (flat index) and direction,
 * written at offset o of each non-null output. */
static void voxel_model(const ogeom *g, const double *u, const double *f, double depth,
                        double ulp, double lam, double corr, int64_t flat, int slot, oblock *bp,
                        int64_t o, double *lse_v, double *lse_d, double *w_b, double *nb_v,
                        double *nb_d, double *e_v, double *e_d)
{
    const int64_t S = 2 * g->M + 1, W = S * S * S;
    int64_t i, x, y, z;
    unflatten(g, flat, &i, &x, &y, &z);
    const double fi = f ? f[flat] : 0.0;
    oblock b = *bp;
    block_eval(g, u, f, depth, ulp, i, slot, x, y, z, &b);
    double V, D;
    if (lse_v || lse_d) {
        V = 0.0;
        D = 0.0;
        double wa = 0.0;
        for (int64_t k = 0; k < b.n; ++k) {
            V += b.w[k] * b.w[k] * b.tb[k] * b.tb[k];
            D -= b.w[k] * b.a[k];
            wa += b.w[k] * b.a[k];
        }
        /* the log of the sum and the removal of the shift: two roundings
         * relative to about a_0 + log W */
        const double lz = ulp * (2.0 * b.a0 + 2.0 * log((double)W) + wa);
        V += lz * lz;
        if (lse_v)
            lse_v[o] = V;
        if (lse_d)
            lse_d[o] = D;
    }
    if (w_b) {
        double s2 = 0.0, sa = 0.0, best = 0.0;
        for (int64_t k = 0; k < b.n; ++k) {
            s2 += b.w[k] * b.w[k] * b.tb[k] * b.tb[k];
            sa += b.w[k] * b.a[k];
        }
        for (int64_t k = 0; k < b.n; ++k) {
            const double wk = b.w[k], tk = b.tb[k];
            /* sum_m (w_k (w_m - [m=k]))^2 tb_m^2 */
            const double Vk = wk * wk * (s2 - wk * wk * tk * tk + (wk - 1.0) * (wk - 1.0) * tk * tk);
            const double Dk = wk * (sa - b.a[k]);
            const double bk = lam * sqrt(Vk) + corr * fabs(Dk);
            if (bk > best)
                best = bk;
        }
        w_b[o] = best;
    }
    if (nb_v || nb_d) {
        fwd_avg(&b, 0, fi, &V, &D);
        if (nb_v)
            nb_v[o] = V;
        if (nb_d)
            nb_d[o] = D;
    }
    if (e_v || e_d) {
        fwd_avg(&b, 1, fi, &V, &D);
        if (e_v)
            e_v[o] = V;
        if (e_d)
            e_d[o] = D;
    }
}

/* The per-voxel outputs of tnlmo_error_model at flat indices idx[0..n):
 * each output [n][2] (direction slot fastest). */
void tnlmo_error_model_at(const ogeom *g, const double *u, const double *f, double depth,
                          double ulp, double lam, double corr, const int64_t *idx, int64_t n,
                          double *lse_v, double *lse_d, double *w_b, double *nb_v, double *nb_d,
                          double *e_v, double *e_d)
{
    const int64_t S = 2 * g->M + 1, W = S * S * S;
#pragma omp parallel
    {
        oblock bl;
        double *mem = (double *)malloc(sizeof(double) * 4 * W);
        bl.a = mem;
        bl.tb = mem + W;
        bl.w = mem + 2 * W;
        bl.c = mem + 3 * W;
#pragma omp for schedule(dynamic, 4)
        for (int64_t t = 0; t < n; ++t) {
            if (!mem)
                continue;
            for (int slot = 0; slot < 2; ++slot)
                voxel_model(g, u, f, depth, ulp, lam, corr, idx[t], slot, &bl, t * 2 + slot,
                            lse_v, lse_d, w_b, nb_v, nb_d, e_v, e_d);
        }
        free(mem);
    }
}

/* Scatter of one block's gradient-error terms (see above) into the
 * accumulators gfv, gfd, guv, gud ([np][N] each). mem: 4W + 2 ni + 2 nj +
 * 2 ni doubles of scratch, touched: ni + nj bytes (ni = (2d+1)^3,
 * nj = (2(M+d)+1)^3). */
static void block_scatter(const ogeom *g, const double *u, const double *f, double depth,
                          double ulp, int64_t i, int slot, int64_t x, int64_t y, int64_t z,
                          double *mem, unsigned char *touched, int want_f, int want_u,
                          double *gfv, double *gfd, double *guv, double *gud)
{
    const int64_t S = 2 * g->M + 1, W = S * S * S;
    const int64_t Li = 2 * g->d + 1, Lj = 2 * (g->M + g->d) + 1;
    const int64_t ni = Li * Li * Li, nj = Lj * Lj * Lj;
    oblock b;
    b.a = mem;
    b.tb = mem + W;
    b.w = mem + 2 * W;
    b.c = mem + 3 * W;
    /* P0 = sum_k w_k G_k(q), P1 = sum_k w_k (r_k^2 - e) G_k(q) for the
     * outputs q the block touches: phase i within d of v, phase j within
     * M+d of v (clamped coordinates, so clamped copies merge) */
    double *P0i = mem + 4 * W, *P1i = P0i + ni, *P0j = P1i + ni, *P1j = P0j + nj;
    int64_t *lq = (int64_t *)(P1j + nj); /* per (k, side): (output, G) pairs */
    double *lG = (double *)(lq + ni);
    const double k8 = 1.0 / (8.0 * g->h * g->h);
    const int64_t j = neighbour(g, i, slot);
    block_eval(g, u, f, depth, ulp, i, slot, x, y, z, &b);
    const int64_t vi = vidx(g, i, x, y, z);
    const double fi = f[vi], e = b.ebar;
    /* per-block sums over the F sources */
    double S0 = 0.0, S1 = 0.0, S2 = 0.0, T0 = 0.0, T1 = 0.0;
    for (int64_t m = 0; m < b.n; ++m) {
        const double rm = fi - b.c[m], q2 = rm * rm - e;
        const double wt = b.w[m] * b.w[m] * b.tb[m] * b.tb[m];
        S0 += wt;
        S1 += wt * q2;
        S2 += wt * q2 * q2;
        T0 += b.w[m] * b.a[m];
        T1 += b.w[m] * b.a[m] * q2;
    }
    /* image part, self: X = 1/2 sum_k w_k r_k (-dA_k + sum_m w_m dF_m) */
    if (want_f) {
        double v = 0.25 * b.rbar * b.rbar * S0, d = 0.0;
        for (int64_t k = 0; k < b.n; ++k) {
            const double r = fi - b.c[k];
            v += 0.25 * b.w[k] * b.w[k] * r * r * b.tb[k] * b.tb[k];
            d += -0.5 * b.w[k] * r * b.a[k] + 0.5 * b.w[k] * r * T0;
        }
        gfv[vi] += v;
        gfd[vi] += d;
    }
    memset(touched, 0, (size_t)(ni + nj));
    int64_t k = 0;
    for (int64_t ox = -g->M; ox <= g->M; ++ox)
        for (int64_t oy = -g->M; oy <= g->M; ++oy)
            for (int64_t oz = -g->M; oz <= g->M; ++oz) {
                if (!inside(g, x + ox, y + oy, z + oz))
                    continue;
                const double wk = b.w[k], r = fi - b.c[k];
                const double q2 = r * r - e, tk = b.tb[k], ak = b.a[k];
                ++k;
                /* image part, other, to (j, v+delta):
                 * X = -1/2 w_k r (-dA_k + sum_m w_m dF_m) */
                if (want_f) {
                    const int64_t qo = vidx(g, j, x + ox, y + oy, z + oz);
                    gfv[qo] += 0.25 * wk * wk * r * r * (tk * tk + S0);
                    gfd[qo] += 0.5 * wk * r * ak - 0.5 * wk * r * T0;
                }
                if (!want_u)
                    continue;
                /* weight part: +2 Delta dDbar_k to clamp(v+p) (phase i) and
                 * -2 Delta dDbar_k to clamp(v+delta+p) (phase j) */
                for (int side = 0; side < 2; ++side) {
                    const int64_t L = side == 0 ? Li : Lj;
                    const int64_t R = side == 0 ? g->d : g->M + g->d;
                    int64_t nl = 0;
                    for (int64_t px = -g->d; px <= g->d; ++px)
                        for (int64_t py = -g->d; py <= g->d; ++py)
                            for (int64_t pz = -g->d; pz <= g->d; ++pz) {
                                const int64_t ax = x + px, ay = y + py, az = z + pz;
                                const int64_t bx = ax + ox, by = ay + oy, bz = az + oz;
                                const double Delta = ext(g, u, i, ax, ay, az) - ext(g, u, j, bx, by, bz);
                                const int64_t cx = clampi(side == 0 ? ax : bx, 0, g->nx - 1);
                                const int64_t cy = clampi(side == 0 ? ay : by, 0, g->ny - 1);
                                const int64_t cz = clampi(side == 0 ? az : bz, 0, g->nz - 1);
                                const int64_t l = ((cx - x + R) * L + (cy - y + R)) * L + (cz - z + R);
                                int64_t t = 0;
                                while (t < nl && lq[t] != l)
                                    ++t;
                                if (t == nl) {
                                    lq[nl] = l;
                                    lG[nl] = 0.0;
                                    ++nl;
                                }
                                lG[t] += (side == 0 ? 2.0 : -2.0) * Delta;
                            }
                    double *P0 = side == 0 ? P0i : P0j, *P1 = side == 0 ? P1i : P1j;
                    unsigned char *tch = side == 0 ? touched : touched + ni;
                    const int64_t ph = side == 0 ? i : j;
                    for (int64_t t = 0; t < nl; ++t) {
                        const int64_t l = lq[t];
                        if (!tch[l]) {
                            tch[l] = 1;
                            P0[l] = 0.0;
                            P1[l] = 0.0;
                        }
                        P0[l] += wk * lG[t];
                        P1[l] += wk * q2 * lG[t];
                        const int64_t lz = l % L, ly = (l / L) % L, lx = l / (L * L);
                        const int64_t q = vidx(g, ph, x - R + lx, y - R + ly, z - R + lz);
                        const double ca = k8 * wk * q2 * lG[t]; /* coefficient of dA_k */
                        guv[q] += ca * ca * tk * tk;
                        /* correlated: through a_k, and through the factor
                         * 1/(8h^2) of the term itself (-ca), which scales
                         * with 1/(2h^2) */
                        gud[q] += ca * ak - ca;
                    }
                }
            }
    if (!want_u)
        return;
    /* F part of every touched output: coefficient of dF_m is
     * -k8 w_m (P1 + (r_m^2 - e) P0) */
    for (int side = 0; side < 2; ++side) {
        const int64_t n = side == 0 ? ni : nj, L = side == 0 ? Li : Lj;
        const int64_t R = side == 0 ? g->d : g->M + g->d;
        const unsigned char *tch = side == 0 ? touched : touched + ni;
        const double *P0 = side == 0 ? P0i : P0j, *P1 = side == 0 ? P1i : P1j;
        const int64_t ph = side == 0 ? i : j;
        for (int64_t l = 0; l < n; ++l) {
            if (!tch[l])
                continue;
            const int64_t lz = l % L, ly = (l / L) % L, lx = l / (L * L);
            const int64_t q = vidx(g, ph, x - R + lx, y - R + ly, z - R + lz);
            guv[q] += k8 * k8 * (P1[l] * P1[l] * S0 + 2.0 * P1[l] * P0[l] * S1 + P0[l] * P0[l] * S2);
            gud[q] += -k8 * (P1[l] * T0 + P0[l] * T1);
        }
    }
}

void tnlmo_error_model(const ogeom *g, const double *u, const double *f, double depth, double ulp,
                       double lam, double corr, double *lse_v, double *lse_d, double *w_b,
                       double *nb_v, double *nb_d, double *e_v, double *e_d, double *gf_v,
                       double *gf_d, double *gu_v, double *gu_d)
{
    const int64_t N = nvox_phase(g);
    const int64_t S = 2 * g->M + 1, W = S * S * S;
    if (lse_v || lse_d || w_b || nb_v || nb_d || e_v || e_d) {
#pragma omp parallel
        {
            oblock bl;
            double *mem = (double *)malloc(sizeof(double) * 4 * W);
            bl.a = mem;
            bl.tb = mem + W;
            bl.w = mem + 2 * W;
            bl.c = mem + 3 * W;
#pragma omp for schedule(dynamic, 64)
            for (int64_t flat = 0; flat < g->np * N; ++flat) {
                if (!mem)
                    continue;
                const int64_t i = flat / N, v = flat - i * N;
                for (int slot = 0; slot < 2; ++slot)
                    voxel_model(g, u, f, depth, ulp, lam, corr, flat, slot, &bl,
                                (i * 2 + slot) * N + v, lse_v, lse_d, w_b, nb_v, nb_d, e_v, e_d);
            }
            free(mem);
        }
    }
    if (!(gf_v || gf_d || gu_v || gu_d))
        return;
    const int64_t tot = g->np * N;
    double *outs[4] = {gf_v, gf_d, gu_v, gu_d};
    for (int q = 0; q < 4; ++q)
        if (outs[q])
            memset(outs[q], 0, sizeof(double) * tot);
    /* blocks in parallel, each thread scattering into private copies that
     * are added up at the end */
#pragma omp parallel
    {
        double *acc = (double *)calloc((size_t)(4 * tot), sizeof(double));
        const int64_t Li = 2 * g->d + 1, Lj = 2 * (g->M + g->d) + 1;
        const int64_t ni = Li * Li * Li, nj = Lj * Lj * Lj;
        double *mem = (double *)malloc(sizeof(double) * (4 * W + 2 * ni + 2 * nj + 2 * ni));
        unsigned char *touched = (unsigned char *)calloc((size_t)(ni + nj), 1);
        const int ok = acc && mem && touched;
#pragma omp for schedule(dynamic, 16)
        for (int64_t flat = 0; flat < tot; ++flat) {
            if (!ok)
                continue;
            int64_t i, x, y, z;
            unflatten(g, flat, &i, &x, &y, &z);
            for (int slot = 0; slot < 2; ++slot)
                block_scatter(g, u, f, depth, ulp, i, slot, x, y, z, mem, touched,
                              gf_v || gf_d, gu_v || gu_d, acc, acc + tot, acc + 2 * tot,
                              acc + 3 * tot);
        }
#pragma omp critical
        {
            if (ok)
                for (int q = 0; q < 4; ++q)
                    if (outs[q])
                        for (int64_t t = 0; t < tot; ++t)
                            outs[q][t] += acc[q * tot + t];
        }
        free(acc);
        free(mem);
        free(touched);
    }
}
