/*
 * Host-side AddressSanitizer / UndefinedBehaviorSanitizer driver for the C
 * oracles (test infrastructure). Built by tests/test_oracle_sanitizers.py
 * together with oracle/tnlm_oracle.c and oracle/ct_oracle.c, without OpenMP,
 * and run once: it calls every exported oracle function on small grids that
 * reach the awkward cases (ragged extents, a window wider than the grid,
 * Np = 2, d = 0, sampled index lists, voxels on corners, a detector that
 * overhangs the volume) and checks a few invariants on the way, so that an
 * out-of-bounds access or undefined operation in any code path is reported
 * by the sanitizers.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int64_t np, nx, ny, nz, d, M;
    double h;
} ogeom;
typedef struct {
    int64_t np, nx, ny, nz, nu, nv, na;
    double sid, sdd, du, dv;
} ctgeom;

void tnlmo_weights(const ogeom *, const double *, double *, double *);
void tnlmo_jacobi(const ogeom *, const double *, const double *, const double *, double,
                  const int64_t *, int64_t, double *);
void tnlmo_grad_eq6(const ogeom *, const double *, const double *, const int64_t *, int64_t,
                    double *);
void tnlmo_stats(const ogeom *, const double *, const double *, const int64_t *, int64_t,
                 double *);
double tnlmo_energy(const ogeom *, const double *, const double *, double *);
void tnlmo_grad_exact_scatter(const ogeom *, const double *, const double *, double *,
                              double *);
void tnlmo_grad_exact_at(const ogeom *, const double *, const double *, const int64_t *,
                         int64_t, double *, double *);
double tnlmo_local_energy(const ogeom *, const double *, const double *, int64_t, int64_t,
                          int64_t, int64_t);
void tnlmo_error_model_at(const ogeom *, const double *, const double *, double, double,
                          double, double, const int64_t *, int64_t, double *, double *,
                          double *, double *, double *, double *, double *);
void tnlmo_error_model(const ogeom *, const double *, const double *, double, double, double,
                       double, double *, double *, double *, double *, double *, double *,
                       double *, double *, double *, double *, double *);
void ctor_project(const ctgeom *, const double *, const double *, double *, double *,
                  double *);
void ctor_backproject(const ctgeom *, const double *, const double *, double *, double *,
                      double *);
double ctor_box_chord(const ctgeom *, double, int64_t, int64_t, const double *,
                      const double *);
void ctor_error_model(const ctgeom *, const double *, const double *, const double *, double *,
                      double *);
double ctor_pair_error(const ctgeom *, double, int64_t, int64_t, int64_t, int64_t, int64_t,
                       double *);

static int failures = 0;
#define CHECK(c, ...)                                    \
    do {                                                 \
        if (!(c)) {                                      \
            fprintf(stderr, "check failed: " __VA_ARGS__); \
            fputc('\n', stderr);                         \
            ++failures;                                  \
        }                                                \
    } while (0)

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double urand(void) /* splitmix64, uniform in [0, 1) */
{
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53;
}

static double *vol(int64_t n, double lo, double hi)
{
    double *p = malloc(sizeof(double) * n);
    for (int64_t k = 0; k < n; ++k)
        p[k] = lo + (hi - lo) * urand();
    return p;
}

static void tnlm_case(int64_t np, int64_t nx, int64_t ny, int64_t nz, int64_t d, int64_t M,
                      double h)
{
    const ogeom g = {np, nx, ny, nz, d, M, h};
    const int64_t N = nx * ny * nz, T = np * N, S = 2 * M + 1, W = S * S * S;
    double *u = vol(T, 0.0, 1.0), *f = vol(T, 0.0, 1.0), *gin = vol(T, 0.0, 1.0);
    double *w = malloc(sizeof(double) * np * 2 * W * N);
    double *lse = malloc(sizeof(double) * np * 2 * N);
    double *out = malloc(sizeof(double) * T), *st = malloc(sizeof(double) * np * 4 * N);
    double *gf = malloc(sizeof(double) * T), *gu = malloc(sizeof(double) * T);
    double *gf2 = malloc(sizeof(double) * T), *gu2 = malloc(sizeof(double) * T);

    tnlmo_weights(&g, u, w, lse);
    for (int64_t v = 0; v < np * 2 * N; ++v) {
        const int64_t i = v / (2 * N), rest = v % (2 * N), s = rest / N, x = rest % N;
        double sum = 0.0;
        for (int64_t k = 0; k < W; ++k)
            sum += w[((i * 2 + s) * W + k) * N + x];
        CHECK(fabs(sum - 1.0) < 1e-12, "weights row %lld sums to %.17g", (long long)v, sum);
    }
    tnlmo_weights(&g, u, NULL, lse);
    tnlmo_jacobi(&g, u, f, gin, 0.5, NULL, 0, out);
    tnlmo_grad_eq6(&g, u, f, NULL, 0, out);
    tnlmo_stats(&g, u, f, NULL, 0, st);
    const double E = tnlmo_energy(&g, u, f, st);
    const double E2 = tnlmo_energy(&g, u, f, NULL);
    CHECK(E >= 0.0 && E == E2, "energy %.17g vs %.17g", E, E2);

    /* sampled paths: first, last and corner voxels of every phase */
    int64_t idx[8];
    const int64_t corners[4][3] = {{0, 0, 0}, {nx - 1, ny - 1, nz - 1}, {0, ny - 1, 0},
                                   {nx - 1, 0, nz - 1}};
    for (int c = 0; c < 8; ++c) {
        const int64_t i = c % np, *q = corners[c % 4];
        idx[c] = i * N + (q[0] * ny + q[1]) * nz + q[2];
    }
    tnlmo_jacobi(&g, u, f, gin, 2.0, idx, 8, out);
    tnlmo_grad_eq6(&g, u, f, idx, 8, out);
    tnlmo_stats(&g, u, f, idx, 8, st);
    tnlmo_grad_exact_at(&g, u, f, idx, 8, gf2, gu2);
    tnlmo_grad_exact_at(&g, u, f, idx, 8, gf2, NULL);
    tnlmo_grad_exact_scatter(&g, u, f, gf, gu);
    tnlmo_grad_exact_scatter(&g, u, f, gf, NULL);
    for (int c = 0; c < 8; ++c) {
        const double le = tnlmo_local_energy(&g, u, f, c % np, corners[c % 4][0],
                                             corners[c % 4][1], corners[c % 4][2]);
        CHECK(le >= 0.0, "local energy %.17g", le);
    }

    /* error model: whole grid (with gradients) and sampled */
    double *em[18];
    for (int k = 0; k < 18; ++k)
        em[k] = malloc(sizeof(double) * (k < 7 ? np * 2 * N : T));
    tnlmo_error_model(&g, u, f, 8.0, 0x1.0p-24, 6.0, 3.0 * 0x1.0p-24, em[0], em[1], em[2],
                      em[3], em[4], em[5], em[6], em[7], em[8], em[9], em[10]);
    tnlmo_error_model(&g, u, f, 8.0, 0x1.0p-24, 6.0, 3.0 * 0x1.0p-24, em[0], em[1], em[2],
                      em[3], em[4], em[5], em[6], NULL, NULL, NULL, NULL);
    tnlmo_error_model_at(&g, u, f, 8.0, 0x1.0p-24, 6.0, 3.0 * 0x1.0p-24, idx, 8, em[11],
                         em[12], em[13], em[14], em[15], em[16], em[17]);
    for (int k = 0; k < 18; ++k)
        free(em[k]);

    /* a constant stack: the energy is zero */
    for (int64_t k = 0; k < T; ++k)
        u[k] = f[k] = 0.25;
    const double E0 = tnlmo_energy(&g, u, f, NULL);
    CHECK(E0 == 0.0, "energy of a constant stack %.17g", E0);

    free(u); free(f); free(gin); free(w); free(lse); free(out); free(st);
    free(gf); free(gu); free(gf2); free(gu2);
}

static void ct_case(int64_t nx, int64_t ny, int64_t nz, int64_t nu, int64_t nv, int64_t na,
                    double du)
{
    const ctgeom g = {2, nx, ny, nz, nu, nv, na, 30.0, 50.0, du, du};
    const int64_t N = nx * ny * nz, R = na * nu * nv;
    double *ang = malloc(sizeof(double) * 2 * na);
    for (int64_t k = 0; k < 2 * na; ++k)
        ang[k] = 6.283185307179586 * k / (2.0 * na) + 1e-3;
    ang[0] = 0.0; /* an axis-aligned ray set */
    double *x = vol(2 * N, 0.0, 1.0), *y = vol(2 * R, 0.0, 1.0);
    double *p = malloc(sizeof(double) * 2 * R), *b = malloc(sizeof(double) * 2 * N);
    double *pc = malloc(sizeof(double) * 2 * R), *ps = malloc(sizeof(double) * 2 * R);
    double *bc = malloc(sizeof(double) * 2 * N), *bs = malloc(sizeof(double) * 2 * N);
    ctor_project(&g, ang, x, p, pc, ps);
    ctor_project(&g, ang, x, p, NULL, NULL);
    ctor_backproject(&g, ang, y, b, bc, bs);
    ctor_backproject(&g, ang, y, b, NULL, NULL);
    /* adjointness <Ax, y> = <x, A^T y> */
    double l = 0.0, r = 0.0;
    for (int64_t k = 0; k < 2 * R; ++k)
        l += p[k] * y[k];
    for (int64_t k = 0; k < 2 * N; ++k)
        r += x[k] * b[k];
    CHECK(fabs(l - r) <= 1e-10 * fabs(l), "adjointness %.17g vs %.17g", l, r);
    /* FP32 error model: both outputs, then each alone; one pair per voxel */
    ctor_error_model(&g, ang, x, y, pc, bc);
    ctor_error_model(&g, ang, x, NULL, ps, NULL);
    ctor_error_model(&g, ang, NULL, y, NULL, bs);
    for (int64_t k = 0; k < 2 * R; ++k)
        CHECK(pc[k] >= 0.0 && pc[k] == ps[k], "projection bound %.17g", pc[k]);
    for (int64_t ix = 0; ix < nx; ++ix)
        for (int64_t iz = 0; iz < nz; ++iz) {
            double len;
            const double e = ctor_pair_error(&g, 0.7, nu / 2, nv / 2, ix, ny / 2, iz, &len);
            CHECK(len >= 0.0 && e >= 0.0, "pair %.17g %.17g", len, e);
        }
    const double lo[3] = {-2.0, -1.5, -1.0}, hi[3] = {2.0, 1.5, 1.0};
    for (int64_t iu = 0; iu < nu; ++iu)
        for (int64_t iv = 0; iv < nv; ++iv) {
            const double c = ctor_box_chord(&g, 0.3, iu, iv, lo, hi);
            CHECK(c >= 0.0, "chord %.17g", c);
        }
    free(ang); free(x); free(y); free(p); free(b); free(pc); free(ps); free(bc); free(bs);
}

int main(void)
{
    tnlm_case(2, 4, 3, 5, 1, 1, 0.3);   /* Np = 2, ragged extents */
    tnlm_case(3, 3, 4, 2, 0, 2, 0.05);  /* d = 0, window wider than z */
    tnlm_case(2, 2, 2, 3, 1, 5, 1e6);   /* window wider than the grid */
    tnlm_case(3, 5, 4, 4, 1, 0, 0.1);   /* M = 0 */
    ct_case(6, 5, 4, 9, 7, 3, 1.5);     /* detector overhangs the volume */
    ct_case(3, 4, 5, 4, 3, 2, 0.7);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer run: all cases passed\n");
    return 0;
}
