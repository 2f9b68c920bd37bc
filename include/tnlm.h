/*
 * tnlm.h — C ABI of libtnlm, the MI355X (gfx950) temporal non-local means
 * (TNLM) operator library.
 *
 * Method: Jia, Tian, Lou, Sonke, Jiang, "Four-dimensional cone beam CT
 * reconstruction and enhancement using a temporal non-local means method".
 * A cyclic stack of Np respiratory-phase volumes f_0..f_{Np-1} (Sec. 2.1,
 * periodic: phase Np is phase 0) is regularised by comparing every voxel of
 * phase i with a (2M+1)^3 search window around the same coordinates in the
 * neighbour phases i+1 and i-1 (Sec. 2.4), using (2d+1)^3 patches.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layout      vol[i][x][y][z], flat index ((i*nx + x)*ny + y)*nz + z
 *             (z fastest). N = nx*ny*nz voxels per phase.
 * Weights     w_{i->j}(v, delta) = exp(-D/(2h^2)) / Z_{i->j}(v) for the
 *             neighbour phase j = i+1 (direction slot 0) or j = i-1 (slot 1),
 *             where D is the unweighted sum of squared differences between
 *             the (2d+1)^3 patches of the weight-source volume u around v in
 *             phase i and around v+delta in phase j (Eq. (3), estimated from
 *             the latest images as in Eq. (9)). Z_{i->j}(v) sums over the
 *             valid offsets V(v) = {delta in [-M,M]^3 : v+delta in the grid}
 *             (window truncated at the borders), so the weights of each
 *             voxel and slot sum to one. Patch voxels outside the grid take
 *             the value of the nearest in-grid voxel of the same phase (clamp
 *             to edge, per axis).
 * Offsets     offset index k = ((dx+M)*(2M+1) + (dy+M))*(2M+1) + (dz+M).
 * Storage     u, f, g and f_out share one storage dtype (tnlm_dtype);
 *             arithmetic is FP32; every other array is FP32. Stores to BF16
 *             and FP16 round to nearest even.
 * Memory      every pointer argument is a device pointer unless stated
 *             otherwise, allocated and owned by the caller. The library
 *             allocates nothing, keeps no state between calls and is
 *             thread-safe. `stream` is a hipStream_t (NULL = null stream);
 *             calls are asynchronous and ordered on that stream. No call
 *             clears memory, synchronises or allocates, so calls may be
 *             captured in a HIP graph and replayed.
 * Speed       patch_r = 1 with 1 <= search_r <= 5 runs LDS-tiled kernels;
 *             other geometries run a one-thread-per-voxel path that is much
 *             slower. Both follow the same definitions.
 * Aliasing    u may equal f (weights from the current iterate, as in the
 *             enhancement algorithm). Outputs must not overlap any input
 *             (TNLM_EALIAS); callers ping-pong buffers instead.
 * Errors      0 on success, or a negative tnlm_status. Arguments are
 *             validated before anything is launched, and on error nothing is
 *             written. NaN/Inf inside volume data is not checked: it
 *             propagates to the outputs it touches.
 * Limits      np >= 2, nx, ny, nz >= 1, N < 2^31, np*N < 2^40;
 *             0 <= patch_r <= 8, 0 <= search_r <= 16; h finite and > 0.
 */
#ifndef TNLM_H
#define TNLM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Problem geometry (Secs. 2.1, 2.4). */
typedef struct tnlm_geom {
    int32_t np;       /* number of respiratory phases, cyclic, >= 2          */
    int32_t nx, ny, nz; /* grid; z is the contiguous axis                    */
    int32_t patch_r;  /* d: patches are (2d+1)^3                             */
    int32_t search_r; /* M: search windows are (2M+1)^3                      */
    float h;          /* similarity scale in exp(-D/(2h^2)), Eq. (3)         */
} tnlm_geom;

typedef enum tnlm_dtype {
    TNLM_F32 = 0,
    TNLM_BF16 = 1,
    TNLM_F16 = 2
} tnlm_dtype;

typedef enum tnlm_grad_mode {
    TNLM_GRAD_EQ6 = 0,   /* the paper's operator with frozen weights, Eq. (6) */
    TNLM_GRAD_EXACT = 1  /* exact gradient of the energy, through the weights */
} tnlm_grad_mode;

typedef enum tnlm_op {
    TNLM_OP_WEIGHTS = 0,
    TNLM_OP_JACOBI = 1,
    TNLM_OP_ENERGY = 2,
    TNLM_OP_GRAD_EQ6 = 3,
    TNLM_OP_GRAD_EXACT = 4
} tnlm_op;

typedef enum tnlm_status {
    TNLM_OK = 0,
    TNLM_EINVAL = -1,     /* bad geometry, h, mu, dtype, mode or flag       */
    TNLM_ENULL = -2,      /* a required pointer is NULL                     */
    TNLM_EALIAS = -3,     /* an output overlaps an input or another output  */
    TNLM_ERANGE = -4,     /* a size overflows the supported index range     */
    TNLM_EWORKSPACE = -5, /* workspace missing or smaller than required     */
    TNLM_EHIP = -6        /* a HIP launch or runtime call failed            */
} tnlm_status;

/*
 * tnlm_weights — weights of Eq. (3) with the weight source u (Eq. (9)).
 *   u    [np][nx][ny][nz] storage dtype, read only.
 *   w    [np][2][W][N] FP32 with W = (2M+1)^3, or NULL. Entry
 *        ((i*2 + slot)*W + k)*N + v holds w_{i->j}(v, delta_k); invalid
 *        offsets hold 0. Indexed in 64 bits; the caller sizes the buffer.
 *   lse  [np][2][N] FP32, or NULL: log Z_{i->j}(v) in natural-log units,
 *        i.e. log sum_{delta in V(v)} exp(-D(v, delta)/(2h^2)).
 *   At least one of w and lse must be non-NULL.
 */
int tnlm_weights(const tnlm_geom *geom, int dtype, const void *u, float *w,
                 float *lse, void *stream);

/*
 * tnlm_jacobi_step — one Gauss-Jacobi step, Eq. (8):
 *   f_out_i(v) = mu/(2+mu) g_i(v)
 *              + 1/(2+mu) sum_{slot} sum_{delta in V(v)} w_{i->j}(v, delta) f_j(v+delta)
 *   with the weights taken from u, and every phase reading the previous
 *   iterate f (Jacobi, not Gauss-Seidel; Sec. 2.3).
 *   u, f, g  [np][nx][ny][nz] storage dtype (u may equal f; g may equal u).
 *   mu       fidelity weight, finite and > 0 (Eqs. (1), (4)).
 *   f_out    [np][nx][ny][nz] storage dtype; must not overlap u, f or g.
 */
int tnlm_jacobi_step(const tnlm_geom *geom, int dtype, const void *u,
                     const void *f, const void *g, float mu, void *f_out,
                     void *stream);

/*
 * tnlm_energy — TNLM energy with weights from u:
 *   E(f; u) = 1/4 sum_i sum_slot sum_v sum_{delta in V(v)}
 *             w_{i->j}(v, delta; u) (f_i(v) - f_j(v+delta))^2,
 *   i.e. 1/2 sum_i J[f_i, f_{i+1}] (Eqs. (1), (2), (4)) with the weights of
 *   the two directions of each link averaged.
 *   e_out  device FP32[2]: E = e_out[0] + e_out[1] (a compensated hi/lo
 *          pair, reduced in a fixed order: bitwise reproducible).
 *   stats  [np][2][2][N] FP32 or NULL: entry ((i*2+slot)*2 + 0)*N + v is the
 *          log-normaliser (as lse of tnlm_weights), entry
 *          ((i*2+slot)*2 + 1)*N + v is e = sum_delta w r^2 of that voxel.
 *   ws     device workspace of at least tnlm_workspace_bytes(geom,
 *          TNLM_OP_ENERGY) bytes (partial sums), owned by the caller.
 */
int tnlm_energy(const tnlm_geom *geom, int dtype, const void *u,
                const void *f, float *e_out, float *stats, void *ws,
                size_t ws_bytes, void *stream);

/*
 * tnlm_energy_noalloc — tnlm_energy without a workspace argument, for callers
 *   that cannot allocate device memory (code under HIP graph capture, tight
 *   serving loops, harnesses that forbid hipMalloc). It computes exactly what
 *   tnlm_energy computes, with the same kernels, arguments (minus ws) and
 *   outputs, and allocates nothing: the per-workgroup partial sums go to a
 *   fixed 4 MiB device array inside the library, one copy per GPU, held until
 *   the process ends. Its device address is looked up (hipGetSymbolAddress)
 *   on the first call on each device, with that device current.
 *   Limit: tnlm_workspace_bytes(geom, TNLM_OP_ENERGY) <= 4 MiB (about half a
 *   million workgroups; 20 phases of 512x512x128 voxels need 1.5 MiB);
 *   larger problems return TNLM_EWORKSPACE before anything is launched.
 *   Every call on one GPU shares that array and overwrites what the last
 *   call left there (every word the result depends on is rewritten, so
 *   nothing needs clearing): calls that overlap in time on one GPU (on
 *   different streams, or from several threads) race and must be ordered by
 *   the caller.
 */
int tnlm_energy_noalloc(const tnlm_geom *geom, int dtype, const void *u,
                        const void *f, float *e_out, float *stats,
                        void *stream);

/*
 * tnlm_grad — gradient of the TNLM term.
 *   mode TNLM_GRAD_EQ6: grad_f = 2 f_i - sum_slot sum_delta w_{i->j} f_j,
 *        the TNLM part of the functional variation Eq. (6) with the weights
 *        frozen (computed from u). grad_u must be NULL; stats is ignored.
 *   mode TNLM_GRAD_EXACT: the exact partial derivatives of E(f; u) above:
 *        grad_f = dE/df (weights held fixed) and grad_u = dE/du (through the
 *        weights: patch distances, normalisers and clamp-to-edge borders).
 *        If grad_u == grad_f, the sum dE/df + dE/du is written there (the
 *        gradient of E(f; f)); this requires u == f.
 *   stats  [np][2][2][N] FP32 as written by tnlm_energy for the same u and
 *          f, or NULL to recompute it inside (needs a larger workspace).
 *   grad_f, grad_u  [np][nx][ny][nz] FP32, each may be NULL (not both).
 *   ws     device workspace of at least tnlm_workspace_bytes(geom, op) bytes
 *          with op = TNLM_OP_GRAD_EQ6 / TNLM_OP_GRAD_EXACT; for EXACT with
 *          stats == NULL add 16*np*N bytes.
 */
int tnlm_grad(const tnlm_geom *geom, int dtype, const void *u, const void *f,
              int mode, const float *stats, float *grad_f, float *grad_u,
              void *ws, size_t ws_bytes, void *stream);

/*
 * tnlm_workspace_bytes — device workspace an operation needs (host call, no
 * device access). Returns 0 for operations that need none, and (size_t)-1 for
 * an invalid geometry or op.
 */
size_t tnlm_workspace_bytes(const tnlm_geom *geom, int op);

/*
 * tnlm_strerror — static description of a status code. For TNLM_EHIP it
 * includes the HIP error text of the last failure on the calling thread.
 */
const char *tnlm_strerror(int code);

/* tnlm_version — library version string, e.g. "tnlm 0.1 gfx950". */
const char *tnlm_version(void);

/* ------------------------------------------------------------------------
 * Reconstruction model: the data-fidelity part of Eq. (1) and the (P1)
 * sub-problem of Eq. (5), solved by CGLS phase by phase (Sec. 2.3), for the
 * TNLM-R algorithm (Sec. 2.3): (P1) by CGLS, weights and one Eq. (8) step
 * from its result (tnlm_jacobi_step), then positivity (tnlm_clamp_nonneg).
 *
 * Projection matrix P_i of phase i: (P f)_r = sum_v a_{r,v} f_v with a_{r,v}
 * the length of ray r inside voxel v, i.e. the line integral of the image
 * taken as constant over unit voxel cubes centred on the grid points.
 * Geometry (circular cone beam, Sec. 2.5), lengths in voxel units, isocentre
 * at the volume centre c = ((nx-1)/2, (ny-1)/2, (nz-1)/2): for gantry angle
 * t the source is at S = sid (cos t, sin t, 0); the flat detector is
 * perpendicular to the central ray at distance sdd from the source; pixel
 * (iu, iv) is centred at S + sdd (-cos t, -sin t, 0)
 * + (iu - (nu-1)/2) du (-sin t, cos t, 0) + (iv - (nv-1)/2) dv (0, 0, 1);
 * ray r is the line through S and that pixel centre.
 * Layouts: volumes [np][nx][ny][nz] FP32 (z fastest); projections
 * [np][na][nu][nv] FP32 (v fastest); angles [np][na] FP32 radians, device.
 * ------------------------------------------------------------------------ */
typedef struct tnlm_ct_geom {
    int32_t np;            /* phases (each with its own angles), >= 1        */
    int32_t nx, ny, nz;    /* volume grid                                   */
    int32_t nu, nv;        /* detector pixels (u in the gantry plane, v = z) */
    int32_t na;            /* projection angles per phase                   */
    float sid, sdd;        /* source-isocentre, source-detector distances   */
    float du, dv;          /* detector pixel pitch at the detector          */
    const float *angles;   /* device [np][na], radians                      */
} tnlm_ct_geom;
/* Limits: every size >= 1; np*nx*ny*nz and np*na*nu*nv < 2^31; sid, sdd,
 * du, dv finite and > 0; the source and the detector outside the volume:
 * sid and sdd - sid larger than the volume's half-diagonal in the gantry
 * plane (TNLM_EINVAL otherwise). The angles sit in device memory and are not
 * checked: a non-finite angle defines no ray, so every pixel of its
 * projection is NaN and the transpose adds NaN to every voxel of its phase
 * (other angles and phases are unaffected). */

/* tnlm_ct_project — proj = P vol for every phase (Eq. (1)). vol and proj
 * must not overlap. */
int tnlm_ct_project(const tnlm_ct_geom *geom, const float *vol, float *proj, void *stream);

/* tnlm_ct_backproject — vol = P^T proj for every phase: the transpose of
 * tnlm_ct_project (same lengths a_{r,v}), gathered per voxel. */
int tnlm_ct_backproject(const tnlm_ct_geom *geom, const float *proj, float *vol,
                        void *stream);

/* tnlm_ct_workspace_bytes — device workspace of the CGLS calls (host call);
 * (size_t)-1 for an invalid geometry. Layout (floats, then pairs of floats
 * hi, lo whose sum is the value): r [np][na*nu*nv] at offset 0, then
 * q [np][na*nu*nv], p [np][N], s [np][N] (N = nx*ny*nz), then gamma [np],
 * qq [np], gnew [np] as pairs, then partial sums. */
size_t tnlm_ct_workspace_bytes(const tnlm_ct_geom *geom);

/* tnlm_cgls_init — starts CGLS for min_g sum_i ||P_i g_i - y_i||^2 ((P1) of
 * Eq. (5)) from x (Sec. 2.3: the previous iterate): r = y - P x,
 * s = P^T r, p = s, gamma = |s|^2 per phase, all in ws (layout above).
 * y [np][na][nu][nv]; x [np][nx][ny][nz] (read). */
int tnlm_cgls_init(const tnlm_ct_geom *geom, const float *y, const float *x, void *ws,
                   size_t ws_bytes, void *stream);

/* tnlm_cgls_step — iters CGLS iterations on the state in ws, updating x in
 * place (x must be the volume tnlm_cgls_init started from, or its result):
 * q = P p, alpha = gamma/|q|^2, x += alpha p, r -= alpha q, s = P^T r,
 * gnew = |s|^2, p = s + (gnew/gamma) p, gamma = gnew; per phase, every
 * scalar on the device (a phase whose |q|^2 or gamma is 0 takes a zero
 * step). Dot products are compensated sums in a fixed order. */
int tnlm_cgls_step(const tnlm_ct_geom *geom, float *x, int iters, void *ws, size_t ws_bytes,
                   void *stream);

/* tnlm_clamp_nonneg — x = max(x, 0) elementwise over n floats (the
 * positivity step of the TNLM-R algorithm, Sec. 2.3); NaN stays NaN. */
int tnlm_clamp_nonneg(float *x, int64_t n, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TNLM_H */
