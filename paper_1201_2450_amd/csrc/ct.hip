// Reconstruction model kernels (Eq. (1), (P1) of Eq. (5)): the cone-beam
// projector P of every phase, its transpose, and the CGLS iteration for the
// per-phase least-squares problem, with every scalar kept on the device.
//
// P: a_{r,v} = length of ray r inside voxel v (unit cubes centred on the
// grid points, isocentre at the volume centre). Forward: one thread per ray
// walks the voxels it crosses in order (the next x, y and z plane crossings
// taken from the plane index each step, so errors do not accumulate) and
// sums length x value. Transpose: one thread per voxel and angle loop: the
// voxel's eight corners are projected to the detector, and every pixel whose
// centre falls in that footprint has its ray clipped against the voxel's
// cube; length x projection value is summed. Both enumerate the same
// (ray, voxel) pairs with the same lengths (up to rounding), in gather form:
// no atomics, deterministic. A ray parallel to an axis that runs exactly in
// the face plane between two voxel layers is counted in the upper layer only
// (the walk's floor of the entry coordinate; half-open cubes in the
// transpose), so the lengths of every ray add up to its chord.
//
// Geometry (voxel units): for gantry angle t the source is at
// sid (cos t, sin t, 0); pixel (iu, iv) is centred at
// S + sdd (-cos t, -sin t, 0) + (iu - (nu-1)/2) du e_u + (iv - (nv-1)/2) dv e_v,
// e_u = (-sin t, cos t, 0), e_v = (0, 0, 1). Projections [np][na][nu][nv].
#include <math.h>

#include "tnlm_internal.h"

namespace tnlm {
namespace {

constexpr int kBlock = 256;
constexpr float kFootMargin = 1e-2f;  // pixels added around a voxel's footprint

struct CTG {
    int np, nx, ny, nz, nu, nv, na;
    float sid, sdd, du, dv;
    const float *angles;
    int64_t N, R;  // voxels per phase, rays per phase
};

__device__ __forceinline__ void ray_of(const CTG &g, float th, int iu, int iv, float S[3],
                                       float d[3])
{
    float s, c;
    sincosf(th, &s, &c);
    const float ou = (iu - 0.5f * (g.nu - 1)) * g.du;
    const float ov = (iv - 0.5f * (g.nv - 1)) * g.dv;
    S[0] = g.sid * c;
    S[1] = g.sid * s;
    S[2] = 0.f;
    d[0] = -g.sdd * c - ou * s;
    d[1] = -g.sdd * s + ou * c;
    d[2] = ov;
}

// parameter interval of the ray inside [lo, hi] along one axis
__device__ __forceinline__ bool slab(float S, float d, float lo, float hi, float &t0, float &t1)
{
    if (d == 0.f) {
        t0 = -INFINITY;
        t1 = INFINITY;
        return S >= lo && S <= hi;
    }
    const float inv = 1.f / d;
    const float a = (lo - S) * inv, b = (hi - S) * inv;
    t0 = fminf(a, b);
    t1 = fmaxf(a, b);
    return true;
}

// slab() for one voxel's cube in the transpose: a ray parallel to the axis
// that lies in the face plane between two voxels belongs to the upper one
// (the cube is half-open, [lo, hi), except for the last voxel along the
// axis), as the projector's walk assigns it. The reciprocal of d is the
// hardware estimate refined by one Newton step (within about one ulp; the
// correctly rounded quotient costs some ten instructions more).
__device__ __forceinline__ bool vslab(float S, float d, float lo, float hi, bool last, float &t0,
                                      float &t1)
{
    if (d == 0.f) {
        t0 = -INFINITY;
        t1 = INFINITY;
        return S >= lo && (S < hi || (S == hi && last));
    }
    float inv = __builtin_amdgcn_rcpf(d);
    inv = fmaf(fmaf(-d, inv, 1.f), inv, inv);
    const float a = (lo - S) * inv, b = (hi - S) * inv;
    t0 = fminf(a, b);
    t1 = fmaxf(a, b);
    return true;
}

__global__ void __launch_bounds__(kBlock) project_kernel(CTG g, const float *vol, float *proj)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)g.np * g.R)
        return;
    const int i = (int)(t / g.R);
    const int64_t rr = t - (int64_t)i * g.R;
    const int a = (int)(rr / ((int64_t)g.nu * g.nv));
    const int iu = (int)((rr / g.nv) % g.nu), iv = (int)(rr % g.nv);
    const float th = g.angles[(int64_t)i * g.na + a];
    // a non-finite angle defines no ray: its projection is NaN
    if (!isfinite(th)) {
        proj[t] = __builtin_nanf("");
        return;
    }
    float S[3], d[3];
    ray_of(g, th, iu, iv, S, d);
    const int n[3] = {g.nx, g.ny, g.nz};
    float c[3];
    for (int k = 0; k < 3; ++k)
        c[k] = 0.5f * (n[k] - 1);
    float tin = -INFINITY, tout = INFINITY;
    for (int k = 0; k < 3; ++k) {
        float a0, a1;
        if (!slab(S[k], d[k], -c[k] - 0.5f, c[k] + 0.5f, a0, a1)) {
            proj[t] = 0.f;
            return;
        }
        tin = fmaxf(tin, a0);
        tout = fminf(tout, a1);
    }
    if (!(tout > tin)) {
        proj[t] = 0.f;
        return;
    }
    const float L = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    // voxel of the entry point, clamped to the grid (on the entry face the
    // coordinate is at the box boundary; where it lies on a plane between two
    // voxels either is right: the walk then takes a zero-length step).
    // Per axis the walk keeps the coordinate of the next plane it will cross
    // (an exact half-integer); the crossing parameter is recomputed from it
    // every step, so errors do not accumulate. An axis the ray runs parallel
    // to gets plane +inf and slope 1, i.e. crossing parameter +inf.
    float pl[3], inv[3], pstep[3];
    int off = 0, ostep[3];
    const int stride[3] = {g.ny * g.nz, g.nz, 1};
    for (int k = 0; k < 3; ++k) {
        const float p = S[k] + tin * d[k] + c[k] + 0.5f;
        const int q = (int)floorf(p);
        const int ik = q < 0 ? 0 : (q > n[k] - 1 ? n[k] - 1 : q);
        off += ik * stride[k];
        const int sk = d[k] > 0.f ? 1 : (d[k] < 0.f ? -1 : 0);
        pl[k] = sk == 0 ? INFINITY : (float)(ik + (sk > 0 ? 1 : 0)) - 0.5f - c[k];
        inv[k] = sk == 0 ? 1.f : 1.f / d[k];
        pstep[k] = (float)sk;
        ostep[k] = sk * stride[k];
    }
    const float *v = vol + (int64_t)i * g.N;
    const unsigned nvox = (unsigned)g.N;
    float acc = 0.f, tc = tin;
    const int maxsteps = g.nx + g.ny + g.nz + 3;
    for (int it = 0; it < maxsteps; ++it) {
        const float t0 = (pl[0] - S[0]) * inv[0];
        const float t1 = (pl[1] - S[1]) * inv[1];
        const float t2 = (pl[2] - S[2]) * inv[2];
        const float tm = fminf(fminf(t0, t1), t2);
        const float te = fminf(tm, tout);
        const float nacc = fmaf((te - tc) * L, v[off], acc);
        acc = te > tc ? nacc : acc;
        if (te >= tout)
            break;
        tc = te;
        // step every axis whose crossing is the nearest (a tie is a ray
        // through an edge or corner: the voxels skipped have zero length)
        const bool h0 = t0 == tm, h1 = t1 == tm, h2 = t2 == tm;
        pl[0] += h0 ? pstep[0] : 0.f;
        pl[1] += h1 ? pstep[1] : 0.f;
        pl[2] += h2 ? pstep[2] : 0.f;
        off += (h0 ? ostep[0] : 0) + (h1 ? ostep[1] : 0) + (h2 ? ostep[2] : 0);
        // the exit face ends the walk through te >= tout (its crossing is
        // computed exactly as the box's exit parameter); this guard only
        // keeps the reads inside the phase
        if ((unsigned)off >= nvox)
            break;
    }
    proj[t] = acc;
}

// The transpose reads two per-block tables from LDS when they fit
// (kTabBytes): the sine and cosine of every angle of the phases the block's
// voxels belong to, and for every detector row iv the ray's axial component
// ov = (iv - (nv-1)/2) dv and the z slab's parameters: with r = 1/ov and the
// voxel's z range [zlo, zlo + 1], the entry and exit are fma(zlo, r, c0) and
// fma(zlo, r, c1), (c0, c1) = (r, 0) below the detector centre (ov < 0) and
// (0, r) above it, i.e. zhi r and zlo r or the reverse, each rounded once;
// the centre row of an odd nv (ov = 0, no z bound) has r = 0 and (c0, c1) =
// (-inf, +inf). They hold the values the threads would compute themselves, so
// the results do not depend on whether the tables are used.
constexpr int kTabBytes = 32 * 1024;

// max and min of two floats as single instructions: fmaxf/fminf re-quiet
// (canonicalise) loop-invariant operands on every iteration; the operands
// here are never NaN (angles are finite by then, the geometry is checked)
__device__ __forceinline__ float vmaxf(float a, float b)
{
    float r;
    asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ float vminf(float a, float b)
{
    float r;
    asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// four consecutive floats at a 4-byte boundary: one global_load_dwordx4
// (the HSA targets allow dword-aligned multi-dword loads)
struct __attribute__((packed, aligned(4))) Float4u {
    float x, y, z, w;
};

// start (in floats) of the per-row table, after nang (sin, cos) pairs and
// aligned for 16-byte reads
__host__ __device__ inline int row_tab_offset(int nang)
{
    return (2 * nang + 3) & ~3;
}

// phases a block of kBlock consecutive voxels can touch
__host__ __device__ inline int block_phase_span(const CTG &g)
{
    const int64_t s = (kBlock - 1) / g.N + 2;
    return (int)(s < g.np ? s : g.np);
}

template <bool TAB>
__global__ void __launch_bounds__(kBlock) backproject_kernel(CTG g, const float *proj, float *vol)
{
    // [span][na] (sin, cos) pairs, then from a 16-byte boundary [nv] (r, c0, c1, ov)
    extern __shared__ float4 tab4[];
    float *tab = (float *)tab4;
    const int64_t tb = (int64_t)blockIdx.x * kBlock;
    const int ib = (int)(tb / g.N);  // first phase of the block
    const int nang = TAB ? block_phase_span(g) * g.na : 0;
    const float vcen = 0.5f * (g.nv - 1);
    if (TAB) {
        for (int k = threadIdx.x; k < nang; k += kBlock) {
            const int ph = ib + k / g.na;
            float sn = 0.f, cs = 1.f;
            if (ph < g.np)
                sincosf(g.angles[(int64_t)ph * g.na + k % g.na], &sn, &cs);
            tab[2 * k] = sn;
            tab[2 * k + 1] = cs;
        }
        for (int k = threadIdx.x; k < g.nv; k += kBlock) {
            const float ov = (k - vcen) * g.dv;
            const float r = 1.f / ov;
            float *row = tab + row_tab_offset(nang) + 4 * k;
            row[0] = ov == 0.f ? 0.f : r;
            row[1] = ov == 0.f ? -INFINITY : (ov < 0.f ? r : 0.f);
            row[2] = ov == 0.f ? INFINITY : (ov < 0.f ? 0.f : r);
            row[3] = ov;
        }
        __syncthreads();
    }
    const int64_t t = tb + threadIdx.x;
    if (t >= (int64_t)g.np * g.N)
        return;
    const int i = (int)(t / g.N);
    const int64_t vv = t - (int64_t)i * g.N;
    const int z = (int)(vv % g.nz), y = (int)((vv / g.nz) % g.ny), x = (int)(vv / ((int64_t)g.nz * g.ny));
    const float cen[3] = {x - 0.5f * (g.nx - 1), y - 0.5f * (g.ny - 1), z - 0.5f * (g.nz - 1)};
    const float ucen = 0.5f * (g.nu - 1);
    const float rdu = 1.f / g.du, rdv = 1.f / g.dv;
    const float zlo = cen[2] - 0.5f, zhi = cen[2] + 0.5f;
    // a ray with no axial component (z = 0): inside the half-open cube
    const bool zin0 = zlo <= 0.f && (zhi > 0.f || (zhi == 0.f && z == g.nz - 1));
    float acc = 0.f;
    for (int a = 0; a < g.na; ++a) {
        const float th = g.angles[(int64_t)i * g.na + a];
        float s, c;
        if (TAB) {
            const int k = (i - ib) * g.na + a;
            s = tab[2 * k];
            c = tab[2 * k + 1];
        } else {
            sincosf(th, &s, &c);
        }
        // a non-finite angle (whose sine and cosine are NaN) defines no ray:
        // it adds NaN, as its projection holds NaN, and its footprint, which
        // would span the whole detector, is never visited
        if (!(fabsf(s) <= 1.f)) {
            acc = __builtin_nanf("");
            continue;
        }
        // footprint: bounding box of the corners projected onto the detector
        // (pixel units). The detector coordinate u and the magnification m
        // depend on a corner's (X, Y) only, v on Z times m (m > 0: the depth
        // w stays above zero, the source lies outside the volume). The box
        // only selects candidate pixels, each of which is clipped exactly
        // below, so it is built with approximate reciprocals and widened by
        // kFootMargin pixels, far more than their rounding.
        float umin = INFINITY, umax = -INFINITY, mmin = INFINITY, mmax = -INFINITY;
        for (int k = 0; k < 4; ++k) {
            const float X = cen[0] + ((k & 1) ? 0.5f : -0.5f);
            const float Y = cen[1] + ((k & 2) ? 0.5f : -0.5f);
            const float m = g.sdd * __builtin_amdgcn_rcpf(g.sid - (X * c + Y * s));
            const float u = (-X * s + Y * c) * m;
            umin = fminf(umin, u);
            umax = fmaxf(umax, u);
            mmin = fminf(mmin, m);
            mmax = fmaxf(mmax, m);
        }
        const float vmin = zlo * (zlo < 0.f ? mmax : mmin) * rdv + vcen - kFootMargin;
        const float vmax = zhi * (zhi < 0.f ? mmin : mmax) * rdv + vcen + kFootMargin;
        umin = umin * rdu + ucen - kFootMargin;
        umax = umax * rdu + ucen + kFootMargin;
        // clamped in float before converting
        const int u0 = (int)fmaxf(0.f, ceilf(umin)), u1 = (int)fminf(g.nu - 1.f, floorf(umax));
        const int v0 = (int)fmaxf(0.f, ceilf(vmin)), v1 = (int)fminf(g.nv - 1.f, floorf(vmax));
        // the centre row of an odd nv (rays in the plane z = 0) reaches this
        // voxel only if its half-open z range holds 0; where it does not, that
        // row can only be the footprint's last (the voxel's top face is z = 0)
        const int v1c = (TAB && (g.nv & 1) && !zin0 && v1 == (g.nv - 1) / 2) ? v1 - 1 : v1;
        const float *pa = proj + ((int64_t)i * g.na + a) * g.nu * g.nv;
        for (int iu = u0; iu <= u1; ++iu) {
            // the ray of pixel (iu, iv): source S = sid (c, s, 0), direction
            // d = (dxy, ov) with dxy from iu alone and ov from iv alone
            const float ou = (iu - ucen) * g.du;
            const float S0 = g.sid * c, S1 = g.sid * s;
            const float d0 = -g.sdd * c - ou * s, d1 = -g.sdd * s + ou * c;
            float txy0, txy1, a0, a1;
            bool hxy = vslab(S0, d0, cen[0] - 0.5f, cen[0] + 0.5f, x == g.nx - 1, a0, a1);
            txy0 = fmaxf(-INFINITY, a0);
            txy1 = fminf(INFINITY, a1);
            hxy = vslab(S1, d1, cen[1] - 0.5f, cen[1] + 0.5f, y == g.ny - 1, a0, a1) && hxy;
            txy0 = fmaxf(txy0, a0);
            txy1 = fminf(txy1, a1);
            // a column whose rays miss the voxel's x-y extent adds nothing
            if (!hxy || !(txy1 > txy0))
                continue;
            const float d01 = d0 * d0 + d1 * d1;
            const float *pcol = pa + (int64_t)iu * g.nv;
            // length x value of pixel iv's ray inside the voxel; the value is
            // read only where the ray meets the voxel (add) or handed in (addv)
            auto addv = [&](bool use, float val, float ov, float z0, float z1) {
                const float tin = vmaxf(txy0, z0), tout = vminf(txy1, z1);
                if (use && tout > tin) {
                    // the hardware square root (within 1 ulp; the argument
                    // is at least sdd^2, far from denormals)
                    const float L = __builtin_amdgcn_sqrtf(d01 + ov * ov);
                    acc = fmaf((tout - tin) * L, val, acc);
                }
            };
            auto add = [&](int iv, float ov, float z0, float z1) {
                const float tin = vmaxf(txy0, z0), tout = vminf(txy1, z1);
                if (tout > tin) {
                    const float L = __builtin_amdgcn_sqrtf(d01 + ov * ov);
                    acc = fmaf((tout - tin) * L, pcol[iv], acc);
                }
            };
            if (TAB) {
                const float4 *rtab = (const float4 *)(tab + row_tab_offset(nang));
                int iv = v0;
                if (g.nv >= 4 && v0 <= v1c) {
                    // the first rows of the column come from one 16-byte load
                    // (a gather's cost is set by its address count, not its
                    // width), placed inside the column; rows of it outside
                    // [v0, v1c] are skipped, so the same rows are summed in
                    // the same order
                    const int vs = min(v0, g.nv - 4);
                    Float4u q;
                    __builtin_memcpy(&q, pcol + vs, sizeof(q));
                    const float qv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float4 r = rtab[vs + k];
                        addv(vs + k >= v0 && vs + k <= v1c, qv[k], r.w, fmaf(zlo, r.x, r.y),
                             fmaf(zlo, r.x, r.z));
                    }
                    iv = vs + 4;
                }
                for (; iv <= v1c; ++iv) {
                    const float4 r = rtab[iv];
                    add(iv, r.w, fmaf(zlo, r.x, r.y), fmaf(zlo, r.x, r.z));
                }
            } else {
                for (int iv = v0; iv <= v1; ++iv) {
                    const float ov = (iv - vcen) * g.dv;
                    float z0, z1;
                    if (vslab(0.f, ov, zlo, zhi, z == g.nz - 1, z0, z1))
                        add(iv, ov, z0, z1);
                }
            }
        }
    }
    vol[t] = acc;
}

// ---- CGLS (per phase, scalars on the device) ------------------------------
// Workspace: r [np][R], q [np][R], p [np][N], s [np][N] (floats), then the
// per-phase scalars gamma, qq, gnew (compensated pairs), then the partial
// sums of the dot products.
constexpr int kDotBlocks = 64;  // partial sums per phase

__global__ void __launch_bounds__(kBlock) sub_kernel(int64_t n, const float *a, const float *b,
                                                     float *out)
{
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlock)
        out[t] = a[t] - b[t];
}

__global__ void __launch_bounds__(kBlock) copy_kernel(int64_t n, const float *a, float *out)
{
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlock)
        out[t] = a[t];
}

// partial[i][b]: compensated sum of a.b over block b's share of phase i
__global__ void __launch_bounds__(kBlock) pdot_kernel(int64_t len, const float *a, const float *b,
                                                      dfloat *partial)
{
    const int i = blockIdx.y, blk = blockIdx.x;
    const float *pa = a + (int64_t)i * len, *pb = b + (int64_t)i * len;
    dfloat acc{0.f, 0.f};
    for (int64_t t = (int64_t)blk * kBlock + threadIdx.x; t < len; t += (int64_t)kDotBlocks * kBlock)
        acc = df_add(acc, dfloat{pa[t] * pb[t], fmaf(pa[t], pb[t], -pa[t] * pb[t])});
    __shared__ dfloat sh[kBlock];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            sh[threadIdx.x] = df_add(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        partial[(int64_t)i * kDotBlocks + blk] = sh[0];
}

__global__ void pdot_final_kernel(int np, const dfloat *partial, dfloat *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np)
        return;
    dfloat acc = partial[(int64_t)i * kDotBlocks];
    for (int b = 1; b < kDotBlocks; ++b)
        acc = df_add(acc, partial[(int64_t)i * kDotBlocks + b]);
    out[i] = acc;
}

__device__ __forceinline__ float ratio(dfloat num, dfloat den)
{
    const float d = den.hi + den.lo;
    return d > 0.f ? (num.hi + num.lo) / d : 0.f;
}

// x += alpha p (volume), alpha = gamma / qq per phase
__global__ void __launch_bounds__(kBlock) axpy_vol_kernel(int np, int64_t len, const dfloat *gamma,
                                                          const dfloat *qq, const float *p, float *x)
{
    const int64_t n = (int64_t)np * len;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlock) {
        const int i = (int)(t / len);
        x[t] = fmaf(ratio(gamma[i], qq[i]), p[t], x[t]);
    }
}

// r -= alpha q (projections)
__global__ void __launch_bounds__(kBlock) axmy_proj_kernel(int np, int64_t len, const dfloat *gamma,
                                                           const dfloat *qq, const float *q, float *r)
{
    const int64_t n = (int64_t)np * len;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlock) {
        const int i = (int)(t / len);
        r[t] = fmaf(-ratio(gamma[i], qq[i]), q[t], r[t]);
    }
}

// p = s + beta p, beta = gnew / gamma per phase
__global__ void __launch_bounds__(kBlock) pupdate_kernel(int np, int64_t len, const dfloat *gnew,
                                                         const dfloat *gamma, const float *s, float *p)
{
    const int64_t n = (int64_t)np * len;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlock) {
        const int i = (int)(t / len);
        p[t] = fmaf(ratio(gnew[i], gamma[i]), p[t], s[t]);
    }
}

__global__ void scalar_copy_kernel(int np, const dfloat *a, dfloat *b)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np)
        b[i] = a[i];
}

__global__ void __launch_bounds__(kBlock) clamp_kernel(int64_t n, float *x)
{
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlock) {
        const float v = x[t];
        x[t] = v < 0.f ? 0.f : v;  // NaN stays NaN
    }
}

int64_t grid1(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    return b < 1 ? 1 : (b > 65536 ? 65536 : b);
}

struct CGWs {
    float *r, *q, *p, *s;
    dfloat *gamma, *qq, *gnew, *partial;
};

CGWs carve(const CTG &g, void *ws)
{
    CGWs w;
    char *c = (char *)ws;
    const int64_t pr = (int64_t)g.np * g.R, pv = (int64_t)g.np * g.N;
    w.r = (float *)c;
    w.q = w.r + pr;
    w.p = w.q + pr;
    w.s = w.p + pv;
    w.gamma = (dfloat *)(w.s + pv);
    w.qq = w.gamma + g.np;
    w.gnew = w.qq + g.np;
    w.partial = w.gnew + g.np;
    return w;
}

hipError_t pdot(const CTG &g, int64_t len, const float *a, const float *b, dfloat *partial,
                dfloat *out, hipStream_t s)
{
    pdot_kernel<<<dim3(kDotBlocks, g.np), kBlock, 0, s>>>(len, a, b, partial);
    pdot_final_kernel<<<(g.np + 63) / 64, 64, 0, s>>>(g.np, partial, out);
    return hipGetLastError();
}

}  // namespace

// ---- launchers used by the C ABI ------------------------------------------
size_t ct_workspace_bytes_impl(int np, int64_t N, int64_t R)
{
    return (size_t)np * (2 * R + 2 * N) * sizeof(float) +
           (size_t)np * (3 + kDotBlocks) * sizeof(dfloat);
}

static CTG make(const tnlm_ct_geom *p)
{
    CTG g;
    g.np = p->np;
    g.nx = p->nx;
    g.ny = p->ny;
    g.nz = p->nz;
    g.nu = p->nu;
    g.nv = p->nv;
    g.na = p->na;
    g.sid = p->sid;
    g.sdd = p->sdd;
    g.du = p->du;
    g.dv = p->dv;
    g.angles = p->angles;
    g.N = (int64_t)p->nx * p->ny * p->nz;
    g.R = (int64_t)p->na * p->nu * p->nv;
    return g;
}

hipError_t ct_project(const tnlm_ct_geom *p, const float *vol, float *proj, hipStream_t s)
{
    const CTG g = make(p);
    const int64_t n = (int64_t)g.np * g.R;
    project_kernel<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(g, vol, proj);
    return hipGetLastError();
}

hipError_t ct_backproject(const tnlm_ct_geom *p, const float *proj, float *vol, hipStream_t s)
{
    const CTG g = make(p);
    const int64_t n = (int64_t)g.np * g.N;
    const int64_t grid = (n + kBlock - 1) / kBlock;
    const int64_t nang = (int64_t)block_phase_span(g) * g.na;
    const int64_t tab = nang > (1 << 20) ? INT64_MAX
                                         : ((int64_t)row_tab_offset((int)nang) + 4 * g.nv) * sizeof(float);
    if (tab <= kTabBytes)
        backproject_kernel<true><<<grid, kBlock, (size_t)tab, s>>>(g, proj, vol);
    else
        backproject_kernel<false><<<grid, kBlock, 0, s>>>(g, proj, vol);
    return hipGetLastError();
}

hipError_t ct_cgls_init(const tnlm_ct_geom *p, const float *y, const float *x, void *ws,
                        hipStream_t s)
{
    const CTG g = make(p);
    CGWs w = carve(g, ws);
    const int64_t pr = (int64_t)g.np * g.R, pv = (int64_t)g.np * g.N;
    hipError_t e = ct_project(p, x, w.q, s);  // q = P x
    if (e != hipSuccess)
        return e;
    sub_kernel<<<grid1(pr), kBlock, 0, s>>>(pr, y, w.q, w.r);  // r = y - P x
    if ((e = ct_backproject(p, w.r, w.s, s)) != hipSuccess)    // s = P^T r
        return e;
    copy_kernel<<<grid1(pv), kBlock, 0, s>>>(pv, w.s, w.p);    // p = s
    return pdot(g, g.N, w.s, w.s, w.partial, w.gamma, s);      // gamma = |s|^2
}

hipError_t ct_cgls_step(const tnlm_ct_geom *p, float *x, void *ws, hipStream_t s)
{
    const CTG g = make(p);
    CGWs w = carve(g, ws);
    const int64_t pr = (int64_t)g.np * g.R, pv = (int64_t)g.np * g.N;
    hipError_t e = ct_project(p, w.p, w.q, s);  // q = P p
    if (e != hipSuccess)
        return e;
    if ((e = pdot(g, g.R, w.q, w.q, w.partial, w.qq, s)) != hipSuccess)  // qq = |q|^2
        return e;
    axpy_vol_kernel<<<grid1(pv), kBlock, 0, s>>>(g.np, g.N, w.gamma, w.qq, w.p, x);
    axmy_proj_kernel<<<grid1(pr), kBlock, 0, s>>>(g.np, g.R, w.gamma, w.qq, w.q, w.r);
    if ((e = ct_backproject(p, w.r, w.s, s)) != hipSuccess)  // s = P^T r
        return e;
    if ((e = pdot(g, g.N, w.s, w.s, w.partial, w.gnew, s)) != hipSuccess)
        return e;
    pupdate_kernel<<<grid1(pv), kBlock, 0, s>>>(g.np, g.N, w.gnew, w.gamma, w.s, w.p);
    scalar_copy_kernel<<<(g.np + 63) / 64, 64, 0, s>>>(g.np, w.gnew, w.gamma);
    return hipGetLastError();
}

hipError_t ct_clamp(float *x, int64_t n, hipStream_t s)
{
    clamp_kernel<<<grid1(n), kBlock, 0, s>>>(n, x);
    return hipGetLastError();
}

}  // namespace tnlm
