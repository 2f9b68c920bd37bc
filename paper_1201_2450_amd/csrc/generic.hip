// Generic TNLM kernels: one thread per output voxel, any patch radius d and
// search radius M, reading the volumes straight from global memory.
//
// These are the path for (d, M) outside the specialised tiled kernels and
// the baseline the tiled kernels are measured against. Arithmetic follows
// Eq. (3) (weights), Eq. (8) (Gauss-Jacobi step), Eq. (6) (frozen-weight
// operator) and the symmetrised energy of Eqs. (1)-(2) and its derivatives.
//
// Normalisation: the exponent of every candidate is taken relative to the
// patch distance D0 of the zero offset (always a valid candidate), so the
// zero-offset term is exactly 1 and the sum Z >= 1 never underflows. When a
// far better match than the zero offset makes Z overflow (Z >= 2^100), the
// voxel is redone relative to the exact minimum distance over its window.
#include <math.h>

#include "tnlm_internal.h"

namespace tnlm {
namespace {

constexpr int kBlock = 256;
constexpr float kZOverflow = 1.2676506e30f;  // 2^100

__device__ __forceinline__ int clampi(int a, int lo, int hi)
{
    return a < lo ? lo : (a > hi ? hi : a);
}

template <typename T>
__device__ __forceinline__ float ext(const Geo &g, const T *u, int i, int x, int y, int z)
{
    x = clampi(x, 0, g.nx - 1);
    y = clampi(y, 0, g.ny - 1);
    z = clampi(z, 0, g.nz - 1);
    return load_f(u, ((int64_t)i * g.nx + x) * (int64_t)g.ny * g.nz + (int64_t)y * g.nz + z);
}

template <typename T>
__device__ float patch_dist(const Geo &g, const T *u, int i, int j, int x, int y, int z,
                            int ox, int oy, int oz)
{
    float s = 0.f;
    for (int px = -g.d; px <= g.d; ++px)
        for (int py = -g.d; py <= g.d; ++py)
            for (int pz = -g.d; pz <= g.d; ++pz) {
                float a = ext(g, u, i, x + px, y + py, z + pz);
                float b = ext(g, u, j, x + ox + px, y + oy + py, z + oz + pz);
                float t = a - b;
                s = fmaf(t, t, s);
            }
    return s;
}

__device__ __forceinline__ int neighbour(const Geo &g, int i, int slot)
{
    return slot == 0 ? (i + 1 == g.np ? 0 : i + 1) : (i == 0 ? g.np - 1 : i - 1);
}

struct Acc {
    float Z, num, er2;
};

// Sums over the valid window of voxel (i; x,y,z) towards phase j, with every
// exponent taken relative to distance `ref`.
template <typename T, bool WANT_F, bool WANT_R2>
__device__ Acc window_sums(const Geo &g, const T *u, const T *f, int i, int j, int x,
                           int y, int z, float ref, float fi)
{
    Acc a{0.f, 0.f, 0.f};
    const int x0 = max(-g.M, -x), x1 = min(g.M, g.nx - 1 - x);
    const int y0 = max(-g.M, -y), y1 = min(g.M, g.ny - 1 - y);
    const int z0 = max(-g.M, -z), z1 = min(g.M, g.nz - 1 - z);
    for (int ox = x0; ox <= x1; ++ox)
        for (int oy = y0; oy <= y1; ++oy)
            for (int oz = z0; oz <= z1; ++oz) {
                float D = patch_dist(g, u, i, j, x, y, z, ox, oy, oz);
                float e = __builtin_amdgcn_exp2f((ref - D) * g.c2);
                a.Z += e;
                if (WANT_F) {
                    int64_t q = (((int64_t)j * g.nx + x + ox) * g.ny + y + oy) * g.nz + z + oz;
                    float fj = load_f(f, q);
                    a.num = fmaf(e, fj, a.num);
                    if (WANT_R2) {
                        float r = fi - fj;
                        a.er2 = fmaf(e * r, r, a.er2);
                    }
                }
            }
    return a;
}

template <typename T>
__device__ float window_min_dist(const Geo &g, const T *u, int i, int j, int x, int y, int z)
{
    float m = INFINITY;
    const int x0 = max(-g.M, -x), x1 = min(g.M, g.nx - 1 - x);
    const int y0 = max(-g.M, -y), y1 = min(g.M, g.ny - 1 - y);
    const int z0 = max(-g.M, -z), z1 = min(g.M, g.nz - 1 - z);
    for (int ox = x0; ox <= x1; ++ox)
        for (int oy = y0; oy <= y1; ++oy)
            for (int oz = z0; oz <= z1; ++oz)
                m = fminf(m, patch_dist(g, u, i, j, x, y, z, ox, oy, oz));
    return m;
}

// Normalised sums for one voxel and direction; returns the reference
// distance used so that log Z = log(a.Z) - ref * inv2h2.
template <typename T, bool WANT_F, bool WANT_R2>
__device__ float voxel_dir(const Geo &g, const T *u, const T *f, int i, int j, int x, int y,
                           int z, float fi, Acc &a)
{
    float ref = patch_dist(g, u, i, j, x, y, z, 0, 0, 0);
    a = window_sums<T, WANT_F, WANT_R2>(g, u, f, i, j, x, y, z, ref, fi);
    if (!(a.Z < kZOverflow)) {
        float m = window_min_dist(g, u, i, j, x, y, z);
        if (m == m) {  // NaN inputs: keep the NaN result
            ref = m;
            a = window_sums<T, WANT_F, WANT_R2>(g, u, f, i, j, x, y, z, ref, fi);
        }
    }
    return ref;
}

template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock) fwd_generic_kernel(Geo g, FwdArgs a)
{
    const T *u = (const T *)a.u;
    const T *f = (const T *)a.f;
    const int64_t total = (int64_t)g.np * g.N;
    dfloat part{0.f, 0.f};
    for (int64_t flat = (int64_t)blockIdx.x * kBlock + threadIdx.x; flat < total;
         flat += (int64_t)gridDim.x * kBlock) {
        const int i = (int)(flat / g.N);
        const int64_t v = flat - (int64_t)i * g.N;
        const int z = (int)(v % g.nz);
        const int y = (int)((v / g.nz) % g.ny);
        const int x = (int)(v / ((int64_t)g.nz * g.ny));
        constexpr bool WF = MODE != FWD_WEIGHTS;
        constexpr bool WR = MODE == FWD_ENERGY;
        const float fi = WF ? load_f(f, flat) : 0.f;
        float nbsum = 0.f;
        dfloat esum{0.f, 0.f};
        for (int slot = 0; slot < 2; ++slot) {
            const int j = neighbour(g, i, slot);
            Acc acc;
            float ref = voxel_dir<T, WF, WR>(g, u, f, i, j, x, y, z, fi, acc);
            const float invZ = 1.f / acc.Z;
            const float lse = logf(acc.Z) - ref * g.inv2h2;
            if (MODE == FWD_WEIGHTS) {
                if (a.lse)
                    a.lse[((int64_t)i * 2 + slot) * g.N + v] = lse;
                if (a.w) {
                    for (int ox = -g.M; ox <= g.M; ++ox)
                        for (int oy = -g.M; oy <= g.M; ++oy)
                            for (int oz = -g.M; oz <= g.M; ++oz) {
                                const int k = ((ox + g.M) * g.S + (oy + g.M)) * g.S + (oz + g.M);
                                float wv = 0.f;
                                if (x + ox >= 0 && x + ox < g.nx && y + oy >= 0 && y + oy < g.ny &&
                                    z + oz >= 0 && z + oz < g.nz) {
                                    float D = patch_dist(g, u, i, j, x, y, z, ox, oy, oz);
                                    wv = __builtin_amdgcn_exp2f((ref - D) * g.c2) * invZ;
                                }
                                a.w[(((int64_t)i * 2 + slot) * g.W + k) * g.N + v] = wv;
                            }
                }
            } else if (MODE == FWD_ENERGY) {
                const float e = acc.er2 * invZ;
                if (a.stats) {
                    a.stats[(((int64_t)i * 2 + slot) * 2 + 0) * g.N + v] = lse;
                    a.stats[(((int64_t)i * 2 + slot) * 2 + 1) * g.N + v] = e;
                }
                esum = df_add(esum, dfloat{e, 0.f});
            } else {
                nbsum += acc.num * invZ;
            }
        }
        if (MODE == FWD_JACOBI) {
            const float gi = load_f((const T *)a.g, flat);
            const float r = 1.f / (2.f + a.mu);
            store_f((T *)a.out, flat, fmaf(a.mu * r, gi, nbsum * r));
        } else if (MODE == FWD_EQ6) {
            ((float *)a.out)[flat] = 2.f * fi - nbsum;
        } else if (MODE == FWD_ENERGY) {
            part = df_add(part, esum);
        }
    }
    if (MODE == FWD_ENERGY) {
        // fixed-order block reduction of (hi, lo) pairs
        __shared__ dfloat sh[kBlock];
        sh[threadIdx.x] = part;
        __syncthreads();
        for (int off = kBlock / 2; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off)
                sh[threadIdx.x] = df_add(sh[threadIdx.x], sh[threadIdx.x + off]);
            __syncthreads();
        }
        if (threadIdx.x == 0)
            a.partial[blockIdx.x] = sh[0];
    }
}

// ---------------------------------------------------------------------------
// Exact gradient, gather form. For output voxel q of phase k:
//   dE/df_k(q) = 1/2 sum_s sum_{delta in V(q)} [w_{k->j}(q,delta) +
//                w_{j->k}(q+delta,-delta)] (f_k(q) - f_j(q+delta)),   j = k+s;
//   dE/du_k(q) = sum over padded positions q' that clamp to q of
//                2 sum_s sum_delta (U_k(q') - U_j(q'+delta)) G_s(q', delta),
//   G_s(q',delta) = sum_p [Dbar_{k,s}(q'-p, delta) + Dbar_{j,-s}(q'-p+delta, -delta)],
//   Dbar_{i,s}(v, delta) = -(1/(8h^2)) w_{i->j}(v,delta) (r^2 - e_{i,s}(v)),
// with Dbar = 0 unless v and v+delta are both in the grid. The weights are
// rebuilt from the saved log-normalisers: w = exp(-D/(2h^2) - lse).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) grad_exact_generic_kernel(Geo g, GradArgs a)
{
    const T *u = (const T *)a.u;
    const T *f = (const T *)a.f;
    const float L2E = 1.4426950408889634f;
    const int64_t total = (int64_t)g.np * g.N;
    for (int64_t flat = (int64_t)blockIdx.x * kBlock + threadIdx.x; flat < total;
         flat += (int64_t)gridDim.x * kBlock) {
        const int k = (int)(flat / g.N);
        const int64_t q = flat - (int64_t)k * g.N;
        const int z = (int)(q % g.nz);
        const int y = (int)((q / g.nz) % g.ny);
        const int x = (int)(q / ((int64_t)g.nz * g.ny));
        auto st = [&](int ph, int slot, int comp, int64_t v) {
            return a.stats[(((int64_t)ph * 2 + slot) * 2 + comp) * g.N + v];
        };
        auto vflat = [&](int xx, int yy, int zz) {
            return ((int64_t)xx * g.ny + yy) * g.nz + zz;
        };
        auto inside = [&](int xx, int yy, int zz) {
            return xx >= 0 && xx < g.nx && yy >= 0 && yy < g.ny && zz >= 0 && zz < g.nz;
        };
        float gimg = 0.f, gw = 0.f;
        const float fk = load_f(f, flat);
        if (a.grad_f) {
            for (int slot = 0; slot < 2; ++slot) {
                const int j = neighbour(g, k, slot), back = 1 - slot;
                const float lse_c = st(k, slot, 0, q);
                for (int ox = -g.M; ox <= g.M; ++ox)
                    for (int oy = -g.M; oy <= g.M; ++oy)
                        for (int oz = -g.M; oz <= g.M; ++oz) {
                            if (!inside(x + ox, y + oy, z + oz))
                                continue;
                            const int64_t qn = vflat(x + ox, y + oy, z + oz);
                            const float av = -patch_dist(g, u, k, j, x, y, z, ox, oy, oz) * g.inv2h2;
                            const float w1 = __builtin_amdgcn_exp2f((av - lse_c) * L2E);
                            const float w2 = __builtin_amdgcn_exp2f((av - st(j, back, 0, qn)) * L2E);
                            gimg = fmaf(0.5f * (w1 + w2), fk - load_f(f, (int64_t)j * g.N + qn), gimg);
                        }
            }
        }
        if (a.grad_u) {
            const float s8 = -0.25f * g.inv2h2;  // -1/(8h^2)
            int lo[3], hi[3];
            const int qq[3] = {x, y, z}, nn[3] = {g.nx, g.ny, g.nz};
            for (int ax = 0; ax < 3; ++ax) {
                lo[ax] = qq[ax] == 0 ? -g.d : qq[ax];
                hi[ax] = qq[ax] == nn[ax] - 1 ? nn[ax] - 1 + g.d : qq[ax];
            }
            for (int qx = lo[0]; qx <= hi[0]; ++qx)
                for (int qy = lo[1]; qy <= hi[1]; ++qy)
                    for (int qz = lo[2]; qz <= hi[2]; ++qz)
                        for (int slot = 0; slot < 2; ++slot) {
                            const int j = neighbour(g, k, slot), back = 1 - slot;
                            for (int ox = -g.M; ox <= g.M; ++ox)
                                for (int oy = -g.M; oy <= g.M; ++oy)
                                    for (int oz = -g.M; oz <= g.M; ++oz) {
                                        float G = 0.f;
                                        for (int px = -g.d; px <= g.d; ++px)
                                            for (int py = -g.d; py <= g.d; ++py)
                                                for (int pz = -g.d; pz <= g.d; ++pz) {
                                                    const int vx = qx - px, vy = qy - py, vz = qz - pz;
                                                    if (!inside(vx, vy, vz) ||
                                                        !inside(vx + ox, vy + oy, vz + oz))
                                                        continue;
                                                    const int64_t v = vflat(vx, vy, vz);
                                                    const int64_t vn = vflat(vx + ox, vy + oy, vz + oz);
                                                    const float av =
                                                        -patch_dist(g, u, k, j, vx, vy, vz, ox, oy, oz) *
                                                        g.inv2h2;
                                                    const float r = load_f(f, (int64_t)k * g.N + v) -
                                                                    load_f(f, (int64_t)j * g.N + vn);
                                                    const float r2 = r * r;
                                                    const float w1 = __builtin_amdgcn_exp2f(
                                                        (av - st(k, slot, 0, v)) * L2E);
                                                    const float w2 = __builtin_amdgcn_exp2f(
                                                        (av - st(j, back, 0, vn)) * L2E);
                                                    G = fmaf(w1, r2 - st(k, slot, 1, v), G);
                                                    G = fmaf(w2, r2 - st(j, back, 1, vn), G);
                                                }
                                        if (G == 0.f)
                                            continue;
                                        const float Delta = ext(g, u, k, qx, qy, qz) -
                                                            ext(g, u, j, qx + ox, qy + oy, qz + oz);
                                        gw = fmaf(2.f * s8 * Delta, G, gw);
                                    }
                        }
        }
        if (a.grad_f && a.grad_u == a.grad_f) {
            a.grad_f[flat] = gimg + gw;
        } else {
            if (a.grad_f)
                a.grad_f[flat] = gimg;
            if (a.grad_u)
                a.grad_u[flat] = gw;
        }
    }
}

__global__ void __launch_bounds__(1024) energy_final_kernel(const dfloat *partial, int64_t n,
                                                             float *e_out)
{
    __shared__ dfloat sh[1024];
    dfloat acc{0.f, 0.f};
    for (int64_t b = threadIdx.x; b < n; b += 1024)
        acc = df_add(acc, partial[b]);
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            sh[threadIdx.x] = df_add(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // E = 1/4 of the sum (exact scaling by a power of two)
        e_out[0] = 0.25f * sh[0].hi;
        e_out[1] = 0.25f * sh[0].lo;
    }
}

int64_t grid_for(int64_t total)
{
    int64_t b = (total + kBlock - 1) / kBlock;
    return b < 1 ? 1 : (b > 65536 ? 65536 : b);
}

template <typename T>
hipError_t fwd_dispatch(const Geo &g, int mode, const FwdArgs &a, hipStream_t s)
{
    const int64_t blocks = grid_for((int64_t)g.np * g.N);
    switch (mode) {
    case FWD_WEIGHTS:
        fwd_generic_kernel<T, FWD_WEIGHTS><<<blocks, kBlock, 0, s>>>(g, a);
        break;
    case FWD_JACOBI:
        fwd_generic_kernel<T, FWD_JACOBI><<<blocks, kBlock, 0, s>>>(g, a);
        break;
    case FWD_EQ6:
        fwd_generic_kernel<T, FWD_EQ6><<<blocks, kBlock, 0, s>>>(g, a);
        break;
    default:
        fwd_generic_kernel<T, FWD_ENERGY><<<blocks, kBlock, 0, s>>>(g, a);
        break;
    }
    return hipGetLastError();
}

}  // namespace

int64_t energy_blocks_generic(const Geo &g) { return grid_for((int64_t)g.np * g.N); }

hipError_t launch_fwd_generic(const Geo &g, int dtype, int mode, const FwdArgs &a, hipStream_t s)
{
    switch (dtype) {
    case TNLM_F32:
        return fwd_dispatch<float>(g, mode, a, s);
    case TNLM_BF16:
        return fwd_dispatch<bf16_t>(g, mode, a, s);
    default:
        return fwd_dispatch<_Float16>(g, mode, a, s);
    }
}

hipError_t launch_grad_exact_generic(const Geo &g, int dtype, const GradArgs &a, hipStream_t s)
{
    const int64_t blocks = grid_for((int64_t)g.np * g.N);
    switch (dtype) {
    case TNLM_F32:
        grad_exact_generic_kernel<float><<<blocks, kBlock, 0, s>>>(g, a);
        break;
    case TNLM_BF16:
        grad_exact_generic_kernel<bf16_t><<<blocks, kBlock, 0, s>>>(g, a);
        break;
    default:
        grad_exact_generic_kernel<_Float16><<<blocks, kBlock, 0, s>>>(g, a);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_energy_final(const dfloat *partial, int64_t n, float *e_out, hipStream_t s)
{
    energy_final_kernel<<<1, 1024, 0, s>>>(partial, n, e_out);
    return hipGetLastError();
}

}  // namespace tnlm
