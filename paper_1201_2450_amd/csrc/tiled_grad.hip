// Tiled exact gradient of the TNLM energy for 3x3x3 patches (d = 1) and
// search radius M = 1..5, gather form, from the saved per-voxel statistics
// (log-normaliser and e of every voxel and direction).
//
// For output phase k, neighbour j = k+s and search offset delta:
//   image part   dE/df_k(q) += 1/2 (w1 + w2) r,      q in the grid,
//   weight part  dE/dU_k(q') += 2 Delta(q') sum_p Gv(q'-p),
// with, at every position v with v and v+delta in the grid,
//   D  = patch distance between u_k around v and u_j around v+delta,
//   w1 = exp(-D/(2h^2) - lse_{k,s}(v)),  w2 = exp(-D/(2h^2) - lse_{j,-s}(v+delta)),
//   r  = f_k(v) - f_j(v+delta),
//   Gv = -(1/(8h^2)) [w1 (r^2 - e_{k,s}(v)) + w2 (r^2 - e_{j,-s}(v+delta))],
//   Delta(q') = U_k(q') - U_j(q'+delta)  (clamp-to-edge values).
// The weight part lives on the padded grid (every q' within one voxel of the
// grid, since patches reach one voxel out); a second kernel folds each padded
// position onto the grid voxel it clamps to, which is the chain rule through
// the clamp-to-edge extension.
//
// Work layout: a workgroup owns 2 (x) x 56 (y) x 4*ZB (z) padded outputs of
// one phase (ZB z-blocks: 2 when u = f, else 4); lanes run along y in 32-lane
// segments (two halo rows on each side: one for the distance box, one for the
// Gv box, so 28 outputs per segment); each lane keeps 2 (x) x 4 (z) outputs.
// Two waves own each z-block and split the (dy, dz) offset pairs between them
// (alternate pairs), sharing one LDS tile; their partial sums are added in a
// fixed order at the end. With ZB = 2 two workgroups (8 waves) share a CU, so
// one stages its tile while the other computes. Per
// search offset a lane builds D on its block grown by one voxel in x and z
// (box sums of squared differences as in the forward kernel), forms Gv there,
// and box-sums Gv back onto its outputs; the 3-tap box sums along z and x
// share the pair sums of neighbouring outputs, and the y box runs across
// lanes with DPP. The neighbour phase's u_j, f_j and statistics are staged in
// LDS one dx at a time, clamped to the grid; the two statistics of a position
// sit side by side, so one ds_read2 fetches both.
#include <math.h>

#include <type_traits>

#include "tnlm_internal.h"

namespace tnlm {
namespace {

constexpr int kBX = 2;            // outputs per lane in x
constexpr int kBZ = 4;            // outputs per lane in z
static_assert(kBX % 2 == 0 && kBZ % 2 == 0, "pair-shared box sums need even blocks");
constexpr int kEX = kBX + 2;      // Gv positions per lane in x
constexpr int kEZ = kBZ + 2;      // Gv positions per lane in z
constexpr int kSX = kBX + 4;      // squared-difference planes per lane
constexpr int kSZ = kBZ + 4;      // squared-difference z per lane
constexpr int kSegOut = 28;       // outputs per 32-lane segment
#ifndef TNLM_GRAD_SETS
#define TNLM_GRAD_SETS 2
#endif
constexpr int kSets = TNLM_GRAD_SETS;  // waves per z-block, splitting the offset pairs
constexpr int kTY = 2 * kSegOut;  // 56
constexpr float kLog2e = 1.4426950408889634f;

// Workgroup shape per instance: the u = f instance (no f_j tile) takes two
// z-blocks up to M = 4, so its LDS tile (~67 KB at M = 3, 77 KB at M = 4)
// lets two workgroups share a CU and one stages while the other computes;
// the general instance, with f_j staged too, and M = 5 take four z-blocks
// (one workgroup of eight waves per CU).
constexpr int kMaxTiledM = 5;  // search radii with a tiled instance
template <bool SAME, int M>
struct Lay {
    static constexpr int ZB = (SAME && M <= 4) ? 2 : 4;  // z-blocks per workgroup
    static constexpr int THREADS = kSets * 64 * ZB;
    static constexpr int TZ = ZB * kBZ;                 // padded z outputs per workgroup
};
constexpr int kMinTZ = Lay<true, 1>::TZ;

template <int M, bool SAME>
struct GG {
    static constexpr int YL = kTY + 4 + 2 * M;              // rows Y0-2-M .. Y0+kTY+1+M
    static constexpr int ZL = Lay<SAME, M>::TZ + 4 + 2 * M;  // z    Z0-2-M .. Z0+TZ+1+M
    static constexpr int RU = (kSX * ZL) | 1;      // u_j row: kSX planes
    static constexpr int RV = (kEX * ZL) | 1;      // f_j row: kEX planes
    static constexpr int RS = (2 * kEX * ZL) | 1;  // (L2, e2) row: pairs, kEX planes
    static_assert((kSX - 1) * ZL + kSZ < 256, "ds_read2 offsets");
    static_assert(2 * ((kEX - 1) * ZL + kEZ) < 256, "ds_read2 offsets");
};

struct GradGrid {
    int ntx, nty, ntz, nblocks;
};

__device__ __forceinline__ float from_below(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_above(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}

__device__ __forceinline__ int clampi(int a, int lo, int hi)
{
    return a < lo ? lo : (a > hi ? hi : a);
}

// SAME: the image is the weight source (f and u are one volume), so f_j is
// the staged u_j and the residual r is the centre squared-difference term.
template <typename T, int M, bool SAME>
__global__ void __launch_bounds__((Lay<SAME, M>::THREADS))
    grad_tiled_kernel(Geo g, GradArgs a, float *gpad, GradGrid gg)
{
    using G = GG<M, SAME>;
    constexpr int kWaves = Lay<SAME, M>::ZB;
    constexpr int kThreads = Lay<SAME, M>::THREADS;
    constexpr int kTZ = Lay<SAME, M>::TZ;
    __shared__ float sU[G::YL * G::RU];
    __shared__ float sF[SAME ? 1 : G::YL * G::RV];  // f_j (u_j when SAME)
    __shared__ float sS[G::YL * G::RS];  // (-lse*log2e, e2) side by side

    const int b = blockIdx.x;
    const int q8 = gg.nblocks >> 3, r8 = gg.nblocks & 7, xcd = b & 7;
    int t = xcd * q8 + min(xcd, r8) + (b >> 3);
    const int tz = t % gg.ntz;
    t /= gg.ntz;
    const int ty = t % gg.nty;
    t /= gg.nty;
    const int tx = t % gg.ntx;
    const int k = t / gg.ntx;
    // padded coordinates: P = grid + 1, P in [0, N+2)
    const int X0 = tx * kBX, Y0 = ty * kTY, Z0 = tz * kTZ;

    const int tid = threadIdx.x;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wave = wid & (kWaves - 1);  // z-block
    const int half = wid / kWaves;        // which (dy, dz) pairs this wave takes (set)
    const int lane = tid & 63, seg = lane >> 5, l = lane & 31;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int64_t N = g.N;
    const int Yp = Y0 - 2 + kSegOut * seg + l;  // this lane's padded y
    const int y = Yp - 1;                         // grid y (may be outside)
    const int zb = Z0 + kBZ * wave;               // first padded output z (uniform)
    const bool yout = l >= 2 && l <= kSegOut + 1 && Yp < ny + 2;
    const int ry = kSegOut * seg + l + M;          // LDS row of this lane's y
    const int zoffU = kBZ * wave + M;              // LDS z of padded zb-2 (dz = 0)
    const int zoffV = kBZ * wave + M + 1;          // LDS z of padded zb-1 (dz = 0)

    const T *u = (const T *)a.u;
    const T *f = (const T *)a.f;
    auto vox = [&](int ph, int xx, int yy, int zz) -> int64_t {
        return (int64_t)ph * N + ((int64_t)xx * ny + yy) * nz + zz;
    };
    auto st = [&](int ph, int slot, int comp, int xx, int yy, int zz) -> float {
        return a.stats[(((int64_t)ph * 2 + slot) * 2 + comp) * N + ((int64_t)xx * ny + yy) * nz + zz];
    };
    const int yc = clampi(y, 0, ny - 1);
    const bool yin = (unsigned)y < (unsigned)ny;

    // u_k on the squared-difference block: padded x X0-2 .. X0+kBX+1, z zb-2 .. zb+kBZ+1
    float uk[kSX][kSZ];
#pragma unroll
    for (int xs = 0; xs < kSX; ++xs)
#pragma unroll
        for (int zs = 0; zs < kSZ; ++zs)
            uk[xs][zs] = load_f(u, vox(k, clampi(X0 - 3 + xs, 0, nx - 1), yc,
                                       clampi(zb - 3 + zs, 0, nz - 1)));
    // f_k on the Gv block (padded X0-1 .. X0+kBX, zb-1 .. zb+kBZ)
    float fk[SAME ? 1 : kEX][SAME ? 1 : kEZ];
    if (!SAME) {
#pragma unroll
        for (int xe = 0; xe < kEX; ++xe)
#pragma unroll
            for (int ze = 0; ze < kEZ; ++ze)
                fk[xe][ze] = load_f(f, vox(k, clampi(X0 - 2 + xe, 0, nx - 1), yc,
                                           clampi(zb - 2 + ze, 0, nz - 1)));
    }

    float gw[kBX][kBZ], gi[kBX][kBZ];
#pragma unroll
    for (int xo = 0; xo < kBX; ++xo)
#pragma unroll
        for (int zo = 0; zo < kBZ; ++zo) {
            gw[xo][zo] = 0.f;
            gi[xo][zo] = 0.f;
        }

    // waves whose every Gv position v has v and v+delta in the grid for all
    // offsets skip the masks: x and y decided per workgroup, z per wave (its
    // z-block), uniform over the wave; both sweeps meet the same barriers
    const bool border = (X0 - 2 - M < 1) || (X0 + kBX + 1 + M > nx) || (Y0 - 2 - M < 1) ||
                        (Y0 + kTY + 1 + M > ny) || (zb - 2 - M < 1) || (zb + kBZ + 1 + M > nz);
    const float nc2 = in_vgpr(-g.c2);  // the exponent's factor, in a vector register

    for (int slot = 0; slot < 2; ++slot) {
        const int j = slot == 0 ? (k + 1 == g.np ? 0 : k + 1) : (k == 0 ? g.np - 1 : k - 1);
        const int back = 1 - slot;
        // own-side statistics on the Gv block
        float L1[kEX][kEZ], e1[kEX][kEZ];
#pragma unroll
        for (int xe = 0; xe < kEX; ++xe)
#pragma unroll
            for (int ze = 0; ze < kEZ; ++ze) {
                const int xx = clampi(X0 - 2 + xe, 0, nx - 1), zz = clampi(zb - 2 + ze, 0, nz - 1);
                L1[xe][ze] = -st(k, slot, 0, xx, yc, zz) * kLog2e;  // negated, log2 units
                e1[xe][ze] = st(k, slot, 1, xx, yc, zz);
            }

        auto sweep = [&](auto bord_c) {
            constexpr bool bord = decltype(bord_c)::value;
            for (int dx = -M; dx <= M; ++dx) {
                __syncthreads();
                {
                    // stage u_j (kSX planes from padded X0-2+dx) and f_j, L2, e2
                    // (kEX planes from padded X0-1+dx), clamped to the grid. A
                    // lane takes (row, z) cells, clamps each once and loads it
                    // from every plane through uniform plane bases.
                    const int64_t plane = (int64_t)ny * nz;
                    const T *up[kSX];
                    const T *fp[kEX];
                    const float *lp[kEX], *ep[kEX];
#pragma unroll
                    for (int p = 0; p < kSX; ++p)
                        up[p] = u + (int64_t)j * N + clampi(X0 - 3 + dx + p, 0, nx - 1) * plane;
#pragma unroll
                    for (int p = 0; p < kEX; ++p) {
                        const int64_t gx = clampi(X0 - 2 + dx + p, 0, nx - 1) * plane;
                        fp[p] = f + (int64_t)j * N + gx;
                        lp[p] = a.stats + ((int64_t)j * 2 + back) * 2 * N + gx;
                        ep[p] = lp[p] + N;
                    }
                    constexpr int kCells = G::YL * G::ZL;
                    for (int c = tid; c < kCells; c += kThreads) {
                        const int r = c / G::ZL, zc = c - r * G::ZL;
                        const int gy = clampi(Y0 - 3 - M + r, 0, ny - 1);
                        const int gz = clampi(Z0 - 3 - M + zc, 0, nz - 1);
                        // offset of the cell within a plane: ny*nz*4 < 2^32
                        const unsigned co = (unsigned)(gy * nz + gz);
                        auto at = [co](const auto *pl) {
                            using E = std::remove_cv_t<std::remove_reference_t<decltype(*pl)>>;
                            return load_f((const E *)((const char *)pl + co * (unsigned)sizeof(E)), 0);
                        };
                        float *su = sU + r * G::RU + zc;
#pragma unroll
                        for (int p = 0; p < kSX; ++p)
                            su[p * G::ZL] = at(up[p]);
                        float *sf = sF + r * G::RV + zc;
                        float *ss = sS + r * G::RS + 2 * zc;
#pragma unroll
                        for (int p = 0; p < kEX; ++p) {
                            if (!SAME)
                                sf[p * G::ZL] = at(fp[p]);
                            ss[2 * p * G::ZL] = -at(lp[p]) * kLog2e;  // negated, log2 units
                            ss[2 * p * G::ZL + 1] = at(ep[p]);
                        }
                    }
                }
                __syncthreads();
                constexpr int S = 2 * M + 1;
                for (int pr = half; pr < S * S; pr += kSets) {
                    const int dy = pr / S - M, dz = pr - (pr / S) * S - M;
                    const bool yval = yin && (unsigned)(y + dy) < (unsigned)ny;
                    {
                        lds_float *bu = lds_base(sU + (ry + dy) * G::RU + zoffU + dz);
                        lds_float *bf = lds_base(SAME ? sU : sF + (ry + dy) * G::RV + zoffV + dz);
                        lds_float *bs = lds_base(sS + (ry + dy) * G::RS + 2 * (zoffV + dz));
                        // D on the Gv block: box sums along z, x, then y (DPP);
                        // neighbouring outputs 2q, 2q+1 share the sum of
                        // inputs 2q+1 and 2q+2 (squares fused along z)
                        //
                        // When u = f each phase first reads all its LDS operands
                        // into registers behind a scheduling fence, so the reads
                        // are in flight together; left alone, the scheduler
                        // issues one read, waits for it and issues the next. (The
                        // u != f instance holds f_k too and has no registers to
                        // spare for the batches.)
                        float ub[kSX][kSZ];
#pragma unroll
                        for (int xs = 0; xs < kSX; ++xs)
#pragma unroll
                            for (int zs = 0; zs < kSZ; ++zs)
                                ub[xs][zs] = bu[xs * G::ZL + zs];
                        if (SAME)
                            __builtin_amdgcn_sched_barrier(0);
                        float D[kEX][kEZ];
                        float pz[kSX][kEZ];
                        float rc[SAME ? kEX : 1][SAME ? kEZ : 1];  // u_k - u_j on the Gv block
#pragma unroll
                        for (int xs = 0; xs < kSX; ++xs) {
                            float dd[kSZ];
#pragma unroll
                            for (int zs = 0; zs < kSZ; ++zs)
                                dd[zs] = uk[xs][zs] - ub[xs][zs];
                            if (SAME && xs >= 1 && xs <= kEX) {
#pragma unroll
                                for (int ze = 0; ze < kEZ; ++ze)
                                    rc[xs - 1][ze] = dd[ze + 1];
                            }
#pragma unroll
                            for (int ze = 0; ze < kEZ; ze += 2) {
                                const float pr = fmaf(dd[ze + 1], dd[ze + 1], dd[ze + 2] * dd[ze + 2]);
                                pz[xs][ze] = fmaf(dd[ze], dd[ze], pr);
                                pz[xs][ze + 1] = fmaf(dd[ze + 3], dd[ze + 3], pr);
                            }
                        }
#pragma unroll
                        for (int xe = 0; xe < kEX; xe += 2)
#pragma unroll
                            for (int ze = 0; ze < kEZ; ++ze) {
                                const float pr = pz[xe + 1][ze] + pz[xe + 2][ze];
                                D[xe][ze] = pz[xe][ze] + pr;
                                D[xe + 1][ze] = pr + pz[xe + 3][ze];
                            }
                        // y box across lanes, all reads of a pass after all writes
                        // of the previous one (no DPP read-after-write stalls)
                        float Dy[kEX][kEZ];
#pragma unroll
                        for (int xe = 0; xe < kEX; ++xe)
#pragma unroll
                            for (int ze = 0; ze < kEZ; ++ze)
                                Dy[xe][ze] = from_below(D[xe][ze]) + D[xe][ze];
#pragma unroll
                        for (int xe = 0; xe < kEX; ++xe)
#pragma unroll
                            for (int ze = 0; ze < kEZ; ++ze)
                                D[xe][ze] = Dy[xe][ze] + from_above(D[xe][ze]);
                        // Gv on the block; image part at the grid outputs
                        float sl[kEX][kEZ], se[kEX][kEZ];
#pragma unroll
                        for (int xe = 0; xe < kEX; ++xe)
#pragma unroll
                            for (int ze = 0; ze < kEZ; ++ze) {
                                sl[xe][ze] = bs[2 * (xe * G::ZL + ze)];
                                se[xe][ze] = bs[2 * (xe * G::ZL + ze) + 1];
                            }
                        if (SAME)
                            __builtin_amdgcn_sched_barrier(0);
                        float Gv[kEX][kEZ];
#pragma unroll
                        for (int xe = 0; xe < kEX; ++xe)
#pragma unroll
                            for (int ze = 0; ze < kEZ; ++ze) {
                                const float w1 = __builtin_amdgcn_exp2f(fmaf(D[xe][ze], nc2, L1[xe][ze]));
                                const float w2 = __builtin_amdgcn_exp2f(fmaf(D[xe][ze], nc2, sl[xe][ze]));
                                const float r = SAME ? rc[xe][ze] : fk[xe][ze] - bf[xe * G::ZL + ze];
                                const float r2 = r * r;
                                float gv = fmaf(w2, r2 - se[xe][ze], w1 * (r2 - e1[xe][ze]));
                                float wr = (w1 + w2) * r;
                                if (bord) {
                                    // v = padded (X0-1+xe, Yp, zb-1+ze) - 1 and v + delta in the grid
                                    const int vx = X0 - 2 + xe, vz = zb - 2 + ze;
                                    const bool ok = yval & ((unsigned)vx < (unsigned)nx) &
                                                    ((unsigned)(vx + dx) < (unsigned)nx) &
                                                    ((unsigned)vz < (unsigned)nz) &
                                                    ((unsigned)(vz + dz) < (unsigned)nz);
                                    gv = ok ? gv : 0.f;
                                    wr = ok ? wr : 0.f;
                                }
                                Gv[xe][ze] = gv;
                                if (xe >= 1 && xe <= kBX && ze >= 1 && ze <= kBZ)
                                    gi[xe - 1][ze - 1] += wr;
                            }
                        // box of Gv onto the outputs (z, x, then y), times Delta,
                        // with the same pair sharing
                        float gz[kEX][kBZ];
#pragma unroll
                        for (int xe = 0; xe < kEX; ++xe)
#pragma unroll
                            for (int zo = 0; zo < kBZ; zo += 2) {
                                const float pr = Gv[xe][zo + 1] + Gv[xe][zo + 2];
                                gz[xe][zo] = Gv[xe][zo] + pr;
                                gz[xe][zo + 1] = pr + Gv[xe][zo + 3];
                            }
                        float gx[kBX][kBZ], gy[kBX][kBZ];
#pragma unroll
                        for (int xo = 0; xo < kBX; xo += 2)
#pragma unroll
                            for (int zo = 0; zo < kBZ; ++zo) {
                                const float pr = gz[xo + 1][zo] + gz[xo + 2][zo];
                                gx[xo][zo] = gz[xo][zo] + pr;
                                gx[xo + 1][zo] = pr + gz[xo + 3][zo];
                            }
#pragma unroll
                        for (int xo = 0; xo < kBX; ++xo)
#pragma unroll
                            for (int zo = 0; zo < kBZ; ++zo)
                                gy[xo][zo] = from_below(gx[xo][zo]) + gx[xo][zo];
#pragma unroll
                        for (int xo = 0; xo < kBX; ++xo)
#pragma unroll
                            for (int zo = 0; zo < kBZ; ++zo) {
                                const float G3 = gy[xo][zo] + from_above(gx[xo][zo]);
                                // Delta at the output (the centre difference when u = f)
                                const float Dl = SAME ? rc[xo + 1][zo + 1]
                                                      : uk[xo + 2][zo + 2] - bu[(xo + 2) * G::ZL + zo + 2];
                                gw[xo][zo] = fmaf(Dl, G3, gw[xo][zo]);
                            }
                    }
                }
            }
        };
        if (border)
            sweep(std::true_type{});
        else
            sweep(std::false_type{});
    }

    // combine the sets in a fixed order: sets 1.. hand their sums over
    // through LDS, set 0 adds them in set order and writes
    __syncthreads();
    float *xfer = sU;  // the staging tile is free now
    constexpr int kPer = 2 * kBX * kBZ;
    static_assert((kSets - 1) * kWaves * 64 * kPer <= G::YL * G::RU, "transfer fits");
    if (half > 0) {
        float *xs = xfer + (((half - 1) * kWaves + wave) * 64 + lane) * kPer;
#pragma unroll
        for (int xo = 0; xo < kBX; ++xo)
#pragma unroll
            for (int zo = 0; zo < kBZ; ++zo) {
                xs[xo * kBZ + zo] = gw[xo][zo];
                xs[kBX * kBZ + xo * kBZ + zo] = gi[xo][zo];
            }
    }
    __syncthreads();
    if (half > 0)
        return;
    for (int h = 1; h < kSets; ++h) {
        const float *xs = xfer + (((h - 1) * kWaves + wave) * 64 + lane) * kPer;
#pragma unroll
        for (int xo = 0; xo < kBX; ++xo)
#pragma unroll
            for (int zo = 0; zo < kBZ; ++zo) {
                gw[xo][zo] += xs[xo * kBZ + zo];
                gi[xo][zo] += xs[kBX * kBZ + xo * kBZ + zo];
            }
    }

    // write: weight part to the padded buffer, image part to grad_f
    const float sw = -0.5f * g.inv2h2;  // 2 * (-1/(8h^2))
    const int64_t NP = (int64_t)(nx + 2) * (ny + 2) * (nz + 2);
#pragma unroll
    for (int xo = 0; xo < kBX; ++xo)
#pragma unroll
        for (int zo = 0; zo < kBZ; ++zo) {
            const int Xp = X0 + xo, Zp = zb + zo;
            if (!yout || Xp >= nx + 2 || Zp >= nz + 2)
                continue;
            if (gpad)
                gpad[(int64_t)k * NP + ((int64_t)Xp * (ny + 2) + Yp) * (nz + 2) + Zp] = sw * gw[xo][zo];
            const int xg = Xp - 1, zg = Zp - 1;
            if (a.grad_f && (unsigned)xg < (unsigned)nx && yin && (unsigned)zg < (unsigned)nz)
                a.grad_f[vox(k, xg, y, zg)] = 0.5f * gi[xo][zo];
        }
}

// grad_u(q) = sum of the padded weight-part values at every padded position
// that clamps to q (plus grad_f when the total gradient is asked for).
__global__ void __launch_bounds__(256) fold_kernel(Geo g, const float *gpad, float *grad_u,
                                                   const float *add)
{
    const int64_t total = (int64_t)g.np * g.N;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int64_t NP = (int64_t)(nx + 2) * (ny + 2) * (nz + 2);
    for (int64_t flat = (int64_t)blockIdx.x * 256 + threadIdx.x; flat < total;
         flat += (int64_t)gridDim.x * 256) {
        const int k = (int)(flat / g.N);
        const int64_t v = flat - (int64_t)k * g.N;
        const int z = (int)(v % nz), y = (int)((v / nz) % ny), x = (int)(v / ((int64_t)nz * ny));
        const int xl = x == 0 ? 0 : x + 1, xh = x == nx - 1 ? nx + 1 : x + 1;
        const int yl = y == 0 ? 0 : y + 1, yh = y == ny - 1 ? ny + 1 : y + 1;
        const int zl = z == 0 ? 0 : z + 1, zh = z == nz - 1 ? nz + 1 : z + 1;
        float s = 0.f;
        for (int X = xl; X <= xh; ++X)
            for (int Y = yl; Y <= yh; ++Y)
                for (int Z = zl; Z <= zh; ++Z)
                    s += gpad[(int64_t)k * NP + ((int64_t)X * (ny + 2) + Y) * (nz + 2) + Z];
        grad_u[flat] = add ? s + add[flat] : s;
    }
}

// ---------------------------------------------------------------------------
// Two-stage adjoint for u = f (the gradient of E(f; f)), M <= 3.
//
// The per-lane blocks above evaluate the distance and Gv on positions grown
// by a halo around each lane's outputs (4 x 6 Gv positions for 2 x 4
// outputs, two exponentials each). Here a workgroup evaluates Gv once per
// position of its tile (stage 1) into an LDS field, and box-sums that field
// back onto its outputs (stage 2), so every exponential serves the 27
// outputs around its position:
//   * tile: TX = 4 (x) x TY = 28 (y) x TZ = 14 (z) padded outputs of one
//     phase, 8 32-lane segments (256 threads, so two workgroups share a CU);
//     lane l of every segment sits on grid row Y0 - 3 + l;
//   * stage 1: segment s takes a 3 (x) x 4 (z) block of the 6 x 16 Gv
//     positions (grid x X0-2 .. X0+3, z Z0-2 .. Z0+13): squared differences
//     on its 5 x 6 block, box sums along z, x (pair sums shared) and y (DPP),
//     both weights, Gv and the image part; Gv goes to LDS;
//   * stage 2: segment s < 7 owns 4 (x) x 2 (z) outputs: reads the 6 x 4
//     Gv block around them, box sums along z, x and y (DPP), multiplies by
//     Delta = U_k(q') - U_j(q' + delta) and accumulates;
//   * u_j and the neighbour's statistics are staged per dx as above; per
//     (dy, dz) pair one barrier sits between stage 1's arithmetic and its
//     Gv stores (so the previous pair's stage-2 reads are done) and one
//     between the stores and stage 2.
// ---------------------------------------------------------------------------
namespace v2 {
constexpr int TX = 4, TY = 28, TZ = 14;  // padded outputs per tile
constexpr int GX = TX + 2, GZ = TZ + 2;  // Gv positions (x, z)
constexpr int SX = TX + 4, SZ = TZ + 4;  // squared-difference positions
constexpr int B1X = 3, B1Z = 4;          // stage-1 block (Gv positions)
constexpr int B2X = TX, B2Z = 2;         // stage-2 block (outputs)
constexpr int NSEG = 8, THREADS = 32 * NSEG;
constexpr int NSEG2 = TZ / B2Z;  // segments with stage-2 outputs (15)
static_assert(GX == 2 * B1X && GZ == (NSEG / 2) * B1Z, "stage-1 blocks tile the Gv field");
static_assert(NSEG2 <= NSEG && TZ % B2Z == 0, "stage-2 blocks tile the outputs");
// up to M = 3 the LDS (u_j, statistics, Gv) stays within 80 KB, so two
// workgroups share a CU; beyond, one 4-wave workgroup per CU leaves one wave
// per SIMD and the per-lane kernel is faster (fbs512, M = 4: 3.40 s against
// 2.22 s)
constexpr int kMaxM = 3;

template <int M>
struct Lay {
    static constexpr int UR = 32 + 2 * M;  // u_j rows (lanes 0..31, +-M)
    static constexpr int UZ = SZ + 2 * M;  // u_j z
    static constexpr int RU = (SX * UZ) | 1;
    static constexpr int SR = 32 + 2 * M;  // statistics rows
    static constexpr int SZL = GZ + 2 * M; // statistics z
    static constexpr int RS = (2 * GX * SZL) | 1;
    static constexpr int RG = (GX * GZ) | 1;  // Gv field row stride
    // Gv rows of lanes 1..30, plus one row that lanes 0 and 31 (incomplete
    // distances, unused outputs) write to; they read rows of lanes 1 and 30
    static constexpr int NU = UR * RU, NS = SR * RS, NG = 31 * RG;
    static_assert((B1X + 1) * UZ + B1Z + 2 < 256, "stage-1 u_j reads reach by ds_read2 offsets");
    static_assert(2 * ((B1X - 1) * SZL + B1Z) < 256, "statistics reads reach");
    static_assert((GX - 1) * GZ + 4 < 256, "stage-2 Gv reads reach");
    static_assert((NU + NS + NG) * 4 <= 160 * 1024, "fits the LDS of one CU");
    // up to M = 3 two workgroups share a CU (one computes while the other
    // waits at a barrier)
    static_assert((NU + NS + NG) * 4 <= 80 * 1024, "two workgroups per CU");
};

struct Grid {
    int ntx, nty, ntz, nblocks;
};

template <typename T, int M>
__global__ void __launch_bounds__(THREADS) grad_lds_kernel(Geo g, GradArgs a, float *gpad, Grid gg)
{
    using L = Lay<M>;
    __shared__ float lds[L::NU + L::NS + L::NG];
    float *sU = lds, *sS = lds + L::NU, *sG = lds + L::NU + L::NS;

    const int b = blockIdx.x;
    const int q8 = gg.nblocks >> 3, r8 = gg.nblocks & 7, xcd = b & 7;
    int t = xcd * q8 + min(xcd, r8) + (b >> 3);
    const int tz = t % gg.ntz;
    t /= gg.ntz;
    const int ty = t % gg.nty;
    t /= gg.nty;
    const int tx = t % gg.ntx;
    const int k = t / gg.ntx;
    const int X0 = tx * TX, Y0 = ty * TY, Z0 = tz * TZ;  // padded tile origin

    const int tid = threadIdx.x;
    const int seg = tid >> 5;  // 32-lane segment (two per wave)
    const int l = tid & 31;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int64_t N = g.N;
    const T *u = (const T *)a.u;
    const int y = Y0 - 3 + l;  // grid row of this lane
    const int yc = clampi(y, 0, ny - 1);
    auto vox = [&](int ph, int xx, int yy, int zz) -> int64_t {
        return (int64_t)ph * N + ((int64_t)xx * ny + yy) * nz + zz;
    };
    auto st = [&](int ph, int slot, int comp, int xx, int yy, int zz) -> float {
        return a.stats[(((int64_t)ph * 2 + slot) * 2 + comp) * N + ((int64_t)xx * ny + yy) * nz + zz];
    };

    // stage-1 block: Gv x [ex0, ex0+3), z [ez0, ez0+4); squared differences
    // on x [ex0, ex0+5) (sq index s <-> grid X0-3+s), z [ez0, ez0+6)
    const int ex0 = B1X * (seg / (NSEG / 2)), ez0 = B1Z * (seg % (NSEG / 2));
    float uk[B1X + 2][B1Z + 2];
#pragma unroll
    for (int s = 0; s < B1X + 2; ++s)
#pragma unroll
        for (int c = 0; c < B1Z + 2; ++c)
            uk[s][c] = load_f(u, vox(k, clampi(X0 - 3 + ex0 + s, 0, nx - 1), yc,
                                     clampi(Z0 - 3 + ez0 + c, 0, nz - 1)));
    // stage-2 block: outputs padded x X0 .. X0+3, z Z0+2 seg .. +1 (grid = padded - 1)
    const bool has2 = seg < NSEG2;
    const int oz0 = B2Z * (has2 ? seg : 0);
    float uk2[B2X][B2Z], gw[B2X][B2Z];
#pragma unroll
    for (int xo = 0; xo < B2X; ++xo)
#pragma unroll
        for (int zo = 0; zo < B2Z; ++zo) {
            uk2[xo][zo] = load_f(u, vox(k, clampi(X0 + xo - 1, 0, nx - 1), yc,
                                        clampi(Z0 + oz0 + zo - 1, 0, nz - 1)));
            gw[xo][zo] = 0.f;
        }
    float gi[B1X][B1Z];
#pragma unroll
    for (int ex = 0; ex < B1X; ++ex)
#pragma unroll
        for (int ez = 0; ez < B1Z; ++ez)
            gi[ex][ez] = 0.f;

    // masks are needed when some Gv position of the tile (rows of lanes
    // 0..31 included) has v or v + delta outside the grid
    const bool border = (X0 - 2 - M < 0) || (X0 + TX - 1 + M >= nx) || (Y0 - 3 - M < 0) ||
                        (Y0 + 28 + M >= ny) || (Z0 - 2 - M < 0) || (Z0 + TZ - 1 + M >= nz);
    const float nc2 = in_vgpr(-g.c2);  // the exponent's factor, in a vector register
    constexpr int S = 2 * M + 1;
    const bool want_u = gpad != nullptr;  // uniform: without dE/du only stage 1 runs

    for (int slot = 0; slot < 2; ++slot) {
        const int j = slot == 0 ? (k + 1 == g.np ? 0 : k + 1) : (k == 0 ? g.np - 1 : k - 1);
        const int back = 1 - slot;
        float L1[B1X][B1Z], e1[B1X][B1Z];
#pragma unroll
        for (int ex = 0; ex < B1X; ++ex)
#pragma unroll
            for (int ez = 0; ez < B1Z; ++ez) {
                const int xx = clampi(X0 - 2 + ex0 + ex, 0, nx - 1);
                const int zz = clampi(Z0 - 2 + ez0 + ez, 0, nz - 1);
                L1[ex][ez] = -st(k, slot, 0, xx, yc, zz) * kLog2e;
                e1[ex][ez] = st(k, slot, 1, xx, yc, zz);
            }
        auto sweep = [&](auto bord_c) {
            constexpr bool bord = decltype(bord_c)::value;
            for (int dx = -M; dx <= M; ++dx) {
                __syncthreads();
                {
                    const int64_t plane = (int64_t)ny * nz;
                    const T *up[SX];
                    const float *lp[GX];
#pragma unroll
                    for (int p = 0; p < SX; ++p)
                        up[p] = u + (int64_t)j * N + clampi(X0 - 3 + dx + p, 0, nx - 1) * plane;
#pragma unroll
                    for (int p = 0; p < GX; ++p)
                        lp[p] = a.stats + ((int64_t)j * 2 + back) * 2 * N +
                                clampi(X0 - 2 + dx + p, 0, nx - 1) * plane;
                    for (int c = tid; c < L::UR * L::UZ; c += THREADS) {
                        const int r = c / L::UZ, zc = c - r * L::UZ;
                        const int gy = clampi(Y0 - 3 - M + r, 0, ny - 1);
                        const int gz = clampi(Z0 - 3 - M + zc, 0, nz - 1);
                        const unsigned co = (unsigned)(gy * nz + gz) * (unsigned)sizeof(T);
                        float *su = sU + r * L::RU + zc;
#pragma unroll
                        for (int p = 0; p < SX; ++p)
                            su[p * L::UZ] = load_f((const T *)((const char *)up[p] + co), 0);
                    }
                    for (int c = tid; c < L::SR * L::SZL; c += THREADS) {
                        const int r = c / L::SZL, zc = c - r * L::SZL;
                        const int gy = clampi(Y0 - 3 - M + r, 0, ny - 1);
                        const int gz = clampi(Z0 - 2 - M + zc, 0, nz - 1);
                        const unsigned co = (unsigned)(gy * nz + gz);
                        float *ss = sS + r * L::RS + 2 * zc;
#pragma unroll
                        for (int p = 0; p < GX; ++p) {
                            ss[2 * p * L::SZL] = -lp[p][co] * kLog2e;
                            ss[2 * p * L::SZL + 1] = lp[p][co + N];
                        }
                    }
                }
                __syncthreads();
                for (int pr = 0; pr < S * S; ++pr) {
                    const int dy = pr / S - M, dz = pr - (pr / S) * S - M;
                    // ---- stage 1: D and Gv on this segment's block
                    {
                        lds_float *bu = lds_base(sU + (l + M + dy) * L::RU + ex0 * L::UZ + ez0 + M + dz);
                        lds_float *bs = lds_base(sS + (l + M + dy) * L::RS + 2 * (ex0 * L::SZL + ez0 + M + dz));
                        float ub[B1X + 2][B1Z + 2];
#pragma unroll
                        for (int s = 0; s < B1X + 2; ++s)
#pragma unroll
                            for (int c = 0; c < B1Z + 2; ++c)
                                ub[s][c] = bu[s * L::UZ + c];
                        float sl[B1X][B1Z], se[B1X][B1Z];
#pragma unroll
                        for (int ex = 0; ex < B1X; ++ex)
#pragma unroll
                            for (int ez = 0; ez < B1Z; ++ez) {
                                sl[ex][ez] = bs[2 * (ex * L::SZL + ez)];
                                se[ex][ez] = bs[2 * (ex * L::SZL + ez) + 1];
                            }
                        __builtin_amdgcn_sched_barrier(0);
                        float pz[B1X + 2][B1Z], rc[B1X][B1Z];
#pragma unroll
                        for (int s = 0; s < B1X + 2; ++s) {
                            float dd[B1Z + 2];
#pragma unroll
                            for (int c = 0; c < B1Z + 2; ++c)
                                dd[c] = uk[s][c] - ub[s][c];
                            if (s >= 1 && s <= B1X) {
#pragma unroll
                                for (int ez = 0; ez < B1Z; ++ez)
                                    rc[s - 1][ez] = dd[ez + 1];
                            }
#pragma unroll
                            for (int ez = 0; ez < B1Z; ez += 2) {
                                const float p2 = fmaf(dd[ez + 1], dd[ez + 1], dd[ez + 2] * dd[ez + 2]);
                                pz[s][ez] = fmaf(dd[ez], dd[ez], p2);
                                pz[s][ez + 1] = fmaf(dd[ez + 3], dd[ez + 3], p2);
                            }
                        }
                        float D[B1X][B1Z];
#pragma unroll
                        for (int ez = 0; ez < B1Z; ++ez) {
                            const float p12 = pz[1][ez] + pz[2][ez];
                            D[0][ez] = pz[0][ez] + p12;
                            D[1][ez] = p12 + pz[3][ez];
                            D[2][ez] = (pz[2][ez] + pz[3][ez]) + pz[4][ez];
                        }
                        float Dy[B1X][B1Z];
#pragma unroll
                        for (int ex = 0; ex < B1X; ++ex)
#pragma unroll
                            for (int ez = 0; ez < B1Z; ++ez)
                                Dy[ex][ez] = from_below(D[ex][ez]) + D[ex][ez];
#pragma unroll
                        for (int ex = 0; ex < B1X; ++ex)
#pragma unroll
                            for (int ez = 0; ez < B1Z; ++ez)
                                D[ex][ez] = Dy[ex][ez] + from_above(D[ex][ez]);
                        float gvv[B1X][B1Z];
#pragma unroll
                        for (int ex = 0; ex < B1X; ++ex)
#pragma unroll
                            for (int ez = 0; ez < B1Z; ++ez) {
                                const float w1 = __builtin_amdgcn_exp2f(fmaf(D[ex][ez], nc2, L1[ex][ez]));
                                const float w2 = __builtin_amdgcn_exp2f(fmaf(D[ex][ez], nc2, sl[ex][ez]));
                                const float r = rc[ex][ez];
                                const float r2 = r * r;
                                float gv = fmaf(w2, r2 - se[ex][ez], w1 * (r2 - e1[ex][ez]));
                                float wr = (w1 + w2) * r;
                                if (bord) {
                                    const int vx = X0 - 2 + ex0 + ex, vz = Z0 - 2 + ez0 + ez;
                                    const bool ok = ((unsigned)y < (unsigned)ny) &
                                                    ((unsigned)(y + dy) < (unsigned)ny) &
                                                    ((unsigned)vx < (unsigned)nx) &
                                                    ((unsigned)(vx + dx) < (unsigned)nx) &
                                                    ((unsigned)vz < (unsigned)nz) &
                                                    ((unsigned)(vz + dz) < (unsigned)nz);
                                    gv = ok ? gv : 0.f;
                                    wr = ok ? wr : 0.f;
                                }
                                gvv[ex][ez] = gv;
                                gi[ex][ez] += wr;
                            }
                        if (!want_u)
                            continue;
                        // every wave has read the previous pair's Gv field by
                        // now: the long stage-1 arithmetic above ran between
                        // its stage 2 and this barrier
                        __syncthreads();
                        const int grow = (l >= 1 && l <= 30) ? l - 1 : 30;
                        float *gwr = sG + grow * L::RG + ex0 * GZ + ez0;
#pragma unroll
                        for (int ex = 0; ex < B1X; ++ex)
#pragma unroll
                            for (int ez = 0; ez < B1Z; ++ez)
                                gwr[ex * GZ + ez] = gvv[ex][ez];
                    }
                    __syncthreads();
                    // ---- stage 2: box sums of Gv onto this segment's outputs
                    if (has2) {
                        const int grow = l < 1 ? 0 : (l > 30 ? 29 : l - 1);
                        lds_float *bg = lds_base(sG + grow * L::RG + oz0);
                        lds_float *bu = lds_base(sU + (l + M + dy) * L::RU + 2 * L::UZ + oz0 + 2 + M + dz);
                        float gv[GX][B2Z + 2], ub[B2X][B2Z];
#pragma unroll
                        for (int ex = 0; ex < GX; ++ex)
#pragma unroll
                            for (int c = 0; c < B2Z + 2; ++c)
                                gv[ex][c] = bg[ex * GZ + c];
#pragma unroll
                        for (int xo = 0; xo < B2X; ++xo)
#pragma unroll
                            for (int zo = 0; zo < B2Z; ++zo)
                                ub[xo][zo] = bu[xo * L::UZ + zo];
                        __builtin_amdgcn_sched_barrier(0);
                        float gz[GX][B2Z];
#pragma unroll
                        for (int ex = 0; ex < GX; ++ex) {
                            const float p12 = gv[ex][1] + gv[ex][2];
                            gz[ex][0] = gv[ex][0] + p12;
                            gz[ex][1] = p12 + gv[ex][3];
                        }
                        float gx[B2X][B2Z], gyb[B2X][B2Z];
#pragma unroll
                        for (int xo = 0; xo < B2X; xo += 2)
#pragma unroll
                            for (int zo = 0; zo < B2Z; ++zo) {
                                const float p12 = gz[xo + 1][zo] + gz[xo + 2][zo];
                                gx[xo][zo] = gz[xo][zo] + p12;
                                gx[xo + 1][zo] = p12 + gz[xo + 3][zo];
                            }
#pragma unroll
                        for (int xo = 0; xo < B2X; ++xo)
#pragma unroll
                            for (int zo = 0; zo < B2Z; ++zo)
                                gyb[xo][zo] = from_below(gx[xo][zo]) + gx[xo][zo];
#pragma unroll
                        for (int xo = 0; xo < B2X; ++xo)
#pragma unroll
                            for (int zo = 0; zo < B2Z; ++zo) {
                                const float G3 = gyb[xo][zo] + from_above(gx[xo][zo]);
                                gw[xo][zo] = fmaf(uk2[xo][zo] - ub[xo][zo], G3, gw[xo][zo]);
                            }
                    }
                }
            }
        };
        if (border)
            sweep(std::true_type{});
        else
            sweep(std::false_type{});
    }

    // writes: weight part at the padded outputs, image part at the grid
    // voxels of this tile (Gv positions 1..4 in x, lanes 2..29, 1..30 in z)
    const float sw = -0.5f * g.inv2h2;
    const int64_t NP = (int64_t)(nx + 2) * (ny + 2) * (nz + 2);
    const int Yp = y + 1;
    const bool lrow = l >= 2 && l <= TY + 1 && Yp < ny + 2;
    if (has2 && gpad) {
#pragma unroll
        for (int xo = 0; xo < B2X; ++xo)
#pragma unroll
            for (int zo = 0; zo < B2Z; ++zo) {
                const int Xp = X0 + xo, Zp = Z0 + oz0 + zo;
                if (lrow && Xp < nx + 2 && Zp < nz + 2)
                    gpad[(int64_t)k * NP + ((int64_t)Xp * (ny + 2) + Yp) * (nz + 2) + Zp] = sw * gw[xo][zo];
            }
    }
    if (a.grad_f) {
#pragma unroll
        for (int ex = 0; ex < B1X; ++ex)
#pragma unroll
            for (int ez = 0; ez < B1Z; ++ez) {
                const int e_x = ex0 + ex, e_z = ez0 + ez;
                const int xg = X0 - 2 + e_x, zg = Z0 - 2 + e_z;
                if (e_x >= 1 && e_x <= TX && e_z >= 1 && e_z <= TZ && lrow &&
                    (unsigned)xg < (unsigned)nx && (unsigned)y < (unsigned)ny &&
                    (unsigned)zg < (unsigned)nz)
                    a.grad_f[vox(k, xg, y, zg)] = 0.5f * gi[ex][ez];
            }
    }
}

Grid grid_for(const Geo &g)
{
    Grid gg;
    gg.ntx = (g.nx + 2 + TX - 1) / TX;
    gg.nty = (g.ny + 2 + TY - 1) / TY;
    gg.ntz = (g.nz + 2 + TZ - 1) / TZ;
    gg.nblocks = g.np * gg.ntx * gg.nty * gg.ntz;
    return gg;
}

template <typename T, int M>
void launch(const Geo &g, const GradArgs &a, float *gpad, hipStream_t s)
{
    const Grid gg = grid_for(g);
    grad_lds_kernel<T, M><<<gg.nblocks, THREADS, 0, s>>>(g, a, gpad, gg);
}

template <typename T>
void launch_m(const Geo &g, const GradArgs &a, float *gpad, hipStream_t s)
{
    switch (g.M) {
    case 1:
        launch<T, 1>(g, a, gpad, s);
        break;
    case 2:
        launch<T, 2>(g, a, gpad, s);
        break;
    default:
        launch<T, 3>(g, a, gpad, s);
        break;
    }
}
}  // namespace v2

GradGrid grad_grid(const Geo &g, int tz)
{
    GradGrid gg;
    gg.ntx = (g.nx + 2 + kBX - 1) / kBX;
    gg.nty = (g.ny + 2 + kTY - 1) / kTY;
    gg.ntz = (g.nz + 2 + tz - 1) / tz;
    gg.nblocks = g.np * gg.ntx * gg.nty * gg.ntz;
    return gg;
}

template <typename T, int M, bool SAME>
void launch_one(const Geo &g, const GradArgs &a, float *gpad, hipStream_t s)
{
    using L = Lay<SAME, M>;
    const GradGrid gg = grad_grid(g, L::TZ);
    grad_tiled_kernel<T, M, SAME><<<gg.nblocks, L::THREADS, 0, s>>>(g, a, gpad, gg);
}

template <typename T, bool SAME>
void launch_m(const Geo &g, const GradArgs &a, float *gpad, hipStream_t s)
{
    switch (g.M) {
    case 1:
        launch_one<T, 1, SAME>(g, a, gpad, s);
        break;
    case 2:
        launch_one<T, 2, SAME>(g, a, gpad, s);
        break;
    case 3:
        launch_one<T, 3, SAME>(g, a, gpad, s);
        break;
    case 4:
        launch_one<T, 4, SAME>(g, a, gpad, s);
        break;
    default:
        launch_one<T, 5, SAME>(g, a, gpad, s);
        break;
    }
}

template <typename T>
hipError_t launch_t(const Geo &g, const GradArgs &a, float *gpad, hipStream_t s)
{
    if (a.u == a.f && g.M <= v2::kMaxM)
        v2::launch_m<T>(g, a, gpad, s);
    else if (a.u == a.f)
        launch_m<T, true>(g, a, gpad, s);
    else
        launch_m<T, false>(g, a, gpad, s);
    return hipGetLastError();
}


}  // namespace

bool grad_tiled_supported(const Geo &g)
{
    if (g.d != 1 || g.M < 1 || g.M > kMaxTiledM)
        return false;
    // staging addresses a cell within an x-plane by a 32-bit byte offset
    if ((int64_t)g.ny * g.nz * (int64_t)sizeof(float) >= (int64_t(1) << 32))
        return false;
    const int64_t nb = (int64_t)g.np * ((g.nx + 2 + kBX - 1) / kBX) *
                       ((g.ny + 2 + kTY - 1) / kTY) * ((g.nz + 2 + kMinTZ - 1) / kMinTZ);
    return nb < (int64_t(1) << 31);
}

size_t grad_tiled_pad_bytes(const Geo &g)
{
    return (size_t)g.np * (g.nx + 2) * (g.ny + 2) * (g.nz + 2) * sizeof(float);
}

hipError_t launch_grad_tiled(const Geo &g, int dtype, const GradArgs &a, float *gpad, hipStream_t s)
{
    hipError_t e;
    // weight part needed for grad_u; the kernel always writes it to gpad
    float *gp = a.grad_u ? gpad : nullptr;
    switch (dtype) {
    case TNLM_F32:
        e = launch_t<float>(g, a, gp, s);
        break;
    case TNLM_BF16:
        e = launch_t<bf16_t>(g, a, gp, s);
        break;
    default:
        e = launch_t<_Float16>(g, a, gp, s);
        break;
    }
    if (e != hipSuccess || !a.grad_u)
        return e;
    int64_t blocks = ((int64_t)g.np * g.N + 255) / 256;
    blocks = blocks > 65536 ? 65536 : blocks;
    const float *add = (a.grad_u == a.grad_f) ? a.grad_f : nullptr;
    fold_kernel<<<blocks, 256, 0, s>>>(g, gpad, a.grad_u, add);
    return hipGetLastError();
}

}  // namespace tnlm
