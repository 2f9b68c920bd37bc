// Internal declarations shared by the HIP translation units of libtnlm.
// Not part of the public ABI (include/tnlm.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tnlm.h"

namespace tnlm {

// Derived geometry passed by value to every kernel.
struct Geo {
    int np, nx, ny, nz;  // phases and grid, z fastest
    int d, M;            // patch radius, search radius
    int S;               // 2M+1
    int W;               // (2M+1)^3 offsets
    int64_t N;           // voxels per phase
    float inv2h2;        // 1/(2h^2): exponent of Eq. (3) is -D * inv2h2
    float c2;            // log2(e)/(2h^2): same exponent in base-2 units
};

// ---- storage types ---------------------------------------------------------
// u, f, g and f_out are stored as float, bfloat16 (raw uint16 bits) or
// float16; arithmetic is always float.
struct bf16_t {
    uint16_t bits;
};

__device__ __forceinline__ float load_f(const float *p, int64_t i) { return p[i]; }
__device__ __forceinline__ float load_f(const bf16_t *p, int64_t i)
{
    return __uint_as_float(((uint32_t)p[i].bits) << 16);
}
__device__ __forceinline__ float load_f(const _Float16 *p, int64_t i) { return (float)p[i]; }

// An LDS pointer whose address the compiler treats as an unknown register
// value: reads through it use that one register plus small immediate
// offsets (ds_read2 reaches 255 dwords), instead of folding the array's
// absolute LDS address into every read and overflowing the offset field.
// A wave-uniform float held in a vector register: gfx950 issues an FP32
// VALU instruction whose operands are all vector registers (or inline
// constants) in about 2 cycles per wave64, one that reads a scalar register
// in about 4. Kernel arguments live in scalar registers; a loop-invariant
// factor used in every iteration is worth one copy.
__device__ __forceinline__ float in_vgpr(float v)
{
    asm volatile("" : "+v"(v));
    return v;
}

using lds_float = __attribute__((address_space(3))) const float;
__device__ __forceinline__ lds_float *lds_base(const float *p)
{
    unsigned a = (unsigned)(size_t)(lds_float *)p;
    asm("" : "+v"(a));
    return (lds_float *)(size_t)a;
}

__device__ __forceinline__ void store_f(float *p, int64_t i, float v) { p[i] = v; }
__device__ __forceinline__ void store_f(bf16_t *p, int64_t i, float v)
{
    // round to nearest even; quiet NaN stays NaN
    uint32_t x = __float_as_uint(v);
    uint16_t r;
    if ((x & 0x7fffffffu) > 0x7f800000u)
        r = (uint16_t)((x >> 16) | 0x0040u);
    else
        r = (uint16_t)((x + 0x7fffu + ((x >> 16) & 1u)) >> 16);
    p[i].bits = r;
}
__device__ __forceinline__ void store_f(_Float16 *p, int64_t i, float v) { p[i] = (_Float16)v; }

// ---- compensated (double-float) accumulation for the energy ---------------
struct dfloat {
    float hi, lo;
};

// Knuth's TwoSum of the high parts, low parts added, then renormalised.
__device__ __forceinline__ dfloat df_add(dfloat a, dfloat b)
{
    float s = a.hi + b.hi;
    float bb = s - a.hi;
    float err = (a.hi - (s - bb)) + (b.hi - bb);
    float lo = err + a.lo + b.lo;
    float hi = s + lo;
    lo = lo - (hi - s);
    return dfloat{hi, lo};
}

// ---- kernel launchers (defined in the .hip files) --------------------------
enum FwdMode { FWD_WEIGHTS = 0, FWD_JACOBI = 1, FWD_EQ6 = 2, FWD_ENERGY = 3 };

struct FwdArgs {
    const void *u, *f, *g;
    float mu;
    void *out;       // JACOBI: storage dtype volume; EQ6: float volume
    float *w;        // WEIGHTS: [np][2][W][N] or null
    float *lse;      // WEIGHTS: [np][2][N] or null
    float *stats;    // ENERGY: [np][2][2][N] or null
    dfloat *partial; // ENERGY: per-block partial sums
};

struct GradArgs {
    const void *u, *f;
    const float *stats;
    float *grad_f, *grad_u;  // grad_u may equal grad_f (sum written)
};

// Number of blocks (= partial sums) of the generic / tiled energy pass.
int64_t energy_blocks_generic(const Geo &g);
int64_t energy_blocks_tiled(const Geo &g);

// Tiled forward kernels (d = 1, M = 1..4; weights mode: log-normalisers only).
bool fwd_tiled_supported(const Geo &g, int mode);
hipError_t launch_fwd_tiled(const Geo &g, int dtype, int mode, const FwdArgs &a,
                            hipStream_t s);

// Tiled exact gradient (d = 1, M = 1..4): weight part on the padded grid in
// gpad (np*(nx+2)*(ny+2)*(nz+2) floats of workspace), then folded into grad_u.
bool grad_tiled_supported(const Geo &g);
size_t grad_tiled_pad_bytes(const Geo &g);
hipError_t launch_grad_tiled(const Geo &g, int dtype, const GradArgs &a, float *gpad,
                             hipStream_t s);

hipError_t launch_fwd_generic(const Geo &g, int dtype, int mode, const FwdArgs &a,
                              hipStream_t s);
hipError_t launch_grad_exact_generic(const Geo &g, int dtype, const GradArgs &a,
                                     hipStream_t s);
hipError_t launch_energy_final(const dfloat *partial, int64_t n, float *e_out,
                               hipStream_t s);

// Reconstruction model (ct.hip): projector, transpose, CGLS, positivity.
size_t ct_workspace_bytes_impl(int np, int64_t N, int64_t R);
hipError_t ct_project(const tnlm_ct_geom *g, const float *vol, float *proj, hipStream_t s);
hipError_t ct_backproject(const tnlm_ct_geom *g, const float *proj, float *vol, hipStream_t s);
hipError_t ct_cgls_init(const tnlm_ct_geom *g, const float *y, const float *x, void *ws,
                        hipStream_t s);
hipError_t ct_cgls_step(const tnlm_ct_geom *g, float *x, void *ws, hipStream_t s);
hipError_t ct_clamp(float *x, int64_t n, hipStream_t s);

}  // namespace tnlm
