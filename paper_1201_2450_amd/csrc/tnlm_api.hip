// C-ABI entry points of libtnlm: argument validation, workspace layout and
// kernel dispatch. Declarations and conventions: include/tnlm.h.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "tnlm_internal.h"

using namespace tnlm;

namespace {

thread_local char g_hip_msg[256] = "HIP error";

int hip_fail(hipError_t e)
{
    snprintf(g_hip_msg, sizeof g_hip_msg, "HIP error %d: %s", (int)e, hipGetErrorString(e));
    return TNLM_EHIP;
}

constexpr int64_t kMaxPhaseVox = (int64_t(1) << 31) - 1;
constexpr int64_t kMaxVox = int64_t(1) << 40;

// Validates the geometry and fills the derived values.
int make_geo(const tnlm_geom *p, Geo *g)
{
    if (!p)
        return TNLM_ENULL;
    if (p->np < 2 || p->nx < 1 || p->ny < 1 || p->nz < 1)
        return TNLM_EINVAL;
    if (p->patch_r < 0 || p->patch_r > 8 || p->search_r < 0 || p->search_r > 16)
        return TNLM_EINVAL;
    if (!(p->h > 0.f) || !isfinite(p->h))
        return TNLM_EINVAL;
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    if (N > kMaxPhaseVox || N * p->np > kMaxVox)
        return TNLM_ERANGE;
    const double h = p->h;
    const double inv2h2 = 1.0 / (2.0 * h * h);
    if (!isfinite(inv2h2) || !isfinite((float)(inv2h2 * 1.4426950408889634)))
        return TNLM_EINVAL;
    g->np = p->np;
    g->nx = p->nx;
    g->ny = p->ny;
    g->nz = p->nz;
    g->d = p->patch_r;
    g->M = p->search_r;
    g->S = 2 * p->search_r + 1;
    g->W = g->S * g->S * g->S;
    g->N = N;
    g->inv2h2 = (float)inv2h2;
    g->c2 = (float)(inv2h2 * 1.4426950408889634);
    return TNLM_OK;
}

int elem_size(int dtype) { return dtype == TNLM_F32 ? 4 : 2; }

bool valid_dtype(int dtype)
{
    return dtype == TNLM_F32 || dtype == TNLM_BF16 || dtype == TNLM_F16;
}

// [a, a+na) and [b, b+nb) overlap (byte ranges)?
bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    if (!a || !b || na == 0 || nb == 0)
        return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Forward kernels: the tiled path where it applies, else the generic one.
bool tiled(const Geo &g, int mode) { return fwd_tiled_supported(g, mode); }

hipError_t launch_fwd(const Geo &g, int dtype, int mode, const FwdArgs &a, hipStream_t s)
{
    if (tiled(g, mode) && !(mode == FWD_WEIGHTS && a.w))
        return launch_fwd_tiled(g, dtype, mode, a, s);
    return launch_fwd_generic(g, dtype, mode, a, s);
}

int64_t energy_blocks(const Geo &g)
{
    return tiled(g, FWD_ENERGY) ? energy_blocks_tiled(g) : energy_blocks_generic(g);
}

size_t partial_bytes(const Geo &g) { return align256((size_t)energy_blocks(g) * sizeof(dfloat)); }

size_t stats_bytes(const Geo &g) { return (size_t)g.np * g.N * 4 * sizeof(float); }

// Exact gradient workspace: [partial sums][padded weight part]; the caller
// appends room for the statistics when it passes none.
size_t pad_bytes(const Geo &g) { return grad_tiled_supported(g) ? align256(grad_tiled_pad_bytes(g)) : 0; }
size_t grad_exact_bytes(const Geo &g) { return partial_bytes(g) + pad_bytes(g); }

// Fixed device scratch of tnlm_energy_noalloc: the per-workgroup partial
// sums of the energy. One copy per GPU, held until the process ends. Host
// code never uses this name as an address (on the host it is only a
// stand-in for the symbol): the device address of each GPU's copy comes from
// hipGetSymbolAddress, looked up once per device.
constexpr size_t kScratchBytes = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch (looked up on the first
// call on that device, with it current), or null with *err set.
void *scratch_ptr(hipError_t *err)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *err = e;
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

const char *tnlm_strerror(int code)
{
    switch (code) {
    case TNLM_OK:
        return "success";
    case TNLM_EINVAL:
        return "invalid argument (geometry, h, mu, dtype, mode or flag)";
    case TNLM_ENULL:
        return "required pointer is NULL";
    case TNLM_EALIAS:
        return "output overlaps an input or another output";
    case TNLM_ERANGE:
        return "size exceeds the supported index range";
    case TNLM_EWORKSPACE:
        return "workspace missing or too small";
    case TNLM_EHIP:
        return g_hip_msg;
    default:
        return "unknown tnlm status";
    }
}

const char *tnlm_version(void) { return "tnlm 0.1 gfx950"; }

size_t tnlm_workspace_bytes(const tnlm_geom *geom, int op)
{
    Geo g;
    if (make_geo(geom, &g) != TNLM_OK)
        return (size_t)-1;
    switch (op) {
    case TNLM_OP_WEIGHTS:
    case TNLM_OP_JACOBI:
    case TNLM_OP_GRAD_EQ6:
        return 0;
    case TNLM_OP_ENERGY:
        return partial_bytes(g);
    case TNLM_OP_GRAD_EXACT:
        return grad_exact_bytes(g);
    default:
        return (size_t)-1;
    }
}

int tnlm_weights(const tnlm_geom *geom, int dtype, const void *u, float *w, float *lse,
                 void *stream)
{
    Geo g;
    int rc = make_geo(geom, &g);
    if (rc)
        return rc;
    if (!valid_dtype(dtype))
        return TNLM_EINVAL;
    if (!u || (!w && !lse))
        return TNLM_ENULL;
    const size_t vb = (size_t)g.np * g.N * elem_size(dtype);
    // w holds np*2*W*N floats: check the 64-bit byte count
    const double wbytes = (double)g.np * 2.0 * g.W * (double)g.N * 4.0;
    if (w && wbytes > 9.0e18)
        return TNLM_ERANGE;
    const size_t wb = w ? (size_t)g.np * 2 * g.W * g.N * sizeof(float) : 0;
    const size_t lb = (size_t)g.np * 2 * g.N * sizeof(float);
    if (overlap(w, wb, u, vb) || overlap(lse, lb, u, vb) || overlap(w, wb, lse, lb))
        return TNLM_EALIAS;
    FwdArgs a{};
    a.u = u;
    a.w = w;
    a.lse = lse;
    hipError_t e = launch_fwd(g, dtype, FWD_WEIGHTS, a, (hipStream_t)stream);
    return e == hipSuccess ? TNLM_OK : hip_fail(e);
}

int tnlm_jacobi_step(const tnlm_geom *geom, int dtype, const void *u, const void *f,
                     const void *gin, float mu, void *f_out, void *stream)
{
    Geo g;
    int rc = make_geo(geom, &g);
    if (rc)
        return rc;
    if (!valid_dtype(dtype) || !(mu > 0.f) || !isfinite(mu))
        return TNLM_EINVAL;
    if (!u || !f || !gin || !f_out)
        return TNLM_ENULL;
    const size_t vb = (size_t)g.np * g.N * elem_size(dtype);
    if (overlap(f_out, vb, u, vb) || overlap(f_out, vb, f, vb) || overlap(f_out, vb, gin, vb))
        return TNLM_EALIAS;
    FwdArgs a{};
    a.u = u;
    a.f = f;
    a.g = gin;
    a.mu = mu;
    a.out = f_out;
    hipError_t e = launch_fwd(g, dtype, FWD_JACOBI, a, (hipStream_t)stream);
    return e == hipSuccess ? TNLM_OK : hip_fail(e);
}

static int energy_impl(const Geo &g, int dtype, const void *u, const void *f, float *e_out,
                       float *stats, dfloat *partial, hipStream_t s)
{
    FwdArgs a{};
    a.u = u;
    a.f = f;
    a.stats = stats;
    a.partial = partial;
    hipError_t e = launch_fwd(g, dtype, FWD_ENERGY, a, s);
    if (e != hipSuccess)
        return hip_fail(e);
    if (e_out) {
        e = launch_energy_final(partial, energy_blocks(g), e_out, s);
        if (e != hipSuccess)
            return hip_fail(e);
    }
    return TNLM_OK;
}

int tnlm_energy(const tnlm_geom *geom, int dtype, const void *u, const void *f, float *e_out,
                float *stats, void *ws, size_t ws_bytes, void *stream)
{
    Geo g;
    int rc = make_geo(geom, &g);
    if (rc)
        return rc;
    if (!valid_dtype(dtype))
        return TNLM_EINVAL;
    if (!u || !f || !e_out)
        return TNLM_ENULL;
    const size_t need = partial_bytes(g);
    if (!ws || ws_bytes < need)
        return TNLM_EWORKSPACE;
    const size_t vb = (size_t)g.np * g.N * elem_size(dtype);
    const size_t sb = stats ? stats_bytes(g) : 0;
    const void *outs[3] = {e_out, stats, ws};
    const size_t outb[3] = {2 * sizeof(float), sb, need};
    for (int a = 0; a < 3; ++a) {
        if (overlap(outs[a], outb[a], u, vb) || overlap(outs[a], outb[a], f, vb))
            return TNLM_EALIAS;
        for (int b = a + 1; b < 3; ++b)
            if (overlap(outs[a], outb[a], outs[b], outb[b]))
                return TNLM_EALIAS;
    }
    return energy_impl(g, dtype, u, f, e_out, stats, (dfloat *)ws, (hipStream_t)stream);
}

int tnlm_energy_noalloc(const tnlm_geom *geom, int dtype, const void *u, const void *f,
                        float *e_out, float *stats, void *stream)
{
    Geo g;
    int rc = make_geo(geom, &g);
    if (rc)
        return rc;
    if (!valid_dtype(dtype))
        return TNLM_EINVAL;
    if (!u || !f || !e_out)
        return TNLM_ENULL;
    if (partial_bytes(g) > kScratchBytes)
        return TNLM_EWORKSPACE;
    const size_t vb = (size_t)g.np * g.N * elem_size(dtype);
    const size_t sb = stats ? stats_bytes(g) : 0;
    if (overlap(e_out, 2 * sizeof(float), u, vb) || overlap(e_out, 2 * sizeof(float), f, vb) ||
        overlap(stats, sb, u, vb) || overlap(stats, sb, f, vb) ||
        overlap(e_out, 2 * sizeof(float), stats, sb))
        return TNLM_EALIAS;
    hipError_t e = hipSuccess;
    void *part = scratch_ptr(&e);
    if (!part)
        return hip_fail(e);
    // every partial sum the final reduction reads is written by the energy
    // kernel of this call: nothing needs clearing
    return energy_impl(g, dtype, u, f, e_out, stats, (dfloat *)part, (hipStream_t)stream);
}

int tnlm_grad(const tnlm_geom *geom, int dtype, const void *u, const void *f, int mode,
              const float *stats, float *grad_f, float *grad_u, void *ws, size_t ws_bytes,
              void *stream)
{
    Geo g;
    int rc = make_geo(geom, &g);
    if (rc)
        return rc;
    if (!valid_dtype(dtype))
        return TNLM_EINVAL;
    if (mode != TNLM_GRAD_EQ6 && mode != TNLM_GRAD_EXACT)
        return TNLM_EINVAL;
    if (mode == TNLM_GRAD_EQ6 && grad_u)
        return TNLM_EINVAL;
    if (!u || !f || (!grad_f && !grad_u))
        return TNLM_ENULL;
    if (grad_u && grad_u == grad_f && u != f)
        return TNLM_EINVAL;
    const size_t vb = (size_t)g.np * g.N * elem_size(dtype);
    const size_t gb = (size_t)g.np * g.N * sizeof(float);
    const hipStream_t s = (hipStream_t)stream;
    const void *ins[3] = {u, f, stats};
    const size_t inb[3] = {vb, vb, stats ? stats_bytes(g) : 0};
    for (int a = 0; a < 3; ++a)
        if (overlap(grad_f, gb, ins[a], inb[a]) || overlap(grad_u, gb, ins[a], inb[a]))
            return TNLM_EALIAS;
    if (grad_f && grad_u && grad_f != grad_u && overlap(grad_f, gb, grad_u, gb))
        return TNLM_EALIAS;
    if (mode == TNLM_GRAD_EQ6) {
        FwdArgs a{};
        a.u = u;
        a.f = f;
        a.out = grad_f;
        hipError_t e = launch_fwd(g, dtype, FWD_EQ6, a, s);
        return e == hipSuccess ? TNLM_OK : hip_fail(e);
    }
    size_t need = grad_exact_bytes(g) + (stats ? 0 : stats_bytes(g));
    if (!ws || ws_bytes < need)
        return TNLM_EWORKSPACE;
    for (int a = 0; a < 3; ++a)
        if (overlap(ws, need, ins[a], inb[a]))
            return TNLM_EALIAS;
    if (overlap(ws, need, grad_f, grad_f ? gb : 0) || overlap(ws, need, grad_u, grad_u ? gb : 0))
        return TNLM_EALIAS;
    const float *st = stats;
    if (!st) {
        float *own = (float *)((char *)ws + grad_exact_bytes(g));
        rc = energy_impl(g, dtype, u, f, nullptr, own, (dfloat *)ws, s);
        if (rc)
            return rc;
        st = own;
    }
    GradArgs a{};
    a.u = u;
    a.f = f;
    a.stats = st;
    a.grad_f = grad_f;
    a.grad_u = grad_u;
    if (!grad_f && grad_u) {
        a.grad_f = nullptr;
    }
    hipError_t e;
    if (grad_tiled_supported(g))
        e = launch_grad_tiled(g, dtype, a, (float *)((char *)ws + partial_bytes(g)), s);
    else
        e = launch_grad_exact_generic(g, dtype, a, s);
    return e == hipSuccess ? TNLM_OK : hip_fail(e);
}

// ---- reconstruction model ---------------------------------------------------
static int check_ct(const tnlm_ct_geom *g, int64_t *N, int64_t *R)
{
    if (!g)
        return TNLM_ENULL;
    if (g->np < 1 || g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nu < 1 || g->nv < 1 || g->na < 1)
        return TNLM_EINVAL;
    const float vals[4] = {g->sid, g->sdd, g->du, g->dv};
    for (float v : vals)
        if (!(v > 0.f) || !isfinite(v))
            return TNLM_EINVAL;
    const double half = 0.5 * sqrt((double)g->nx * g->nx + (double)g->ny * g->ny);
    if (!(g->sid > half) || !(g->sdd - g->sid > half))
        return TNLM_EINVAL;
    *N = (int64_t)g->nx * g->ny * g->nz;
    *R = (int64_t)g->na * g->nu * g->nv;
    if (*N * g->np >= (int64_t(1) << 31) || *R * g->np >= (int64_t(1) << 31))
        return TNLM_ERANGE;
    if (!g->angles)
        return TNLM_ENULL;
    return TNLM_OK;
}

size_t tnlm_ct_workspace_bytes(const tnlm_ct_geom *geom)
{
    int64_t N, R;
    if (check_ct(geom, &N, &R) != TNLM_OK)
        return (size_t)-1;
    return ct_workspace_bytes_impl(geom->np, N, R);
}

int tnlm_ct_project(const tnlm_ct_geom *geom, const float *vol, float *proj, void *stream)
{
    int64_t N, R;
    int rc = check_ct(geom, &N, &R);
    if (rc)
        return rc;
    if (!vol || !proj)
        return TNLM_ENULL;
    if (overlap(vol, (size_t)geom->np * N * 4, proj, (size_t)geom->np * R * 4) ||
        overlap(geom->angles, (size_t)geom->np * geom->na * 4, proj, (size_t)geom->np * R * 4))
        return TNLM_EALIAS;
    hipError_t e = ct_project(geom, vol, proj, (hipStream_t)stream);
    return e == hipSuccess ? TNLM_OK : hip_fail(e);
}

int tnlm_ct_backproject(const tnlm_ct_geom *geom, const float *proj, float *vol, void *stream)
{
    int64_t N, R;
    int rc = check_ct(geom, &N, &R);
    if (rc)
        return rc;
    if (!vol || !proj)
        return TNLM_ENULL;
    if (overlap(vol, (size_t)geom->np * N * 4, proj, (size_t)geom->np * R * 4) ||
        overlap(geom->angles, (size_t)geom->np * geom->na * 4, vol, (size_t)geom->np * N * 4))
        return TNLM_EALIAS;
    hipError_t e = ct_backproject(geom, proj, vol, (hipStream_t)stream);
    return e == hipSuccess ? TNLM_OK : hip_fail(e);
}

int tnlm_cgls_init(const tnlm_ct_geom *geom, const float *y, const float *x, void *ws,
                   size_t ws_bytes, void *stream)
{
    int64_t N, R;
    int rc = check_ct(geom, &N, &R);
    if (rc)
        return rc;
    if (!y || !x)
        return TNLM_ENULL;
    const size_t need = ct_workspace_bytes_impl(geom->np, N, R);
    if (!ws || ws_bytes < need)
        return TNLM_EWORKSPACE;
    const size_t vb = (size_t)geom->np * N * 4, pb = (size_t)geom->np * R * 4;
    if (overlap(ws, need, y, pb) || overlap(ws, need, x, vb) ||
        overlap(ws, need, geom->angles, (size_t)geom->np * geom->na * 4))
        return TNLM_EALIAS;
    hipError_t e = ct_cgls_init(geom, y, x, ws, (hipStream_t)stream);
    return e == hipSuccess ? TNLM_OK : hip_fail(e);
}

int tnlm_cgls_step(const tnlm_ct_geom *geom, float *x, int iters, void *ws, size_t ws_bytes,
                   void *stream)
{
    int64_t N, R;
    int rc = check_ct(geom, &N, &R);
    if (rc)
        return rc;
    if (iters < 0)
        return TNLM_EINVAL;
    if (!x)
        return TNLM_ENULL;
    const size_t need = ct_workspace_bytes_impl(geom->np, N, R);
    if (!ws || ws_bytes < need)
        return TNLM_EWORKSPACE;
    if (overlap(ws, need, x, (size_t)geom->np * N * 4) ||
        overlap(ws, need, geom->angles, (size_t)geom->np * geom->na * 4))
        return TNLM_EALIAS;
    for (int k = 0; k < iters; ++k) {
        hipError_t e = ct_cgls_step(geom, x, ws, (hipStream_t)stream);
        if (e != hipSuccess)
            return hip_fail(e);
    }
    return TNLM_OK;
}

int tnlm_clamp_nonneg(float *x, int64_t n, void *stream)
{
    if (n < 0)
        return TNLM_EINVAL;
    if (n == 0)
        return TNLM_OK;
    if (!x)
        return TNLM_ENULL;
    hipError_t e = ct_clamp(x, n, (hipStream_t)stream);
    return e == hipSuccess ? TNLM_OK : hip_fail(e);
}

}  // extern "C"
