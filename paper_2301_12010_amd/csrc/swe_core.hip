// swe_core.hip - single-scenario context, stage kernels and shared host code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "swe_internal.hpp"

namespace swe {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Wave speeds (slot 0) and runup of the initial state.
__global__ __launch_bounds__(256) void k_init(Geo G)
{
    __shared__ unsigned int ru[3 * 4];
    __shared__ double rd[4];
    unsigned int sx = 0, sy = 0, rb = 0;
    double hs = 0.0;
    const long long n = (long long)G.nx * G.ny;
    for (long long e = blockIdx.x * 256ll + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const int j = (int)(e / G.nx), i = (int)(e - (long long)j * G.nx);
        const int gi = j * G.pitch + i;
        const float b = G.b[gi], lo = fminf(b, 0.f);
        const float h = G.U[0][gi] - lo, hu = G.U[1][gi], hv = G.U[2][gi];
        const bool wet = h > G.h_dry;
        const float cel = fsqrt(G.g * fmaxf(h, 0.f));
        const float inv = wet ? 1.f / h : 0.f;
        const bool fin = fabsf(h) <= 3.4e38f && fabsf(hu) <= 3.4e38f && fabsf(hv) <= 3.4e38f;
        const unsigned int bx = fin ? speed_bits(fabsf(hu * inv) + cel) : 0x7f800000u;
        const unsigned int by = fin ? speed_bits(fabsf(hv * inv) + cel) : 0x7f800000u;
        sx = bx > sx ? bx : sx;
        sy = by > sy ? by : sy;
        hs += (double)G.U[0][gi] - (double)lo;
        if (wet && b > 0.f) rb = __float_as_uint(b) > rb ? __float_as_uint(b) : rb;
    }
    sx = wave_max_u32(sx);
    sy = wave_max_u32(sy);
    rb = wave_max_u32(rb);
    hs = wave_sum_f64(hs);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        ru[wv] = sx;
        ru[4 + wv] = sy;
        ru[8 + wv] = rb;
        rd[wv] = hs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int mx = 0, my = 0, mr = 0;
        double s = 0.0;
        for (int w = 0; w < 4; ++w) {
            mx = ru[w] > mx ? ru[w] : mx;
            my = ru[4 + w] > my ? ru[4 + w] : my;
            mr = ru[8 + w] > mr ? ru[8 + w] : mr;
            s += rd[w];
        }
        atomicMax(&G.sd->alpha[0][0], mx);
        atomicMax(&G.sd->alpha[0][1], my);
        if (mr) atomicMax(&G.sd->runup, mr);
        (void)s;
        if (mx >= 0x7f800000u || my >= 0x7f800000u) atomicOr(&G.sd->flags, 1u);
    }
}

// FP64 mass: MASS_BLOCKS blocks write fixed-order partial sums of h, then one
// block adds them in order, so the result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_mass_part(Geo G)
{
    __shared__ double rd[4];
    double hs = 0.0;
    const long long n = (long long)G.nx * G.ny;
    for (long long e = blockIdx.x * 256ll + threadIdx.x; e < n; e += (long long)MASS_BLOCKS * 256) {
        const int j = (int)(e / G.nx), i = (int)(e - (long long)j * G.nx);
        const int gi = j * G.pitch + i;
        // depth from the stored level, in FP64
        hs += (double)G.U[0][gi] - (double)fminf(G.b[gi], 0.f);
        if (G.Rl[0]) hs += (double)G.Rl[0][gi];  // residual of the compensated level
    }
    hs = wave_sum_f64(hs);
    if ((threadIdx.x & 63) == 0) rd[threadIdx.x >> 6] = hs;
    __syncthreads();
    if (threadIdx.x == 0) G.mass_part[blockIdx.x] = ((rd[0] + rd[1]) + rd[2]) + rd[3];
}

__global__ __launch_bounds__(64) void k_mass_final(Geo G)
{
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < MASS_BLOCKS; ++b) s += G.mass_part[b];
        G.sd->mass_sum = s;
    }
}

int launch_mass(const Geo &g, hipStream_t stream)
{
    hipLaunchKernelGGL(k_mass_part, dim3(MASS_BLOCKS), dim3(256), 0, stream, g);
    hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(64), 0, stream, g);
    return hipGetLastError() == hipSuccess ? SWE_OK : SWE_EDEVICE;
}

// Depth h = s - min(b, 0) of a stored-level plane, over whole padded planes
// (four floats per access: the pitch is a multiple of 64; padding is zero).
__global__ __launch_bounds__(256) void k_depth(Geo G, const float *lev, float *out)
{
    const size_t q = (size_t)G.pitch * G.ny / 4;
    const float4 *s4 = reinterpret_cast<const float4 *>(lev);
    const float4 *b4 = reinterpret_cast<const float4 *>(G.b);
    float4 *o4 = reinterpret_cast<float4 *>(out);
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < q; i += (size_t)gridDim.x * 256) {
        const float4 a = s4[i], b = b4[i];
        o4[i] = make_float4(a.x - fminf(b.x, 0.f), a.y - fminf(b.y, 0.f), a.z - fminf(b.z, 0.f),
                            a.w - fminf(b.w, 0.f));
    }
}

int launch_depth(const Geo &g, const float *lev, float *out, hipStream_t stream)
{
    const size_t q = (size_t)g.pitch * g.ny / 4;
    size_t blocks = (q + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_depth, dim3((unsigned)blocks), dim3(256), 0, stream, g, lev, out);
    return hipGetLastError() == hipSuccess ? SWE_OK : SWE_EDEVICE;
}

// ---------------------------------------------------------------------------
// outputs during a run: snapshots at output times, maximum-depth map
// ---------------------------------------------------------------------------
// Device bookkeeping of an output request: `next` is the first output not yet
// taken; hdr[k] describes output k once taken (src: the output whose slot
// holds the state, when one step served several output times).
struct SnapHeader {
    double t;
    long long step;
    int src;
    int pad[3];
};
struct SnapMeta {
    int next, n;
    int pad[6];
    SnapHeader hdr[1];  // n entries
};

static size_t snap_meta_bytes(int n) { return offsetof(SnapMeta, hdr) + (size_t)n * sizeof(SnapHeader); }

// Copy u^n (depth, hu, hv) into output slot `next` if the step just
// completed reached its time.  Every block takes the same decision: nothing writes `next` or t in
// this kernel.  Planes are copied whole (pitch included), four floats per
// access (the pitch is a multiple of 64).
__global__ __launch_bounds__(256) void k_snap_copy(Geo G, const double *times, const SnapMeta *m,
                                                   float *slots)
{
    const int j = m->next;
    if (j >= m->n || !(G.sd->t >= times[j])) return;
    const size_t plane = (size_t)G.pitch * G.ny;
    const size_t q = plane / 4;
    float4 *dst = reinterpret_cast<float4 *>(slots + (size_t)j * 3 * plane);
    const float4 *s0 = reinterpret_cast<const float4 *>(G.U[0]);
    const float4 *s1 = reinterpret_cast<const float4 *>(G.U[1]);
    const float4 *s2 = reinterpret_cast<const float4 *>(G.U[2]);
    const float4 *b4 = reinterpret_cast<const float4 *>(G.b);
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < q; i += (size_t)gridDim.x * 256) {
        const float4 a = s0[i], b = b4[i];  // depth from the stored level
        dst[i] = make_float4(a.x - fminf(b.x, 0.f), a.y - fminf(b.y, 0.f), a.z - fminf(b.z, 0.f),
                             a.w - fminf(b.w, 0.f));
        dst[q + i] = s1[i];
        dst[2 * q + i] = s2[i];
    }
}

// Advance `next` past every output time the step reached (one thread).
__global__ __launch_bounds__(64) void k_snap_advance(Geo G, const double *times, SnapMeta *m)
{
    if (threadIdx.x != 0) return;
    int j = m->next;
    const double t = G.sd->t;
    if (j >= m->n || !(t >= times[j])) return;
    const int src = j;
    const long long step = G.sd->step;
    while (j < m->n && t >= times[j]) {
        m->hdr[j].t = t;
        m->hdr[j].step = step;
        m->hdr[j].src = src;
        ++j;
    }
    m->next = j;
}

static int launch_snap(const Geo &g, const double *times, SnapMeta *m, float *slots, hipStream_t stream)
{
    const size_t q = (size_t)g.pitch * g.ny / 4;
    size_t blocks = (q + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_snap_copy, dim3((unsigned)blocks), dim3(256), 0, stream, g, times, m, slots);
    hipLaunchKernelGGL(k_snap_advance, dim3(1), dim3(64), 0, stream, g, times, m);
    return hipGetLastError() == hipSuccess ? SWE_OK : SWE_EDEVICE;
}

// ---------------------------------------------------------------------------
// tile variants
// ---------------------------------------------------------------------------
#define SWE_VARIANT(TX, TY, R, W)                                                                    \
    {TX, TY, R, TileCfg<TX, TY, R>::NT, W, sizeof(float) * TileCfg<TX, TY, R>::LDS_FLOATS,          \
     {k_stage<TileCfg<TX, TY, R>, 1, W>, k_stage<TileCfg<TX, TY, R>, 2, W>, k_stage<TileCfg<TX, TY, R>, 3, W>}},

static const Variant g_variants[] = {SWE_TILE_LIST(SWE_VARIANT)};

int variant_count() { return (int)(sizeof(g_variants) / sizeof(g_variants[0])); }
const Variant &variant(int i) { return g_variants[i]; }

int launch_stage(const Variant &v, int stage, const Geo &g, hipStream_t stream)
{
    const int ntx = (g.nx + v.tx - 1) / v.tx, nty = (g.ny + v.ty - 1) / v.ty;
    const int nb = ntx * nty;
    const int mode = (g.Rl[0] ? 1 : 0) + (g.fric_implicit ? 2 : 0) + (g.local_split ? 4 : 0);
    const int vi = (int)(&v - g_variants);
    static const StageSet *const sets[8] = {nullptr, g_stage_mode1, g_stage_mode2, g_stage_mode3,
                                            g_stage_mode4, g_stage_mode5, g_stage_mode6, g_stage_mode7};
    void (*k)(Geo, int, int) = mode ? sets[mode][vi].k[stage - 1] : v.stage[stage - 1];
    hipLaunchKernelGGL(k, dim3(nb), dim3(v.nt), 0, stream, g, ntx, nb);
    return hipGetLastError() == hipSuccess ? SWE_OK : SWE_EDEVICE;
}

int launch_init(const Geo &g, hipStream_t stream)
{
    const long long n = (long long)g.nx * g.ny;
    long long blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(256), 0, stream, g);
    return hipGetLastError() == hipSuccess ? SWE_OK : SWE_EDEVICE;
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
double now_seconds()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int validate_params(const swe_params *p)
{
    if (!p) return SWE_EINVAL;
    if (p->nx < 3 || p->ny < 3) return SWE_EINVAL;
    // every plane (row pitch x ny) must stay below 2^30 elements: the kernels
    // address planes with 32-bit byte offsets
    if ((long long)plane_pitch(p->nx) * p->ny >= (1ll << 30)) return SWE_EINVAL;
    if (!(p->dx > 0.0) || !(p->dy > 0.0) || !std::isfinite(p->dx) || !std::isfinite(p->dy))
        return SWE_EINVAL;
    if (!(p->g > 0.0) || !std::isfinite(p->g)) return SWE_EINVAL;
    if (!std::isfinite(p->cfl)) return SWE_EINVAL;
    if (p->cfl <= 0.0 && !(p->dt_fixed > 0.0 && std::isfinite(p->dt_fixed))) return SWE_EINVAL;
    if (!(p->h_dry >= 0.0) || !std::isfinite(p->h_dry)) return SWE_EINVAL;
    if (!(p->weno_eps > 0.0) || !std::isfinite(p->weno_eps)) return SWE_EINVAL;
    if (!std::isfinite(p->kappa_cap)) return SWE_EINVAL;
    for (int s = 0; s < 4; ++s)
        if (p->bc[s] != SWE_BC_REFLECT && p->bc[s] != SWE_BC_FIXED) return SWE_EINVAL;
    return SWE_OK;
}

static int fetch(const float *src, size_t n, std::vector<float> &dst)
{
    if (!src) return SWE_EINVAL;
    dst.resize(n);
    hipPointerAttribute_t attr;
    bool dev = false;
    if (hipPointerGetAttributes(&attr, src) == hipSuccess)
        dev = attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
    (void)hipGetLastError();
    if (dev) {
        SWE_HIP_TRY(hipMemcpy(dst.data(), src, n * sizeof(float), hipMemcpyDefault));
    } else {
        std::memcpy(dst.data(), src, n * sizeof(float));
    }
    return SWE_OK;
}

int load_fields(const swe_params *p, const float *b, const float *n, const float *h,
                const float *hu, const float *hv, HostFields &f)
{
    int rc = validate_params(p);
    if (rc) return rc;
    const size_t N = (size_t)p->nx * p->ny;
    f.nx = p->nx;
    f.ny = p->ny;
    if ((rc = fetch(b, N, f.b)) || (rc = fetch(n, N, f.n)) || (rc = fetch(h, N, f.h)) ||
        (rc = fetch(hu, N, f.hu)) || (rc = fetch(hv, N, f.hv)))
        return rc;
    for (size_t k = 0; k < N; ++k) {
        if (!std::isfinite(f.b[k]) || !std::isfinite(f.n[k]) || !std::isfinite(f.h[k]) ||
            !std::isfinite(f.hu[k]) || !std::isfinite(f.hv[k]))
            return SWE_EINVAL;
        if (f.h[k] < 0.f || f.n[k] < 0.f) return SWE_EINVAL;
    }
    return SWE_OK;
}

std::vector<float> build_ghosts(const swe_params &p, const HostFields &f)
{
    const int nx = p.nx, ny = p.ny;
    std::vector<float> g((size_t)24 * ny + (size_t)24 * nx, 0.f);
    auto at = [&](const std::vector<float> &a, int i, int j) { return a[(size_t)j * nx + i]; };
    for (int side = 0; side < 4; ++side) {
        const int len = side < 2 ? ny : nx;
        const size_t base = side == 0 ? 0 : side == 1 ? (size_t)12 * ny : side == 2 ? (size_t)24 * ny
                                                                                     : (size_t)24 * ny + (size_t)12 * nx;
        for (int k = 0; k < HALO; ++k)
            for (int q = 0; q < len; ++q) {
                int i0, j0, i1, j1;  // nearest and second-nearest interior cell
                if (side == 0) { i0 = 0; j0 = q; i1 = 1; j1 = q; }
                else if (side == 1) { i0 = nx - 1; j0 = q; i1 = nx - 2; j1 = q; }
                else if (side == 2) { i0 = q; j0 = 0; i1 = q; j1 = 1; }
                else { i0 = q; j0 = ny - 1; i1 = q; j1 = ny - 2; }
                const double b0 = at(f.b, i0, j0), b1 = at(f.b, i1, j1);
                const float bg = (float)(b0 + (k + 1) * (b0 - b1));
                // the frozen depth stored as a level over the ghost's own bed
                const float sg = (float)((double)at(f.h, i0, j0) + std::min((double)bg, 0.0));
                const float vals[4] = {sg, at(f.hu, i0, j0), at(f.hv, i0, j0), bg};
                for (int fld = 0; fld < 4; ++fld) g[base + (size_t)(fld * 3 + k) * len + q] = vals[fld];
            }
    }
    return g;
}

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

size_t scenario_bytes(int nx, int ny)
{
    const size_t plane = align256((size_t)plane_pitch(nx) * ny * sizeof(float));
    const size_t ghost = align256(((size_t)24 * ny + (size_t)24 * nx) * sizeof(float));
    return 11 * plane + ghost + align256(sizeof(DevScen)) + align256(MASS_BLOCKS * sizeof(double));
}

void geo_layout(void *mem, const swe_params &p, Geo &g)
{
    const int nx = p.nx, ny = p.ny, pitch = plane_pitch(nx);
    const size_t plane = align256((size_t)pitch * ny * sizeof(float));
    char *base = static_cast<char *>(mem);
    g.nx = nx;
    g.ny = ny;
    g.pitch = pitch;
    for (int s = 0; s < 4; ++s) g.bc[s] = p.bc[s];
    g.dx = (float)p.dx;
    g.dy = (float)p.dy;
    g.inv_dx = (float)(1.0 / p.dx);
    g.inv_dy = (float)(1.0 / p.dy);
    g.g = (float)p.g;
    g.half_g = (float)(0.5 * p.g);
    g.h_dry = (float)p.h_dry;
    g.eps16 = (float)(16.0 * p.weno_eps);
    g.kappa_cap = (float)p.kappa_cap;
    g.fric_implicit = 0;
    g.local_split = 0;
    g.cfl = (float)p.cfl;
    g.dt_fixed = (float)p.dt_fixed;
    float *planes[11];
    for (int k = 0; k < 11; ++k) planes[k] = reinterpret_cast<float *>(base + k * plane);
    g.b = planes[0];
    g.gn2 = planes[1];
    for (int c = 0; c < 3; ++c) {
        g.U[c] = planes[2 + c];
        g.A[c] = planes[5 + c];
        g.B[c] = planes[8 + c];
    }
    float *ghost = reinterpret_cast<float *>(base + 11 * plane);
    g.ghost = ghost;
    const size_t ghost_b = align256(((size_t)24 * ny + (size_t)24 * nx) * sizeof(float));
    g.sd = reinterpret_cast<DevScen *>(base + 11 * plane + ghost_b);
    g.mass_part = reinterpret_cast<double *>(base + 11 * plane + ghost_b + align256(sizeof(DevScen)));
    g.hmax = nullptr;
    for (int c = 0; c < 3; ++c) g.Rl[c] = nullptr;
}

int scenario_upload_into(void *mem, const swe_params &p, const HostFields &f, hipStream_t stream,
                         DevScenario &d)
{
    const int nx = p.nx, ny = p.ny, pitch = plane_pitch(nx);
    const size_t plane = align256((size_t)pitch * ny * sizeof(float));
    char *base = static_cast<char *>(mem);
    d.base = mem;
    d.bytes = scenario_bytes(nx, ny);
    Geo &g = d.geo;
    geo_layout(mem, p, g);
    float *planes[11];
    for (int k = 0; k < 11; ++k) planes[k] = reinterpret_cast<float *>(base + k * plane);
    float *ghost = reinterpret_cast<float *>(base + 11 * plane);

    const size_t N = (size_t)nx * ny;
    std::vector<float> gn2(N), s0(N);
    for (size_t k = 0; k < N; ++k) {
        gn2[k] = (float)(p.g * (double)f.n[k] * (double)f.n[k]);
        s0[k] = (float)((double)f.h[k] + std::min((double)f.b[k], 0.0));  // stored level
    }
    std::vector<float> gh = build_ghosts(p, f);
    const size_t row = (size_t)nx * sizeof(float), dpitch = (size_t)pitch * sizeof(float);
    SWE_HIP_TRY(hipMemsetAsync(base, 0, 11 * plane, stream));
    SWE_HIP_TRY(hipMemcpy2DAsync(planes[0], dpitch, f.b.data(), row, row, ny, hipMemcpyHostToDevice, stream));
    SWE_HIP_TRY(hipMemcpy2DAsync(planes[1], dpitch, gn2.data(), row, row, ny, hipMemcpyHostToDevice, stream));
    SWE_HIP_TRY(hipMemcpy2DAsync(planes[2], dpitch, s0.data(), row, row, ny, hipMemcpyHostToDevice, stream));
    SWE_HIP_TRY(hipMemcpy2DAsync(planes[3], dpitch, f.hu.data(), row, row, ny, hipMemcpyHostToDevice, stream));
    SWE_HIP_TRY(hipMemcpy2DAsync(planes[4], dpitch, f.hv.data(), row, row, ny, hipMemcpyHostToDevice, stream));
    SWE_HIP_TRY(hipMemcpyAsync(ghost, gh.data(), gh.size() * sizeof(float), hipMemcpyHostToDevice, stream));
    SWE_HIP_TRY(hipMemsetAsync(g.sd, 0, sizeof(DevScen), stream));
    int rc = launch_init(g, stream);
    if (rc) return rc;
    // the host vectors are freed on return: wait for the copies
    SWE_HIP_TRY(hipStreamSynchronize(stream));
    return SWE_OK;
}

// ---- device allocations ---------------------------------------------------
namespace {
struct AllocHook {
    swe_alloc_fn alloc = nullptr;
    swe_release_fn release = nullptr;
    void *user = nullptr;
    int device = 0;
};
std::mutex g_alloc_mu;
AllocHook g_hook;                              // guarded by g_alloc_mu
std::unordered_map<void *, AllocHook> g_owned;  // caller-allocated blocks, with their allocator
}  // namespace

int dev_alloc(void **p, size_t bytes)
{
    *p = nullptr;
    AllocHook h;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        h = g_hook;
    }
    if (!h.alloc) {
        if (hipMalloc(p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return SWE_ENOMEM;
        }
        return SWE_OK;
    }
    if (hipGetDevice(&h.device) != hipSuccess) return SWE_EDEVICE;
    void *m = h.alloc(bytes, h.device, h.user);
    if (!m) return SWE_ENOMEM;
    if (reinterpret_cast<uintptr_t>(m) % 256 != 0) {
        h.release(m, h.device, h.user);
        return SWE_EINVAL;
    }
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        g_owned[m] = h;
    }
    *p = m;
    return SWE_OK;
}

void dev_free(void *p)
{
    if (!p) return;
    AllocHook h;
    bool caller = false;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        auto it = g_owned.find(p);
        if (it != g_owned.end()) {
            h = it->second;
            caller = true;
            g_owned.erase(it);
        }
    }
    if (!caller) {
        (void)hipFree(p);  // waits for the device itself
        return;
    }
    // the allocator may hand the block out again at once: no kernel or copy
    // of this library may still be using it
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != h.device) (void)hipSetDevice(h.device);
    (void)hipDeviceSynchronize();
    if (cur != h.device) (void)hipSetDevice(cur);
    h.release(p, h.device, h.user);
}

static int set_alloc_hook(swe_alloc_fn a, swe_release_fn r, void *user)
{
    if (!a != !r) return SWE_EINVAL;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_hook.alloc = a;
    g_hook.release = r;
    g_hook.user = a ? user : nullptr;
    return SWE_OK;
}

int scenario_upload(const swe_params &p, const HostFields &f, hipStream_t stream, DevScenario &d)
{
    void *mem = nullptr;
    const size_t bytes = scenario_bytes(p.nx, p.ny);
    const int arc = dev_alloc(&mem, bytes);
    if (arc) return arc;
    const int rc = scenario_upload_into(mem, p, f, stream, d);
    if (rc) {
        dev_free(mem);
        d.base = nullptr;
    }
    return rc;
}

int attach_residuals(Geo &g, float *mem, hipStream_t stream)
{
    const size_t plane = (size_t)g.pitch * g.ny;
    for (int k = 0; k < 3; ++k) g.Rl[k] = mem ? mem + k * plane : nullptr;
    // the stored FP32 level is exact as it stands: residuals start at 0
    if (mem) SWE_HIP_TRY(hipMemsetAsync(mem, 0, residual_bytes(g.nx, g.ny), stream));
    return SWE_OK;
}

void scenario_free(DevScenario &d)
{
    dev_free(d.base);
    d.base = nullptr;
}

int stats_from_dev(const Geo &g, const DevScen &ds, swe_stats *st)
{
    const bool bad = (ds.flags & 1u) || ds.alpha[0][0] >= 0x7f800000u || ds.alpha[0][1] >= 0x7f800000u;
    if (st) {
        float ax, ay, ru;
        std::memcpy(&ax, &ds.alpha[0][0], 4);
        std::memcpy(&ay, &ds.alpha[0][1], 4);
        std::memcpy(&ru, &ds.runup, 4);
        st->t = ds.t;
        st->step = ds.step;
        st->mass = ds.mass_sum * (double)g.dx * (double)g.dy;
        st->clamp_mass = ds.clamp_sum * (double)g.dx * (double)g.dy;
        double dt = g.dt_fixed;
        if (g.cfl > 0.f) {
            const double den = (double)ax * (double)g.inv_dx + (double)ay * (double)g.inv_dy;
            dt = (den > 0.0 && den < 1e300) ? (double)(float)((double)g.cfl / den) : 0.0;
        }
        st->dt = dt;
        st->alpha_x = ax;
        st->alpha_y = ay;
        st->runup = ru;
        st->status = bad ? SWE_ENONFINITE : SWE_OK;
    }
    return bad ? SWE_ENONFINITE : SWE_OK;
}

int scenario_read(const DevScenario &d, hipStream_t stream, float *h, float *hu, float *hv,
                  swe_stats *st)
{
    const Geo &g = d.geo;
    const size_t row = (size_t)g.nx * sizeof(float), spitch = (size_t)g.pitch * sizeof(float);
    float *outs[3] = {h, hu, hv};
    const float *src[3] = {g.A[0], g.U[1], g.U[2]};
    if (h) {
        // depth from the stored level into u^(1)'s first plane, free between steps
        const int rc = launch_depth(g, g.U[0], g.A[0], stream);
        if (rc) return rc;
    }
    for (int c = 0; c < 3; ++c)
        if (outs[c])
            SWE_HIP_TRY(hipMemcpy2DAsync(outs[c], row, src[c], spitch, row, g.ny, hipMemcpyDefault, stream));
    int rc = launch_mass(g, stream);
    if (rc) return rc;
    DevScen ds;
    SWE_HIP_TRY(hipMemcpyAsync(&ds, g.sd, sizeof ds, hipMemcpyDeviceToHost, stream));
    SWE_HIP_TRY(hipStreamSynchronize(stream));
    return stats_from_dev(g, ds, st);
}

}  // namespace swe

// ---------------------------------------------------------------------------
// single-scenario context (C ABI)
// ---------------------------------------------------------------------------
using namespace swe;

// Output request of a context (swe_set_outputs).  Snapshot slots and headers
// live on the device; `meta` is copied to one of two pinned buffers after
// every swe_step (double-buffered, each with an event), and once a copy has
// landed the host enqueues the transfers of newly taken snapshots on the
// copy stream behind that event.
struct OutputSet {
    int n = 0;
    double *d_times = nullptr;
    SnapMeta *d_meta = nullptr;
    float *d_slots = nullptr;  // n x 3 planes (pitch x ny)
    float *h_data = nullptr;   // pinned, n x 3 x ny x nx
    SnapMeta *h_meta[2] = {nullptr, nullptr};
    hipEvent_t ev_meta[2] = {nullptr, nullptr};
    bool meta_pending[2] = {false, false};
    int meta_turn = 0;
    bool post_owed = false;        // steps enqueued since the last metadata copy
    int known = 0;                 // outputs known to be taken
    std::vector<SnapHeader> hdr;   // headers of taken outputs
    std::vector<hipEvent_t> ev_copy;
    std::vector<char> queued;
};

struct swe_ctx {
    swe_params p{};
    DevScenario d;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    int tile = -1;        // -1: automatic
    int graph_steps = 32;
    hipGraphExec_t graph = nullptr;
    int graph_k = 0;
    int graph_tile = -1;
    OutputSet out;
    hipStream_t copy_stream = nullptr;
    float *d_hmax = nullptr;
    float *d_resid = nullptr;  // 3 residual planes of the compensated level
};

static int ctx_tile(const swe_ctx *c)
{
    return c->tile >= 0 ? c->tile : default_variant(c->p.nx, c->p.ny);
}

static int enqueue_steps(swe_ctx *c, int n)
{
    const Variant &v = variant(ctx_tile(c));
    for (int s = 0; s < n; ++s) {
        for (int st = 1; st <= 3; ++st) {
            const int rc = launch_stage(v, st, c->d.geo, c->stream);
            if (rc) return rc;
        }
        if (c->out.n > 0) {
            const int rc = launch_snap(c->d.geo, c->out.d_times, c->out.d_meta, c->out.d_slots, c->stream);
            if (rc) return rc;
        }
    }
    return SWE_OK;
}

// ---- outputs ----------------------------------------------------------------

static void outputs_free(swe_ctx *c)
{
    OutputSet &o = c->out;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->copy_stream) (void)hipStreamSynchronize(c->copy_stream);
    for (hipEvent_t e : o.ev_copy)
        if (e) (void)hipEventDestroy(e);
    for (int b = 0; b < 2; ++b) {
        if (o.ev_meta[b]) (void)hipEventDestroy(o.ev_meta[b]);
        if (o.h_meta[b]) (void)hipHostFree(o.h_meta[b]);
    }
    if (o.h_data) (void)hipHostFree(o.h_data);
    dev_free(o.d_slots);
    dev_free(o.d_meta);
    dev_free(o.d_times);
    o = OutputSet();
}

// Enqueue the host transfer of output k (its state sits in slot hdr[k].src)
// on the copy stream, behind the event of the metadata copy that reported it.
static int outputs_queue_copy(swe_ctx *c, int k, hipEvent_t after)
{
    OutputSet &o = c->out;
    const Geo &g = c->d.geo;
    const size_t plane = (size_t)g.pitch * g.ny;
    const size_t cells = (size_t)g.nx * g.ny;
    const size_t row = (size_t)g.nx * sizeof(float), spitch = (size_t)g.pitch * sizeof(float);
    const int src = o.hdr[k].src;
    SWE_HIP_TRY(hipStreamWaitEvent(c->copy_stream, after, 0));
    for (int f = 0; f < 3; ++f)
        SWE_HIP_TRY(hipMemcpy2DAsync(o.h_data + ((size_t)k * 3 + f) * cells, row,
                                     o.d_slots + ((size_t)src * 3 + f) * plane, spitch, row, g.ny,
                                     hipMemcpyDeviceToHost, c->copy_stream));
    SWE_HIP_TRY(hipEventRecord(o.ev_copy[k], c->copy_stream));
    o.queued[k] = 1;
    return SWE_OK;
}

// Take in the metadata copies that have landed (waiting for them if block)
// and queue the transfers of outputs they report as taken.
static int outputs_service(swe_ctx *c, bool block)
{
    OutputSet &o = c->out;
    for (int i = 0; i < 2; ++i) {
        const int b = (o.meta_turn + i) & 1;  // older copy first
        if (!o.meta_pending[b]) continue;
        const hipError_t e = block ? hipEventSynchronize(o.ev_meta[b]) : hipEventQuery(o.ev_meta[b]);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return SWE_EDEVICE;
        o.meta_pending[b] = false;
        const SnapMeta *m = o.h_meta[b];
        const int next = m->next < o.n ? m->next : o.n;
        for (int k = o.known; k < next; ++k) {
            o.hdr[k] = m->hdr[k];
            if (o.hdr[k].src < 0 || o.hdr[k].src > k) return SWE_EDEVICE;
            const int rc = outputs_queue_copy(c, k, o.ev_meta[b]);
            if (rc) return rc;
        }
        if (next > o.known) o.known = next;
    }
    return SWE_OK;
}

// After new steps (or when a copy is owed): copy the metadata to a free
// pinned buffer.  With both buffers in flight the copy is owed and made by
// the next swe_step or swe_output_get call that finds a buffer free.
static int outputs_post(swe_ctx *c)
{
    OutputSet &o = c->out;
    if (o.n == 0) return SWE_OK;
    int rc = outputs_service(c, false);
    if (rc) return rc;
    int b = o.meta_turn;
    if (o.meta_pending[b]) {
        b ^= 1;
        if (o.meta_pending[b]) {
            o.post_owed = true;
            return SWE_OK;
        }
    }
    SWE_HIP_TRY(hipMemcpyAsync(o.h_meta[b], o.d_meta, snap_meta_bytes(o.n), hipMemcpyDeviceToHost, c->stream));
    SWE_HIP_TRY(hipEventRecord(o.ev_meta[b], c->stream));
    o.meta_pending[b] = true;
    o.meta_turn = b ^ 1;
    o.post_owed = false;
    return SWE_OK;
}

// Destroys the captured step graph after any launch of it has finished (the
// buffers it refers to may be released next).
static void drop_graph(swe_ctx *c)
{
    if (c->graph) {
        if (c->stream) (void)hipStreamSynchronize(c->stream);
        (void)hipGraphExecDestroy(c->graph);
    }
    c->graph = nullptr;
    c->graph_k = 0;
}

static int build_graph(swe_ctx *c, int k)
{
    drop_graph(c);
    hipGraph_t g = nullptr;
    SWE_HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_steps(c, k);
    const hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (rc || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : SWE_EDEVICE;
    }
    const hipError_t ie = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
        c->graph = nullptr;
        return SWE_EDEVICE;
    }
    c->graph_k = k;
    c->graph_tile = ctx_tile(c);
    return SWE_OK;
}

extern "C" {

int swe_create(const swe_params *p, const float *b, const float *manning_n, const float *h0,
               const float *hu0, const float *hv0, void *hip_stream, swe_ctx **out)
{
    if (!out) return SWE_EINVAL;
    *out = nullptr;
    HostFields f;
    int rc = load_fields(p, b, manning_n, h0, hu0, hv0, f);
    if (rc) return rc;
    swe_ctx *c = new (std::nothrow) swe_ctx();
    if (!c) return SWE_ENOMEM;
    c->p = *p;
    (void)hipGetDevice(&c->device);
    if (hip_stream) {
        c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return SWE_EDEVICE;
        }
        c->own_stream = true;
    }
    rc = scenario_upload(*p, f, c->stream, c->d);
    if (rc) {
        swe_destroy(c);
        return rc;
    }
    *out = c;
    return SWE_OK;
}

int swe_step(swe_ctx *c, int32_t nsteps)
{
    if (!c || nsteps < 0) return SWE_EINVAL;
    int n = nsteps;
    if (c->graph_steps > 0 && n >= c->graph_steps) {
        if (!c->graph || c->graph_k != c->graph_steps || c->graph_tile != ctx_tile(c)) {
            const int rc = build_graph(c, c->graph_steps);
            if (rc) return rc;
        }
        while (n >= c->graph_k) {
            SWE_HIP_TRY(hipGraphLaunch(c->graph, c->stream));
            n -= c->graph_k;
        }
    }
    const int rc = enqueue_steps(c, n);
    if (rc) return rc;
    return nsteps > 0 ? outputs_post(c) : SWE_OK;
}

int swe_read(swe_ctx *c, float *h, float *hu, float *hv, swe_stats *st)
{
    if (!c) return SWE_EINVAL;
    return scenario_read(c->d, c->stream, h, hu, hv, st);
}

void swe_destroy(swe_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_graph(c);
    outputs_free(c);
    dev_free(c->d_hmax);
    dev_free(c->d_resid);
    if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
    scenario_free(c->d);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

int swe_set_outputs(swe_ctx *c, const double *times, int32_t n)
{
    if (!c || n < 0 || n > 65536 || (n > 0 && !times)) return SWE_EINVAL;
    for (int k = 0; k < n; ++k)
        if (!std::isfinite(times[k]) || (k > 0 && times[k] < times[k - 1])) return SWE_EINVAL;
    drop_graph(c);  // captured steps refer to the old request
    outputs_free(c);
    if (n == 0) return SWE_OK;
    OutputSet &o = c->out;
    const Geo &g = c->d.geo;
    const size_t plane = (size_t)g.pitch * g.ny, cells = (size_t)g.nx * g.ny;
    int rc = SWE_ENOMEM;
    if (!c->copy_stream && hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking) != hipSuccess) {
        c->copy_stream = nullptr;
        return SWE_EDEVICE;
    }
    o.n = n;
    o.hdr.assign(n, SnapHeader{});
    o.ev_copy.assign(n, nullptr);
    o.queued.assign(n, 0);
    if (dev_alloc((void **)&o.d_times, n * sizeof(double)) != SWE_OK ||
        dev_alloc((void **)&o.d_meta, snap_meta_bytes(n)) != SWE_OK ||
        dev_alloc((void **)&o.d_slots, (size_t)n * 3 * plane * sizeof(float)) != SWE_OK ||
        hipHostMalloc(&o.h_data, (size_t)n * 3 * cells * sizeof(float), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&o.h_meta[0], snap_meta_bytes(n), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&o.h_meta[1], snap_meta_bytes(n), hipHostMallocDefault) != hipSuccess)
        goto fail;
    rc = SWE_EDEVICE;
    for (int b = 0; b < 2; ++b)
        if (hipEventCreateWithFlags(&o.ev_meta[b], hipEventDisableTiming) != hipSuccess) goto fail;
    for (int k = 0; k < n; ++k)
        if (hipEventCreateWithFlags(&o.ev_copy[k], hipEventDisableTiming) != hipSuccess) goto fail;
    {
        std::vector<char> meta(snap_meta_bytes(n), 0);
        SnapMeta *m = reinterpret_cast<SnapMeta *>(meta.data());
        m->next = 0;
        m->n = n;
        if (hipMemcpyAsync(o.d_times, times, n * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            hipMemcpyAsync(o.d_meta, meta.data(), meta.size(), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            goto fail;
    }
    return SWE_OK;
fail:
    (void)hipGetLastError();
    outputs_free(c);
    return rc;
}

int swe_output_get(swe_ctx *c, int32_t k, int32_t wait, float *h, float *hu, float *hv, double *t,
                   int64_t *step)
{
    if (!c || k < 0 || k >= c->out.n) return SWE_EINVAL;
    OutputSet &o = c->out;
    int rc = o.post_owed ? outputs_post(c) : outputs_service(c, false);
    if (rc) return rc;
    if (!o.queued[k] && wait) {
        // everything enqueued so far: wait for it and read the metadata
        SWE_HIP_TRY(hipStreamSynchronize(c->stream));
        rc = outputs_service(c, true);
        if (rc) return rc;
        if (!o.queued[k]) {
            SWE_HIP_TRY(hipMemcpyAsync(o.h_meta[0], o.d_meta, snap_meta_bytes(o.n), hipMemcpyDeviceToHost,
                                       c->stream));
            SWE_HIP_TRY(hipStreamSynchronize(c->stream));
            const SnapMeta *m = o.h_meta[0];
            const int next = m->next < o.n ? m->next : o.n;
            if (next > o.known) {
                SWE_HIP_TRY(hipEventRecord(o.ev_meta[0], c->stream));
                for (int j = o.known; j < next; ++j) {
                    o.hdr[j] = m->hdr[j];
                    if (o.hdr[j].src < 0 || o.hdr[j].src > j) return SWE_EDEVICE;
                    rc = outputs_queue_copy(c, j, o.ev_meta[0]);
                    if (rc) return rc;
                }
                o.known = next;
            }
        }
    }
    if (!o.queued[k]) return 0;
    const hipError_t e = wait ? hipEventSynchronize(o.ev_copy[k]) : hipEventQuery(o.ev_copy[k]);
    if (e == hipErrorNotReady) return 0;
    if (e != hipSuccess) return SWE_EDEVICE;
    const Geo &g = c->d.geo;
    const size_t cells = (size_t)g.nx * g.ny;
    float *outs[3] = {h, hu, hv};
    for (int f = 0; f < 3; ++f)
        if (outs[f]) std::memcpy(outs[f], o.h_data + ((size_t)k * 3 + f) * cells, cells * sizeof(float));
    if (t) *t = o.hdr[k].t;
    if (step) *step = o.hdr[k].step;
    return 1;
}

int swe_track_max_depth(swe_ctx *c, int32_t enable)
{
    if (!c) return SWE_EINVAL;
    drop_graph(c);  // captured steps carry the plane's address
    if (c->d_hmax) {
        SWE_HIP_TRY(hipStreamSynchronize(c->stream));
        dev_free(c->d_hmax);
        c->d_hmax = nullptr;
        c->d.geo.hmax = nullptr;
    }
    if (!enable) return SWE_OK;
    const Geo &g = c->d.geo;
    const size_t bytes = (size_t)g.pitch * g.ny * sizeof(float);
    const int arc = dev_alloc((void **)&c->d_hmax, bytes);
    if (arc) return arc;
    // start from the current depth, after the work already enqueued
    const int drc = launch_depth(g, g.U[0], c->d_hmax, c->stream);
    if (drc) return drc;
    c->d.geo.hmax = c->d_hmax;
    return SWE_OK;
}

int swe_read_max_depth(swe_ctx *c, float *hmax)
{
    if (!c || !hmax || !c->d_hmax) return SWE_EINVAL;
    const Geo &g = c->d.geo;
    const size_t row = (size_t)g.nx * sizeof(float), spitch = (size_t)g.pitch * sizeof(float);
    SWE_HIP_TRY(hipMemcpy2DAsync(hmax, row, c->d_hmax, spitch, row, g.ny, hipMemcpyDeviceToHost, c->stream));
    SWE_HIP_TRY(hipStreamSynchronize(c->stream));
    return SWE_OK;
}

int swe_set_option(swe_ctx *c, int32_t key, int64_t value)
{
    if (!c) return SWE_EINVAL;
    if (key == SWE_OPT_GRAPH_STEPS) {
        if (value < 0 || value > 100000) return SWE_EINVAL;
        c->graph_steps = (int)value;
        drop_graph(c);
        return SWE_OK;
    }
    if (key == SWE_OPT_TILE) {
        if (value < -1 || value >= variant_count()) return SWE_EINVAL;
        c->tile = (int)value;
        drop_graph(c);
        return SWE_OK;
    }
    if (key == SWE_OPT_FRICTION_IMPLICIT) {
        if (value != 0 && value != 1) return SWE_EINVAL;
        drop_graph(c);  // captured steps carry the flag in their arguments
        c->d.geo.fric_implicit = (int)value;
        return SWE_OK;
    }
    if (key == SWE_OPT_LOCAL_SPLIT) {
        if (value != 0 && value != 1) return SWE_EINVAL;
        drop_graph(c);  // captured steps launch the kernels of the mode
        c->d.geo.local_split = (int)value;
        return SWE_OK;
    }
    if (key == SWE_OPT_COMPENSATED) {
        if (value != 0 && value != 1) return SWE_EINVAL;
        drop_graph(c);  // captured steps carry the planes' addresses
        Geo &g = c->d.geo;
        if (c->d_resid) {
            SWE_HIP_TRY(hipStreamSynchronize(c->stream));
            dev_free(c->d_resid);
            c->d_resid = nullptr;
            for (int k = 0; k < 3; ++k) g.Rl[k] = nullptr;
        }
        if (!value) return SWE_OK;
        const int arc = dev_alloc((void **)&c->d_resid, residual_bytes(g.nx, g.ny));
        if (arc) return arc;
        return attach_residuals(g, c->d_resid, c->stream);
    }
    return SWE_EINVAL;
}

int swe_state_device(swe_ctx *c, float **h, float **hu, float **hv, int64_t *pitch)
{
    if (!c) return SWE_EINVAL;
    if (h) {
        // the depth is derived from the stored level: refreshed into u^(1)'s
        // first plane, which no call but swe_step overwrites
        const int rc = launch_depth(c->d.geo, c->d.geo.U[0], c->d.geo.A[0], c->stream);
        if (rc) return rc;
        *h = c->d.geo.A[0];
    }
    if (hu) *hu = c->d.geo.U[1];
    if (hv) *hv = c->d.geo.U[2];
    if (pitch) *pitch = c->d.geo.pitch;
    return SWE_OK;
}

int swe_time_stages(swe_ctx *c, int32_t nsteps, double *ms)
{
    if (!c || nsteps <= 0 || !ms) return SWE_EINVAL;
    hipEvent_t ev[6];
    for (int k = 0; k < 6; ++k)
        if (hipEventCreate(&ev[k]) != hipSuccess) {
            for (int q = 0; q < k; ++q) (void)hipEventDestroy(ev[q]);
            return SWE_EDEVICE;
        }
    double acc[3] = {0, 0, 0};
    int rc = SWE_OK;
    const Variant &v = variant(ctx_tile(c));
    for (int s = 0; s < nsteps && !rc; ++s) {
        for (int st = 0; st < 3 && !rc; ++st) {
            if (hipEventRecord(ev[2 * st], c->stream) != hipSuccess) rc = SWE_EDEVICE;
            if (!rc) rc = launch_stage(v, st + 1, c->d.geo, c->stream);
            if (!rc && hipEventRecord(ev[2 * st + 1], c->stream) != hipSuccess) rc = SWE_EDEVICE;
        }
        // the timed steps are ordinary steps: outputs requested are still taken
        if (!rc && c->out.n > 0)
            rc = launch_snap(c->d.geo, c->out.d_times, c->out.d_meta, c->out.d_slots, c->stream);
        if (!rc && hipEventSynchronize(ev[5]) != hipSuccess) rc = SWE_EDEVICE;
        for (int st = 0; st < 3 && !rc; ++st) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, ev[2 * st], ev[2 * st + 1]) != hipSuccess) rc = SWE_EDEVICE;
            acc[st] += t;
        }
    }
    for (int k = 0; k < 6; ++k) (void)hipEventDestroy(ev[k]);
    for (int st = 0; st < 3; ++st) ms[st] = acc[st] / nsteps;
    return rc ? rc : outputs_post(c);
}

int swe_tile_count(void) { return variant_count(); }

int swe_tile_info(int32_t index, int32_t *tx, int32_t *ty, int32_t *r, int32_t *threads)
{
    if (index < 0 || index >= variant_count()) return SWE_ENOTFOUND;
    const Variant &v = variant(index);
    if (tx) *tx = v.tx;
    if (ty) *ty = v.ty;
    if (r) *r = v.r;
    if (threads) *threads = v.nt;
    return SWE_OK;
}

size_t swe_footprint(int32_t nx, int32_t ny)
{
    if (nx < 1 || ny < 1) return 0;
    return scenario_bytes(nx, ny);
}

int swe_set_allocator(swe_alloc_fn alloc, swe_release_fn release, void *user)
{
    return swe::set_alloc_hook(alloc, release, user);
}

const char *swe_strerror(int code)
{
    switch (code) {
    case SWE_OK: return "ok";
    case SWE_EINVAL: return "invalid argument";
    case SWE_ENOMEM: return "out of device memory or over the memory budget";
    case SWE_EDEVICE: return "HIP runtime error";
    case SWE_ENONFINITE: return "non-finite wave speed (state poisoned)";
    case SWE_EBUSY: return "request queue full";
    case SWE_ENOTFOUND: return "unknown ticket or index";
    default: return "unknown error";
    }
}

}  // extern "C"
