// swe_noalloc.hip - swe_run_noalloc: the single-scenario step on caller device
// arrays, with every intermediate in a fixed device array of the library.
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation).  The
// scenario's working storage (the same 11 planes, frozen ghosts, DevScen and
// mass partials that swe_create allocates) lives in `scratch`, a file-scope
// device array of NOALLOC_BYTES.  Each device holds its own copy; host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device, taken once per device on the first call there.  The
// kernels compute exactly what swe_create / swe_step / swe_read compute (the
// same conversions, stage kernels and tile choice), so the results are
// bitwise those of a context.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "swe_internal.hpp"

namespace swe {

constexpr size_t NOALLOC_BYTES = SWE_NOALLOC_MAX_BYTES;

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_na_mu;
static void *g_na_ptr[NOALLOC_MAX_DEVICES];  // device address of `scratch`, per device

// Address of this device's `scratch` (looked up once per device).
static int scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return SWE_EDEVICE;
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SWE_EDEVICE;
        g_na_ptr[dev] = p;
    }
    *out = g_na_ptr[dev];
    return SWE_OK;
}

// Clears the scenario scalars (a kernel, not a memset, so the call can be
// captured into a graph and replayed).
__global__ __launch_bounds__(64) void k_na_clear(Geo G)
{
    unsigned int *w = reinterpret_cast<unsigned int *>(G.sd);
    for (int i = threadIdx.x; i < (int)(sizeof(DevScen) / 4); i += 64) w[i] = 0u;
}

// Caller fields [ny][nx] -> the pitched planes b, g n^2 and the stored level
// s = h + min(b, 0) (both in FP64, rounded once, as the host upload does),
// hu, hv; padding columns are zero.  Non-finite fields, h < 0 or n < 0 set
// bit 1 of DevScen::flags.
__global__ __launch_bounds__(256) void k_na_load(Geo G, const float *b, const float *n, const float *h,
                                                 const float *hu, const float *hv, double g)
{
    const long long total = (long long)G.pitch * G.ny;
    bool bad = false;
    for (long long e = blockIdx.x * 256ll + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
        const int j = (int)(e / G.pitch), i = (int)(e - (long long)j * G.pitch);
        float vb = 0.f, vg = 0.f, vs = 0.f, vu = 0.f, vv = 0.f;
        if (i < G.nx) {
            const long long k = (long long)j * G.nx + i;
            vb = b[k];
            const float vn = n[k], vh = h[k];
            vu = hu[k];
            vv = hv[k];
            bad |= !(std::isfinite(vb) && std::isfinite(vn) && std::isfinite(vh) && std::isfinite(vu) &&
                     std::isfinite(vv)) ||
                   vh < 0.f || vn < 0.f;
            vg = (float)(g * (double)vn * (double)vn);
            const double bd = (double)vb;
            vs = (float)((double)vh + (0.0 < bd ? 0.0 : bd));
        }
        const_cast<float *>(G.b)[e] = vb;
        G.U[0][e] = vs;
        G.U[1][e] = vu;
        G.U[2][e] = vv;
        const_cast<float *>(G.gn2)[e] = vg;
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&G.sd->flags, 2u);
}

// Frozen FIXED ghosts from the caller's initial fields (the values the host
// builds for a context): (h, hu, hv) of the nearest interior cell, b extended
// linearly from the two nearest cells, the depth stored as a level over the
// ghost's own bed.  One thread per (side, layer, position).
__global__ __launch_bounds__(256) void k_na_ghost(Geo G, const float *b, const float *h, const float *hu,
                                                  const float *hv)
{
    const int nx = G.nx, ny = G.ny;
    const int per_x = HALO * ny, per_y = HALO * nx;
    const int total = 2 * per_x + 2 * per_y;
    float *gh = const_cast<float *>(G.ghost);
    for (int e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256) {
        int side, r;
        if (e < 2 * per_x) {
            side = e / per_x;
            r = e - side * per_x;
        } else {
            side = 2 + (e - 2 * per_x) / per_y;
            r = e - 2 * per_x - (side - 2) * per_y;
        }
        const int len = side < 2 ? ny : nx;
        const int k = r / len, q = r - k * len;
        int i0, j0, i1, j1;
        if (side == 0) { i0 = 0; j0 = q; i1 = 1; j1 = q; }
        else if (side == 1) { i0 = nx - 1; j0 = q; i1 = nx - 2; j1 = q; }
        else if (side == 2) { i0 = q; j0 = 0; i1 = q; j1 = 1; }
        else { i0 = q; j0 = ny - 1; i1 = q; j1 = ny - 2; }
        const long long c0 = (long long)j0 * nx + i0, c1 = (long long)j1 * nx + i1;
        const double b0 = b[c0], b1 = b[c1];
        const float bg = (float)(b0 + (double)(k + 1) * (b0 - b1));
        const double bgd = (double)bg;
        const float sg = (float)((double)h[c0] + (0.0 < bgd ? 0.0 : bgd));
        gh[ghost_index(G, side, 0, k, q)] = sg;
        gh[ghost_index(G, side, 1, k, q)] = hu[c0];
        gh[ghost_index(G, side, 2, k, q)] = hv[c0];
        gh[ghost_index(G, side, 3, k, q)] = bg;
    }
}

// The state back into the caller's arrays: depth h = s - min(b, 0), hu, hv.
__global__ __launch_bounds__(256) void k_na_store(Geo G, float *h, float *hu, float *hv)
{
    const long long total = (long long)G.nx * G.ny;
    for (long long k = blockIdx.x * 256ll + threadIdx.x; k < total; k += (long long)gridDim.x * 256) {
        const int j = (int)(k / G.nx), i = (int)(k - (long long)j * G.nx);
        const int gi = j * G.pitch + i;
        h[k] = G.U[0][gi] - fminf(G.b[gi], 0.f);
        hu[k] = G.U[1][gi];
        hv[k] = G.U[2][gi];
    }
}

static unsigned grid_for(long long n)
{
    long long blocks = (n + 255) / 256;
    return (unsigned)(blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks));
}

static bool is_device_ptr(const void *p)
{
    hipPointerAttribute_t a;
    const bool ok = hipPointerGetAttributes(&a, p) == hipSuccess &&
                    (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged);
    (void)hipGetLastError();
    return ok;
}

}  // namespace swe

using namespace swe;

extern "C" {

int swe_run_noalloc(const swe_params *p, const float *b, const float *manning_n, float *h, float *hu,
                    float *hv, int32_t nsteps, void *hip_stream, swe_stats *stats)
{
    int rc = validate_params(p);
    if (rc) return rc;
    if (nsteps < 0 || !b || !manning_n || !h || !hu || !hv) return SWE_EINVAL;
    if (scenario_bytes(p->nx, p->ny) > NOALLOC_BYTES) return SWE_EINVAL;
    const void *ptrs[5] = {b, manning_n, h, hu, hv};
    for (const void *q : ptrs)
        if (!is_device_ptr(q)) return SWE_EINVAL;
    int dev = 0;
    SWE_HIP_TRY(hipGetDevice(&dev));
    void *mem = nullptr;
    if ((rc = scratch_address(dev, &mem))) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Geo g{};
    geo_layout(mem, *p, g);
    hipLaunchKernelGGL(k_na_clear, dim3(1), dim3(64), 0, s, g);
    hipLaunchKernelGGL(k_na_load, dim3(grid_for((long long)g.pitch * g.ny)), dim3(256), 0, s, g, b, manning_n,
                       h, hu, hv, p->g);
    hipLaunchKernelGGL(k_na_ghost, dim3(grid_for(6ll * (p->nx + p->ny))), dim3(256), 0, s, g, b, h, hu, hv);
    SWE_HIP_TRY(hipGetLastError());
    if ((rc = launch_init(g, s))) return rc;
    const Variant &v = variant(default_variant(p->nx, p->ny));
    for (int k = 0; k < nsteps; ++k)
        for (int st = 1; st <= 3; ++st)
            if ((rc = launch_stage(v, st, g, s))) return rc;
    hipLaunchKernelGGL(k_na_store, dim3(grid_for((long long)p->nx * p->ny)), dim3(256), 0, s, g, h, hu, hv);
    SWE_HIP_TRY(hipGetLastError());
    if (!stats) return SWE_OK;
    if ((rc = launch_mass(g, s))) return rc;
    DevScen ds;
    SWE_HIP_TRY(hipMemcpyAsync(&ds, g.sd, sizeof ds, hipMemcpyDeviceToHost, s));
    SWE_HIP_TRY(hipStreamSynchronize(s));
    if (ds.flags & 2u) return SWE_EINVAL;
    return stats_from_dev(g, ds, stats);
}

}  // extern "C"
