// swe_internal.hpp - host-side pieces shared by the single-scenario context,
// the batched launcher and the server: validation, frozen ghosts, device
// scenario storage and the tile-variant registry.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <utility>
#include <vector>

#include "../../include/swe.h"
#include "swe_stage.hpp"

namespace swe {

#define SWE_HIP_TRY(expr)                       \
    do {                                        \
        if ((expr) != hipSuccess) return SWE_EDEVICE; \
    } while (0)

// Host copy of a scenario's inputs (validated).
struct HostFields {
    int nx = 0, ny = 0;
    std::vector<float> b, n, h, hu, hv;
};

int validate_params(const swe_params *p);

// Device memory of the library: hipMalloc, or the caller's allocator when
// swe_set_allocator has set one.  dev_alloc returns SWE_OK, SWE_ENOMEM or
// SWE_EINVAL (memory not aligned to 256 bytes); dev_free (NULL-safe) hands
// memory back to the allocator that made it, after the device is idle.
int dev_alloc(void **p, size_t bytes);
void dev_free(void *p);

// Copies the five fields (host or device pointers) and validates them.
int load_fields(const swe_params *p, const float *b, const float *n, const float *h,
                const float *hu, const float *hv, HostFields &out);

// Row pitch (elements) of every plane: nx rounded up to 64 floats.
inline int plane_pitch(int nx) { return (nx + 63) / 64 * 64; }

// Frozen FIXED ghosts (see ghost_index in swe_stage.hpp): (h, hu, hv) of the
// nearest interior cell, b extended linearly from the two nearest cells; the
// depth is stored as the level h + min(b, 0) over the ghost's own bed.
std::vector<float> build_ghosts(const swe_params &p, const HostFields &f);

// Device storage of one scenario: 11 planes + ghosts + DevScen in one block.
struct DevScenario {
    void *base = nullptr;
    size_t bytes = 0;
    Geo geo{};
};

size_t scenario_bytes(int nx, int ny);
// Geometry, parameters and plane addresses of a scenario stored in `mem`
// (scenario_bytes() of it, 256-byte aligned): 11 planes, FIXED ghosts,
// DevScen, mass partials.  Fills g only; touches no memory.
void geo_layout(void *mem, const swe_params &p, Geo &g);

// Allocates (dev_alloc) and uploads on `stream`, then runs the init kernel.
int scenario_upload(const swe_params &p, const HostFields &f, hipStream_t stream, DevScenario &d);
// Uploads into caller-provided device memory of scenario_bytes() size.
int scenario_upload_into(void *mem, const swe_params &p, const HostFields &f, hipStream_t stream,
                         DevScenario &d);
void scenario_free(DevScenario &d);

// Wave speeds of u^n into DevScen slot 0 and the initial runup (after a
// zeroing of DevScen).
int launch_init(const Geo &g, hipStream_t stream);
// Deterministic FP64 sum of h into DevScen::mass_sum.
int launch_mass(const Geo &g, hipStream_t stream);

// Reads state planes (any may be NULL; host or device) and the diagnostics.
int scenario_read(const DevScenario &d, hipStream_t stream, float *h, float *hu, float *hv,
                  swe_stats *st);
int stats_from_dev(const Geo &g, const DevScen &ds, swe_stats *st);

// ---- tile variants -------------------------------------------------------
struct Variant {
    int tx, ty, r, nt, waves;
    size_t lds_bytes;
    void (*stage[3])(Geo, int, int);    // single-scenario stage kernels
};
// (tile width, tile height, cells per thread per sweep, minimum waves per SIMD)
#define SWE_TILE_LIST(X) \
    X(64, 16, 8, 2)      \
    X(64, 32, 8, 2)      \
    X(32, 32, 8, 2)      \
    X(64, 16, 4, 2)      \
    X(128, 16, 8, 2)     \
    X(64, 16, 4, 3)      \
    X(32, 32, 4, 3)      \
    X(32, 16, 2, 2)      \
    X(16, 16, 2, 2)      \
    X(16, 16, 1, 2)
// Stage kernels of every tile variant (in SWE_TILE_LIST order) in the
// optional modes of a context, mode = CMP + 2 IMP + 4 LLF: 1 the compensated
// level, 2 point-implicit friction, 4 local Lax-Friedrichs splitting, and
// their sums.  One translation unit per mode (swe_mode<N>.hip), so the sets
// compile in parallel.
struct StageSet {
    void (*k[3])(Geo, int, int);
};
#define SWE_STAGE_SET_L(TX, TY, R, W, CMP, IMP, LLF)                                                 \
    {{k_stage<TileCfg<TX, TY, R>, 1, W, CMP, IMP, LLF>, k_stage<TileCfg<TX, TY, R>, 2, W, CMP, IMP, LLF>, \
      k_stage<TileCfg<TX, TY, R>, 3, W, CMP, IMP, LLF>}},
#define SWE_STAGE_SET(TX, TY, R, W, CMP, IMP) SWE_STAGE_SET_L(TX, TY, R, W, CMP, IMP, false)
extern const StageSet g_stage_mode1[], g_stage_mode2[], g_stage_mode3[], g_stage_mode4[], g_stage_mode5[],
    g_stage_mode6[], g_stage_mode7[];
// depth h = s - min(b, 0) of a stored-level plane into out (same pitch)
int launch_depth(const Geo &g, const float *lev, float *out, hipStream_t stream);
int variant_count();
const Variant &variant(int i);
int default_variant(int nx, int ny);
// variant of one launch over scenarios of these (nx, ny) sizes
int batch_variant_for(const std::vector<std::pair<int, int>> &sizes);
int launch_stage(const Variant &v, int stage, const Geo &g, hipStream_t stream);

double now_seconds();

// Builds the round/ticket tables of one run over `geos` (scenario i advances
// ksteps[i] >= 0 steps) and launches it on `stream` with tile variant vi, in
// SWE_BATCH_PERSISTENT or SWE_BATCH_ROUNDS mode, optionally as a hipGraph.
// Asynchronous; the tables stay valid until the next run (which first waits
// for `stream`).
struct SegmentLauncher {
    void *dmem = nullptr;
    size_t dbytes = 0;
    char *hbuf = nullptr;  // pinned host copy of the tables (asynchronous upload)
    size_t hbytes = 0;
    hipGraphExec_t graph = nullptr;
    int cus = 0;
    int group = 0;  // tickets taken per atomic in persistent mode (0: automatic)
    ~SegmentLauncher();
    // implicit: the point-implicit friction kernels; compensated: the
    // compensated-level kernels (every geo then has residual planes);
    // local_split: the local Lax-Friedrichs kernels
    int run(const std::vector<Geo> &geos, const std::vector<int> &ksteps, int vi, int mode, bool use_graph,
            hipStream_t stream, bool implicit = false, bool compensated = false, bool local_split = false);
};

// Residual planes of the compensated level for one scenario: `mem` holds
// three planes of the scenario's pitch x ny floats; they are zeroed on
// `stream` and attached to g (mem == nullptr detaches them).
int attach_residuals(Geo &g, float *mem, hipStream_t stream);
inline size_t residual_bytes(int nx, int ny) { return (size_t)plane_pitch(nx) * ny * sizeof(float) * 3; }

}  // namespace swe
