// swe_batch.hip - many scenarios of uneven sizes and step counts advanced
// together.
//
// Schedule.  A run advances scenario s by k_s = min(max_steps, remaining_s)
// steps.  Scenarios are ordered by k_s (descending), so the scenarios taking
// part in round r (round = one stage of one step: r = 3*step + stage - 1)
// are a prefix of that order, of length A(r).  The tiles of round r are the
// tiles of those scenarios, numbered scenario after scenario.
//
// PERSISTENT mode: one kernel for the whole run.  Tiles are numbered round
// after round ("tickets"); each block repeatedly takes the next group of
// tickets with one atomic and maps them to (round, scenario, tile) by binary
// search in two small tables.  The group is handled in runs that stay inside
// one round: a run waits until every tile of the previous round of each
// scenario it touches has completed (per-scenario counters, one acquire at
// agent scope), runs its tiles, and publishes them with one release.  A
// ticket only ever waits on smaller tickets, and tickets are taken by running
// blocks, so the smallest unfinished ticket can always proceed: the kernel
// cannot deadlock and needs no co-residency guarantee.
//
// ROUNDS mode: one launch per round over the tiles of all its scenarios;
// kernel boundaries order the rounds.  Optionally captured as one hipGraph.
//
// Both modes run the same stage code per tile, so every scenario's state is
// bitwise identical to a run of that scenario alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "swe_batch_kernels.hpp"
#include "swe_internal.hpp"
#include "swe_schedule.hpp"

namespace swe {

// Clears the run's counters (a kernel, so graph replays need no memset node).
__global__ void k_zero_counters(unsigned int *done, int n, unsigned long long *ticket)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) done[i] = 0u;
    if (threadIdx.x == 0) *ticket = 0ull;
}

#define SWE_BK_EXPLICIT(TX, TY, R, W) SWE_BK(TX, TY, R, W, false)
const BatchKernels g_bk[] = {SWE_TILE_LIST(SWE_BK_EXPLICIT)};

// ---------------------------------------------------------------------------
// segment launcher (shared by swe_batch and the server)
// ---------------------------------------------------------------------------
static size_t al(size_t x) { return (x + 255) / 256 * 256; }

SegmentLauncher::~SegmentLauncher()
{
    if (graph) (void)hipGraphExecDestroy(graph);
    dev_free(dmem);
    if (hbuf) (void)hipHostFree(hbuf);
}

int SegmentLauncher::run(const std::vector<Geo> &geos, const std::vector<int> &ksteps, int vi, int mode,
                         bool use_graph, hipStream_t stream, bool implicit, bool compensated, bool local_split)
{
    const Variant &v = variant(vi);
    static const BatchKernels *const sets[8] = {g_bk,     g_bk_cmp,     g_bk_imp,     g_bk_cmp_imp,
                                                g_bk_llf, g_bk_llf_cmp, g_bk_llf_imp, g_bk_llf_cmp_imp};
    const BatchKernels &K = sets[(compensated ? 1 : 0) + (implicit ? 2 : 0) + (local_split ? 4 : 0)][vi];
    const int n = (int)geos.size();
    std::vector<int> nxs(n), nys(n);
    for (int i = 0; i < n; ++i) {
        nxs[i] = geos[i].nx;
        nys[i] = geos[i].ny;
    }
    const Schedule S = build_schedule(nxs, nys, ksteps, v.tx, v.ty);
    if (S.nact == 0) return SWE_OK;
    const int nact = S.nact, nrounds = S.nrounds;
    const std::vector<int> &prefix = S.prefix, &ntx = S.ntx, &order = S.order, &ractive = S.ractive;
    const std::vector<long long> &rstart = S.rstart;

    const size_t o_geo = 0, o_order = o_geo + al(n * sizeof(Geo));
    const size_t o_prefix = o_order + al(nact * sizeof(int));
    const size_t o_ntx = o_prefix + al((nact + 1) * sizeof(int));
    const size_t o_rstart = o_ntx + al(nact * sizeof(int));
    const size_t o_ract = o_rstart + al((nrounds + 1) * sizeof(long long));
    const size_t o_blk = o_ract + al(nrounds * sizeof(int));
    const int ntiles = prefix[nact];
    const size_t o_done = o_blk + al((size_t)ntiles * sizeof(int2));
    const size_t o_ticket = o_done + al(nact * sizeof(unsigned int));
    const size_t need = o_ticket + al(sizeof(unsigned long long));
    SWE_HIP_TRY(hipStreamSynchronize(stream));  // the previous segment's tables are free
    if (graph) {
        (void)hipGraphExecDestroy(graph);
        graph = nullptr;
    }
    if (need > dbytes) {
        dev_free(dmem);
        dmem = nullptr;
        dbytes = 0;
        const int arc = dev_alloc(&dmem, need);
        if (arc) return arc;
        dbytes = need;
    }
    if (cus <= 0) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (cus <= 0) cus = 256;
    }
    if (o_done > hbytes) {
        // pinned, so that the upload below is asynchronous; reused while
        // large enough (the previous run's copy is complete: see above)
        if (hbuf) (void)hipHostFree(hbuf);
        hbuf = nullptr;
        hbytes = 0;
        SWE_HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&hbuf), o_done * 2, hipHostMallocDefault));
        hbytes = o_done * 2;
    }
    char *hb = hbuf;
    std::memset(hb, 0, o_done);
    std::memcpy(hb + o_geo, geos.data(), n * sizeof(Geo));
    std::memcpy(hb + o_order, order.data(), nact * sizeof(int));
    std::memcpy(hb + o_prefix, prefix.data(), (nact + 1) * sizeof(int));
    std::memcpy(hb + o_ntx, ntx.data(), nact * sizeof(int));
    std::memcpy(hb + o_rstart, rstart.data(), (nrounds + 1) * sizeof(long long));
    std::memcpy(hb + o_ract, ractive.data(), nrounds * sizeof(int));
    int2 *blk = reinterpret_cast<int2 *>(hb + o_blk);
    for (int q = 0; q < nact; ++q)
        for (int l = prefix[q]; l < prefix[q + 1]; ++l) blk[l] = make_int2(order[q], l - prefix[q]);
    SWE_HIP_TRY(hipMemcpyAsync(dmem, hb, o_done, hipMemcpyHostToDevice, stream));

    char *dm = static_cast<char *>(dmem);
    BatchTables T;
    T.geo = reinterpret_cast<const Geo *>(dm + o_geo);
    T.order = reinterpret_cast<const int *>(dm + o_order);
    T.prefix = reinterpret_cast<const int *>(dm + o_prefix);
    T.ntx = reinterpret_cast<const int *>(dm + o_ntx);
    T.rstart = reinterpret_cast<const long long *>(dm + o_rstart);
    T.ractive = reinterpret_cast<const int *>(dm + o_ract);
    T.blk = reinterpret_cast<const int2 *>(dm + o_blk);
    T.done = reinterpret_cast<unsigned int *>(dm + o_done);
    T.ticket = reinterpret_cast<unsigned long long *>(dm + o_ticket);
    T.nrounds = nrounds;
    T.nact = nact;
    T.group = group;
    int per_cu = 0;
    if (mode == SWE_BATCH_PERSISTENT &&
        (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, K.persistent, v.nt, 0) != hipSuccess || per_cu <= 0))
        per_cu = 1;
    long long grid = (long long)(per_cu > 0 ? per_cu : 1) * cus;
    if (grid > rstart[nrounds]) grid = rstart[nrounds];
    // about one run of tickets per block and round: one acquire and one
    // release per block per round, as many as a kernel boundary costs
    if (group <= 0) T.group = ticket_group(S, grid);

    auto enqueue = [&]() -> int {
        if (mode == SWE_BATCH_PERSISTENT) {
            hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(256), 0, stream, T.done, nact, T.ticket);
            hipLaunchKernelGGL(K.persistent, dim3((unsigned)grid), dim3(v.nt), 0, stream, T);
        } else {
            for (int r = 0; r < nrounds; ++r) {
                const int nb = prefix[ractive[r]];
                hipLaunchKernelGGL(K.round[r % 3], dim3(nb), dim3(v.nt), 0, stream, T, ractive[r], nb);
            }
        }
        return hipGetLastError() == hipSuccess ? SWE_OK : SWE_EDEVICE;
    };

    if (use_graph) {
        hipGraph_t g = nullptr;
        SWE_HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue();
        const hipError_t e = hipStreamEndCapture(stream, &g);
        if (rc || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return rc ? rc : SWE_EDEVICE;
        }
        const hipError_t ie = hipGraphInstantiate(&graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            graph = nullptr;
            return SWE_EDEVICE;
        }
        SWE_HIP_TRY(hipGraphLaunch(graph, stream));
        return SWE_OK;
    }
    return enqueue();
}

}  // namespace swe

using namespace swe;

struct BatchScen {
    swe_params p{};
    DevScenario d;
    int total = 0;  // requested steps
    int done = 0;   // steps enqueued so far
    float *hmax = nullptr;  // maximum-depth plane, when tracked
    float *resid = nullptr; // residual planes of the compensated level, when on
};

struct swe_batch {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<BatchScen> sc;
    int mode = SWE_BATCH_ROUNDS;
    bool use_graph = true;
    int tile = -1;
    bool implicit = false;     // point-implicit friction
    bool compensated = false;  // compensated level (residual planes per scenario)
    bool local_split = false;  // local Lax-Friedrichs splitting
    SegmentLauncher seg;
};

// Gives scenario s residual planes (zeroed) or takes them away.
static int batch_residuals(swe_batch *bt, BatchScen &s, bool on)
{
    if (s.resid) {
        SWE_HIP_TRY(hipStreamSynchronize(bt->stream));
        dev_free(s.resid);
        s.resid = nullptr;
        (void)attach_residuals(s.d.geo, nullptr, bt->stream);
    }
    if (!on) return SWE_OK;
    const int arc = dev_alloc((void **)&s.resid, residual_bytes(s.p.nx, s.p.ny));
    if (arc) return arc;
    return attach_residuals(s.d.geo, s.resid, bt->stream);
}

static int batch_variant(const swe_batch *bt)
{
    if (bt->tile >= 0) return bt->tile;
    std::vector<std::pair<int, int>> sizes;
    for (const auto &s : bt->sc) sizes.emplace_back(s.p.nx, s.p.ny);
    return batch_variant_for(sizes);
}

extern "C" {

int swe_batch_create(void *hip_stream, swe_batch **out)
{
    if (!out) return SWE_EINVAL;
    *out = nullptr;
    swe_batch *bt = new (std::nothrow) swe_batch();
    if (!bt) return SWE_ENOMEM;
    if (hip_stream) {
        bt->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&bt->stream, hipStreamNonBlocking) != hipSuccess) {
            delete bt;
            return SWE_EDEVICE;
        }
        bt->own_stream = true;
    }
    *out = bt;
    return SWE_OK;
}

int swe_batch_add(swe_batch *bt, const swe_params *p, const float *b, const float *n, const float *h0,
                  const float *hu0, const float *hv0, int32_t nsteps, int32_t *index)
{
    if (!bt || nsteps < 0) return SWE_EINVAL;
    HostFields f;
    int rc = load_fields(p, b, n, h0, hu0, hv0, f);
    if (rc) return rc;
    BatchScen s;
    s.p = *p;
    s.total = nsteps;
    SWE_HIP_TRY(hipStreamSynchronize(bt->stream));
    rc = scenario_upload(*p, f, bt->stream, s.d);
    if (rc) return rc;
    if (bt->compensated && (rc = batch_residuals(bt, s, true))) {
        scenario_free(s.d);
        return rc;
    }
    bt->sc.push_back(s);
    if (index) *index = (int32_t)bt->sc.size() - 1;
    return SWE_OK;
}

int swe_batch_set_mode(swe_batch *bt, int32_t mode, int32_t use_graph)
{
    if (!bt || (mode != SWE_BATCH_PERSISTENT && mode != SWE_BATCH_ROUNDS)) return SWE_EINVAL;
    bt->mode = mode;
    bt->use_graph = use_graph != 0;
    return SWE_OK;
}

int swe_batch_set_tile(swe_batch *bt, int32_t tile)
{
    if (!bt || tile < -1 || tile >= variant_count()) return SWE_EINVAL;
    bt->tile = tile;
    return SWE_OK;
}

int swe_batch_set_option(swe_batch *bt, int32_t key, int64_t value)
{
    if (!bt || (value != 0 && value != 1)) return SWE_EINVAL;
    if (key == SWE_OPT_FRICTION_IMPLICIT) {
        bt->implicit = value != 0;
        return SWE_OK;
    }
    if (key == SWE_OPT_LOCAL_SPLIT) {
        bt->local_split = value != 0;
        return SWE_OK;
    }
    if (key != SWE_OPT_COMPENSATED) return SWE_EINVAL;
    for (auto &s : bt->sc) {
        const int rc = batch_residuals(bt, s, value != 0);
        if (rc) {
            for (auto &q : bt->sc) (void)batch_residuals(bt, q, false);
            bt->compensated = false;
            return rc;
        }
    }
    bt->compensated = value != 0;
    return SWE_OK;
}

int swe_batch_run(swe_batch *bt, int32_t max_steps)
{
    if (!bt) return SWE_EINVAL;
    std::vector<Geo> geos;
    std::vector<int> ks;
    for (auto &s : bt->sc) {
        int k = s.total - s.done;
        if (max_steps >= 0 && k > max_steps) k = max_steps;
        geos.push_back(s.d.geo);
        ks.push_back(k);
    }
    const int rc = bt->seg.run(geos, ks, batch_variant(bt), bt->mode, bt->use_graph, bt->stream, bt->implicit,
                               bt->compensated, bt->local_split);
    if (rc) return rc;
    for (size_t i = 0; i < bt->sc.size(); ++i) bt->sc[i].done += ks[i];
    return SWE_OK;
}

int swe_batch_read(swe_batch *bt, int32_t index, float *h, float *hu, float *hv, swe_stats *st)
{
    if (!bt) return SWE_EINVAL;
    if (index < 0 || index >= (int)bt->sc.size()) return SWE_ENOTFOUND;
    return scenario_read(bt->sc[index].d, bt->stream, h, hu, hv, st);
}

int swe_batch_track_max_depth(swe_batch *bt, int32_t index, int32_t enable)
{
    if (!bt) return SWE_EINVAL;
    if (index < 0 || index >= (int)bt->sc.size()) return SWE_ENOTFOUND;
    BatchScen &s = bt->sc[index];
    if (s.hmax) {
        SWE_HIP_TRY(hipStreamSynchronize(bt->stream));
        dev_free(s.hmax);
        s.hmax = nullptr;
        s.d.geo.hmax = nullptr;
    }
    if (!enable) return SWE_OK;
    const Geo &g = s.d.geo;
    const size_t bytes = (size_t)g.pitch * g.ny * sizeof(float);
    const int arc = dev_alloc((void **)&s.hmax, bytes);
    if (arc) return arc;
    // start from the current depth, after the work already enqueued
    const int drc = launch_depth(g, g.U[0], s.hmax, bt->stream);
    if (drc) return drc;
    s.d.geo.hmax = s.hmax;
    return SWE_OK;
}

int swe_batch_read_max_depth(swe_batch *bt, int32_t index, float *hmax)
{
    if (!bt || !hmax) return SWE_EINVAL;
    if (index < 0 || index >= (int)bt->sc.size()) return SWE_ENOTFOUND;
    const BatchScen &s = bt->sc[index];
    if (!s.hmax) return SWE_EINVAL;
    const Geo &g = s.d.geo;
    const size_t row = (size_t)g.nx * sizeof(float), spitch = (size_t)g.pitch * sizeof(float);
    SWE_HIP_TRY(hipMemcpy2DAsync(hmax, row, s.hmax, spitch, row, g.ny, hipMemcpyDeviceToHost, bt->stream));
    SWE_HIP_TRY(hipStreamSynchronize(bt->stream));
    return SWE_OK;
}

void swe_batch_destroy(swe_batch *bt)
{
    if (!bt) return;
    if (bt->stream) (void)hipStreamSynchronize(bt->stream);
    for (auto &s : bt->sc) {
        dev_free(s.hmax);
        dev_free(s.resid);
        scenario_free(s.d);
    }
    if (bt->own_stream && bt->stream) (void)hipStreamDestroy(bt->stream);
    delete bt;  // the segment launcher frees its tables
}

}  // extern "C"
