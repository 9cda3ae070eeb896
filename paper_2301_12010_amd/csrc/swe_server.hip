// swe_server.hip - continuous batching of scenario requests.
//
// The server owns a device arena of the memory budget and two host threads.
// Requests wait in a FIFO queue.  The upload thread admits the queue's head
// when a slot is free and its footprint (swe_footprint) fits a first-fit hole
// of the arena, so admission is by HBM footprint and allocates no device
// memory after create; it prepares the request's device planes on its own
// stream and hands the request to the segment thread.  The segment thread
// advances every resident scenario in segments: one launch sequence advances
// each by min(segment_steps, its remaining steps); uploaded requests join at
// the next segment.  While a segment runs, the segment thread copies the
// results of scenarios finished in the previous segment back to host memory,
// and those leave the arena.  Neither host-side preparation nor transfers
// hold up the compute stream while resident work remains.  Every scenario
// runs the same per-tile stage code as alone, so its result does not depend
// on what else is in the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "swe_internal.hpp"

namespace swe {

// First-fit allocator over one device block; offsets aligned to 256 bytes.
class Arena {
  public:
    int init(size_t bytes)
    {
        bytes_ = bytes / 256 * 256;
        const int rc = dev_alloc(&base_, bytes_);
        if (rc) return rc;
        free_[0] = bytes_;
        return SWE_OK;
    }
    ~Arena()
    {
        dev_free(base_);
    }
    void *alloc(size_t n)
    {
        n = (n + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > n) free_[off + n] = len - n;
                used_ += n;
                high_ = std::max(high_, used_);
                return static_cast<char *>(base_) + off;
            }
        }
        return nullptr;
    }
    void release(void *p, size_t n)
    {
        n = (n + 255) / 256 * 256;
        size_t off = static_cast<char *>(p) - static_cast<char *>(base_);
        used_ -= n;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            free_.erase(next);
        }
        auto prev = free_.lower_bound(off);
        if (prev != free_.begin()) {
            --prev;
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }
    size_t capacity() const { return bytes_; }
    size_t used() const { return used_; }
    size_t high_water() const { return high_; }

  private:
    void *base_ = nullptr;
    size_t bytes_ = 0, used_ = 0, high_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
};

struct Request {
    uint64_t ticket = 0;
    swe_params p{};
    HostFields f;
    int nsteps = 0;
    int status = SWE_PENDING;
    int error = SWE_OK;
    std::atomic<bool> cancel{false};  // set by swe_cancel, read by the server thread
    bool track_max = false;  // keep the maximum-depth map (SWE_SUBMIT_MAX_DEPTH)
    double t_submit = 0, t_admit = 0, t_done = 0;
    // resident state
    DevScenario d;
    int done_steps = 0;
    // result
    swe_stats st{};
    std::vector<float> h, hu, hv, hmax;
};

// Device bytes of a request: its scenario, plus one plane for the
// maximum-depth map when it keeps one, plus three residual planes when the
// server runs the compensated level.
static size_t map_bytes(const swe_params &p)
{
    return ((size_t)plane_pitch(p.nx) * p.ny * sizeof(float) + 255) / 256 * 256;
}
static size_t request_bytes(const swe_params &p, bool track_max, bool compensated)
{
    return scenario_bytes(p.nx, p.ny) + (track_max ? map_bytes(p) : 0) +
           (compensated ? residual_bytes(p.nx, p.ny) : 0);
}

}  // namespace swe

using namespace swe;

struct swe_server {
    int device = 0;
    int max_slots = 64;
    int segment_steps = 100;
    int mode = SWE_BATCH_ROUNDS;
    bool implicit = false;     // point-implicit friction (set before the first submit)
    bool local_split = false;  // local Lax-Friedrichs splitting (set before the first submit)
    std::atomic<bool> compensated{false};  // compensated level (set before the first submit)
    size_t max_queue = 1 << 16;
    Arena arena;
    hipStream_t compute = nullptr, copy = nullptr, upload = nullptr;
    DevScen *ds_host = nullptr;  // pinned: the resident scenarios' scalars after a segment
    SegmentLauncher seg;
    std::thread th, up;  // segment thread, upload thread
    std::mutex mu;
    std::condition_variable cv;     // segment thread: requests ready, cancel, stop
    std::condition_variable cv_up;  // upload thread: submit, memory released, cancel, stop
    bool stop = false;
    uint64_t next_ticket = 1;
    std::deque<Request *> queue;
    std::vector<Request *> ready;   // uploaded, joining at the next segment
    std::vector<Request *> active;  // resident in the segment thread
    int uploading = 0;              // admitted, upload in progress
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    int64_t submitted = 0, completed = 0, failed = 0, cancelled = 0, segments = 0;
    int fatal = SWE_OK;

    void loop();
    void uploader();
    Request *admit_one_locked();
    void release_locked(Request *r);
    void finish(Request *r, int status, int error);
};

void swe_server::finish(Request *r, int status, int error)
{
    r->status = status;
    r->error = error;
    r->t_done = now_seconds();
    if (status == SWE_DONE) ++completed;
    else if (status == SWE_CANCELLED) ++cancelled;
    else ++failed;
}

// Admits the queue's head if a slot is free and its footprint fits a hole of
// the arena (first in, first out: a head that does not fit waits for memory);
// cancelled heads end here.  Caller holds `mu`.
Request *swe_server::admit_one_locked()
{
    while (!queue.empty() && (int)(active.size() + ready.size()) + uploading < max_slots) {
        Request *r = queue.front();
        if (r->cancel) {
            queue.pop_front();
            r->f = HostFields();
            finish(r, SWE_CANCELLED, SWE_OK);
            continue;
        }
        void *mem = arena.alloc(request_bytes(r->p, r->track_max, compensated));
        if (!mem) return nullptr;
        queue.pop_front();
        r->d.base = mem;
        r->t_admit = now_seconds();
        ++uploading;
        return r;
    }
    return nullptr;
}

// Returns a request's device memory to the arena; caller holds `mu`.
void swe_server::release_locked(Request *r)
{
    arena.release(r->d.base, request_bytes(r->p, r->track_max, compensated));
    r->d.base = nullptr;
    cv_up.notify_one();
}

void swe_server::uploader()
{
    (void)hipSetDevice(device);
    for (;;) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (stop) return;
                if ((r = admit_one_locked())) break;
                cv_up.wait(lk);
            }
        }
        int urc = scenario_upload_into(r->d.base, r->p, r->f, upload, r->d);
        if (!urc && r->track_max) {
            // the map's plane follows the scenario; it starts at the depth
            r->d.geo.hmax =
                reinterpret_cast<float *>(static_cast<char *>(r->d.base) + scenario_bytes(r->p.nx, r->p.ny));
            urc = launch_depth(r->d.geo, r->d.geo.U[0], r->d.geo.hmax, upload);
        }
        if (!urc && compensated) {
            // the residual planes come last
            char *rp = static_cast<char *>(r->d.base) + scenario_bytes(r->p.nx, r->p.ny) +
                       (r->track_max ? map_bytes(r->p) : 0);
            urc = attach_residuals(r->d.geo, reinterpret_cast<float *>(rp), upload);
        }
        // the segment thread uses the planes only after this wait
        if (!urc && hipStreamSynchronize(upload) != hipSuccess) urc = SWE_EDEVICE;
        std::lock_guard<std::mutex> lk(mu);
        --uploading;
        r->f = HostFields();
        if (urc) {
            release_locked(r);
            finish(r, SWE_FAILED, urc);
        } else {
            ready.push_back(r);
            cv.notify_one();
        }
    }
}

void swe_server::loop()
{
    (void)hipSetDevice(device);
    std::vector<Request *> retiring;  // finished in the previous segment, results not yet copied
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            if (stop) break;
            active.insert(active.end(), ready.begin(), ready.end());
            ready.clear();
            if (active.empty() && retiring.empty()) {
                cv.wait_for(lk, std::chrono::milliseconds(20));
                continue;
            }
        }
        // one segment over every resident scenario with steps left
        std::vector<Geo> geos;
        std::vector<int> ks;
        std::vector<Request *> in_seg;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (Request *r : active) {
                if (r->cancel || r->done_steps >= r->nsteps) continue;
                geos.push_back(r->d.geo);
                ks.push_back(std::min(segment_steps, r->nsteps - r->done_steps));
                in_seg.push_back(r);
            }
        }
        int rc = SWE_OK;
        if (!in_seg.empty()) {
            std::vector<std::pair<int, int>> sizes;
            for (const Geo &g : geos) sizes.emplace_back(g.nx, g.ny);
            int launch_mode;
            bool launch_implicit, launch_local;
            {
                std::lock_guard<std::mutex> lk(mu);
                launch_mode = mode;
                launch_implicit = implicit;
                launch_local = local_split;
            }
            rc = seg.run(geos, ks, batch_variant_for(sizes), launch_mode, false, compute, launch_implicit,
                         compensated, launch_local);
            std::lock_guard<std::mutex> lk(mu);
            ++segments;
            if (rc) fatal = rc;
        }
        // while the segment runs: copy out the results of the previous
        // segment's finishers
        for (Request *r : retiring) {
            int rrc = SWE_OK;
            if (!r->cancel) {
                const size_t N = (size_t)r->p.nx * r->p.ny;
                r->h.resize(N);
                r->hu.resize(N);
                r->hv.resize(N);
                if (r->track_max) {
                    // ordered before the read's own synchronisation
                    r->hmax.resize(N);
                    const size_t row = (size_t)r->p.nx * sizeof(float);
                    const size_t spitch = (size_t)r->d.geo.pitch * sizeof(float);
                    if (hipMemcpy2DAsync(r->hmax.data(), row, r->d.geo.hmax, spitch, row, r->p.ny,
                                         hipMemcpyDeviceToHost, copy) != hipSuccess)
                        rrc = SWE_EDEVICE;
                }
                const int src = scenario_read(r->d, copy, r->h.data(), r->hu.data(), r->hv.data(), &r->st);
                if (!rrc) rrc = src;
            }
            std::lock_guard<std::mutex> lk(mu);
            release_locked(r);
            if (r->cancel) finish(r, SWE_CANCELLED, SWE_OK);
            else if (rrc == SWE_OK) finish(r, SWE_DONE, SWE_OK);
            else finish(r, SWE_FAILED, rrc);
        }
        retiring.clear();
        if (hipStreamSynchronize(compute) != hipSuccess) rc = SWE_EDEVICE;
        // account the segment, detect failures, pick the finishers
        DevScen *ds = ds_host;
        for (size_t i = 0; i < in_seg.size(); ++i)
            (void)hipMemcpyAsync(&ds[i], in_seg[i]->d.geo.sd, sizeof(DevScen), hipMemcpyDeviceToHost, copy);
        (void)hipStreamSynchronize(copy);
        std::lock_guard<std::mutex> lk(mu);
        for (size_t i = 0; i < in_seg.size(); ++i) {
            in_seg[i]->done_steps += ks[i];
            if (rc) in_seg[i]->error = rc;
        }
        std::vector<Request *> keep;
        for (Request *r : active) {
            bool out = r->cancel || r->done_steps >= r->nsteps || rc != SWE_OK;
            for (size_t i = 0; i < in_seg.size(); ++i)
                if (in_seg[i] == r && ((ds[i].flags & 1u) || ds[i].alpha[0][0] >= 0x7f800000u)) {
                    r->error = SWE_ENONFINITE;
                    out = true;
                }
            if (out) {
                if (r->error != SWE_OK && !r->cancel) {
                    release_locked(r);
                    finish(r, SWE_FAILED, r->error);
                } else {
                    retiring.push_back(r);
                }
            } else {
                keep.push_back(r);
            }
        }
        active.swap(keep);
    }
    // shutdown: drop whatever is resident
    (void)hipStreamSynchronize(compute);
    (void)hipStreamSynchronize(copy);
}

extern "C" {

int swe_server_create(int32_t device, size_t mem_budget, int32_t max_slots, int32_t segment_steps,
                      swe_server **out)
{
    if (!out || max_slots <= 0 || segment_steps <= 0) return SWE_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SWE_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return SWE_EDEVICE;
    if (mem_budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return SWE_EDEVICE;
        mem_budget = fr / 2;
    }
    swe_server *sv = new (std::nothrow) swe_server();
    if (!sv) return SWE_ENOMEM;
    sv->device = device;
    sv->max_slots = max_slots;
    sv->segment_steps = segment_steps;
    int rc = sv->arena.init(mem_budget);
    if (rc) {
        delete sv;
        return rc;
    }
    if (hipStreamCreateWithFlags(&sv->compute, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&sv->copy, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&sv->upload, hipStreamNonBlocking) != hipSuccess) {
        if (sv->compute) (void)hipStreamDestroy(sv->compute);
        if (sv->copy) (void)hipStreamDestroy(sv->copy);
        delete sv;
        return SWE_EDEVICE;
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&sv->ds_host), (size_t)max_slots * sizeof(DevScen),
                      hipHostMallocDefault) != hipSuccess) {
        (void)hipStreamDestroy(sv->compute);
        (void)hipStreamDestroy(sv->copy);
        (void)hipStreamDestroy(sv->upload);
        delete sv;
        return SWE_ENOMEM;
    }
    sv->th = std::thread([sv] { sv->loop(); });
    sv->up = std::thread([sv] { sv->uploader(); });
    *out = sv;
    return SWE_OK;
}

int swe_submit_ex(swe_server *sv, const swe_params *p, const float *b, const float *n, const float *h0,
                  const float *hu0, const float *hv0, int32_t nsteps, int32_t flags, uint64_t *ticket)
{
    if (!sv || !ticket || nsteps < 0 || (flags & ~SWE_SUBMIT_MAX_DEPTH)) return SWE_EINVAL;
    auto r = std::make_unique<Request>();
    int rc = load_fields(p, b, n, h0, hu0, hv0, r->f);
    if (rc) return rc;
    r->track_max = (flags & SWE_SUBMIT_MAX_DEPTH) != 0;
    if (request_bytes(*p, r->track_max, sv->compensated) > sv->arena.capacity()) return SWE_ENOMEM;
    r->p = *p;
    r->nsteps = nsteps;
    r->t_submit = now_seconds();
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->queue.size() >= sv->max_queue) return SWE_EBUSY;
    r->ticket = sv->next_ticket++;
    *ticket = r->ticket;
    sv->queue.push_back(r.get());
    sv->reqs[r->ticket] = std::move(r);
    ++sv->submitted;
    sv->cv_up.notify_one();
    return SWE_OK;
}

int swe_submit(swe_server *sv, const swe_params *p, const float *b, const float *n, const float *h0,
               const float *hu0, const float *hv0, int32_t nsteps, uint64_t *ticket)
{
    return swe_submit_ex(sv, p, b, n, h0, hu0, hv0, nsteps, 0, ticket);
}

int swe_poll_ex(swe_server *sv, uint64_t ticket, swe_result *res, float *h, float *hu, float *hv, float *hmax)
{
    if (!sv || !res) return SWE_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return SWE_ENOTFOUND;
    Request *r = it->second.get();
    if (hmax && !r->track_max) return SWE_EINVAL;  // no map kept: the ticket stays
    std::memset(res, 0, sizeof *res);
    res->status = r->status;
    res->error = r->error;
    res->t_submit = r->t_submit;
    res->t_admit = r->t_admit;
    res->t_done = r->t_done;
    if (r->status == SWE_PENDING) return SWE_OK;
    if (r->status == SWE_DONE) {
        res->t = r->st.t;
        res->mass = r->st.mass;
        res->runup = r->st.runup;
        res->steps = r->st.step;
        const size_t N = r->h.size();
        if (h) std::memcpy(h, r->h.data(), N * sizeof(float));
        if (hu) std::memcpy(hu, r->hu.data(), N * sizeof(float));
        if (hv) std::memcpy(hv, r->hv.data(), N * sizeof(float));
        if (hmax) std::memcpy(hmax, r->hmax.data(), N * sizeof(float));
    }
    sv->reqs.erase(it);  // a final status is reported once
    return SWE_OK;
}

int swe_poll(swe_server *sv, uint64_t ticket, swe_result *res, float *h, float *hu, float *hv)
{
    return swe_poll_ex(sv, ticket, res, h, hu, hv, nullptr);
}

int swe_server_set_mode(swe_server *sv, int32_t mode)
{
    if (!sv || (mode != SWE_BATCH_PERSISTENT && mode != SWE_BATCH_ROUNDS)) return SWE_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->mode = mode;
    return SWE_OK;
}

int swe_server_set_option(swe_server *sv, int32_t key, int64_t value)
{
    if (!sv || (key != SWE_OPT_FRICTION_IMPLICIT && key != SWE_OPT_COMPENSATED && key != SWE_OPT_LOCAL_SPLIT) ||
        (value != 0 && value != 1))
        return SWE_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->submitted > 0) return SWE_EBUSY;  // one treatment for every request
    if (key == SWE_OPT_FRICTION_IMPLICIT) sv->implicit = value != 0;
    else if (key == SWE_OPT_LOCAL_SPLIT) sv->local_split = value != 0;
    else sv->compensated = value != 0;
    return SWE_OK;
}

int swe_cancel(swe_server *sv, uint64_t ticket)
{
    if (!sv) return SWE_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return SWE_ENOTFOUND;
    it->second->cancel = true;
    sv->cv.notify_one();
    sv->cv_up.notify_one();
    return SWE_OK;
}

int swe_server_get_stats(swe_server *sv, swe_server_stats *st)
{
    if (!sv || !st) return SWE_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    st->submitted = sv->submitted;
    st->completed = sv->completed;
    st->failed = sv->failed;
    st->cancelled = sv->cancelled;
    st->queued = (int64_t)sv->queue.size();
    st->active = (int64_t)(sv->active.size() + sv->ready.size()) + sv->uploading;
    st->mem_in_use = sv->arena.used();
    st->mem_high_water = sv->arena.high_water();
    st->mem_budget = sv->arena.capacity();
    st->segments = sv->segments;
    return sv->fatal;
}

void swe_server_destroy(swe_server *sv)
{
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv.notify_all();
    sv->cv_up.notify_all();
    if (sv->up.joinable()) sv->up.join();
    if (sv->th.joinable()) sv->th.join();
    (void)hipStreamDestroy(sv->compute);
    (void)hipStreamDestroy(sv->copy);
    (void)hipStreamDestroy(sv->upload);
    (void)hipHostFree(sv->ds_host);
    delete sv;
}

}  // extern "C"
