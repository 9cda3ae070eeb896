// Host-thread model of the persistent batch kernel's ticket protocol.
//
// Each std::thread plays one block of the persistent kernel: it takes groups
// of tickets with one atomic add, splits a group into runs that stay inside
// one round, waits (relaxed spin, then an acquire fence) until every tile of
// the previous round of each scenario in the run has been published, "runs"
// its tiles, and publishes the run with one release add per scenario.  A
// tile's work is emulated with plain (non-atomic) memory: it reads every tile
// value of its scenario's previous round (a superset of the halo it needs)
// and writes its own.  Under ThreadSanitizer a missing happens-before edge is
// reported as a data race; without it, the value checks catch reordering.
// The kernel spins with relaxed loads and then issues one acquire fence;
// ThreadSanitizer does not model standalone fences, so the model spins with
// acquire loads, which the C++ memory model treats as the same
// synchronisation for the value that ends the wait.  Building with
// -DPLANT_MISSING_RELEASE publishes runs with relaxed adds instead, a
// protocol mistake the sanitizer must report.
// The schedule tables come from the launcher's own builder.  Threads may be
// descheduled at any time, which also exercises the claim that the protocol
// needs no co-residency.  Exit status 0 and "OK" on success.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "../../paper_2301_12010_amd/csrc/swe_schedule.hpp"

using swe::Schedule;

static int upper_index_ll(const std::vector<long long> &a, int n, long long v)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

static int upper_index_i(const std::vector<int> &a, int n, int v)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct Model {
    Schedule S;
    int group = 4;
    std::atomic<long long> ticket{0};
    std::vector<std::atomic<unsigned>> done;
    // plain "state": value[slot][round][tile] = round + 1 once written
    std::vector<std::vector<std::vector<int>>> value;
    std::atomic<int> errors{0};

    void tile_work(int slot, int r, int tl)
    {
        const int nt = S.prefix[slot + 1] - S.prefix[slot];
        if (r > 0) {
            long sum = 0;
            for (int k = 0; k < nt; ++k) {
                const int v = value[slot][r - 1][k];  // plain read of the previous round
                if (v != r) errors.fetch_add(1);
                sum += v;
            }
            if (sum != (long)nt * r) errors.fetch_add(1);
        }
        if (value[slot][r][tl] != 0) errors.fetch_add(1);  // each tile runs once
        value[slot][r][tl] = r + 1;                       // plain write of this tile
    }

    void block(unsigned seed)
    {
        std::mt19937 rng(seed);
        const long long total = S.rstart[S.nrounds];
        for (;;) {
            const long long t0 = ticket.fetch_add(group, std::memory_order_relaxed);
            if (t0 >= total) break;
            const long long t1 = std::min(t0 + group, total);
            int r = upper_index_ll(S.rstart, S.nrounds, t0);
            long long t = t0;
            while (t < t1) {
                const long long te = std::min(t1, S.rstart[r + 1]);
                const int l0 = (int)(t - S.rstart[r]), l1 = (int)(te - S.rstart[r]);
                const int s0 = upper_index_i(S.prefix, S.ractive[r], l0);
                const int s1 = upper_index_i(S.prefix, S.ractive[r], l1 - 1);
                for (int sl = s0; sl <= s1; ++sl) {
                    const unsigned need = (unsigned)(S.prefix[sl + 1] - S.prefix[sl]) * (unsigned)r;
                    while (done[sl].load(std::memory_order_acquire) < need) std::this_thread::yield();
                }
                int slot = s0;
                for (int l = l0; l < l1; ++l) {
                    while (l >= S.prefix[slot + 1]) ++slot;
                    tile_work(slot, r, l - S.prefix[slot]);
                    if ((rng() & 15) == 0) std::this_thread::yield();
                }
                for (int sl = s0; sl <= s1; ++sl) {
                    const int a = std::max(l0, S.prefix[sl]), b = std::min(l1, S.prefix[sl + 1]);
#ifdef PLANT_MISSING_RELEASE
                    done[sl].fetch_add((unsigned)(b - a), std::memory_order_relaxed);
#else
                    done[sl].fetch_add((unsigned)(b - a), std::memory_order_release);
#endif
                }
                t = te;
                ++r;
            }
        }
    }
};

static bool run_case(int nscen, int maxsteps, int threads, int group, unsigned seed)
{
    std::mt19937 rng(seed);
    std::vector<int> nx(nscen), ny(nscen), ks(nscen);
    for (int i = 0; i < nscen; ++i) {
        nx[i] = 3 + (int)(rng() % 300);
        ny[i] = 3 + (int)(rng() % 200);
        ks[i] = (int)(rng() % (maxsteps + 1));  // some scenarios take no steps
    }
    Model M;
    M.S = swe::build_schedule(nx, ny, ks, 64, 32);
    M.group = group > 0 ? group : swe::ticket_group(M.S, threads);
    if (M.S.nact == 0) return true;
    M.done = std::vector<std::atomic<unsigned>>(M.S.nact);
    M.value.resize(M.S.nact);
    for (int q = 0; q < M.S.nact; ++q) {
        const int nt = M.S.prefix[q + 1] - M.S.prefix[q];
        M.value[q].assign(M.S.nrounds, std::vector<int>(nt, 0));
    }
    std::atomic<bool> finished{false};
    std::thread watchdog([&] {
        for (int i = 0; i < 600 && !finished.load(); ++i) std::this_thread::sleep_for(std::chrono::milliseconds(100));
        if (!finished.load()) {
            std::fprintf(stderr, "deadlock: case nscen=%d threads=%d group=%d seed=%u\n", nscen, threads, group, seed);
            std::_Exit(3);
        }
    });
    std::vector<std::thread> ws;
    for (int b = 0; b < threads; ++b) ws.emplace_back([&, b] { M.block(seed * 977u + b); });
    for (auto &w : ws) w.join();
    finished.store(true);
    watchdog.join();
    // every participating tile of every round ran exactly once
    for (int q = 0; q < M.S.nact; ++q) {
        const int steps = ks[M.S.order[q]];
        for (int r = 0; r < M.S.nrounds; ++r)
            for (int v : M.value[q][r])
                if (v != (r < 3 * steps ? r + 1 : 0)) M.errors.fetch_add(1);
        if (M.done[q].load() != (unsigned)(3 * steps * (M.S.prefix[q + 1] - M.S.prefix[q]))) M.errors.fetch_add(1);
    }
    if (M.errors.load()) {
        std::fprintf(stderr, "ordering errors: %d (nscen=%d threads=%d group=%d seed=%u)\n", M.errors.load(), nscen,
                     threads, group, seed);
        return false;
    }
    return true;
}

int main(int argc, char **argv)
{
    const int reps = argc > 1 ? std::atoi(argv[1]) : 6;
    int cases = 0;
    for (int rep = 0; rep < reps; ++rep)
        for (int threads : {1, 3, 8, 24})
            for (int group : {1, 3, 8, 0}) {
                if (!run_case(1 + rep % 5, 6, threads, group, 1234u + 17u * rep + threads * 3u + group)) return 1;
                ++cases;
            }
    // many tiny scenarios: runs of one tile per round, groups spanning rounds
    for (int threads : {2, 16})
        if (!run_case(12, 9, threads, 5, 99u + threads)) return 1;
    std::printf("OK %d cases\n", cases + 2);
    return 0;
}
