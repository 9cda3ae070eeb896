// swe_batch_kernels.hpp - the batched stage kernels (persistent and per-round
// launches) and their tables; the schedule is described in swe_batch.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "swe_internal.hpp"

namespace swe {

__device__ __forceinline__ int xcd_remap_b(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, l = b >> 3;
    return x * q + (x < r ? x : r) + l;
}

// Largest i in [0, n) with a[i] <= v (a ascending, a[0] <= v).
template <class T>
__device__ __forceinline__ int upper_index(const T *a, int n, T v)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Table entries read as kernel arguments are: through the constant address
// space (the tables do not change during a launch), so a block's (uniform)
// entry is read with scalar loads into scalar registers.  The Geo stays a
// reference into the table (a local copy would be spilled to scratch: the
// ghost code indexes its arrays per lane).
template <class T>
__device__ __forceinline__ const T &table_entry(const T *base, int i)
{
    return *(const T *)reinterpret_cast<const __attribute__((address_space(4))) T *>(
        reinterpret_cast<uintptr_t>(base + i));
}

struct BatchTables {
    const Geo *geo;            // per scenario (batch order)
    const int2 *blk;           // per tile of round 0: (scenario index, tile of that scenario)
    const int *order;          // sorted position -> scenario
    const int *prefix;         // tile prefix over sorted positions (size nact + 1)
    const int *ntx;            // tiles along x per sorted position
    const long long *rstart;   // first ticket of each round (size nrounds + 1)
    const int *ractive;        // active prefix length per round
    unsigned int *done;        // completed tiles per sorted position (this run)
    unsigned long long *ticket;
    int nrounds, nact, group;
};

template <class C, int W, bool IMP, bool CMP, bool LLF = false>
__global__ __launch_bounds__(C::NT, W) void k_persistent(BatchTables T)
{
    __shared__ float lds[C::LDS_FLOATS];
    __shared__ long long s_ticket;
    const long long total = T.rstart[T.nrounds];
    for (;;) {
        if (threadIdx.x == 0) s_ticket = (long long)atomicAdd(T.ticket, (unsigned long long)T.group);
        __syncthreads();
        const long long t0 = s_ticket;
        __syncthreads();
        if (t0 >= total) break;
        const long long t1 = t0 + T.group < total ? t0 + T.group : total;
        int r = upper_index(T.rstart, T.nrounds, t0);
        long long t = t0;
        // The grabbed tickets are handled in runs that stay inside one round.
        // Tiles of one round never depend on each other, so a run waits once
        // (one acquire) for the previous round of every scenario it touches,
        // runs its tiles, and publishes them with one release.
        while (t < t1) {
            const long long te = t1 < T.rstart[r + 1] ? t1 : T.rstart[r + 1];
            const int l0 = (int)(t - T.rstart[r]), l1 = (int)(te - T.rstart[r]);
            const int s0 = upper_index(T.prefix, T.ractive[r], l0);
            const int s1 = upper_index(T.prefix, T.ractive[r], l1 - 1);
            if (threadIdx.x == 0) {
                for (int sl = s0; sl <= s1; ++sl) {
                    const unsigned int need = (unsigned int)(T.prefix[sl + 1] - T.prefix[sl]) * (unsigned int)r;
                    while (__hip_atomic_load(&T.done[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need)
                        __builtin_amdgcn_s_sleep(1);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            __syncthreads();
            int slot = s0;
            for (int l = l0; l < l1; ++l) {
                while (l >= T.prefix[slot + 1]) ++slot;
                const int tl = l - T.prefix[slot];
                const int ntx = T.ntx[slot];
                const int sc = __builtin_amdgcn_readfirstlane(T.order[slot]);
                // no early per-cell reads with the compensated level: with the
                // ticket loop's registers they would spill on some tiles
                stage_tile<C, (W <= 2) && !CMP, CMP, IMP, LLF>(table_entry(T.geo, sc), tl % ntx, tl / ntx, lds,
                                                               r % 3 + 1);
                __syncthreads();
            }
            // every wave makes its own stores visible at agent scope before
            // the barrier; then one thread publishes the run
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (threadIdx.x == 0) {
                for (int sl = s0; sl <= s1; ++sl) {
                    const int a = l0 > T.prefix[sl] ? l0 : T.prefix[sl];
                    const int b = l1 < T.prefix[sl + 1] ? l1 : T.prefix[sl + 1];
                    __hip_atomic_fetch_add(&T.done[sl], (unsigned int)(b - a), __ATOMIC_RELEASE,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            t = te;
            ++r;
        }
    }
}

template <class C, int S, int W, bool IMP, bool CMP, bool LLF = false>
__global__ __launch_bounds__(C::NT, W) void k_round(BatchTables T, int nact_round, int nblocks)
{
    __shared__ float lds[C::LDS_FLOATS];
    // the round's tiles are the first nblocks of round 0's (its scenarios are
    // a prefix of the sorted order): one table load names the block's
    // scenario and tile, with no search over the prefix sums
    (void)nact_round;
    const int id = xcd_remap_b(blockIdx.x, nblocks);
    const int2 e = table_entry(T.blk, id);
    const int sc = __builtin_amdgcn_readfirstlane(e.x), tile = __builtin_amdgcn_readfirstlane(e.y);
    const Geo &G = table_entry(T.geo, sc);
    const int ntx = (G.nx + C::TX - 1) / C::TX;
    stage_tile<C, (W <= 2), CMP, IMP, LLF>(G, tile % ntx, tile / ntx, lds, S);
}

struct BatchKernels {
    void (*persistent)(BatchTables);
    void (*round[3])(BatchTables, int, int);
};

// Kernels of one tile variant; IMP: point-implicit friction, CMP: the
// compensated level (every scenario of the run carries residual planes),
// LLF: local Lax-Friedrichs splitting.
#define SWE_BK_L(TX, TY, R, W, IMP, CMP, LLF)                                                              \
    {k_persistent<TileCfg<TX, TY, R>, W, IMP, CMP, LLF>,                                                   \
     {k_round<TileCfg<TX, TY, R>, 1, W, IMP, CMP, LLF>, k_round<TileCfg<TX, TY, R>, 2, W, IMP, CMP, LLF>, \
      k_round<TileCfg<TX, TY, R>, 3, W, IMP, CMP, LLF>}},
#define SWE_BK_M(TX, TY, R, W, IMP, CMP) SWE_BK_L(TX, TY, R, W, IMP, CMP, false)
#define SWE_BK(TX, TY, R, W, IMP) SWE_BK_M(TX, TY, R, W, IMP, false)
// In SWE_TILE_LIST order, the same as the single-scenario variant table;
// one set per translation unit (compiled in parallel): explicit friction in
// swe_batch.hip, implicit in swe_batch_imp.hip, the compensated level with
// either in swe_batch_cmp.hip and swe_batch_cmp_imp.hip, and the same four
// with local Lax-Friedrichs splitting in swe_batch_llf*.hip.
extern const BatchKernels g_bk[], g_bk_imp[], g_bk_cmp[], g_bk_cmp_imp[];
extern const BatchKernels g_bk_llf[], g_bk_llf_imp[], g_bk_llf_cmp[], g_bk_llf_cmp_imp[];

}  // namespace swe
