// swe_schedule.hpp - host-side round/ticket tables of a batched run.
//
// Scenario i advances ksteps[i] >= 0 steps.  Participants are ordered by
// their step count (descending, stable), so the scenarios taking part in
// round r (round = one stage of one step) are a prefix of that order, of
// length ractive[r].  Tiles of a round are numbered scenario after scenario
// (prefix[q] = first tile of sorted position q); rounds are numbered one
// after the other (rstart[r] = first ticket of round r).  Plain C++, shared
// by the launcher and by the host-thread model of the ticket protocol.
#pragma once

#include <algorithm>
#include <vector>

namespace swe {

struct Schedule {
    std::vector<int> order;        // sorted position -> scenario index
    std::vector<int> prefix;       // size nact + 1
    std::vector<int> ntx;          // tiles along x per sorted position
    std::vector<int> ractive;      // size nrounds
    std::vector<long long> rstart; // size nrounds + 1
    int nact = 0, nrounds = 0;
};

inline Schedule build_schedule(const std::vector<int> &nx, const std::vector<int> &ny,
                               const std::vector<int> &ksteps, int tile_x, int tile_y)
{
    Schedule S;
    std::vector<int> act;
    for (int i = 0; i < (int)ksteps.size(); ++i)
        if (ksteps[i] > 0) act.push_back(i);
    if (act.empty()) return S;
    std::stable_sort(act.begin(), act.end(), [&](int a, int b) { return ksteps[a] > ksteps[b]; });
    S.nact = (int)act.size();
    S.nrounds = 3 * ksteps[act[0]];
    S.order = act;
    S.prefix.assign(S.nact + 1, 0);
    S.ntx.assign(S.nact, 0);
    for (int q = 0; q < S.nact; ++q) {
        const int tx = (nx[act[q]] + tile_x - 1) / tile_x, ty = (ny[act[q]] + tile_y - 1) / tile_y;
        S.ntx[q] = tx;
        S.prefix[q + 1] = S.prefix[q] + tx * ty;
    }
    S.ractive.assign(S.nrounds, 0);
    S.rstart.assign(S.nrounds + 1, 0);
    int a = S.nact;
    for (int r = 0; r < S.nrounds; ++r) {
        while (a > 0 && 3 * ksteps[act[a - 1]] <= r) --a;
        S.ractive[r] = a;
        S.rstart[r + 1] = S.rstart[r] + S.prefix[a];
    }
    return S;
}

// Ticket-group size: about one run of tickets per block and round.
inline int ticket_group(const Schedule &S, long long grid)
{
    if (S.nact == 0 || grid <= 0) return 4;
    const long long g = S.prefix[S.nact] / grid;
    return (int)(g < 4 ? 4 : (g > 64 ? 64 : g));
}

}  // namespace swe
