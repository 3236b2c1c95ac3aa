// p2p_common.h -- staging of near-field sources into LDS, shared by the
// forward and the adjoint near-field kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels_common.h"

namespace fmm {

// Entries of a strong list per near-field work chunk, for an item whose leaf
// holds n points.  Every entry of a leaf's strong list is a leaf of the same
// problem and level, whose point counts differ from n by at most one, so a
// chunk holds at most kChunkSrc sources; chunk k of a split item starts at
// entry k * chunk_entries(n), which needs no search of the list.
__host__ __device__ inline int chunk_entries(int n) { return kChunkSrc / (n + 1) > 1 ? kChunkSrc / (n + 1) : 1; }

// Gather sources of the strong list into LDS, resuming at (entry e, offset
// off) and stopping after CAP sources (an entry may be split between
// passes).  Entries are looked at 64 at a time (lane k: entry e + k, its
// first source and the exclusive prefix of the source counts).  The
// non-empty entries that start inside the staged run are compacted in entry
// order (meta) and flag their first staging position (mark); the entry of
// position f = lane + 64 r is then the number of flags at or before f, less
// one, counted with one ballot per row.  Returns the number of sources
// staged (at most `limit`).
template <int CAP, class SRC, class LOADER>
__device__ __forceinline__ int stage_sources(SRC* lds, int2* meta, int* mark, const int32_t* __restrict__ s_ids,
                                             const int32_t* __restrict__ bstart,
                                             const int32_t* __restrict__ bcount, int e0, int e_end, int& e,
                                             int& off, int lane, LOADER load, int limit = CAP)
{
    constexpr int R = CAP / 64;
    const int lim = limit < CAP ? limit : CAP;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));   // lanes before this one
    int staged = 0;
    while (e < e_end && staged < lim) {
        const int k = e + lane;
        int st = 0, avail = 0;
        if (k < e_end) {
            const int S = s_ids[e0 + k];
            st = bstart[S];
            avail = bcount[S];
            if (lane == 0) { st += off; avail -= off; }
        }
        const int x = wave_incl_scan(avail);
        const int excl = x - avail;
        const int total = __builtin_amdgcn_readlane(x, 63);
        const int cap = lim - staged;
        const int take = min(total, cap);
        const bool starts = avail > 0 && excl < take;
        const unsigned long long sm = __ballot(starts);
        if (starts) meta[__popcll(sm & below)] = make_int2(excl, st);
#pragma unroll
        for (int r = 0; r < R; ++r) mark[lane + 64 * r] = 0;
        wave_sync();
        if (starts) mark[excl] = 1;
        wave_sync();
        int src_idx[R];
        int seen = 0;   // flags in earlier rows
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int f = lane + 64 * r;
            const unsigned long long fl = __ballot(mark[f] != 0);
            const int rk = seen + __popcll(fl & below) + (int)((fl >> lane) & 1ull) - 1;
            seen += __popcll(fl);
            const int2 mj = meta[rk < 0 ? 0 : rk];
            src_idx[r] = (f < take) ? mj.y + (f - mj.x) : -1;
        }
        SRC v[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (src_idx[r] >= 0) v[r] = load(src_idx[r]);
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (src_idx[r] >= 0) lds[staged + lane + 64 * r] = v[r];
        // advance the cursor (uniform): the entry of the last staged position
        // is the last non-empty entry starting at or before it
        if (take == total) {
            e = min(e + 64, e_end);
            off = 0;
        } else {
            const unsigned long long lm = __ballot(starts && excl <= take - 1);
            const int L = 63 - __clzll((long long)lm);
            const int consumed = take - __shfl(excl, L, 64);
            if (consumed == __shfl(avail, L, 64)) { e = e + L + 1; off = 0; }
            else { off = (L == 0 ? off : 0) + consumed; e = e + L; }
        }
        staged += take;
        wave_sync();
    }
    return staged;
}

}  // namespace fmm
