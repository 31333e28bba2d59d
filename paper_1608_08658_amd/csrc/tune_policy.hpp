// Choice of the stencil launch shape from the autotuner's timings
// (engine.cpp, Plan::tune), free of HIP so that it can be checked on the CPU.
//
// Timings of near-equal shapes differ by the measurement's noise, so picking
// the plain minimum lets the choice flip from plan to plan.  Candidates within
// `tie` (relative) of the fastest count as equal; of those the longest
// z-chunk is kept (fewest warm-up planes re-read per plane computed), then
// the faster.
#pragma once

#include <cstddef>

namespace awe {

// t[i]: time of candidate i (any unit; 1e30 or more = not timed).
// Returns the index to keep, or -1 when no candidate was timed.
template <class ZchunkOf>
int pick_timed_shape(size_t n, const float* t, ZchunkOf zchunk_of, float tie = 0.01f) {
    float fastest = 1e30f;
    for (size_t i = 0; i < n; ++i)
        if (t[i] < fastest) fastest = t[i];
    if (!(fastest < 1e29f)) return -1;
    int best = -1;
    for (size_t i = 0; i < n; ++i) {
        if (!(t[i] <= (1.0f + tie) * fastest)) continue;
        if (best < 0 || zchunk_of(i) > zchunk_of((size_t)best) ||
            (zchunk_of(i) == zchunk_of((size_t)best) && t[i] < t[best]))
            best = (int)i;
    }
    return best;
}

// Where a plan's launch shape comes from.  exact: the cache holds an entry
// for this very size (exact_timed: timed, not borrowed); nearby: it holds a
// timed entry for a size within the borrowing window; may_time: the plan may
// time candidates now (no other work on the device); own: the plan runs long
// enough to repay timing its own size (plans made directly and gradient
// requests; a server's forward requests borrow instead, since a server meets
// many sizes and timing each costs ~100 launches of it).
enum class ShapeSource { kCached, kBorrowed, kTimed, kBuiltin };
inline ShapeSource shape_source(bool exact, bool exact_timed, bool nearby, bool may_time, bool own) {
    const bool time_own = may_time && own;
    if (exact && (exact_timed || !time_own)) return ShapeSource::kCached;
    if (nearby && !time_own) return ShapeSource::kBorrowed;
    return may_time ? ShapeSource::kTimed : ShapeSource::kBuiltin;
}

// The z-chunk of the same chunk count as `zc` over nz planes with the chunks
// as equal as possible: ceil(nz / ceil(nz / zc)).  A grid of 150 planes cut
// into 28-plane chunks ends with a 10-plane chunk that pays the same warm-up
// as a full one; 25-plane chunks cut it evenly into the same six.
inline int balanced_zchunk(long long nz, int zc) {
    if (nz < 1 || zc < 1) return zc < 1 ? 1 : zc;
    const long long chunks = (nz + zc - 1) / zc;
    return (int)((nz + chunks - 1) / chunks);
}

}  // namespace awe
