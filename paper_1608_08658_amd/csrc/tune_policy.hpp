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

}  // namespace awe
