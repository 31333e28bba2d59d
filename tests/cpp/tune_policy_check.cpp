// CPU checks of the autotuner's choice of launch shape (tune_policy.hpp):
// fixed cases (a clear winner, ties settled by the longer z-chunk and then
// the faster, the tie boundary, nothing timed) and seeded random timings
// checked against the properties that define the choice; balanced z-chunks;
// and where a plan's shape comes from (cached, borrowed, timed, built-in).  Prints "ok" or
// the failed check and exits non-zero on failure.
#include <cstdio>
#include <random>
#include <vector>

#include "tune_policy.hpp"

static int fails = 0;
#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            std::printf("FAILED: %s (line %d)\n", #c, __LINE__);   \
            ++fails;                                               \
        }                                                          \
    } while (0)

static int pick(const std::vector<float>& t, const std::vector<int>& zc) {
    return awe::pick_timed_shape(t.size(), t.data(), [&](size_t i) { return zc[i]; });
}

int main() {
    // a clear winner (other candidates more than 1% slower) whatever its chunk
    CHECK(pick({110.f, 100.f, 120.f}, {56, 8, 84}) == 1);
    // within 1%: the longer chunk
    CHECK(pick({100.f, 100.5f, 103.f}, {42, 56, 84}) == 1);
    // within 1% and equal chunks: the faster
    CHECK(pick({100.8f, 100.f, 100.4f}, {56, 56, 42}) == 1);
    // the boundary: exactly 1% slower is a tie, more is not
    CHECK(pick({100.f, 101.f}, {8, 56}) == 1);
    CHECK(pick({100.f, 101.2f}, {8, 56}) == 0);
    // nothing timed (or nothing at all)
    CHECK(pick({1e30f, 1e30f}, {8, 56}) == -1);
    CHECK(pick({}, {}) == -1);
    // untimed candidates never win
    CHECK(pick({1e30f, 100.f, 1e30f}, {84, 8, 84}) == 1);

    std::mt19937 rng(7);
    std::uniform_real_distribution<float> time(100.f, 104.f);
    const int chunks[] = {8, 14, 21, 28, 42, 56, 70, 84};
    for (int it = 0; it < 20000; ++it) {
        const int n = 1 + (int)(rng() % 40);
        std::vector<float> t(n);
        std::vector<int> zc(n);
        for (int i = 0; i < n; ++i) {
            t[i] = (rng() % 10 == 0) ? 1e30f : time(rng);
            zc[i] = chunks[rng() % 8];
        }
        const int k = pick(t, zc);
        float fastest = 1e30f;
        for (float v : t) fastest = v < fastest ? v : fastest;
        if (fastest >= 1e29f) {
            CHECK(k == -1);
            continue;
        }
        CHECK(k >= 0 && k < n);
        if (k < 0 || k >= n) continue;
        CHECK(t[k] <= 1.01f * fastest);               // a tie with the fastest
        for (int i = 0; i < n; ++i) {
            if (!(t[i] <= 1.01f * fastest)) continue;
            CHECK(zc[i] <= zc[k]);                    // no tied shape has a longer chunk
            if (zc[i] == zc[k]) CHECK(t[k] <= t[i]);  // and among equal chunks it is the fastest
        }
        if (fails) break;
    }
    // balanced z-chunks: the chunk count of zc, lengths differing by at most one
    CHECK(awe::balanced_zchunk(150, 28) == 25);
    CHECK(awe::balanced_zchunk(480, 56) == 54);
    CHECK(awe::balanced_zchunk(480, 84) == 80);
    CHECK(awe::balanced_zchunk(9, 8) == 5);
    CHECK(awe::balanced_zchunk(8, 8) == 8);
    CHECK(awe::balanced_zchunk(3, 8) == 3);
    for (long long nz = 1; nz <= 700; ++nz)
        for (int zc : chunks) {
            const int b = awe::balanced_zchunk(nz, zc);
            const long long n0 = (nz + zc - 1) / zc, n1 = (nz + b - 1) / b;
            CHECK(b >= 1 && b <= zc && n1 == n0);
            CHECK(nz - (n1 - 1) * b >= b - n1);        // the last chunk is short by less than the count
            if (fails) break;
        }
    // where a plan's shape comes from (shape_source): the whole truth table,
    // checked against the rule's statement rather than its code
    using awe::ShapeSource;
    for (int bits = 0; bits < 32; ++bits) {
        const bool exact = bits & 1, exact_timed = exact && (bits & 2), nearby = bits & 4, may_time = bits & 8,
                   own = bits & 16;
        const ShapeSource s = awe::shape_source(exact, exact_timed, nearby, may_time, own);
        // a timed entry for the size itself is always used
        if (exact_timed) CHECK(s == ShapeSource::kCached);
        // nothing is timed unless the plan may time
        if (!may_time) CHECK(s != ShapeSource::kTimed);
        // a plan that may time and repays it never runs a borrowed shape
        if (may_time && own) CHECK(s == ShapeSource::kCached ? exact_timed : s == ShapeSource::kTimed);
        // a plan that does not repay timing borrows before it times
        if (!own && !exact && nearby) CHECK(s == ShapeSource::kBorrowed);
        // and reuses what its size already has, borrowed or not
        if (!own && exact) CHECK(s == ShapeSource::kCached);
        // with nothing cached and nothing near: time if allowed, else the built-in shape
        if (!exact && !nearby) CHECK(s == (may_time ? ShapeSource::kTimed : ShapeSource::kBuiltin));
        if (!may_time && !exact && !nearby) CHECK(s == ShapeSource::kBuiltin);
    }
    // the served-gradient sequence: a serving mix left a borrowed entry for the
    // size; the first gradient request (idle) times its own, the later ones
    // (set up among running work) reuse that timed entry
    CHECK(awe::shape_source(true, false, true, true, true) == ShapeSource::kTimed);
    CHECK(awe::shape_source(true, true, true, false, true) == ShapeSource::kCached);
    // a forward request of a new nearby size, idle or not, borrows
    CHECK(awe::shape_source(false, false, true, true, false) == ShapeSource::kBorrowed);
    CHECK(awe::shape_source(false, false, true, false, false) == ShapeSource::kBorrowed);
    if (fails) return 1;
    std::printf("ok\n");
    return 0;
}
