// Binomial checkpointing for the gradient's reverse sweep.
//
// The adjoint sweep (Eq. 4) visits the forward states x_t = (u[t], u[t-1])
// in reverse order, t = nt-1 .. 0, and the imaging condition (Eq. 3) needs
// u[t] at visit t.  Keeping every state is what the paper's memory-mapped
// full history does (Sec. IV.B, memory-mapping paragraph, which names other forms of checkpointing as
// the alternative under study).  Periodic checkpoints (every K steps) cut
// memory to ~nt/K + K fields at one extra forward sweep.  The binomial
// schedule of Griewank (1992, "Achieving logarithmic growth of temporal and
// spatial complexity in reverse automatic differentiation") and Griewank &
// Walther (2000, ACM TOMS 26, "revolve") needs only `s` stored states and
// the fewest forward steps any schedule with s stored states can take:
//
//   reversing l states that start at a stored x_a with s free snapshots:
//     l == 1 : x_a is restored and visited;
//     s == 0 : for j = l-1 .. 0, restore x_a, advance j steps, visit;
//     else   : advance m steps from x_a, store x_(a+m) in a free snapshot,
//              reverse the l-m states from x_(a+m) with s-1 free snapshots,
//              release that snapshot and reverse the m states from x_a
//              with s free snapshots.
//
// With beta(s, r) = C(s + r, s), the fewest forward steps are
//   T(l, s) = r l - beta(s + 2, r - 1),  r the least with beta(s + 1, r) >= l,
// and T is convex in l, so the best first step m (the one minimising
// m + T(l - m, s - 1) + T(m, s)) is found by bisection on its slope.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "engine.hpp"

namespace awe {
namespace {

constexpr int64_t kSat = int64_t(1) << 62;

// C(s + r, s), saturating at 2^62.
int64_t beta(int64_t s, int64_t r) {
    int64_t b = 1;
    for (int64_t i = 1; i <= r; ++i) {
        if (b > kSat / (s + i)) return kSat;
        b = b * (s + i) / i;   // exact: b (s + i) = C(s + i, i) i
    }
    return b;
}

}  // namespace

int64_t binomial_steps(int64_t l, int s) {
    if (l <= 1) return 0;
    if (s <= 0) return l * (l - 1) / 2;
    const int64_t S = s + 1;   // snapshots counting the one that holds x_a
    int64_t r = 0;
    while (beta(S, r) < l) ++r;
    return r * l - (r >= 1 ? beta(S + 1, r - 1) : 0);
}

namespace {

// The best first advance m in [1, l-1] for l >= 2 states and s >= 1 free
// snapshots: the least m at which m + T(l-m, s-1) + T(m, s) stops falling.
int64_t best_split(int64_t l, int s) {
    auto f = [&](int64_t m) { return m + binomial_steps(l - m, s - 1) + binomial_steps(m, s); };
    int64_t lo = 1, hi = l - 1;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (f(mid + 1) - f(mid) >= 0) hi = mid;
        else lo = mid + 1;
    }
    if (f(lo) != binomial_steps(l, s)) {   // convexity guarantees this; keep a scan as a guard
        int64_t best = 1;
        for (int64_t m = 2; m < l; ++m)
            if (f(m) < f(best)) best = m;
        lo = best;
    }
    return lo;
}

}  // namespace

std::vector<CkptAction> binomial_schedule(int nt, int snapshots) {
    struct Task {
        bool release;   // release snapshot `slot`, else reverse (a, l) from `slot` with s free
        int a, l, s, slot;
    };
    std::vector<CkptAction> out;
    std::vector<Task> stack{{false, 0, nt, snapshots, -1}};
    while (!stack.empty()) {
        const Task k = stack.back();
        stack.pop_back();
        if (k.release) {
            out.push_back({CkptAction::kFree, k.slot});
            continue;
        }
        if (k.l <= 0) continue;
        if (k.l == 1) {
            out.push_back({CkptAction::kRestore, k.slot});
            out.push_back({CkptAction::kYield, k.a});
            continue;
        }
        if (k.s == 0 || binomial_steps(k.l, k.s) == binomial_steps(k.l, k.s - 1)) {
            if (k.s > 0) {   // a snapshot gains nothing here: keep it free
                stack.push_back({false, k.a, k.l, k.s - 1, k.slot});
                continue;
            }
            for (int j = k.l - 1; j >= 0; --j) {
                out.push_back({CkptAction::kRestore, k.slot});
                if (j > 0) out.push_back({CkptAction::kAdvance, k.a + j});
                out.push_back({CkptAction::kYield, k.a + j});
            }
            continue;
        }
        const int m = (int)best_split(k.l, k.s);
        const int slot = k.s - 1;   // snapshots >= s are held by enclosing tasks
        out.push_back({CkptAction::kRestore, k.slot});
        out.push_back({CkptAction::kAdvance, k.a + m});
        out.push_back({CkptAction::kTake, slot});
        stack.push_back({false, k.a, m, k.s, k.slot});
        stack.push_back({true, 0, 0, 0, slot});
        stack.push_back({false, k.a + m, k.l - m, k.s - 1, slot});
    }
    return out;
}

// ---------------------------------------------------------------------------
// Reversal: runs a schedule over a pool of wavefield buffers with reference
// counts.  A stored state is a pair of buffer references, so storing and
// restoring copy nothing, and states one step apart share a buffer.  A step
// writes in place over u[t-1] when nothing but the current state holds it.
// ---------------------------------------------------------------------------
awe_status Reversal::init(int nt_, int snapshots) {
    sized = false;
    nt = nt_;
    sched = binomial_schedule(nt, snapshots);
    snaps.assign(std::max(snapshots, 0), Snap{});
    pool = 0;
    rewind();
    // size the pool and check the schedule by running it without work
    awe_status st = run_impl(false, true, [](int, int, int, int) { return AWE_OK; }, [](int, int) { return AWE_OK; });
    if (st) return st;
    if (visited != nt) return fail(AWE_EINVAL, "checkpoint schedule visits %d of %d states", visited, nt);
    sized = true;
    const int64_t dry_steps = steps;
    rewind();
    steps = dry_steps;   // reported until the next run
    return AWE_OK;
}

awe_status binomial_prepare(Reversal& r, int nt, int snapshots) {
    const int64_t steps = binomial_steps(nt, snapshots);
    if (steps > (int64_t(1) << 31))
        return fail(AWE_EINVAL, "binomial schedule for nt = %d with %d snapshots takes %lld forward steps", nt,
                    snapshots, (long long)steps);
    return r.init(nt, snapshots);
}

void Reversal::rewind() {
    pos = 0;
    ref.assign(pool, 0);
    ua = ub = -1;
    t = 0;
    steps = 0;
    visited = 0;
    for (Snap& s : snaps) s = Snap{};
}

int Reversal::take_buffer(bool grow) {
    if (ub >= 0 && ref[ub] == 1) return ub;   // only the current state holds u[t-1]
    for (int i = 0; i < pool; ++i)
        if (ref[i] == 0) return i;
    if (!grow) return -2;
    ref.push_back(0);
    return pool++;
}

}  // namespace awe
