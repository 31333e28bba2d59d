// CPU simulation of the shot server's admission policy (server_policy.hpp)
// with a fake executor: requests arrive at seeded Poisson times with seeded
// footprints and run times; running requests finish after their run time and
// leave their memory "retired" until the policy frees it.  Checked at every
// decision: the budget holds for running plus retired bytes, at most
// max_active run, admission is first-in first-out, memory is freed only when
// the server has no work (nothing runs, nothing waits) or when that lets the
// head in (and then the head is admitted), and every request completes; and
// the same with one request set up ahead (simulate_ahead).  Prints "ok" and
// the counts, or the failed check, and exits non-zero on failure.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <deque>
#include <random>
#include <vector>

#include "server_policy.hpp"

#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::printf("FAILED: %s (seed %d, line %d)\n", #c, seed, __LINE__); \
            return false;                                                    \
        }                                                                    \
    } while (0)

struct Req {
    double arrive, dur;
    uint64_t bytes;
    double admit = -1, done = -1;
};

static bool simulate(int seed, int max_active, uint64_t budget, int n, long& frees, long& admits) {
    std::mt19937_64 rng(seed);
    std::exponential_distribution<double> gap(1.0), run(0.25);
    std::uniform_int_distribution<uint64_t> size(1, budget);
    std::vector<Req> req(n);
    double t = 0;
    for (Req& r : req) {
        t += gap(rng);
        r.arrive = t;
        r.dur = run(rng);
        r.bytes = (seed % 3 == 0) ? size(rng) : size(rng) / 4 + 1;   // some mixes near the budget
    }
    std::deque<int> queue;
    std::vector<int> running;
    uint64_t reserved = 0, retired = 0;
    int next_arrival = 0, next_admit = 0;
    double now = 0;
    for (int guard = 0; guard < 100 * n + 100; ++guard) {
        while (next_arrival < n && req[next_arrival].arrive <= now) queue.push_back(next_arrival++);
        awe::AdmitState s;
        s.budget = budget;
        s.reserved = reserved;
        s.retired = retired;
        s.running = (int)running.size();
        s.max_active = max_active;
        auto bytes_of = [&](int i) { return req[queue[i]].bytes; };
        const awe::AdmitResult a = awe::admit_fifo(s, (int)queue.size(), bytes_of);
        CHECK(!(a.free_retired && a.count > 0));
        if (a.free_retired) {
            CHECK(retired > 0);
            const bool idle = running.empty() && queue.empty();
            const bool head_fits_after = !queue.empty() && (int)running.size() < max_active &&
                                         reserved + bytes_of(0) <= budget && reserved + retired + bytes_of(0) > budget;
            CHECK(idle || head_fits_after);
            retired = 0;
            ++frees;
            if (head_fits_after) {   // the next decision admits the head
                s.retired = 0;
                CHECK(awe::admit_fifo(s, (int)queue.size(), bytes_of).count >= 1);
            }
            continue;
        }
        for (int k = 0; k < a.count; ++k) {
            const int id = queue.front();
            queue.pop_front();
            CHECK(id == next_admit);   // first in, first out
            ++next_admit;
            req[id].admit = now;
            reserved += req[id].bytes;
            running.push_back(id);
            ++admits;
        }
        CHECK(reserved + retired <= budget);
        CHECK((int)running.size() <= max_active);
        // the head is held back only while it cannot run or fit even with
        // the retired memory freed (else the policy frees that memory)
        if (!queue.empty() && a.count == 0) {
            const uint64_t need = bytes_of(0);
            CHECK((int)running.size() >= max_active || reserved + need > budget);
        }
        // next event: an arrival or a completion
        double t_next = next_arrival < n ? req[next_arrival].arrive : 1e300;
        for (int id : running) t_next = std::min(t_next, req[id].admit + req[id].dur);
        if (t_next >= 1e300) break;
        now = t_next;
        for (size_t i = 0; i < running.size();) {
            const int id = running[i];
            if (req[id].admit + req[id].dur <= now) {
                req[id].done = now;
                reserved -= req[id].bytes;
                retired += req[id].bytes;   // freed later, by the policy
                running.erase(running.begin() + i);
            } else {
                ++i;
            }
        }
    }
    for (const Req& r : req) CHECK(r.done >= r.admit && r.admit >= r.arrive);
    return true;
}

// The engine's use of the policy with one request set up ahead (server.cpp):
// admission runs for max_active + 1 slots, the extra one set up (for
// `setup` time units) while max_active compute; nothing is admitted while a
// request is set up or waits for a slot; it starts computing as soon as a
// slot frees.  Checked: at most max_active compute, at most max_active + 1
// hold memory, the budget holds for them plus retired memory, requests
// start computing in arrival order, and every request completes.
static bool simulate_ahead(int seed, int max_active, uint64_t budget, int n, long& staged_count) {
    std::mt19937_64 rng(seed + 7919);
    std::exponential_distribution<double> gap(1.0), run(0.25), setup(4.0);
    std::uniform_int_distribution<uint64_t> size(1, budget);
    std::vector<Req> req(n);
    std::vector<double> start(n, -1), setup_dur(n);
    double t = 0;
    for (int i = 0; i < n; ++i) {
        t += gap(rng);
        req[i].arrive = t;
        req[i].dur = run(rng);
        setup_dur[i] = setup(rng);
        req[i].bytes = (seed % 3 == 0) ? size(rng) : size(rng) / 4 + 1;
    }
    std::deque<int> queue;
    std::vector<int> running;
    int staged = -1;
    double staged_ready = 0;
    uint64_t reserved = 0, retired = 0;
    int next_arrival = 0, next_start = 0;
    double now = 0;
    auto begin = [&](int id) {
        CHECK(id == next_start);   // computing starts in arrival order
        ++next_start;
        start[id] = now;
        running.push_back(id);
        return true;
    };
    for (int guard = 0; guard < 200 * n + 200; ++guard) {
        while (next_arrival < n && req[next_arrival].arrive <= now) queue.push_back(next_arrival++);
        // promotion of the request set up ahead
        if (staged >= 0 && staged_ready <= now && (int)running.size() < max_active) {
            if (!begin(staged)) return false;
            staged = -1;
        }
        awe::AdmitState s;
        s.budget = budget;
        s.reserved = reserved;
        s.retired = retired;
        s.running = (int)running.size() + (staged >= 0 ? 1 : 0);
        s.max_active = max_active + 1;
        auto bytes_of = [&](int i) { return req[queue[i]].bytes; };
        const awe::AdmitResult a = awe::admit_fifo(s, staged >= 0 ? 0 : (int)queue.size(), bytes_of);
        if (a.free_retired) {
            retired = 0;
            continue;
        }
        for (int k = 0; k < a.count; ++k) {
            const int id = queue.front();
            queue.pop_front();
            req[id].admit = now;
            reserved += req[id].bytes;
            if ((int)running.size() < max_active && staged < 0) {
                if (!begin(id)) return false;
            } else {
                CHECK(staged < 0);   // at most one set up ahead
                staged = id;
                staged_ready = now + setup_dur[id];
                ++staged_count;
            }
        }
        CHECK(reserved + retired <= budget);
        CHECK((int)running.size() <= max_active);
        CHECK((int)running.size() + (staged >= 0 ? 1 : 0) <= max_active + 1);
        double t_next = next_arrival < n ? req[next_arrival].arrive : 1e300;
        for (int id : running) t_next = std::min(t_next, start[id] + req[id].dur);
        if (staged >= 0 && staged_ready > now) t_next = std::min(t_next, staged_ready);
        if (t_next >= 1e300) break;
        now = std::max(now, t_next);
        for (size_t i = 0; i < running.size();) {
            const int id = running[i];
            if (start[id] + req[id].dur <= now) {
                req[id].done = now;
                reserved -= req[id].bytes;
                retired += req[id].bytes;
                running.erase(running.begin() + i);
            } else {
                ++i;
            }
        }
    }
    for (int i = 0; i < n; ++i) CHECK(req[i].done >= start[i] && start[i] >= req[i].admit && req[i].admit >= req[i].arrive);
    return true;
}

int main() {
    long frees = 0, admits = 0, staged = 0;
    int cases = 0;
    for (int seed = 0; seed < 300; ++seed)
        for (int max_active : {1, 2, 4, 16})
            for (uint64_t budget : {1000ull, 1ull << 40}) {
                if (!simulate(seed, max_active, budget, 60, frees, admits)) return 1;
                if (!simulate_ahead(seed, max_active, budget, 60, staged)) return 1;
                ++cases;
            }
    std::printf("ok %d cases, %ld admissions, %ld frees, %ld set up ahead\n", cases, admits, frees, staged);
    return 0;
}
