// Admission policy of the shot server (server.cpp), free of HIP so that it
// can be exercised on the CPU.
//
// Requests wait in arrival order.  The head is admitted while fewer than
// max_active requests run and its footprint fits the device-memory budget;
// a request behind the head never overtakes it.  Device memory of retired
// requests is kept in a pool for the next requests to reuse ("retired
// bytes", counted against the budget): freeing it waits for every stream on
// the device, so it is freed only when the server has no work at all
// (nothing runs and nothing waits) or when the head would fit once it is
// freed.
#pragma once

#include <cstdint>

namespace awe {

struct AdmitState {
    uint64_t budget = 0;     // bytes the running and retired requests may hold
    uint64_t reserved = 0;   // footprints of the running requests
    uint64_t retired = 0;    // bytes of retired requests not freed yet
    int running = 0;
    int max_active = 1;
};

struct AdmitResult {
    int count = 0;           // queue entries to admit, from the head
    bool free_retired = false;   // free the retired bytes first (then decide again)
};

// bytes_of(i): footprint of the i-th queued request (0 = head), i < queued.
template <class BytesOf>
AdmitResult admit_fifo(const AdmitState& s, int queued, BytesOf bytes_of) {
    AdmitResult r;
    if (s.running == 0 && queued == 0 && s.retired > 0) {   // no work at all: freeing stalls no one
        r.free_retired = true;
        return r;
    }
    uint64_t reserved = s.reserved;
    for (int i = 0; i < queued && s.running + r.count < s.max_active; ++i) {
        const uint64_t need = bytes_of(i);
        if (reserved + need > s.budget) break;              // the head waits for retirements
        if (reserved + s.retired + need > s.budget) {       // it fits once retired memory is freed
            r.free_retired = r.count == 0;
            break;
        }
        reserved += need;
        ++r.count;
    }
    return r;
}

}  // namespace awe
