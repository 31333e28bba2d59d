// Shot server with continuous batching (extern "C" awe_server_* of awe.h).
//
// Requests are admitted against a device-memory budget and a cap on running
// requests.  Every running request advances on its own stream in chunks of
// `chunk` time steps, with two chunks in flight: the engine thread polls each
// request's chunk events and enqueues its next chunk as soon as one
// completes, so the kernels of different shots overlap on the device, a
// short request is never held back by a long one (there is no batch-wide
// barrier), and a request that arrives while others run is admitted as soon
// as a slot and memory are free.  Finished requests are retired (traces
// copied out, memory released) when their last chunk completes, which frees
// budget for the queue.  Each request's arithmetic is exactly that of a plan
// run alone: the steps are the same kernels on the same data, only
// interleaved in time with other requests.
//
// The engine never waits for the whole device while requests run: a plan is
// set up on its request's stream (launch shapes are timed only while no other
// request runs; otherwise the autotuner takes a cached or nearby shape, else
// the built-in one), traces are copied out only
// once the request's last chunk has completed, and streams and events are
// reused.  While max_active requests run, the next admitted request is set up
// ahead on a host thread of its own (plan, uploads of the model, wavelet and
// observed traces): it starts computing as soon as a running request
// finishes, whose traces are then copied out while the device already works
// on the next one.  hipFree waits for every stream on the device, so a retired
// request's device memory goes to a pool (counted against the budget) that
// the next plans take their buffers from (same-sized fields of a repeated
// grid need no new allocation), and the pool is freed in one batch only
// when the server has no work or the queue head needs the room.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "awe.h"
#include "engine.hpp"
#include "server_policy.hpp"

using awe::fail;

namespace {

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct Request {
    int64_t id = 0;
    awe_geometry g{};
    std::vector<double> src, rec;
    std::vector<float> m, wavelet, obs;
    float* traces_host = nullptr;
    // gradient requests: checkpoint interval, observed traces (obs, copied at
    // submit) and where the gradient and the misfit go
    bool gradient = false;
    int K = 0;
    float* grad_dev = nullptr;
    double* phi_host = nullptr;
    uint64_t bytes = 0;
    int state = AWE_REQ_QUEUED;
    double t[4] = {-1, -1, -1, -1};
    std::string err;
    // device side while running
    awe_plan plan = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};   // completion of the chunks in flight (ring)
    int ev_head = 0, inflight = 0;
    float* d_m = nullptr;
    float* d_wav = nullptr;
    float* d_tr = nullptr;
    float* d_obs = nullptr;   // gradient: observed traces, then the residual in place
    double* d_phi = nullptr;  // gradient: misfit
    enum Phase { kForward = 0, kAdjoint = 1, kDone = 2 };
    int phase = kForward;
    // set up ahead (see above): the host thread doing it, its outcome
    std::thread setup;
    std::atomic<bool> ready{false};
    bool setup_ok = false;
    std::string setup_err;
};

// A stream with its two chunk events, reused by later requests.
struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
};

}  // namespace

struct awe_server_s {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    int device = 0;
    int chunk = 64;
    int max_active = 8;
    uint64_t budget = 0;
    uint64_t reserved = 0;
    int64_t next_id = 0;
    int64_t n_submitted = 0, n_admitted = 0, n_completed = 0, n_failed = 0, iterations = 0;
    std::mutex mu;
    std::condition_variable wake;     // engine: new work or stop
    std::condition_variable changed;  // waiters: a request changed state
    std::deque<Request*> queue;
    std::vector<Request*> active;
    std::map<int64_t, std::unique_ptr<Request>> all;
    std::vector<Lane> lanes;     // idle streams
    // retired requests' device memory, reused by later plans (engine thread
    // only; pool_bytes mirrors pool.bytes under mu for the stats)
    awe::BufferPool pool;
    uint64_t pool_bytes = 0;
    bool stop = false;
    std::thread engine;
    // engine thread: the request being set up ahead, or set up and waiting
    // for a running slot (at most one)
    Request* staged = nullptr;

    void run();
    void stage(Request* r);
    bool promote();
    bool pump(Request* r, std::string& err, bool alone);
    bool start(Request* r, bool idle, std::string& err);
    void finish(Request* r, int state, const std::string& err);
    void free_pool();
    void release_lanes();
    template <class T>
    bool pool_alloc(T** p, size_t n, std::string& err);
    void sync_pool_bytes();
};

void awe_server_s::sync_pool_bytes() {
    const uint64_t b = pool.held();
    std::lock_guard<std::mutex> lk(mu);
    pool_bytes = b;
}

void awe_server_s::free_pool() {
    // engine thread (or after it has ended); the first hipFree waits for the device
    pool.release_all();
    sync_pool_bytes();
}

// A request buffer: a pooled one of the same size if there is one.
template <class T>
bool awe_server_s::pool_alloc(T** p, size_t n, std::string& err) {
    if ((*p = static_cast<T*>(pool.take(n)))) return true;
    const hipError_t e = hipMalloc(p, n);
    if (e == hipSuccess) return true;
    (void)hipGetLastError();
    err = std::string("hipMalloc: ") + hipGetErrorString(e);
    return false;
}

void awe_server_s::release_lanes() {
    for (Lane& l : lanes) {
        for (hipEvent_t e : l.ev)
            if (e) (void)hipEventDestroy(e);
        if (l.stream) (void)hipStreamDestroy(l.stream);
    }
    lanes.clear();
}

void awe_server_s::finish(Request* r, int state, const std::string& err) {
    // engine thread, caller does not hold mu; waits for r's own stream only:
    // once it is idle nothing uses the request's buffers, and the plan and
    // the buffers go back to the pool without freeing anything
    if (r->stream) (void)hipStreamSynchronize(r->stream);
    delete r->plan;
    const size_t nm = r->m.size(), nw = r->wavelet.size(), ntr = (size_t)r->g.nt * r->g.nrec;
    pool.give(r->d_m, nm * sizeof(float));
    pool.give(r->d_wav, nw * sizeof(float));
    pool.give(r->d_tr, ntr * sizeof(float));
    pool.give(r->d_obs, ntr * sizeof(float));
    pool.give(r->d_phi, sizeof(double));
    Lane ln;
    ln.stream = r->stream;
    ln.ev[0] = r->ev[0];
    ln.ev[1] = r->ev[1];
    r->plan = nullptr;
    r->d_m = r->d_wav = r->d_tr = r->d_obs = nullptr;
    r->d_phi = nullptr;
    r->stream = nullptr;
    r->ev[0] = r->ev[1] = nullptr;
    std::vector<float>().swap(r->m);
    std::vector<float>().swap(r->wavelet);
    std::vector<float>().swap(r->obs);
    const uint64_t held = pool.held();
    std::lock_guard<std::mutex> lk(mu);
    pool_bytes = held;
    if (ln.stream) lanes.push_back(ln);
    else
        for (hipEvent_t e : ln.ev)
            if (e) (void)hipEventDestroy(e);
    r->state = state;
    r->err = err;
    r->t[3] = now_s(t0);
    reserved -= r->bytes;
    if (state == AWE_REQ_DONE) ++n_completed;
    else ++n_failed;
    changed.notify_all();
}

// idle: nothing else runs on the device, so the plan may time its launch
// shapes (timings among other requests' kernels would be distorted and
// would stall them).
bool awe_server_s::start(Request* r, bool idle, std::string& err) {
    auto hip_ok = [&](hipError_t e, const char* what) {
        if (e == hipSuccess) return true;
        err = std::string(what) + ": " + hipGetErrorString(e);
        return false;
    };
    {
        std::lock_guard<std::mutex> lk(mu);
        if (!lanes.empty()) {
            r->stream = lanes.back().stream;
            r->ev[0] = lanes.back().ev[0];
            r->ev[1] = lanes.back().ev[1];
            lanes.pop_back();
        }
    }
    r->ev_head = r->inflight = 0;
    if (!r->stream && !hip_ok(hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking), "hipStreamCreate"))
        return false;
    for (hipEvent_t& e : r->ev)
        if (!e && !hip_ok(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate")) return false;
    awe_status st = AWE_OK;
    try {
        r->plan = new awe_plan_s();
        r->plan->pool = &pool;   // buffers of earlier requests of the same grid are reused
        // a gradient request (long, and typically one of many shots on one
        // grid) times its own size's shapes when it may; forward requests
        // take a nearby size's
        r->plan->own_tune = r->gradient;
        st = r->plan->init(&r->g, r->stream, idle);
    } catch (const std::bad_alloc&) {
        st = fail(AWE_ENOMEM, "host allocation failed");
    } catch (...) {
        st = fail(AWE_EINVAL, "unexpected exception in the library");
    }
    if (st) { err = awe_last_error(); return false; }
    const size_t nm = r->m.size(), nw = r->wavelet.size(), ntr = (size_t)r->g.nt * r->g.nrec;
    if (!pool_alloc(&r->d_m, nm * sizeof(float), err)) return false;
    if (nw && !pool_alloc(&r->d_wav, nw * sizeof(float), err)) return false;
    if (ntr && !pool_alloc(&r->d_tr, ntr * sizeof(float), err)) return false;
    if (!hip_ok(hipMemcpyAsync(r->d_m, r->m.data(), nm * sizeof(float), hipMemcpyHostToDevice, r->stream), "copy m"))
        return false;
    if (nw && !hip_ok(hipMemcpyAsync(r->d_wav, r->wavelet.data(), nw * sizeof(float), hipMemcpyHostToDevice,
                                     r->stream), "copy wavelet"))
        return false;
    if (r->gradient) {
        if (ntr && !pool_alloc(&r->d_obs, ntr * sizeof(float), err)) return false;
        if (!pool_alloc(&r->d_phi, sizeof(double), err)) return false;
        if (ntr && !hip_ok(hipMemcpyAsync(r->d_obs, r->obs.data(), ntr * sizeof(float), hipMemcpyHostToDevice,
                                          r->stream), "copy d_obs"))
            return false;
    }
    st = awe_set_model(r->plan, r->d_m, r->stream);   // synchronises r->stream
    if (st) { err = awe_last_error(); return false; }
    // the forward of awe_forward, advanced a chunk at a time by the engine
    st = r->plan->forward_begin(r->d_wav, r->d_tr, r->gradient ? r->K : 0, r->stream);
    if (st) { err = awe_last_error(); return false; }
    r->phase = Request::kForward;
    return true;
}

// Enqueues the request's next chunk: up to `chunk` forward steps, then (for a
// gradient) the misfit and up to `chunk` steps of the adjoint sweep.  The
// arithmetic is that of awe_forward, awe_misfit and awe_adjoint on a plan
// run alone.
static awe_status advance_request(Request* r, int chunk, bool alone) {
    bool done = false;
    awe_status st;
    if (r->phase == Request::kForward) {
        if ((st = r->plan->forward_advance(chunk, r->stream, &done))) return st;
        if (!done) return AWE_OK;
        if (!r->gradient) {
            r->phase = Request::kDone;
            return AWE_OK;
        }
        // residual = traces - d_obs (in place over d_obs) and its misfit
        const int64_t ntr = (int64_t)r->g.nt * r->g.nrec;
        hipError_t e = awe::launch_misfit(r->d_tr, r->d_obs, ntr, r->d_obs, r->plan->d_mpart, awe::kReduceBlocks,
                                          r->d_phi, r->stream);
        if (e != hipSuccess) return fail(AWE_EHIP, "misfit: %s", hipGetErrorString(e));
        r->plan->timed_tune = alone;   // the imaging step's shape is timed only with the device to itself
        if ((st = r->plan->adjoint_begin(r->d_obs, nullptr, r->grad_dev, r->stream))) return st;
        r->phase = Request::kAdjoint;
        return AWE_OK;
    }
    if (r->phase == Request::kAdjoint) {
        if ((st = r->plan->adjoint_advance(chunk, r->stream, &done))) return st;
        if (done) r->phase = Request::kDone;
    }
    return AWE_OK;
}

// Sets r up on a host thread of its own while the running requests compute.
void awe_server_s::stage(Request* r) {
    staged = r;
    r->ready.store(false);
    r->setup = std::thread([this, r] {
        (void)hipSetDevice(device);
        std::string err;
        const bool ok = start(r, false, err);
        r->setup_ok = ok;
        r->setup_err = err;
        r->ready.store(true, std::memory_order_release);
    });
}

// Moves the staged request, once set up, into a free running slot.  Returns
// true if a request started running.
bool awe_server_s::promote() {
    Request* r = staged;
    if (!r || !r->ready.load(std::memory_order_acquire)) return false;
    if (r->setup_ok) {   // a failed set-up retires at once, without waiting for a slot
        std::lock_guard<std::mutex> lk(mu);
        if ((int)active.size() >= max_active) return false;
    }
    r->setup.join();
    staged = nullptr;
    if (!r->setup_ok) {
        finish(r, AWE_REQ_FAILED, r->setup_err);
        return false;
    }
    std::lock_guard<std::mutex> lk(mu);
    r->t[2] = now_s(t0);
    active.push_back(r);
    return true;
}

// Keeps two chunks of r in flight.  Returns false (err set) on failure.
bool awe_server_s::pump(Request* r, std::string& err, bool alone) {
    while (r->inflight < 2 && r->phase != Request::kDone) {
        if (advance_request(r, chunk, alone)) {
            err = awe_last_error();
            return false;
        }
        const hipError_t e = hipEventRecord(r->ev[r->ev_head], r->stream);
        if (e != hipSuccess) {
            err = hipGetErrorString(e);
            return false;
        }
        r->ev_head = (r->ev_head + 1) % 2;
        ++r->inflight;
    }
    return true;
}

void awe_server_s::run() {
    (void)hipSetDevice(device);
    for (;;) {
        std::vector<Request*> admitted;
        bool flush = false;
        {
            std::unique_lock<std::mutex> lk(mu);
            // with no work left the pooled memory is freed first (below)
            if (!active.empty() || !queue.empty() || staged || pool_bytes == 0) {
                wake.wait(lk, [&] { return stop || !queue.empty() || !active.empty() || staged; });
                if (stop && active.empty() && !staged && pool_bytes == 0) break;
            }
            // FIFO admission (server_policy.hpp) for max_active running
            // requests plus one set up ahead; nothing is admitted past a
            // request set up ahead, which would otherwise start after a
            // younger one
            awe::AdmitState as;
            as.budget = budget;
            as.reserved = reserved;
            as.retired = pool_bytes;
            as.running = (int)active.size() + (staged ? 1 : 0);
            as.max_active = max_active + 1;
            const awe::AdmitResult ar =
                awe::admit_fifo(as, (stop || staged) ? 0 : (int)queue.size(), [&](int i) { return queue[i]->bytes; });
            flush = ar.free_retired;
            for (int i = 0; i < ar.count; ++i) {
                Request* r = queue.front();
                queue.pop_front();
                reserved += r->bytes;
                r->state = AWE_REQ_RUNNING;
                r->t[1] = now_s(t0);
                ++n_admitted;
                admitted.push_back(r);
            }
        }
        if (flush) {
            free_pool();
            continue;
        }
        bool progressed = promote();
        for (Request* r : admitted) {
            std::string err;
            bool idle, slot;
            {
                std::lock_guard<std::mutex> lk(mu);
                idle = active.empty() && !staged;
                slot = (int)active.size() < max_active;
            }
            if (!slot) {   // the admission leaves at most one request beyond max_active
                stage(r);
            } else if (start(r, idle, err)) {
                std::lock_guard<std::mutex> lk(mu);
                r->t[2] = now_s(t0);
                active.push_back(r);
            } else {
                finish(r, AWE_REQ_FAILED, err);
            }
            progressed = true;
        }
        // keep two chunks in flight per running request; retire on completion
        std::vector<Request*> running;
        {
            std::lock_guard<std::mutex> lk(mu);
            running = active;
        }
        // a staged request still uploading shares the device: no shape timing then
        const bool quiet = !staged || staged->ready.load(std::memory_order_acquire);
        for (Request* r : running) {
            std::string err;
            bool failed = false;
            // completed chunks, oldest first (a stream's events complete in order)
            while (r->inflight > 0) {
                const int tail = (r->ev_head - r->inflight + 2) % 2;
                const hipError_t e = hipEventQuery(r->ev[tail]);
                if (e == hipErrorNotReady) break;
                if (e != hipSuccess) {
                    err = hipGetErrorString(e);
                    failed = true;
                    break;
                }
                --r->inflight;
                progressed = true;
            }
            if (!failed && r->inflight < 2 && r->phase != Request::kDone) {
                failed = !pump(r, err, running.size() == 1 && quiet);
                progressed = true;
            }
            if (!failed && !(r->phase == Request::kDone && r->inflight == 0)) continue;
            // r is finished: the staged request takes its slot and gets its
            // first chunks before r's traces are copied out
            { std::lock_guard<std::mutex> lk(mu); active.erase(std::find(active.begin(), active.end(), r)); }
            if (promote()) {
                Request* p;
                {
                    std::lock_guard<std::mutex> lk(mu);
                    p = active.back();
                }
                std::string perr;
                if (!pump(p, perr, false)) {
                    { std::lock_guard<std::mutex> lk(mu); active.erase(std::find(active.begin(), active.end(), p)); }
                    finish(p, AWE_REQ_FAILED, perr);
                }
            }
            if (!failed) {
                // every step of r has completed, so the copy-out waits for nothing else of r
                const size_t ntr = (size_t)r->g.nt * r->g.nrec;
                hipError_t e = hipSuccess;
                if (ntr && r->traces_host)
                    e = hipMemcpyAsync(r->traces_host, r->d_tr, ntr * sizeof(float), hipMemcpyDeviceToHost, r->stream);
                if (e == hipSuccess && r->gradient && r->phi_host)
                    e = hipMemcpyAsync(r->phi_host, r->d_phi, sizeof(double), hipMemcpyDeviceToHost, r->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
                if (e != hipSuccess) {
                    err = hipGetErrorString(e);
                    failed = true;
                }
            }
            finish(r, failed ? AWE_REQ_FAILED : AWE_REQ_DONE, err);
            progressed = true;
        }
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
        std::lock_guard<std::mutex> lk(mu);
        ++iterations;
    }
}

extern "C" {

awe_status awe_server_create(double hbm_fraction, int32_t chunk_steps, int32_t max_active, awe_server* out) {
    if (!out) return fail(AWE_EINVAL, "output pointer is NULL");
    *out = nullptr;
    if (!(hbm_fraction > 0.0 && hbm_fraction <= 1.0)) return fail(AWE_EINVAL, "hbm_fraction must be in (0, 1]");
    if (chunk_steps < 1 || max_active < 1) return fail(AWE_EINVAL, "chunk_steps and max_active must be >= 1");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(AWE_ENODEV, "no HIP device available");
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return fail(AWE_EHIP, "hipMemGetInfo failed");
    awe_server s = new (std::nothrow) awe_server_s();
    if (!s) return fail(AWE_ENOMEM, "host allocation failed");
    s->device = dev;
    s->chunk = chunk_steps;
    s->max_active = max_active;
    s->budget = (uint64_t)(hbm_fraction * (double)free_b);
    if (const char* env = std::getenv("AWE_SERVER_BUDGET_BYTES")) {
        const unsigned long long b = std::strtoull(env, nullptr, 10);
        if (b > 0) s->budget = std::min<uint64_t>(s->budget, b);
    }
    s->engine = std::thread([s] { s->run(); });
    *out = s;
    return AWE_OK;
}

}  // extern "C"

// Copies the request's inputs, sizes its footprint and queues it.
static awe_status submit_request(awe_server srv, std::unique_ptr<Request> r, int64_t* ticket) {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return fail(AWE_EBUSY, "server is shutting down");
    if (r->bytes > srv->budget)
        return fail(AWE_ENOMEM, "request needs %llu bytes, budget is %llu", (unsigned long long)r->bytes,
                    (unsigned long long)srv->budget);
    r->id = srv->next_id++;
    r->t[0] = now_s(srv->t0);
    *ticket = r->id;
    srv->queue.push_back(r.get());
    srv->all[r->id] = std::move(r);
    ++srv->n_submitted;
    srv->wake.notify_all();
    return AWE_OK;
}

static std::unique_ptr<Request> make_request(const awe_geometry* g, const float* m, const float* wavelet,
                                             float* traces) {
    auto r = std::make_unique<Request>();
    r->g = *g;
    r->src.assign(g->src_coords, g->src_coords + (size_t)g->nsrc * g->ndim);
    r->rec.assign(g->rec_coords, g->rec_coords + (size_t)g->nrec * g->ndim);
    r->g.src_coords = r->src.data();
    r->g.rec_coords = r->rec.data();
    size_t nm = 1;
    for (int a = 0; a < g->ndim; ++a) nm *= (size_t)g->shape[a];
    r->m.assign(m, m + nm);
    if (g->nsrc > 0) r->wavelet.assign(wavelet, wavelet + (size_t)g->nt * g->nsrc);
    r->traces_host = traces;
    // plan + model + wavelet + traces on the device
    r->bytes = awe::footprint_bytes(g, 0) + nm * 4 + r->wavelet.size() * 4 + (size_t)g->nt * g->nrec * 4;
    return r;
}

extern "C" {

awe_status awe_server_submit(awe_server srv, const awe_geometry* g, const float* m, const float* wavelet,
                             float* traces, int64_t* ticket) {
    if (!srv || !ticket) return fail(AWE_EINVAL, "NULL argument");
    awe_status st = awe::validate(g);
    if (st) return st;
    if (!m) return fail(AWE_EINVAL, "model is NULL");
    if (g->nsrc > 0 && !wavelet) return fail(AWE_EINVAL, "wavelet is NULL");
    if (g->nrec > 0 && !traces) return fail(AWE_EINVAL, "traces is NULL");
    try {
        return submit_request(srv, make_request(g, m, wavelet, traces), ticket);
    } catch (const std::bad_alloc&) {
        return fail(AWE_ENOMEM, "host allocation failed");
    }
}

awe_status awe_server_submit_gradient(awe_server srv, const awe_geometry* g, const float* m, const float* wavelet,
                                      const float* d_obs, int32_t ckpt_every, float* traces, float* grad_dev,
                                      double* phi, int64_t* ticket) {
    if (!srv || !ticket) return fail(AWE_EINVAL, "NULL argument");
    awe_status st = awe::validate(g);
    if (st) return st;
    if (!m) return fail(AWE_EINVAL, "model is NULL");
    if (g->nsrc > 0 && !wavelet) return fail(AWE_EINVAL, "wavelet is NULL");
    if (g->nrec > 0 && !d_obs) return fail(AWE_EINVAL, "d_obs is NULL");
    if (!grad_dev) return fail(AWE_EINVAL, "grad_dev is NULL");
    if (ckpt_every < 1) return fail(AWE_EINVAL, "ckpt_every must be >= 1");
    try {
        std::unique_ptr<Request> r = make_request(g, m, wavelet, traces);
        const size_t ntr = (size_t)g->nt * g->nrec;
        r->obs.assign(d_obs, d_obs + ntr);
        r->gradient = true;
        r->K = ckpt_every;
        r->grad_dev = grad_dev;
        r->phi_host = phi;
        // + checkpoints, segment slots and adjoint fields, the observed traces
        // (the residual overwrites them) and the misfit
        r->bytes += awe::footprint_bytes(g, ckpt_every) - awe::footprint_bytes(g, 0) + ntr * 4 + sizeof(double);
        return submit_request(srv, std::move(r), ticket);
    } catch (const std::bad_alloc&) {
        return fail(AWE_ENOMEM, "host allocation failed");
    }
}

awe_status awe_server_poll(awe_server srv, int64_t ticket, int32_t* state, double* times) {
    if (!srv || !state) return fail(AWE_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->all.find(ticket);
    if (it == srv->all.end()) return fail(AWE_EINVAL, "unknown ticket %lld", (long long)ticket);
    Request* r = it->second.get();
    *state = r->state;
    if (times)
        for (int i = 0; i < 4; ++i) times[i] = r->t[i];
    if (r->state == AWE_REQ_FAILED) awe::t_err = r->err;
    return AWE_OK;
}

awe_status awe_server_wait(awe_server srv, int64_t ticket, double timeout_s) {
    if (!srv) return fail(AWE_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->all.find(ticket);
    if (it == srv->all.end()) return fail(AWE_EINVAL, "unknown ticket %lld", (long long)ticket);
    Request* r = it->second.get();
    auto done = [&] { return r->state == AWE_REQ_DONE || r->state == AWE_REQ_FAILED; };
    if (!srv->changed.wait_for(lk, std::chrono::duration<double>(timeout_s), done))
        return fail(AWE_EBUSY, "request %lld still running", (long long)ticket);
    if (r->state == AWE_REQ_FAILED) return fail(AWE_EINVAL, "request failed: %s", r->err.c_str());
    return AWE_OK;
}

awe_status awe_server_stats(awe_server srv, int64_t* out) {
    if (!srv || !out) return fail(AWE_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    out[0] = srv->n_submitted;
    out[1] = srv->n_admitted;
    out[2] = srv->n_completed;
    out[3] = srv->n_failed;
    out[4] = (int64_t)srv->active.size();
    out[5] = (int64_t)srv->queue.size();
    out[6] = (int64_t)(srv->reserved + srv->pool_bytes);
    out[7] = srv->iterations;
    return AWE_OK;
}

awe_status awe_server_destroy(awe_server srv) {
    if (!srv) return AWE_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        for (Request* r : srv->queue) {
            r->state = AWE_REQ_FAILED;
            r->err = "server destroyed before the request was admitted";
            ++srv->n_failed;
        }
        srv->queue.clear();
        srv->wake.notify_all();
        srv->changed.notify_all();
    }
    if (srv->engine.joinable()) srv->engine.join();
    srv->free_pool();
    srv->release_lanes();
    delete srv;
    return AWE_OK;
}

}  // extern "C"
