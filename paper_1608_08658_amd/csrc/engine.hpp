// The plan object behind awe_plan and the engine's internal entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "awe.h"
#include "awe_internal.hpp"

namespace awe {

extern thread_local std::string t_err;
awe_status fail(awe_status code, const char* fmt, ...);

void fd_weights(int order, double* w);
double dt_limit(int ndim, int order, const double* h, double vmax);
awe_status validate(const awe_geometry* g);
void padded_zyx(const awe_geometry* g, int64_t pad[3], int64_t phys[3]);
Layout make_layout(int ndim, const int64_t pad[3], int half);
std::vector<int> stored_times(int nt, int K);
int segment_slots(int nt, int K);
uint64_t footprint_bytes(const awe_geometry* g, int K);
// The static conditions under which a 2-D plan advances several forward
// steps per launch (the plan also needs few enough receivers per tile).
bool tb_candidate(const awe_geometry* g, const Layout& L, int64_t src_nodes);

struct LaunchShape {
    int cfg;        // workgroup shape (see launch_step)
    int zchunk;     // z planes per workgroup
};
LaunchShape default_shape(const Layout& L);

// Device buffers kept for reuse by their owner (the shot server): a
// retired plan's buffers come here instead of going to hipFree, and a new
// plan takes one of the same size instead of calling hipMalloc.  The owner
// hands buffers back only once the work that used them has completed.  Not
// thread-safe: one thread owns it.
struct BufferPool {
    std::mutex mu;                       // plans on several host threads share one pool
    std::multimap<size_t, void*> free_list;
    uint64_t bytes = 0;                  // bytes held in the free list (under mu)
    void* take(size_t n);                // a pooled buffer of exactly n bytes, or nullptr
    void give(void* p, size_t n);
    void release_all();                  // hipFree every pooled buffer (waits for the device)
    uint64_t held();
};

struct DeviceCsr {
    int64_t* node = nullptr;
    int32_t* rowptr = nullptr;
    int32_t* pt = nullptr;
    float* w = nullptr;
    int32_t nrows = 0;
};

// Binomial checkpointing (checkpoint.cpp).
struct CkptAction {
    enum Kind : int32_t { kAdvance = 0, kTake = 1, kRestore = 2, kFree = 3, kYield = 4 };
    int32_t kind;
    int32_t arg;   // advance / yield: a time index; take / restore / free: a snapshot (-1 = x_0 = 0)
};
int64_t binomial_steps(int64_t nstates, int free_snapshots);
std::vector<CkptAction> binomial_schedule(int nt, int snapshots);
class Reversal;
awe_status binomial_prepare(Reversal& r, int nt, int snapshots);   // schedule, pool size, step count
uint64_t footprint_binomial_bytes(const awe_geometry* g, int pool_fields);

class Reversal {
public:
    std::vector<CkptAction> sched;
    size_t pos = 0;          // next action
    int pool = 0;            // wavefield buffers the schedule needs
    bool sized = false;
    int64_t steps = 0;       // forward steps taken since rewind()
    int visited = 0;         // states visited since rewind()
    int ua = -1, ub = -1;    // current state (u[t], u[t-1]) as buffer indices; -1 = the zero field
    int t = 0;
    int nt = 0;

    awe_status init(int nt, int snapshots);
    void rewind();
    // Runs actions from `pos`.  step(n, uc, up, out) computes u[n+1] from
    // u[n] (buffer uc) and u[n-1] (up) into out; visit(t, uc) is the visit
    // of state t.  With stop_at_visit the run stops before the first visit.
    template <class Step, class Visit>
    awe_status run(bool stop_at_visit, Step&& step, Visit&& visit) {
        return run_impl(stop_at_visit, false, step, visit);
    }

private:
    struct Snap {
        int ua = -1, ub = -1, t = -1;
    };
    std::vector<Snap> snaps;
    std::vector<int> ref;
    int take_buffer(bool grow);
    void hold(int b) { if (b >= 0) ++ref[b]; }
    void drop(int b) { if (b >= 0) --ref[b]; }
    template <class Step, class Visit>
    awe_status run_impl(bool stop_at_visit, bool grow, Step&& step, Visit&& visit);
};

template <class Step, class Visit>
awe_status Reversal::run_impl(bool stop_at_visit, bool grow, Step&& step, Visit&& visit) {
    for (; pos < sched.size(); ++pos) {
        const CkptAction a = sched[pos];
        switch (a.kind) {
        case CkptAction::kAdvance:
            if (a.arg <= t) return fail(AWE_EINVAL, "checkpoint schedule: advance to %d from %d", a.arg, t);
            while (t < a.arg) {
                const int out = take_buffer(grow);
                if (out < -1) return fail(AWE_EINVAL, "checkpoint schedule: no free buffer at step %d", t);
                awe_status st = step(t, ua, ub, out);
                if (st) return st;
                hold(out);
                drop(ub);
                ub = ua;
                ua = out;
                ++t;
                ++steps;
            }
            break;
        case CkptAction::kTake:
            if (a.arg < 0 || a.arg >= (int)snaps.size() || snaps[a.arg].t >= 0)
                return fail(AWE_EINVAL, "checkpoint schedule: bad snapshot %d", a.arg);
            snaps[a.arg] = Snap{ua, ub, t};
            hold(ua);
            hold(ub);
            break;
        case CkptAction::kRestore: {
            Snap s{-1, -1, 0};
            if (a.arg >= 0) {
                if (a.arg >= (int)snaps.size() || snaps[a.arg].t < 0)
                    return fail(AWE_EINVAL, "checkpoint schedule: restore of empty snapshot %d", a.arg);
                s = snaps[a.arg];
            }
            hold(s.ua);
            hold(s.ub);
            drop(ua);
            drop(ub);
            ua = s.ua;
            ub = s.ub;
            t = s.t;
            break;
        }
        case CkptAction::kFree:
            if (a.arg < 0 || a.arg >= (int)snaps.size() || snaps[a.arg].t < 0)
                return fail(AWE_EINVAL, "checkpoint schedule: free of empty snapshot %d", a.arg);
            drop(snaps[a.arg].ua);
            drop(snaps[a.arg].ub);
            snaps[a.arg] = Snap{};
            break;
        case CkptAction::kYield: {
            if (stop_at_visit) return AWE_OK;
            if (a.arg != t || a.arg != nt - 1 - visited)
                return fail(AWE_EINVAL, "checkpoint schedule: visit of %d at state %d", a.arg, t);
            awe_status st = visit(t, ua);
            if (st) return st;
            ++visited;
            break;
        }
        default:
            return fail(AWE_EINVAL, "checkpoint schedule: bad action");
        }
    }
    return AWE_OK;
}

}  // namespace awe

struct awe_plan_s {
    // geometry (coordinates copied)
    awe_geometry g{};
    std::vector<double> src, rec;
    int half = 0, corners = 0, device = 0;
    int64_t pad[3] = {1, 1, 1}, phys[3] = {1, 1, 1};
    double vol = 1.0;
    awe::Layout L;
    awe::StencilCoef k{};
    awe::LaunchShape fwd_shape{1, 8}, img_shape{1, 8};   // stencil launch shapes (forward / imaging)
    bool img_tuned = false;

    // device buffers owned by the plan
    std::vector<std::pair<void*, size_t>> owned;   // allocation and its size
    awe::BufferPool* pool = nullptr;   // if set: buffers come from and go back to it
    size_t held = 0;
    float* coef = nullptr;
    float *d_ez = nullptr, *d_ey = nullptr, *d_ex = nullptr;
    double *d_ezd = nullptr, *d_eyd = nullptr, *d_exd = nullptr;
    float *w0 = nullptr, *w1 = nullptr;
    int64_t* src_node = nullptr;
    float* src_w = nullptr;
    int64_t* rec_node = nullptr;
    float* rec_w = nullptr;
    awe::DeviceCsr src_csr, rec_csr;
    int32_t* src_zyx = nullptr;     // (z, y, x) of the source nodes when few enough to fuse
    int64_t* d_fold_cells = nullptr;   // edge and corner cells of the gradient fold
    int32_t n_fold_cells = 0;
    bool fuse_sparse = true;        // point operators inside the stencil launch (AWE_FUSE=0: off)
    int tb_T = 0;                   // 2-D plain steps per launch (0: one step per launch; AWE_TB=0)
    float *w2 = nullptr, *w3 = nullptr;   // outputs of blocked 2-D launches
    int32_t *d_rec_zx = nullptr, *d_tile_ptr = nullptr, *d_tile_rec = nullptr;
    float* d_partial = nullptr;
    double* d_mpart = nullptr;
    hipStream_t setup_stream = nullptr;   // stream of init's fills and uploads
    bool timed_tune = true;         // false: take a cached or nearby launch shape, never time candidates
    bool own_tune = true;           // with timed_tune: time this size's own shape rather than borrow a
                                    // nearby size's (server forward requests borrow)

    // wavefield state: u[n] and u[n-1]
    const float* cur = nullptr;
    const float* prev = nullptr;
    bool model_set = false;

    // gradient storage
    int ckpt_K = 0;
    bool storage_ready = false;
    std::map<int, float*> stored;   // time -> wavefield kept by the checkpointed forward
    std::vector<float*> slots;      // recompute buffers of one segment
    float *mu0 = nullptr, *mu1 = nullptr, *grad = nullptr;
    float* wavelet_copy = nullptr;
    float *b_t = nullptr, *b_du0 = nullptr, *b_du1 = nullptr, *b_dm = nullptr;   // linearised modelling
    awe::Reversal rev;              // binomial checkpointing: schedule and executor state
    std::vector<float*> rev_pool;   // its wavefield buffers
    int rev_snaps = -1;             // snapshots of the schedule in rev (-1: none)
    bool rev_mode = false;          // the stored states are binomial (else periodic)
    bool have_ckpt = false, have_grad = false;
    // Sweeps in progress (forward_begin / forward_advance, adjoint_begin /
    // adjoint_advance): where a sweep cut into chunks resumes.
    struct FwdJob {
        const float* wavelet = nullptr;
        float* traces = nullptr;
        int K = 0;
        int n = 0;              // next step: u[n+1] is produced next
        bool active = false;
    } fwd_job;
    struct AdjJob {
        enum Mode { kTranspose = 0, kBinomial = 1, kPeriodic = 2 };
        int mode = kTranspose;
        const float* resid = nullptr;
        float* src_adj = nullptr;
        float* grad_phys = nullptr;
        float *m1 = nullptr, *m2 = nullptr;   // mu[n+1], mu[n+2]
        int n = 0;              // next adjoint step
        int seg = -1;           // periodic: segment being swept (S-1 .. 0)
        bool seg_ready = false; // its state table is set up
        int t = 0;              // next state to recompute in the segment
        int slot = 0;           // next free slot buffer
        std::vector<const float*> ptr;   // u[t] of the segment, t = t0-1 .. t1
        bool active = false;
    } adj_job;
    // Changes whenever the forward state a gradient reads (model, stored
    // states, wavelet copy) is replaced or consumed (awe_forward_id).
    int64_t fwd_id = 0;

    // Optional timing of the step launches (awe_plan_time_kernels): HIP
    // events on the launching stream around every `timer_every`-th launch of
    // each kind (0: stencil steps without imaging, 1: with imaging, 2: point
    // operators launched on their own), resolved by kernel_times().
    int timer_every = 0;
    int64_t timer_seen[3] = {0, 0, 0};
    double timer_ms[3] = {0, 0, 0};
    int64_t timer_count[3] = {0, 0, 0};
    struct TimedLaunch { int kind; hipEvent_t a, b; };
    std::vector<TimedLaunch> timer_pending;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timer_free;
    template <class F>
    hipError_t timed(int kind, hipStream_t s, F&& launch);
    awe_status kernel_times(double* out);
    void timer_reset();

    ~awe_plan_s();
    awe_status init(const awe_geometry* geo, hipStream_t setup = nullptr, bool timed = true);
    awe_status set_model(const float* m, hipStream_t s);
    awe_status forward(const float* wavelet, float* traces, int K, hipStream_t s);
    awe_status forward_binomial(const float* wavelet, float* traces, int snapshots, hipStream_t s);
    awe_status step(int n0, int nsteps, const float* wavelet, float* traces, hipStream_t s);
    awe_status step2_blocked(int npairs, int zchunk, hipStream_t s);   // the temporal-blocking prototype
    awe_status adjoint(const float* resid, float* src_adj, float* grad_phys, hipStream_t s);
    awe_status forward_begin(const float* wavelet, float* traces, int K, hipStream_t s);
    awe_status forward_advance(int max_steps, hipStream_t s, bool* done);
    awe_status adjoint_begin(const float* resid, float* src_adj, float* grad_phys, hipStream_t s);
    awe_status adjoint_advance(int max_steps, hipStream_t s, bool* done);
    awe_status adj_step(int n, const float* usnap, hipStream_t s);
    awe_status born(const float* wavelet, const float* dm_phys, float* traces, hipStream_t s);

    awe_status alloc(void** p, size_t bytes);
    awe_status alloc_field(float** p, hipStream_t s);
    template <class T>
    awe_status upload(T** dst, const std::vector<T>& v);
    void release(void* p);
    awe_status advance(const float* uc, const float* up, float* out, const float* q_row, float* rec_row,
                       hipStream_t s);
    awe_status advance_tb(int n0, int nsteps, const float* wavelet, float* traces, int first_row, hipStream_t s);
    awe::InjectOp src_op(float* field, const float* q_row, float* t_acc) const;
    awe::SampleOp rec_op(float* row, const float* field) const;
    awe_status ensure_gradient_storage(int K, hipStream_t s);
    awe_status ensure_binomial_storage(int snapshots, hipStream_t s);
    awe_status ensure_adjoint_storage(hipStream_t s);
    void release_periodic();
    void release_binomial();
    awe_status tune(bool img, hipStream_t user_stream);
    float* pick_work_dst();
};

namespace awe {
using Plan = awe_plan_s;
}

template <class F>
hipError_t awe_plan_s::timed(int kind, hipStream_t s, F&& launch) {
    if (timer_every <= 0 || (timer_seen[kind]++ % timer_every) != 0 || timer_pending.size() >= 200000) return launch();
    hipEvent_t a = nullptr, b = nullptr;
    if (!timer_free.empty()) {
        a = timer_free.back().first;
        b = timer_free.back().second;
        timer_free.pop_back();
    } else {
        hipError_t e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(a, s);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    timer_pending.push_back({kind, a, b});
    return e;
}
