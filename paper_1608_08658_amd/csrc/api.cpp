// extern "C" entry points of include/awe.h for plans and host utilities.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>

#include "awe.h"
#include "engine.hpp"

using awe::fail;

#define AWE_HIP(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) return fail(AWE_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define AWE_TRY(stmt)                                                     \
    try {                                                                 \
        stmt;                                                             \
    } catch (const std::bad_alloc&) {                                     \
        return fail(AWE_ENOMEM, "host allocation failed");               \
    } catch (...) {                                                       \
        return fail(AWE_EINVAL, "unexpected exception in the library");  \
    }

static inline hipStream_t as_stream(awe_stream s) { return reinterpret_cast<hipStream_t>(s); }

// A plan lives on the device that was current when it was created; calls that
// enqueue work on it must be made with that device current.
#define AWE_PLAN(plan)                                                                              \
    do {                                                                                            \
        if (!(plan)) return fail(AWE_EINVAL, "plan is NULL");                                       \
        int d_ = -1;                                                                                \
        if (hipGetDevice(&d_) != hipSuccess || d_ != (plan)->device)                                \
            return fail(AWE_EINVAL, "the plan was created on device %d but device %d is current",  \
                        (plan)->device, d_);                                                        \
    } while (0)

extern "C" {

const char* awe_last_error(void) { return awe::t_err.c_str(); }

const char* awe_version(void) { return "awe 0.1 gfx950"; }

awe_status awe_fd_weights(int32_t order, double* w) {
    if (!w) return fail(AWE_EINVAL, "output pointer is NULL");
    if (order < 2 || order > 2 * awe::kMaxHalf || order % 2)
        return fail(AWE_EINVAL, "space_order must be even in 2..16 (got %d)", order);
    awe::fd_weights(order, w);
    return AWE_OK;
}

awe_status awe_dt_max(int32_t ndim, int32_t order, const double* spacing, double vmax, double* dt_max) {
    if (!spacing || !dt_max) return fail(AWE_EINVAL, "pointer argument is NULL");
    if (ndim != 2 && ndim != 3) return fail(AWE_EINVAL, "ndim must be 2 or 3");
    if (order < 2 || order > 2 * awe::kMaxHalf || order % 2) return fail(AWE_EINVAL, "bad space_order %d", order);
    for (int a = 0; a < ndim; ++a)
        if (!(spacing[a] > 0.0) || !std::isfinite(spacing[a])) return fail(AWE_EINVAL, "bad spacing");
    if (!(vmax > 0.0) || !std::isfinite(vmax)) return fail(AWE_EINVAL, "vmax must be positive");
    *dt_max = awe::dt_limit(ndim, order, spacing, vmax);
    return AWE_OK;
}

awe_status awe_footprint(const awe_geometry* g, int32_t ckpt_every, uint64_t* bytes) {
    awe_status st = awe::validate(g);
    if (st) return st;
    if (!bytes) return fail(AWE_EINVAL, "output pointer is NULL");
    if (ckpt_every < 0) return fail(AWE_EINVAL, "ckpt_every must be >= 0");
    AWE_TRY(*bytes = awe::footprint_bytes(g, ckpt_every));
    return AWE_OK;
}

awe_status awe_binomial_cost(int32_t nt, int32_t snapshots, int64_t* forward_steps, int32_t* fields) {
    if (!forward_steps || !fields) return fail(AWE_EINVAL, "output pointer is NULL");
    if (nt < 1) return fail(AWE_EINVAL, "nt must be >= 1");
    if (snapshots < 0) return fail(AWE_EINVAL, "snapshots must be >= 0");
    AWE_TRY({
        awe::Reversal r;
        awe_status st = awe::binomial_prepare(r, nt, snapshots);
        if (st) return st;
        *forward_steps = r.steps;
        *fields = r.pool;
    });
    return AWE_OK;
}

awe_status awe_footprint_binomial(const awe_geometry* g, int32_t snapshots, uint64_t* bytes) {
    awe_status st = awe::validate(g);
    if (st) return st;
    if (!bytes) return fail(AWE_EINVAL, "output pointer is NULL");
    if (snapshots < 0) return fail(AWE_EINVAL, "snapshots must be >= 0");
    AWE_TRY({
        awe::Reversal r;
        if ((st = awe::binomial_prepare(r, g->nt, snapshots))) return st;
        *bytes = awe::footprint_binomial_bytes(g, r.pool);
    });
    return AWE_OK;
}

awe_status awe_plan_create(const awe_geometry* g, awe_plan* out) {
    if (!out) return fail(AWE_EINVAL, "output pointer is NULL");
    *out = nullptr;
    awe_status st = awe::validate(g);
    if (st) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(AWE_ENODEV, "no HIP device available");
    }
    awe_plan p = nullptr;
    AWE_TRY(p = new awe_plan_s());
    AWE_TRY(st = p->init(g));
    if (st) {
        delete p;
        return st;
    }
    *out = p;
    return AWE_OK;
}

awe_status awe_plan_destroy(awe_plan plan) {
    if (!plan) return AWE_OK;
    (void)hipDeviceSynchronize();
    delete plan;
    return AWE_OK;
}

awe_status awe_plan_info(awe_plan plan, int64_t* out) {
    if (!plan || !out) return fail(AWE_EINVAL, "NULL argument");
    out[0] = plan->pad[0];
    out[1] = plan->g.ndim == 3 ? plan->pad[1] : plan->pad[2];
    out[2] = plan->g.ndim == 3 ? plan->pad[2] : 1;
    out[3] = (int64_t)plan->held;
    out[4] = plan->fwd_shape.cfg;
    out[5] = plan->fwd_shape.zchunk;
    out[6] = plan->img_shape.cfg;
    out[7] = plan->img_shape.zchunk;
    return AWE_OK;
}

awe_status awe_plan_time_kernels(awe_plan plan, int32_t every) {
    if (!plan) return fail(AWE_EINVAL, "plan is NULL");
    if (every < 0) return fail(AWE_EINVAL, "every must be >= 0");
    plan->timer_reset();
    plan->timer_every = every;
    return AWE_OK;
}

awe_status awe_plan_kernel_times(awe_plan plan, double* out) {
    if (!plan || !out) return fail(AWE_EINVAL, "NULL argument");
    AWE_TRY(return plan->kernel_times(out));
}

awe_status awe_set_model(awe_plan plan, const float* m, awe_stream s) {
    AWE_PLAN(plan);
    AWE_TRY(return plan->set_model(m, as_stream(s)));
}

awe_status awe_forward(awe_plan plan, const float* wavelet, float* traces, int32_t ckpt_every, awe_stream s) {
    AWE_PLAN(plan);
    AWE_TRY(return plan->forward(wavelet, traces, ckpt_every, as_stream(s)));
}

awe_status awe_forward_binomial(awe_plan plan, const float* wavelet, float* traces, int32_t snapshots,
                                awe_stream s) {
    AWE_PLAN(plan);
    AWE_TRY(return plan->forward_binomial(wavelet, traces, snapshots, as_stream(s)));
}

awe_status awe_adjoint(awe_plan plan, const float* resid, float* src_adj, float* grad_m, awe_stream s) {
    AWE_PLAN(plan);
    AWE_TRY(return plan->adjoint(resid, src_adj, grad_m, as_stream(s)));
}

awe_status awe_forward_id(awe_plan plan, int64_t* id) {
    if (!plan || !id) return fail(AWE_EINVAL, "NULL argument");
    *id = plan->fwd_id;
    return AWE_OK;
}

awe_status awe_adjoint_checked(awe_plan plan, int64_t forward_id, const float* resid, float* src_adj, float* grad_m,
                               awe_stream s) {
    AWE_PLAN(plan);
    if (forward_id != plan->fwd_id)
        return fail(AWE_ESTATE, "the plan no longer holds forward state %lld (now %lld): another forward, model "
                                "or linearised run replaced it",
                    (long long)forward_id, (long long)plan->fwd_id);
    AWE_TRY(return plan->adjoint(resid, src_adj, grad_m, as_stream(s)));
}

awe_status awe_born(awe_plan plan, const float* wavelet, const float* dm, float* traces, awe_stream s) {
    AWE_PLAN(plan);
    AWE_TRY(return plan->born(wavelet, dm, traces, as_stream(s)));
}

awe_status awe_get_gradient_padded(awe_plan plan, float* g_pad, awe_stream s) {
    AWE_PLAN(plan);
    if (!g_pad) return fail(AWE_EINVAL, "NULL argument");
    if (!plan->have_grad) return fail(AWE_ESTATE, "no gradient has been computed on this plan");
    AWE_HIP(awe::launch_pack(g_pad, plan->grad, plan->L, (float)(-1.0 / (plan->g.dt * plan->g.dt)), as_stream(s)));
    return AWE_OK;
}

awe_status awe_set_state(awe_plan plan, const float* u, const float* u_prev, awe_stream s) {
    AWE_PLAN(plan);
    if (!u || !u_prev) return fail(AWE_EINVAL, "NULL argument");
    AWE_HIP(awe::launch_unpack(plan->w0, u, plan->L, as_stream(s)));
    AWE_HIP(awe::launch_unpack(plan->w1, u_prev, plan->L, as_stream(s)));
    plan->cur = plan->w0;
    plan->prev = plan->w1;
    return AWE_OK;
}

awe_status awe_step(awe_plan plan, int32_t n0, int32_t nsteps, const float* wavelet, float* traces, awe_stream s) {
    AWE_PLAN(plan);
    AWE_TRY(return plan->step(n0, nsteps, wavelet, traces, as_stream(s)));
}

awe_status awe_step2_blocked(awe_plan plan, int32_t npairs, int32_t zchunk, awe_stream s) {
    AWE_PLAN(plan);
    AWE_TRY(return plan->step2_blocked(npairs, zchunk, as_stream(s)));
}

awe_status awe_get_state(awe_plan plan, float* u, float* u_prev, awe_stream s) {
    AWE_PLAN(plan);
    if (u) AWE_HIP(awe::launch_pack(u, plan->cur, plan->L, 1.f, as_stream(s)));
    if (u_prev) AWE_HIP(awe::launch_pack(u_prev, plan->prev, plan->L, 1.f, as_stream(s)));
    return AWE_OK;
}

awe_status awe_sum_fields(float* out, const float* const* parts, int32_t nparts, int64_t n, awe_stream s) {
    if (!out || !parts) return fail(AWE_EINVAL, "NULL argument");
    if (nparts < 1 || nparts > awe::kMaxSumParts)
        return fail(AWE_EINVAL, "nparts must be in 1..%d (got %d)", awe::kMaxSumParts, nparts);
    if (n < 0) return fail(AWE_EINVAL, "n must be >= 0");
    for (int q = 0; q < nparts; ++q)
        if (!parts[q]) return fail(AWE_EINVAL, "parts[%d] is NULL", q);
    AWE_HIP(awe::launch_sum_parts(out, parts, nparts, n, as_stream(s)));
    return AWE_OK;
}

awe_status awe_misfit(const float* traces, const float* d_obs, int64_t n, float* resid, double* phi, awe_stream s) {
    if (!phi) return fail(AWE_EINVAL, "phi pointer is NULL");
    if (n < 0) return fail(AWE_EINVAL, "n must be >= 0");
    if (n > 0 && (!traces || !d_obs)) return fail(AWE_EINVAL, "NULL trace pointer");
    if (n == 0) {
        *phi = 0.0;
        return AWE_OK;
    }
    double* part = nullptr;
    AWE_HIP(hipMalloc(&part, (awe::kReduceBlocks + 1) * sizeof(double)));
    hipStream_t st = as_stream(s);
    hipError_t e = awe::launch_misfit(traces, d_obs, n, resid, part, awe::kReduceBlocks, part + awe::kReduceBlocks, st);
    if (e == hipSuccess) e = hipMemcpyAsync(phi, part + awe::kReduceBlocks, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(part);
    if (e != hipSuccess) return fail(AWE_EHIP, "misfit: %s", hipGetErrorString(e));
    return AWE_OK;
}

}  // extern "C"
