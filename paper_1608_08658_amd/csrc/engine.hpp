// The plan object behind awe_plan and the engine's internal entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
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

struct LaunchShape {
    int cfg;        // workgroup shape (see launch_step)
    int zchunk;     // z planes per workgroup
};
LaunchShape default_shape(const Layout& L);

struct DeviceCsr {
    int64_t* node = nullptr;
    int32_t* rowptr = nullptr;
    int32_t* pt = nullptr;
    float* w = nullptr;
    int32_t nrows = 0;
};

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
    awe::LaunchShape fwd_shape{3, 56}, img_shape{3, 56};   // stencil launch shapes (forward / imaging)
    bool img_tuned = false;

    // device buffers owned by the plan
    std::vector<void*> owned;
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
    float* d_partial = nullptr;
    double* d_mpart = nullptr;

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
    bool have_ckpt = false, have_grad = false;

    ~awe_plan_s();
    awe_status init(const awe_geometry* geo);
    awe_status set_model(const float* m, hipStream_t s);
    awe_status forward(const float* wavelet, float* traces, int K, hipStream_t s);
    awe_status step(int n0, int nsteps, const float* wavelet, float* traces, hipStream_t s);
    awe_status adjoint(const float* resid, float* src_adj, float* grad_phys, hipStream_t s);
    awe_status born(const float* wavelet, const float* dm_phys, float* traces, hipStream_t s);

    awe_status alloc(void** p, size_t bytes);
    awe_status alloc_field(float** p);
    template <class T>
    awe_status upload(T** dst, const std::vector<T>& v);
    void release(void* p);
    awe_status advance(const float* uc, const float* up, float* out, const float* q_row, hipStream_t s);
    awe_status ensure_gradient_storage(int K);
    awe_status tune(bool img, hipStream_t user_stream);
    float* pick_work_dst();
};

namespace awe {
using Plan = awe_plan_s;
}
