// Host engine behind the C ABI of include/awe.h: validation, FD weights,
// stability limit, damping and off-grid tables, plans, and the forward /
// adjoint / gradient drivers with periodic checkpointing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <string>
#include <vector>

#include "awe.h"
#include "awe_internal.hpp"
#include "engine.hpp"
#include "tune_policy.hpp"

namespace awe {

thread_local std::string t_err;

awe_status fail(awe_status code, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

#define AWE_HIP(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) return fail(AWE_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// FD weights (Sec. IV.A, derivative expressions): central second derivative of order P = 2M,
//   c_k = 2 (-1)^(k+1) (M!)^2 / (k^2 (M-k)! (M+k)!),  c_0 = -2 sum_k c_k
// (closed form of Fornberg, Math. Comp. 1988).  For M <= 8 numerator and
// denominator are integers below 2^53, so each c_k is one correctly rounded
// division.
// ---------------------------------------------------------------------------
void fd_weights(int order, double* w) {
    const int m = order / 2;
    auto fact = [](int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; };
    double sum = 0.0;
    for (int k = 1; k <= m; ++k) {
        const double num = 2.0 * fact(m) * fact(m);
        const double den = double(k) * double(k) * fact(m - k) * fact(m + k);
        w[k] = ((k % 2) ? 1.0 : -1.0) * (num / den);
        sum += w[k];
    }
    w[0] = -2.0 * sum;
}

double dt_limit(int ndim, int order, const double* h, double vmax) {
    double c[kMaxHalf + 1];
    fd_weights(order, c);
    double s = std::fabs(c[0]);
    for (int k = 1; k <= order / 2; ++k) s += 2.0 * std::fabs(c[k]);
    double acc = 0.0;
    for (int a = 0; a < ndim; ++a) acc += s / (h[a] * h[a]);
    return 2.0 / (vmax * std::sqrt(acc));
}

awe_status validate(const awe_geometry* g) {
    if (!g) return fail(AWE_EINVAL, "geometry is NULL");
    if (g->ndim != 2 && g->ndim != 3) return fail(AWE_EINVAL, "ndim must be 2 or 3 (got %d)", g->ndim);
    if (g->space_order < 2 || g->space_order > 2 * kMaxHalf || g->space_order % 2)
        return fail(AWE_EINVAL, "space_order must be even in 2..16 (got %d)", g->space_order);
    if (g->nbl < 0 || g->nbl > 4096) return fail(AWE_EINVAL, "nbl must be in 0..4096 (got %d)", g->nbl);
    for (int a = 0; a < g->ndim; ++a) {
        if (g->shape[a] < 2 || g->shape[a] + 2 * (int64_t)g->nbl > (1 << 20))
            return fail(AWE_EINVAL, "shape[%d] = %lld out of range", a, (long long)g->shape[a]);
        if (!(g->spacing[a] > 0.0) || !std::isfinite(g->spacing[a]))
            return fail(AWE_EINVAL, "spacing[%d] must be positive and finite", a);
    }
    if (g->nbl > 0) {
        if (g->damp_power < 1 || g->damp_power > 4) return fail(AWE_EINVAL, "damp_power must be in 1..4");
        if (!(g->damp_R > 0.0 && g->damp_R < 1.0)) return fail(AWE_EINVAL, "damp_R must be in (0, 1)");
        if (!(g->damp_vref > 0.0) || !std::isfinite(g->damp_vref)) return fail(AWE_EINVAL, "damp_vref must be > 0");
    }
    if (!(g->dt > 0.0) || !std::isfinite(g->dt)) return fail(AWE_EINVAL, "dt must be positive and finite");
    if (g->nt < 1) return fail(AWE_EINVAL, "nt must be >= 1 (got %d)", g->nt);
    if (g->nsrc < 0 || g->nrec < 0) return fail(AWE_EINVAL, "nsrc and nrec must be >= 0");
    if (g->nsrc > 0 && !g->src_coords) return fail(AWE_EINVAL, "src_coords is NULL");
    if (g->nrec > 0 && !g->rec_coords) return fail(AWE_EINVAL, "rec_coords is NULL");
    if (g->reserved != 0) return fail(AWE_EINVAL, "reserved field must be 0");
    int64_t pts = 1;
    for (int a = 0; a < g->ndim; ++a) pts *= g->shape[a] + 2 * (int64_t)g->nbl;
    if (pts > (int64_t(1) << 33)) return fail(AWE_EINVAL, "padded grid too large");
    if ((int64_t)g->nt * std::max(g->nrec, g->nsrc) > (int64_t(1) << 34))
        return fail(AWE_EINVAL, "trace arrays too large");
    return AWE_OK;
}

// Padded extents in (z, y, x) order; y = 1 in 2-D.
void padded_zyx(const awe_geometry* g, int64_t pad[3], int64_t phys[3]) {
    if (g->ndim == 3) {
        for (int a = 0; a < 3; ++a) { phys[a] = g->shape[a]; pad[a] = g->shape[a] + 2 * (int64_t)g->nbl; }
    } else {
        phys[0] = g->shape[0]; phys[1] = 1; phys[2] = g->shape[1];
        pad[0] = phys[0] + 2 * (int64_t)g->nbl; pad[1] = 1; pad[2] = phys[2] + 2 * (int64_t)g->nbl;
    }
}

Layout make_layout(int ndim, const int64_t pad[3], int half) {
    Layout L;
    L.ndim = ndim;
    L.half = half;
    for (int a = 0; a < 3; ++a) L.n[a] = pad[a];
    const int64_t px = ((kXOff + pad[2] + half) + 31) / 32 * 32;
    const int64_t py = ndim == 3 ? pad[1] + 2 * half : 1;
    const int64_t yo = ndim == 3 ? half : 0;
    const int64_t pz = pad[0] + 2 * half;
    L.sy = px;
    L.sz = px * py;
    L.origin = half * L.sz + yo * L.sy + kXOff;
    L.total = pz * L.sz;
    return L;
}

// Times t whose wavefield the checkpointed forward keeps: the pairs
// (u[jK], u[jK-1]) for j = 1 .. S-1 (S = ceil(nt/K)); u[0] = u[-1] = 0 need no storage.
std::vector<int> stored_times(int nt, int K) {
    std::set<int> t;
    const int S = (nt + K - 1) / K;
    for (int j = 1; j < S; ++j) {
        if (j * K >= 1 && j * K <= nt - 1) t.insert(j * K);
        if (j * K - 1 >= 1 && j * K - 1 <= nt - 1) t.insert(j * K - 1);
    }
    return std::vector<int>(t.begin(), t.end());
}

int segment_slots(int nt, int K) { return std::max(0, std::min(K - 1, nt - 1)); }

// Upper bound on the source's grid nodes (its CSR rows): 2^d per source.
static int64_t src_node_bound(const awe_geometry* g) { return (int64_t)g->nsrc << g->ndim; }

bool tb_candidate(const awe_geometry* g, const Layout& L, int64_t src_nodes) {
    const int half = g->space_order / 2;
    const int64_t tb_max_points = half == 1 ? 8000000 : 2500000;
    return g->ndim == 2 && tb_steps(half) > 1 && L.points() <= tb_max_points && src_nodes <= kFuseMaxNodes;
}

// Every device byte a plan for g holds after a forward (K = 0) or after a
// gradient with checkpoints every K steps: the admission test of the server
// relies on this bounding the plan's allocations.
uint64_t footprint_bytes(const awe_geometry* g, int K) {
    int64_t pad[3], phys[3];
    padded_zyx(g, pad, phys);
    const Layout L = make_layout(g->ndim, pad, g->space_order / 2);
    const uint64_t field = (uint64_t)L.total * 4;
    const int corners = 1 << g->ndim;
    uint64_t b = 3 * field;                                                    // C, two wavefields
    b += (uint64_t)(pad[0] + pad[1] + pad[2]) * 12;                            // eta tables (fp32 + fp64)
    // point tables (node int64 + weight fp32) and the two CSR tables (node,
    // row start, point, weight), all with 2^d entries per point
    b += (uint64_t)(g->nsrc + g->nrec) * corners * (8 + 4) * 2 + 8 * corners * (g->nsrc + g->nrec + 2);
    if (src_node_bound(g) <= kFuseMaxNodes) b += (uint64_t)src_node_bound(g) * 3 * 4;   // source node (z, y, x)
    b += (uint64_t)fold_wide_cells(g->ndim, phys, g->nbl).size() * 8;          // gradient fold's wide cells
    b += 3 * 4096 * 4 + (kReduceBlocks + 1) * 8;                               // reduction partials
    if (tb_candidate(g, L, 0)) {
        // blocked steps (whenever the grid allows them, so the bound also
        // holds where the sources rule them out): two more fields, receivers'
        // base nodes and tile lists
        const int64_t t = tb_tile();
        b += 2 * field + (uint64_t)g->nrec * 12 + (uint64_t)((pad[0] + t - 1) / t * ((pad[2] + t - 1) / t) + 1) * 4;
    }
    if (K > 0) {
        b += (uint64_t)(stored_times(g->nt, K).size() + segment_slots(g->nt, K) + 3) * field;  // + mu x2, g
        b += (uint64_t)g->nt * g->nsrc * 4;                                    // wavelet copy
    }
    return b;
}

uint64_t footprint_binomial_bytes(const awe_geometry* g, int pool_fields) {
    int64_t pad[3], phys[3];
    padded_zyx(g, pad, phys);
    const Layout L = make_layout(g->ndim, pad, g->space_order / 2);
    const uint64_t field = (uint64_t)L.total * 4;
    return footprint_bytes(g, 0) + (uint64_t)(pool_fields + 3) * field + (uint64_t)g->nt * g->nsrc * 4;
}

// Physical cells whose padding preimage is wide along two or more axes (the
// edges and corners of the absorbing layer), in ascending linear order: the
// gradient fold gives each of them a workgroup of its own.
std::vector<int64_t> fold_wide_cells(int ndim, const int64_t phys[3], int nbl) {
    std::vector<int64_t> out;
    if (nbl <= 0) return out;
    const int64_t p0 = phys[0], p1 = phys[1], p2 = phys[2];
    auto edge = [](int64_t i, int64_t p) { return i == 0 || i == p - 1; };
    for (int64_t z = 0; z < p0; ++z)
        for (int64_t y = 0; y < p1; ++y) {
            const bool ez = edge(z, p0), ey = ndim == 3 && edge(y, p1);
            const int64_t base = (z * p1 + y) * p2;
            if (ez && ey) {
                for (int64_t x = 0; x < p2; ++x) out.push_back(base + x);
            } else if (ez || ey) {
                out.push_back(base);
                out.push_back(base + p2 - 1);
            }
        }
    return out;
}

// ---------------------------------------------------------------------------
// damping tables and off-grid point tables
// ---------------------------------------------------------------------------
std::vector<double> damping_axis(int64_t n, int nbl, double h, int power, double R, double vref) {
    std::vector<double> e(n + 2 * nbl, 0.0);
    if (nbl == 0) return e;
    const double emax = (power + 1) * std::log(1.0 / R) / (vref * nbl * h);
    for (int64_t i = 0; i < n + 2 * nbl; ++i) {
        const int64_t d = std::max<int64_t>({int64_t(nbl) - i, i - (n + nbl - 1), 0});
        e[i] = emax * std::pow(double(d) / nbl, power);
    }
    return e;
}

struct PointTable {
    std::vector<int64_t> node;   // [npts][corners] pitched indices
    std::vector<float> w;        // [npts][corners]
};

static awe_status build_points(const awe_geometry* g, const Layout& L, const double* coords, int npts,
                               const char* what, PointTable& out) {
    const int d = g->ndim;
    const int corners = 1 << d;
    out.node.resize((size_t)npts * corners);
    out.w.resize((size_t)npts * corners);
    int64_t padn[3];
    for (int a = 0; a < d; ++a) padn[a] = g->shape[a] + 2 * (int64_t)g->nbl;
    for (int p = 0; p < npts; ++p) {
        int64_t i0[3];
        double f[3];
        for (int a = 0; a < d; ++a) {
            const double s = coords[(size_t)p * d + a] / g->spacing[a] + g->nbl;
            if (!std::isfinite(s) || s < 0.0 || s > double(padn[a] - 1))
                return fail(AWE_EINVAL, "%s %d lies outside the padded grid on axis %d", what, p, a);
            int64_t b = (int64_t)std::floor(s);
            if (b > padn[a] - 2) b = padn[a] - 2;
            i0[a] = b;
            f[a] = s - double(b);
        }
        for (int c = 0; c < corners; ++c) {
            int64_t idx[3] = {0, 0, 0};
            double w = 1.0;
            for (int a = 0; a < d; ++a) {
                const int bit = (c >> (d - 1 - a)) & 1;   // axis 0 is the slowest bit
                idx[a] = i0[a] + bit;
                w *= bit ? f[a] : (1.0 - f[a]);
            }
            const int64_t lin = d == 3 ? L.index(idx[0], idx[1], idx[2]) : L.index(idx[0], 0, idx[1]);
            out.node[(size_t)p * corners + c] = lin;
            out.w[(size_t)p * corners + c] = (float)w;
        }
    }
    return AWE_OK;
}

struct CsrHost {
    std::vector<int64_t> node;
    std::vector<int32_t> rowptr, pt;
    std::vector<float> w;
};

// Group the (node, point, weight) triples by node, ascending node then point,
// so injection is a deterministic gather.
static CsrHost build_csr(const PointTable& t, int npts, int corners) {
    std::vector<std::pair<int64_t, int32_t>> keys;
    keys.reserve((size_t)npts * corners);
    for (int p = 0; p < npts; ++p)
        for (int c = 0; c < corners; ++c) keys.push_back({t.node[(size_t)p * corners + c], p * corners + c});
    std::sort(keys.begin(), keys.end());
    CsrHost h;
    for (size_t i = 0; i < keys.size(); ++i) {
        if (i == 0 || keys[i].first != keys[i - 1].first) {
            h.node.push_back(keys[i].first);
            h.rowptr.push_back((int32_t)h.pt.size());
        }
        h.pt.push_back(keys[i].second / corners);
        h.w.push_back(t.w[keys[i].second]);
    }
    h.rowptr.push_back((int32_t)h.pt.size());
    return h;
}

}  // namespace awe

using namespace awe;
using Plan = awe_plan_s;

// ---------------------------------------------------------------------------
// device memory helpers
// ---------------------------------------------------------------------------
void* BufferPool::take(size_t n) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = free_list.find(n);
    if (it == free_list.end()) return nullptr;
    void* p = it->second;
    free_list.erase(it);
    bytes -= n;
    return p;
}

void BufferPool::give(void* p, size_t n) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu);
    free_list.emplace(n, p);
    bytes += n;
}

void BufferPool::release_all() {
    std::lock_guard<std::mutex> lk(mu);
    for (auto& kv : free_list) (void)hipFree(kv.second);
    free_list.clear();
    bytes = 0;
}

uint64_t BufferPool::held() {
    std::lock_guard<std::mutex> lk(mu);
    return bytes;
}

awe_status Plan::alloc(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return AWE_OK;
    if (pool && (*p = pool->take(bytes))) {
        owned.push_back({*p, bytes});
        held += bytes;
        return AWE_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(AWE_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    owned.push_back({*p, bytes});
    held += bytes;
    return AWE_OK;
}

// A wavefield-sized buffer, zeroed once on stream s (the ghost cells must
// stay zero for the plan's lifetime); work that uses it later on s is ordered
// after the fill, so nothing waits for the device.
awe_status Plan::alloc_field(float** p, hipStream_t s) {
    awe_status st = alloc((void**)p, (size_t)L.total * sizeof(float));
    if (st) return st;
    AWE_HIP(launch_fill(*p, L.total, 0.f, s));
    return AWE_OK;
}

template <class T>
awe_status Plan::upload(T** dst, const std::vector<T>& v) {
    awe_status st = alloc((void**)dst, v.size() * sizeof(T));
    if (st) return st;
    if (v.empty()) return AWE_OK;
    AWE_HIP(hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, setup_stream));
    AWE_HIP(hipStreamSynchronize(setup_stream));   // v may be a temporary
    return AWE_OK;
}

void Plan::release(void* p) {
    if (!p) return;
    auto it = std::find_if(owned.begin(), owned.end(), [p](const std::pair<void*, size_t>& o) { return o.first == p; });
    if (it == owned.end()) return;   // not the plan's
    held -= it->second;
    if (pool) pool->give(p, it->second);
    else (void)hipFree(p);
    owned.erase(it);
}

Plan::~awe_plan_s() {
    for (auto& o : owned) {
        if (pool) pool->give(o.first, o.second);
        else (void)hipFree(o.first);
    }
    timer_reset();
    for (auto& pr : timer_free) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
}

void Plan::timer_reset() {
    for (auto& t : timer_pending) timer_free.push_back({t.a, t.b});
    timer_pending.clear();
    for (int i = 0; i < 3; ++i) timer_seen[i] = timer_count[i] = 0, timer_ms[i] = 0.0;
}

// Waits for the recorded launches and returns, per kind, the number timed
// and their mean duration in microseconds (out[2k], out[2k+1]).
awe_status Plan::kernel_times(double* out) {
    for (auto& t : timer_pending) {
        AWE_HIP(hipEventSynchronize(t.b));
        float ms = 0.f;
        AWE_HIP(hipEventElapsedTime(&ms, t.a, t.b));
        timer_ms[t.kind] += ms;
        ++timer_count[t.kind];
        timer_free.push_back({t.a, t.b});
    }
    timer_pending.clear();
    for (int k = 0; k < 3; ++k) {
        out[2 * k] = (double)timer_count[k];
        out[2 * k + 1] = timer_count[k] ? 1e3 * timer_ms[k] / (double)timer_count[k] : 0.0;
    }
    return AWE_OK;
}

// All set-up work runs on `setup` and init waits for that stream only, so a
// plan can be made while other streams keep the device busy.  `timed` =
// false keeps the autotuner from timing launches (for plans made among
// running work, where timings would be distorted and the caller stalled).
awe_status Plan::init(const awe_geometry* geo, hipStream_t setup, bool timed) {
    setup_stream = setup;
    timed_tune = timed;
    g = *geo;
    src.assign(geo->src_coords, geo->src_coords + (size_t)geo->nsrc * geo->ndim);
    rec.assign(geo->rec_coords, geo->rec_coords + (size_t)geo->nrec * geo->ndim);
    g.src_coords = src.data();
    g.rec_coords = rec.data();
    half = g.space_order / 2;
    corners = 1 << g.ndim;
    padded_zyx(&g, pad, phys);
    L = make_layout(g.ndim, pad, half);
    vol = 1.0;
    for (int a = 0; a < g.ndim; ++a) vol *= g.spacing[a];

    // stencil coefficients, axis order (z, y, x)
    double c[kMaxHalf + 1];
    fd_weights(g.space_order, c);
    double hz = g.spacing[0], hy = g.ndim == 3 ? g.spacing[1] : 0.0, hx = g.spacing[g.ndim - 1];
    std::memset(&k, 0, sizeof k);
    double inv_sum = 1.0 / (hz * hz) + 1.0 / (hx * hx) + (g.ndim == 3 ? 1.0 / (hy * hy) : 0.0);
    k.c0 = (float)(c[0] * inv_sum);
    for (int j = 1; j <= half; ++j) {
        k.cz[j] = (float)(c[j] / (hz * hz));
        k.cx[j] = (float)(c[j] / (hx * hx));
        k.cy[j] = g.ndim == 3 ? (float)(c[j] / (hy * hy)) : 0.f;
    }
    k.inv_dt = (float)(1.0 / g.dt);
    k.inv_dt2 = (float)(1.0 / (g.dt * g.dt));

    fwd_shape = img_shape = default_shape(L);

    // damping tables
    std::vector<double> ez, ey, ex;
    if (g.ndim == 3) {
        ez = damping_axis(g.shape[0], g.nbl, g.spacing[0], g.damp_power, g.damp_R, g.damp_vref);
        ey = damping_axis(g.shape[1], g.nbl, g.spacing[1], g.damp_power, g.damp_R, g.damp_vref);
        ex = damping_axis(g.shape[2], g.nbl, g.spacing[2], g.damp_power, g.damp_R, g.damp_vref);
    } else {
        ez = damping_axis(g.shape[0], g.nbl, g.spacing[0], g.damp_power, g.damp_R, g.damp_vref);
        ey.assign(1, 0.0);
        ex = damping_axis(g.shape[1], g.nbl, g.spacing[1], g.damp_power, g.damp_R, g.damp_vref);
    }

    // off-grid tables
    PointTable ts, tr;
    awe_status st;
    if ((st = build_points(&g, L, src.data(), g.nsrc, "source", ts))) return st;
    if ((st = build_points(&g, L, rec.data(), g.nrec, "receiver", tr))) return st;
    CsrHost cs = build_csr(ts, g.nsrc, corners);
    CsrHost cr = build_csr(tr, g.nrec, corners);

    int dev = 0;
    AWE_HIP(hipGetDevice(&dev));
    device = dev;
    if ((st = upload(&d_ezd, ez)) || (st = upload(&d_eyd, ey)) || (st = upload(&d_exd, ex))) return st;
    // the step kernels read eta / dt (one multiply fewer per point update)
    auto over_dt = [&](const std::vector<double>& v) {
        std::vector<float> o(v.size());
        for (size_t i = 0; i < v.size(); ++i) o[i] = (float)(v[i] / g.dt);
        return o;
    };
    if ((st = upload(&d_ez, over_dt(ez))) || (st = upload(&d_ey, over_dt(ey))) || (st = upload(&d_ex, over_dt(ex))))
        return st;
    if ((st = upload(&src_node, ts.node)) || (st = upload(&src_w, ts.w))) return st;
    if ((st = upload(&rec_node, tr.node)) || (st = upload(&rec_w, tr.w))) return st;
    if ((st = upload(&src_csr.node, cs.node)) || (st = upload(&src_csr.rowptr, cs.rowptr)) ||
        (st = upload(&src_csr.pt, cs.pt)) || (st = upload(&src_csr.w, cs.w)))
        return st;
    src_csr.nrows = (int32_t)cs.node.size();
    // grid indices (z, y, x) of the source nodes, for injection fused into the stencil
    if (src_csr.nrows > 0 && src_csr.nrows <= kFuseMaxNodes) {
        std::vector<int32_t> zyx;
        for (int64_t node : cs.node) {
            const int64_t rel = node - L.origin;
            const int64_t z = rel / L.sz, y = (rel % L.sz) / L.sy, x = (rel % L.sz) % L.sy;
            zyx.insert(zyx.end(), {(int32_t)z, (int32_t)y, (int32_t)x});
        }
        if ((st = upload(&src_zyx, zyx))) return st;
    }
    const char* fuse_env = std::getenv("AWE_FUSE");
    fuse_sparse = !(fuse_env && fuse_env[0] == '0');
    if ((st = upload(&rec_csr.node, cr.node)) || (st = upload(&rec_csr.rowptr, cr.rowptr)) ||
        (st = upload(&rec_csr.pt, cr.pt)) || (st = upload(&rec_csr.w, cr.w)))
        return st;
    rec_csr.nrows = (int32_t)cr.node.size();
    {
        const std::vector<int64_t> wide = fold_wide_cells(g.ndim, phys, g.nbl);
        if ((st = upload(&d_fold_cells, wide))) return st;
        n_fold_cells = (int32_t)wide.size();
    }
    // blocked 2-D steps where they beat one step per launch (measured: order
    // 2 up to 2500^2 = 6.25M points and beyond, order 4 up to 1500^2 but not
    // from 1800^2): receivers by tile of their lowest node, and two more fields
    const char* tb_env = std::getenv("AWE_TB");
    if (tb_candidate(&g, L, src_csr.nrows) && fuse_sparse && !(tb_env && tb_env[0] == '0') &&
        (src_csr.nrows == 0 || src_zyx)) {
        const int64_t tile = tb_tile(), gxn = (L.n[2] + tile - 1) / tile, gzn = (L.n[0] + tile - 1) / tile;
        std::vector<int32_t> zx(2 * (size_t)g.nrec), ptr(gxn * gzn + 1, 0), list(g.nrec), tile_of(g.nrec);
        for (int r = 0; r < g.nrec; ++r) {
            const int64_t rel = tr.node[(size_t)r * corners] - L.origin;   // corner 0: the lowest node
            const int64_t z = rel / L.sz, x = rel % L.sz;
            zx[2 * (size_t)r] = (int32_t)z;
            zx[2 * (size_t)r + 1] = (int32_t)x;
            tile_of[r] = (int32_t)((z / tile) * gxn + x / tile);
            ++ptr[tile_of[r] + 1];
        }
        int most = 0;
        for (size_t t = 1; t < ptr.size(); ++t) most = std::max(most, ptr[t]);
        for (size_t t = 1; t < ptr.size(); ++t) ptr[t] += ptr[t - 1];
        if (most <= tb_max_tile_receivers()) {   // else one step per launch
            std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
            for (int r = 0; r < g.nrec; ++r) list[fill[tile_of[r]]++] = r;
            if ((st = upload(&d_rec_zx, zx)) || (st = upload(&d_tile_ptr, ptr)) || (st = upload(&d_tile_rec, list)) ||
                (st = alloc_field(&w2, setup_stream)) || (st = alloc_field(&w3, setup_stream)))
                return st;
            tb_T = tb_steps(half);
        }
    }
    if ((st = alloc_field(&coef, setup_stream)) || (st = alloc_field(&w0, setup_stream)) ||
        (st = alloc_field(&w1, setup_stream)))
        return st;
    if ((st = alloc((void**)&d_partial, 3 * 4096 * sizeof(float)))) return st;
    if ((st = alloc((void**)&d_mpart, (kReduceBlocks + 1) * sizeof(double)))) return st;
    AWE_HIP(hipStreamSynchronize(setup_stream));
    setup_stream = nullptr;
    cur = w0;
    prev = w1;
    return tune(false, nullptr);
}

// ---------------------------------------------------------------------------
// Launch-shape autotuning (the GPU counterpart of the paper's block-size
// autotuning, Sec. IV.B, loop blocking): time each candidate workgroup shape and z-chunk
// length on this plan's own buffers and keep the fastest.  Every shape
// computes the same arithmetic per point, so the choice never changes results.
// Results are cached per (device, dimensions, order, padded grid, kernel).
// AWE_TILE="cfg,zchunk" forces a shape; AWE_AUTOTUNE=0 keeps the default.
// ---------------------------------------------------------------------------
namespace {
struct TuneKey {
    int dev, ndim, half, img;
    int64_t n0, n1, n2;
    bool operator<(const TuneKey& o) const {
        return std::tie(dev, ndim, half, img, n0, n1, n2) < std::tie(o.dev, o.ndim, o.half, o.img, o.n0, o.n1, o.n2);
    }
};
struct TuneEntry {
    LaunchShape shape;
    bool timed;     // false: borrowed from a nearby size
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune_cache;
// Smallest grids worth timing: a 3-D tuning pass times each of its up to 78
// candidates twice for about 1 ms (at least four launches), 0.2-0.4 s, a 2-D
// pass a few tens of milliseconds.
constexpr int64_t kTuneMinPoints3 = 4 << 20;
constexpr int64_t kTuneMinPoints2 = 1 << 16;

// A shape timed for a grid of the same dimensionality, order and mode with a
// point count within 30%, if there is one: taken instead of timing again (a
// server meets many nearby sizes).  The window is narrow because the best
// shape changes where the fields outgrow the 256 MB Infinity Cache (between
// 336^3 and 380^3 at order 8); even inside it a borrowed shape can be ~10%
// slower than the size's own, so plans that run long time their own.
bool nearby_shape(const TuneKey& key, LaunchShape& out) {
    const double pts = (double)key.n0 * key.n1 * key.n2;
    double best = 1.3;
    bool found = false;
    for (const auto& kv : g_tune_cache) {
        const TuneKey& o = kv.first;
        if (!kv.second.timed) continue;
        if (o.dev != key.dev || o.ndim != key.ndim || o.half != key.half || o.img != key.img) continue;
        const double r = std::max(pts, (double)o.n0 * o.n1 * o.n2) / std::min(pts, (double)o.n0 * o.n1 * o.n2);
        if (r <= best) {
            best = r;
            out = kv.second.shape;
            found = true;
        }
    }
    return found;
}
}  // namespace

// The shape used without timing (small grids, AWE_AUTOTUNE=0, plans made
// among running work).  Measured on 3-D grids of 64^3..464^3, orders
// 4/8/16: below ~300^3 points, 64x8 tiles with 8-plane chunks are the
// fastest or within 10% (long chunks leave small grids too few workgroups);
// above, 28-plane chunks are within 10% alone and the fastest with eight
// plans running at once, where the extra halo planes of short chunks cost
// up to 20%.  In 2-D, four-wave blocks of 4-row chunks are within 5% on
// 128^2..2040^2.
LaunchShape awe::default_shape(const Layout& L) {
    if (L.ndim != 3) return LaunchShape{0, 4};
    return LaunchShape{1, balanced_zchunk(L.n[0], L.points() < 27000000 ? 8 : 28)};
}

awe_status Plan::tune(bool img, hipStream_t user_stream) {
    LaunchShape& shape = img ? img_shape : fwd_shape;
    if (const char* env = std::getenv("AWE_TILE")) {
        int cfg = -1, zc = -1;
        if (std::sscanf(env, "%d,%d", &cfg, &zc) == 2 && cfg >= 0 && cfg < num_tile_cfgs(g.ndim) && zc > 0) {
            shape = {cfg, zc};
            return AWE_OK;
        }
    }
    const char* off = std::getenv("AWE_AUTOTUNE");
    if ((off && off[0] == '0') || L.points() < (g.ndim == 3 ? kTuneMinPoints3 : kTuneMinPoints2)) return AWE_OK;
    const TuneKey key{device, g.ndim, half, img ? 1 : 0, L.n[0], L.n[1], L.n[2]};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        LaunchShape near{};
        const bool nearby = g.ndim == 3 && nearby_shape(key, near);
        const ShapeSource src = shape_source(it != g_tune_cache.end(), it != g_tune_cache.end() && it->second.timed,
                                             nearby, timed_tune, own_tune);
        if (src == ShapeSource::kCached) {
            shape = it->second.shape;
            return AWE_OK;
        }
        if (src == ShapeSource::kBorrowed) {
            near.zchunk = balanced_zchunk(L.n[0], near.zchunk);   // the same chunk count, even here
            shape = near;
            g_tune_cache[key] = {near, false};
            return AWE_OK;
        }
        if (src == ShapeSource::kBuiltin) return AWE_OK;
    }
    std::vector<LaunchShape> cand;
    if (g.ndim == 3) {
        // chunks shorter than 28 planes only for the plain step: timed alone
        // they can win the imaging step too, but in the adjoint sweep (which
        // alternates with recomputed forward steps) they were ~3% slower
        // chunks balanced over the z extent (same count, equal lengths); long
        // chunks (a few per column) pay off on deep high-order grids: 64x32
        // tiles with two 240-plane chunks are the fastest 480^3 order-16 step;
        // 35 gives five chunks on 150-plane grids (30 planes each, the
        // fastest order-14 step on the 150 x 281 x 281 grid)
        for (int cfg : {0, 1, 2, 3, 4, 5}) {
            int last = -1;
            for (int zc : {8, 14, 21, 28, 35, 42, 56, 70, 84, 96, 120, 160, 240}) {
                const int bz = balanced_zchunk(L.n[0], zc);
                if ((img && zc < 28) || bz == last) continue;
                cand.push_back({cfg, bz});
                last = bz;
            }
        }
    } else {
        for (int zc : {4, 8, 16, 32, 64}) cand.push_back({0, zc});
        for (int zc : {8, 16, 32, 64}) cand.push_back({1, zc});
    }
    hipStream_t s = user_stream;
    bool own = false;
    if (!s) {
        AWE_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        own = true;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    awe_status st = AWE_OK;
    StepArgs a = img ? StepArgs{mu0, mu1, mu1, coef, d_ez, d_ey, d_ex, w0, grad}
                     : StepArgs{w0, w1, w1, coef, d_ez, d_ey, d_ex, nullptr, nullptr};
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // two interleaved rounds of timed launches (after one untimed); a
    // candidate's time is its faster round.  Each timing spans about 1 ms
    // (at least four launches): with four launches of a ~50 us step, run-to-run
    // noise let a 4% slower shape win now and then.
    std::vector<float> best_of(cand.size(), 1e30f);
    auto time_cand = [&](size_t i, int reps) {
        e = launch_step(L, k, a, img ? kStepImaging : kStepPlain, cand[i].cfg, cand[i].zchunk, s);
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int w = 0; w < reps && e == hipSuccess; ++w)
            e = launch_step(L, k, a, img ? kStepImaging : kStepPlain, cand[i].cfg, cand[i].zchunk, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        return e == hipSuccess ? ms / reps : 1e30f;
    };
    int reps = 4;
    if (e == hipSuccess && !cand.empty()) {
        const float per = time_cand(0, 4);     // a first estimate of one launch
        if (e == hipSuccess && per > 0.f && per < 1e29f)
            reps = std::max(4, std::min(32, (int)std::ceil(1.0f / per)));
    }
    for (int round = 0; round < 2 && e == hipSuccess; ++round)
        for (size_t i = 0; e == hipSuccess && i < cand.size(); ++i) {
            const float per = time_cand(i, reps);
            if (e == hipSuccess) best_of[i] = std::min(best_of[i], per);
        }
    // near-equal timings are a tie, settled by the longest z-chunk (tune_policy.hpp)
    const int pick = pick_timed_shape(cand.size(), best_of.data(), [&](size_t i) { return cand[i].zchunk; });
    const LaunchShape best = pick >= 0 ? cand[pick] : shape;
    if (e != hipSuccess) st = fail(AWE_EHIP, "autotune: %s", hipGetErrorString(e));
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (own) (void)hipStreamDestroy(s);
    if (st) return st;
    shape = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = {best, true};
    return AWE_OK;
}

awe_status Plan::set_model(const float* m, hipStream_t s) {
    if (!m) return fail(AWE_EINVAL, "model pointer is NULL");
    const int64_t n = phys[0] * phys[1] * phys[2];
    const int blocks = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256));
    AWE_HIP(launch_minmax(m, n, d_partial, blocks, s));
    std::vector<float> part(3 * (size_t)blocks);
    AWE_HIP(hipMemcpyAsync(part.data(), d_partial, part.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    AWE_HIP(hipStreamSynchronize(s));
    float lo = INFINITY, hi = -INFINITY, bad = 0.f;
    for (int b = 0; b < blocks; ++b) {
        lo = std::min(lo, part[3 * b]);
        hi = std::max(hi, part[3 * b + 1]);
        bad += part[3 * b + 2];
    }
    if (bad > 0.f) return fail(AWE_EUNSTABLE, "model has %.0f non-finite values", bad);
    if (!(lo > 0.f)) return fail(AWE_EUNSTABLE, "squared slowness must be positive (min %g)", lo);
    const double vmax = std::sqrt(1.0 / (double)lo);
    const double lim = dt_limit(g.ndim, g.space_order, g.spacing, vmax);
    if (g.dt > lim) return fail(AWE_EUNSTABLE, "dt = %g exceeds the stability limit %g (v_max = %g)", g.dt, lim, vmax);
    AWE_HIP(launch_coef(coef, m, L, phys, g.nbl, d_ezd, d_eyd, d_exd, g.dt, s));
    model_set = true;
    have_ckpt = false;
    have_grad = false;
    ++fwd_id;
    return AWE_OK;
}

// Injection of the source row q_row into field (none if q_row is NULL).
InjectOp Plan::src_op(float* field, const float* q_row, float* t_acc) const {
    InjectOp a;
    if (!q_row || g.nsrc == 0) return a;
    a.field = field;
    a.coef = coef;
    a.node = src_csr.node;
    a.rowptr = src_csr.rowptr;
    a.pt = src_csr.pt;
    a.w = src_csr.w;
    a.values = q_row;
    a.grad = t_acc;
    a.scale = (float)(1.0 / vol);
    a.nrows = src_csr.nrows;
    return a;
}

// Receiver sampling of field into row (none if row is NULL).
SampleOp Plan::rec_op(float* row, const float* field) const {
    SampleOp b;
    if (!row || g.nrec == 0) return b;
    b.out = row;
    b.field = field;
    b.node = rec_node;
    b.w = rec_w;
    b.npts = g.nrec;
    b.corners = corners;
    return b;
}

// One step of the recurrence from (uc, up) into out with the point source
// injected into out and, if rec_row is given, the receivers' samples of uc
// (the previous step's result, left untouched by this step) recorded into
// rec_row.  With few source nodes the stencil launch does both itself (one
// launch per step); otherwise a second launch follows it.
awe_status Plan::advance(const float* uc, const float* up, float* out, const float* q_row, float* rec_row,
                         hipStream_t s) {
    StepArgs a{uc, up, out, coef, d_ez, d_ey, d_ex, nullptr, nullptr};
    const InjectOp inj = src_op(out, q_row, nullptr);
    const SampleOp smp = rec_op(rec_row, uc);
    if (fuse_sparse && inj.nrows <= kFuseMaxNodes && (inj.nrows == 0 || src_zyx)) {
        FusedSparse fs;
        fs.inj = inj;
        fs.inj_zyx = src_zyx;
        fs.smp = smp;
        AWE_HIP(timed(0, s, [&] { return launch_step(L, k, a, kStepPlain, fwd_shape.cfg, fwd_shape.zchunk, s, &fs); }));
        return AWE_OK;
    }
    AWE_HIP(timed(0, s, [&] { return launch_step(L, k, a, kStepPlain, fwd_shape.cfg, fwd_shape.zchunk, s); }));
    AWE_HIP(timed(2, s, [&] { return launch_sparse(inj, smp, s); }));
    return AWE_OK;
}

// Steps n0 .. n0+nsteps-1 (nsteps <= tb_T) of a 2-D plain forward in one
// launch, with the source injected at each step and trace rows n0+s for s >=
// first_row recorded from u[n0+s].  The results go to two work buffers other
// than the current pair.
awe_status Plan::advance_tb(int n0, int nsteps, const float* wavelet, float* traces, int first_row, hipStream_t s) {
    float* outs[2] = {nullptr, nullptr};
    int n = 0;
    for (float* b : {w0, w1, w2, w3})
        if (b != cur && b != prev && n < 2) outs[n++] = b;
    TbPoints p;
    if (wavelet && g.nsrc > 0 && src_csr.nrows > 0) {
        p.wavelet = wavelet;
        p.nsrc = g.nsrc;
        p.nrows = src_csr.nrows;
        p.src_node = src_csr.node;
        p.src_rowptr = src_csr.rowptr;
        p.src_pt = src_csr.pt;
        p.src_w = src_csr.w;
        p.src_zyx = src_zyx;
        p.src_scale = (float)(1.0 / vol);
    }
    if (traces && g.nrec > 0) {
        p.traces = traces;
        p.nrec = g.nrec;
        p.first_row = first_row;
        p.rec_zx = d_rec_zx;
        p.rec_w = rec_w;
        p.tile_ptr = d_tile_ptr;
        p.tile_rec = d_tile_rec;
    }
    AWE_HIP(launch_step2d_tb(L, k, cur, prev, outs[0], outs[1], coef, d_ez, d_ex, p, n0, nsteps, s));
    cur = outs[0];
    prev = outs[1];
    return AWE_OK;
}

void Plan::release_periodic() {
    for (auto& kv : stored) release(kv.second);
    stored.clear();
    for (float* p : slots) release(p);
    slots.clear();
    ckpt_K = 0;
    storage_ready = false;
}

void Plan::release_binomial() {
    for (float* p : rev_pool) release(p);
    rev_pool.clear();
    rev_snaps = -1;
}

// Adjoint fields (mu pair, imaging accumulator) and the wavelet copy the
// reverse sweep's recomputation injects.
awe_status Plan::ensure_adjoint_storage(hipStream_t s) {
    awe_status st;
    if (!mu0 && ((st = alloc_field(&mu0, s)) || (st = alloc_field(&mu1, s)))) return st;
    if (!grad && (st = alloc_field(&grad, s))) return st;
    if (!wavelet_copy && g.nsrc > 0 && (st = alloc((void**)&wavelet_copy, (size_t)g.nt * g.nsrc * sizeof(float))))
        return st;
    return AWE_OK;
}

awe_status Plan::ensure_gradient_storage(int K, hipStream_t s) {
    release_binomial();
    if (K == ckpt_K && storage_ready) return AWE_OK;
    release_periodic();
    awe_status st;
    for (int t : stored_times(g.nt, K)) {
        float* p = nullptr;
        if ((st = alloc_field(&p, s))) return st;
        stored[t] = p;
    }
    for (int i = 0; i < segment_slots(g.nt, K); ++i) {
        float* p = nullptr;
        if ((st = alloc_field(&p, s))) return st;
        slots.push_back(p);
    }
    if ((st = ensure_adjoint_storage(s))) return st;
    ckpt_K = K;
    storage_ready = true;
    return AWE_OK;
}

awe_status Plan::ensure_binomial_storage(int snapshots, hipStream_t s) {
    release_periodic();
    awe_status st;
    if (rev_snaps != snapshots) {
        release_binomial();
        if ((st = binomial_prepare(rev, g.nt, snapshots))) return st;
        rev_snaps = snapshots;
    }
    while ((int)rev_pool.size() < rev.pool) {
        float* p = nullptr;
        if ((st = alloc_field(&p, s))) return st;
        rev_pool.push_back(p);
    }
    return ensure_adjoint_storage(s);
}

// The forward of awe_forward in two parts so that a caller (the shot server)
// can advance it a chunk of steps at a time: forward_begin sets up storage
// and the zero initial state, forward_advance takes up to max_steps steps and
// finishes the sweep after the last one.  The steps, their order and their
// buffers do not depend on how the sweep is cut.
awe_status Plan::forward_begin(const float* wavelet, float* traces, int K, hipStream_t s) {
    if (!model_set) return fail(AWE_ESTATE, "awe_set_model has not been called on this plan");
    if (g.nsrc > 0 && !wavelet) return fail(AWE_EINVAL, "wavelet is NULL but nsrc > 0");
    if (K < 0) return fail(AWE_EINVAL, "ckpt_every must be >= 0");
    awe_status st;
    have_ckpt = false;
    ++fwd_id;
    if (K > 0) {
        if ((st = ensure_gradient_storage(K, s))) return st;
        if (g.nsrc > 0)
            AWE_HIP(hipMemcpyAsync(wavelet_copy, wavelet, (size_t)g.nt * g.nsrc * sizeof(float),
                                   hipMemcpyDeviceToDevice, s));
    }
    AWE_HIP(launch_fill(w0, L.total, 0.f, s));
    AWE_HIP(launch_fill(w1, L.total, 0.f, s));
    cur = w0;
    prev = w1;
    fwd_job = FwdJob{wavelet, (traces && g.nrec > 0) ? traces : nullptr, K, 0, true};
    return AWE_OK;
}

awe_status Plan::forward_advance(int max_steps, hipStream_t s, bool* done) {
    FwdJob& j = fwd_job;
    *done = false;
    if (!j.active) return fail(AWE_ESTATE, "no forward sweep in progress");
    awe_status st;
    float* const tr = j.traces;
    const float* const wavelet = j.wavelet;
    // Trace row n is recorded in the launch that injects into u[n+1]; row 0
    // samples u[0] = 0 and the last row follows the loop.
    int budget = max_steps;
    if (j.K == 0 && tb_T > 0) {
        while (j.n + 1 < g.nt && budget > 0) {
            const int m = std::min(tb_T, g.nt - 1 - j.n);
            if ((st = advance_tb(j.n, m, g.nsrc ? wavelet : nullptr, tr, 0, s))) return st;
            j.n += m;
            budget -= m;
        }
    }
    for (; j.n + 1 < g.nt && budget > 0 && !(j.K == 0 && tb_T > 0); ++j.n, --budget) {
        const int n = j.n;
        float* dst = nullptr;
        if (j.K > 0) {
            auto it = stored.find(n + 1);
            if (it != stored.end()) dst = it->second;
        }
        if (!dst) dst = pick_work_dst();
        if ((st = advance(cur, prev, dst, g.nsrc ? wavelet + (size_t)n * g.nsrc : nullptr,
                          tr ? tr + (size_t)n * g.nrec : nullptr, s)))
            return st;
        prev = cur;
        cur = dst;
    }
    if (j.n + 1 < g.nt) return AWE_OK;
    if (tr) AWE_HIP(launch_sparse(InjectOp{}, rec_op(tr + (size_t)(g.nt - 1) * g.nrec, cur), s));
    have_ckpt = j.K > 0;
    rev_mode = false;
    j.active = false;
    *done = true;
    return AWE_OK;
}

awe_status Plan::forward(const float* wavelet, float* traces, int K, hipStream_t s) {
    awe_status st = forward_begin(wavelet, traces, K, s);
    bool done = false;
    while (!st && !done) st = forward_advance(1 << 30, s, &done);
    return st;
}

// The forward sweep of a binomial checkpointing schedule (checkpoint.cpp):
// the schedule's first descent is the plain forward from x_0 to x_(nt-1),
// storing its snapshots as it passes them.  The executor stops before the
// first visit; awe_adjoint runs the rest.
awe_status Plan::forward_binomial(const float* wavelet, float* traces, int snapshots, hipStream_t s) {
    if (!model_set) return fail(AWE_ESTATE, "awe_set_model has not been called on this plan");
    if (g.nsrc > 0 && !wavelet) return fail(AWE_EINVAL, "wavelet is NULL but nsrc > 0");
    if (snapshots < 0) return fail(AWE_EINVAL, "snapshots must be >= 0");
    have_ckpt = false;
    ++fwd_id;
    awe_status st;
    if ((st = ensure_binomial_storage(snapshots, s))) return st;
    if (g.nsrc > 0)
        AWE_HIP(hipMemcpyAsync(wavelet_copy, wavelet, (size_t)g.nt * g.nsrc * sizeof(float), hipMemcpyDeviceToDevice, s));
    AWE_HIP(launch_fill(w0, L.total, 0.f, s));   // x_0 = (0, 0)
    rev.rewind();
    float* const tr = (traces && g.nrec > 0) ? traces : nullptr;
    auto buf = [&](int b) { return b < 0 ? w0 : rev_pool[b]; };
    st = rev.run(
        true,
        [&](int n, int uc, int up, int out) {
            return advance(buf(uc), buf(up), buf(out), g.nsrc ? wavelet + (size_t)n * g.nsrc : nullptr,
                           tr ? tr + (size_t)n * g.nrec : nullptr, s);
        },
        [](int, int) { return AWE_OK; });
    if (st) return st;
    if (rev.t != g.nt - 1) return fail(AWE_EINVAL, "checkpoint schedule: forward sweep ended at %d", rev.t);
    if (tr) AWE_HIP(launch_sparse(InjectOp{}, rec_op(tr + (size_t)(g.nt - 1) * g.nrec, buf(rev.ua)), s));
    cur = buf(rev.ua);
    prev = buf(rev.ub);
    have_ckpt = true;
    rev_mode = true;
    return AWE_OK;
}

float* Plan::pick_work_dst() {
    if (prev == w0 || prev == w1 || (prev && (prev == w2 || prev == w3)))
        return const_cast<float*>(prev);   // in place over u[n-1]
    return cur == w0 ? w1 : w0;
}

awe_status Plan::step(int n0, int nsteps, const float* wavelet, float* traces, hipStream_t s) {
    if (!model_set) return fail(AWE_ESTATE, "awe_set_model has not been called on this plan");
    if (n0 < 0 || nsteps < 0 || (int64_t)n0 + nsteps > (int64_t)g.nt - 1)
        return fail(AWE_EINVAL, "steps %d..%d exceed nt-1 = %d", n0, n0 + nsteps, g.nt - 1);
    awe_status st;
    // Row n+1 receives the sample of u[n+1]: recorded by the next step's
    // injection launch, the last one after the loop.  Row n0 is not written.
    float* const tr = (traces && g.nrec > 0) ? traces : nullptr;
    if (tb_T > 0) {
        for (int n = n0; n < n0 + nsteps;) {
            const int m = std::min(tb_T, n0 + nsteps - n);
            if ((st = advance_tb(n, m, (wavelet && g.nsrc) ? wavelet : nullptr, tr, n == n0 ? 1 : 0, s))) return st;
            n += m;
        }
    }
    for (int n = n0; n < n0 + nsteps && tb_T == 0; ++n) {
        float* dst = pick_work_dst();
        if ((st = advance(cur, prev, dst, (wavelet && g.nsrc) ? wavelet + (size_t)n * g.nsrc : nullptr,
                          (tr && n > n0) ? tr + (size_t)n * g.nrec : nullptr, s)))
            return st;
        prev = cur;
        cur = dst;
    }
    if (tr && nsteps > 0)
        AWE_HIP(launch_sparse(InjectOp{}, rec_op(tr + (size_t)(n0 + nsteps) * g.nrec, cur), s));
    return AWE_OK;
}

// Two plain steps per z-sweep, npairs times (kernels_stencil3d_tb.hip): the
// state (u[n], u[n-1]) becomes (u[n+2], u[n+1]) per launch, bit for bit what
// two awe_step calls give for a plan without sources.  The outputs go to two
// work fields other than the state's, which then become the state.
awe_status Plan::step2_blocked(int npairs, int zchunk, hipStream_t s) {
    if (!model_set) return fail(AWE_ESTATE, "awe_set_model has not been called on this plan");
    if (g.ndim != 3 || half > kTb3MaxHalf)
        return fail(AWE_EINVAL, "two steps per sweep are built for 3-D grids of space order <= %d", 2 * kTb3MaxHalf);
    if (g.nsrc != 0) return fail(AWE_EINVAL, "two steps per sweep apply no point operators: the plan must have no sources");
    if (L.total * 4 > 0x7FFFFFF0ll) return fail(AWE_EINVAL, "two steps per sweep need fields under 2 GB");
    if (npairs < 0 || zchunk < 0) return fail(AWE_EINVAL, "npairs and zchunk must be >= 0");
    if (npairs == 0) return AWE_OK;
    const int zc = zchunk ? zchunk : balanced_zchunk(L.n[0], 56);
    float* bufs[4] = {w0, w1, w2, w3};
    for (int i = 2; i < 4; ++i)
        if (!bufs[i]) {
            const awe_status st = alloc_field(&bufs[i], s);
            if (st) return st;
        }
    w2 = bufs[2];
    w3 = bufs[3];
    for (int p = 0; p < npairs; ++p) {
        float* out[2];
        int nout = 0;
        for (float* b : bufs)
            if (b != cur && b != prev && nout < 2) out[nout++] = b;
        AWE_HIP(launch_step3d_tb2(L, k, cur, prev, out[0], out[1], coef, d_ez, d_ey, d_ex, zc, s));
        prev = out[0];
        cur = out[1];
    }
    return AWE_OK;
}

// Linearised (Born) modelling: J dm, the derivative of the traces with
// respect to m in the direction dm.  The background u and the scattered field
// du advance together: the background step also writes its second time
// difference t = u[n+1] - 2u[n] + u[n-1] (cancellation-free, the injected
// source included), and the scattered step adds -(C/dt^2) dm t.
awe_status Plan::born(const float* wavelet, const float* dm_phys, float* traces, hipStream_t s) {
    if (!model_set) return fail(AWE_ESTATE, "awe_set_model has not been called on this plan");
    if (!dm_phys) return fail(AWE_EINVAL, "dm is NULL");
    if (g.nsrc > 0 && !wavelet) return fail(AWE_EINVAL, "wavelet is NULL but nsrc > 0");
    awe_status st;
    if (!b_t && ((st = alloc_field(&b_t, s)) || (st = alloc_field(&b_du0, s)) || (st = alloc_field(&b_du1, s)) ||
                 (st = alloc_field(&b_dm, s))))
        return st;
    AWE_HIP(launch_pad(b_dm, dm_phys, L, phys, g.nbl, s));
    for (float* f : {w0, w1, b_du0, b_du1}) AWE_HIP(launch_fill(f, L.total, 0.f, s));
    float* const tr = (traces && g.nrec > 0) ? traces : nullptr;
    have_ckpt = false;
    ++fwd_id;
    cur = w0;
    prev = w1;
    float* dcur = b_du0;     // du[n]
    float* dprev = b_du1;    // du[n-1], overwritten in place by du[n+1]
    // 3-D Born launches take their own z-chunk (8 planes below 27M points,
    // as the built-in shape, else 56): the forward's tuned chunk can be long
    // (112 planes at 336^3 order 8), which leaves the one-sweep kernel, with
    // its larger register footprint, too few workgroups (396 against 301 ms
    // in 56-plane chunks)
    const int cfg = g.ndim == 3 ? 3 : 0;
    const int zc = g.ndim == 3 ? balanced_zchunk(L.n[0], L.points() < 27000000 ? 8 : 56) : fwd_shape.zchunk;
    // 3-D steps in one sweep for both fields (1.2-1.3x over the two launches
    // of the save-t and born modes at 336^3 order 8, bit-identical);
    // AWE_BORN_FUSED=0 keeps the two launches (for A/B tests)
    const char* bf = std::getenv("AWE_BORN_FUSED");
    const bool fused_born = g.ndim == 3 && fuse_sparse && !(bf && bf[0] == '0');
    for (int n = 0; n + 1 < g.nt; ++n) {
        float* dst = const_cast<float*>(prev);          // in place over u[n-1]
        StepArgs a{cur, prev, dst, coef, d_ez, d_ey, d_ex, nullptr, b_t};
        StepArgs b{dcur, dprev, dprev, coef, d_ez, d_ey, d_ex, b_dm, b_t};
        // the source into u[n+1] (and t); trace row n samples du[n]
        const InjectOp inj = src_op(dst, g.nsrc ? wavelet + (size_t)n * g.nsrc : nullptr, b_t);
        const SampleOp smp = rec_op(tr ? tr + (size_t)n * g.nrec : nullptr, dcur);
        if (fused_born && inj.nrows <= kFuseMaxNodes && (inj.nrows == 0 || src_zyx)) {
            // one sweep for both fields (3-D): t stays in a register
            FusedSparse f;
            f.inj = inj;
            f.inj_zyx = src_zyx;
            f.smp = smp;
            const BornArgs ba{cur, prev, dcur, dprev, coef, b_dm, d_ez, d_ey, d_ex, dst, dprev};
            AWE_HIP(launch_born3d(L, k, ba, zc, s, f));
        } else if (fuse_sparse && inj.nrows <= kFuseMaxNodes && (inj.nrows == 0 || src_zyx)) {
            // two launches per step: the background step injects, the scattered step samples
            FusedSparse fa, fb;
            fa.inj = inj;
            fa.inj_zyx = src_zyx;
            fb.smp = smp;
            AWE_HIP(launch_step(L, k, a, kStepSaveT, cfg, zc, s, &fa));
            AWE_HIP(launch_step(L, k, b, kStepBorn, cfg, zc, s, &fb));
        } else {
            AWE_HIP(launch_step(L, k, a, kStepSaveT, cfg, zc, s));
            AWE_HIP(launch_sparse(inj, smp, s));
            AWE_HIP(launch_step(L, k, b, kStepBorn, cfg, zc, s));
        }
        prev = cur;
        cur = dst;
        std::swap(dcur, dprev);
    }
    if (tr) AWE_HIP(launch_sparse(InjectOp{}, rec_op(tr + (size_t)(g.nt - 1) * g.nrec, dcur), s));
    return AWE_OK;
}

// mu[n] from (mu[n+1], mu[n+2]) in place over mu[n+2], then one launch that
// injects the residual row n into mu[n] and samples mu[n+1] (left untouched)
// at the sources into row n of the adjoint source.  With usnap = u[n] the
// step also accumulates the imaging condition.
awe_status Plan::adj_step(int n, const float* usnap, hipStream_t s) {
    AdjJob& j = adj_job;
    const bool img = usnap != nullptr;
    StepArgs a{j.m1, j.m2, j.m2, coef, d_ez, d_ey, d_ex, usnap, img ? grad : nullptr};
    const LaunchShape& sh = img ? img_shape : fwd_shape;
    AWE_HIP(timed(img ? 1 : 0, s, [&] { return launch_step(L, k, a, img ? kStepImaging : kStepPlain, sh.cfg, sh.zchunk, s); }));
    InjectOp inj;
    if (g.nrec > 0) {
        inj.field = j.m2;
        inj.coef = coef;
        inj.node = rec_csr.node;
        inj.rowptr = rec_csr.rowptr;
        inj.pt = rec_csr.pt;
        inj.w = rec_csr.w;
        inj.values = j.resid + (size_t)n * g.nrec;
        inj.usnap = usnap;
        inj.grad = img ? grad : nullptr;
        inj.nrows = rec_csr.nrows;
    }
    SampleOp smp;
    if (j.src_adj && g.nsrc > 0 && n <= g.nt - 2) {
        smp.out = j.src_adj + (size_t)n * g.nsrc;
        smp.field = j.m1;
        smp.node = src_node;
        smp.w = src_w;
        smp.scale = (float)(1.0 / vol);
        smp.npts = g.nsrc;
        smp.corners = corners;
    }
    AWE_HIP(timed(2, s, [&] { return launch_sparse(inj, smp, s); }));
    std::swap(j.m1, j.m2);
    return AWE_OK;
}

// The adjoint of awe_adjoint in two parts, like the forward: adjoint_begin
// checks the state and clears the adjoint fields, adjoint_advance takes up
// to max_steps steps (recomputed forward steps and adjoint steps both count)
// and finishes the sweep after the last.  F^T alone and the periodic
// checkpoint gradient resume where they stopped; a binomial gradient runs
// its whole schedule in one call.
awe_status Plan::adjoint_begin(const float* resid, float* src_adj, float* grad_phys, hipStream_t s) {
    if (!model_set) return fail(AWE_ESTATE, "awe_set_model has not been called on this plan");
    if (g.nrec > 0 && !resid) return fail(AWE_EINVAL, "resid is NULL but nrec > 0");
    const bool want_grad = grad_phys != nullptr;
    if (want_grad && !have_ckpt)
        return fail(AWE_ESTATE, "a gradient needs a preceding awe_forward with ckpt_every > 0");
    awe_status st;
    if (!mu0 && ((st = alloc_field(&mu0, s)) || (st = alloc_field(&mu1, s)))) return st;
    if (want_grad && !grad && (st = alloc_field(&grad, s))) return st;
    if (want_grad && rev_mode && rev.pos >= rev.sched.size())
        return fail(AWE_ESTATE, "the binomial checkpoints were used by an earlier gradient; run awe_forward_binomial again");
    if (want_grad && !img_tuned) {
        if ((st = tune(true, s))) return st;
        img_tuned = true;
    }
    AWE_HIP(launch_fill(mu0, L.total, 0.f, s));
    AWE_HIP(launch_fill(mu1, L.total, 0.f, s));
    if (want_grad) AWE_HIP(launch_fill(grad, L.total, 0.f, s));
    if (src_adj && g.nsrc > 0) AWE_HIP(launch_fill(src_adj + (size_t)(g.nt - 1) * g.nsrc, g.nsrc, 0.f, s));
    AdjJob& j = adj_job;
    j = AdjJob{};
    j.resid = resid;
    j.src_adj = src_adj;
    j.grad_phys = grad_phys;
    j.m1 = mu0;   // mu[n+1]
    j.m2 = mu1;   // mu[n+2]
    j.mode = !want_grad ? AdjJob::kTranspose : rev_mode ? AdjJob::kBinomial : AdjJob::kPeriodic;
    j.n = g.nt - 1;
    if (want_grad) {
        AWE_HIP(launch_fill(w0, L.total, 0.f, s));   // w0 serves as u[0] = u[-1] = 0
        const int K = ckpt_K;
        j.seg = j.mode == AdjJob::kPeriodic ? (g.nt + K - 1) / K - 1 : -1;
        j.seg_ready = false;
    }
    j.active = true;
    return AWE_OK;
}

awe_status Plan::adjoint_advance(int max_steps, hipStream_t s, bool* done) {
    AdjJob& j = adj_job;
    *done = false;
    if (!j.active) return fail(AWE_ESTATE, "no adjoint sweep in progress");
    awe_status st;
    float* const zero = w0;
    const float* qsrc = g.nsrc ? wavelet_copy : nullptr;
    int budget = max_steps;
    if (j.mode == AdjJob::kTranspose) {
        for (; j.n >= 0 && budget > 0; --j.n, --budget)
            if ((st = adj_step(j.n, nullptr, s))) return st;
        if (j.n >= 0) return AWE_OK;
        have_grad = false;
        j.active = false;
        *done = true;
        return AWE_OK;
    }
    if (j.mode == AdjJob::kBinomial) {
        // The rest of the binomial schedule: recompute forward steps from
        // stored states and visit t = nt-1 .. 0 with the adjoint step.
        auto buf = [&](int b) { return b < 0 ? zero : rev_pool[b]; };
        st = rev.run(
            false,
            [&](int n, int uc, int up, int out) {
                return advance(buf(uc), buf(up), buf(out), qsrc ? qsrc + (size_t)n * g.nsrc : nullptr, nullptr, s);
            },
            [&](int t, int uc) { return adj_step(t, t >= 1 ? buf(uc) : nullptr, s); });
        if (st) return st;
        AWE_HIP(launch_fold(j.grad_phys, grad, L, phys, g.nbl, (float)(-1.0 / (g.dt * g.dt)), d_fold_cells, n_fold_cells, s));
        cur = prev = zero;   // the wavefield state no longer holds u[nt-1]
        have_ckpt = false;
        ++fwd_id;            // the stored states are consumed
        have_grad = true;
        j.active = false;
        *done = true;
        return AWE_OK;
    }
    // Reverse sweep over segments [jK, min(jK+K, nt) - 1], j = S-1 .. 0: the
    // segment's states are recomputed into the slot buffers (stored states
    // are used in place), then visited from the last to the first.
    const int K = ckpt_K;
    while (j.seg >= 0 && budget > 0) {
        const int t0 = j.seg * K;
        const int t1 = std::min(t0 + K, g.nt) - 1;
        auto at = [&](int t) -> const float*& { return j.ptr[t - (t0 - 1)]; };   // u[t]
        if (!j.seg_ready) {
            j.ptr.assign(t1 - t0 + 2, nullptr);
            for (int t = t0 - 1; t <= t1; ++t) {
                if (t <= 0) at(t) = zero;
                else {
                    auto it = stored.find(t);
                    at(t) = it != stored.end() ? it->second : nullptr;
                }
            }
            j.slot = 0;
            j.t = t0 + 1;
            j.n = t1;
            j.seg_ready = true;
        }
        for (; j.t <= t1 && budget > 0; ++j.t) {
            if (at(j.t)) continue;
            float* dst = slots[j.slot++];
            if ((st = advance(at(j.t - 1), at(j.t - 2), dst, qsrc ? qsrc + (size_t)(j.t - 1) * g.nsrc : nullptr,
                              nullptr, s)))
                return st;
            at(j.t) = dst;
            --budget;
        }
        if (j.t <= t1) break;
        for (; j.n >= t0 && budget > 0; --j.n, --budget)
            if ((st = adj_step(j.n, j.n >= 1 ? at(j.n) : nullptr, s))) return st;
        if (j.n >= t0) break;
        --j.seg;
        j.seg_ready = false;
    }
    if (j.seg >= 0) return AWE_OK;
    // g_phys = fold(-(1/dt^2) * accumulated imaging)
    AWE_HIP(launch_fold(j.grad_phys, grad, L, phys, g.nbl, (float)(-1.0 / (g.dt * g.dt)), d_fold_cells, n_fold_cells, s));
    // w0 served as the zero field: the wavefield state is now (0, 0), as after
    // a binomial gradient (the stored states stay valid for another gradient)
    cur = prev = zero;
    have_grad = true;
    j.active = false;
    *done = true;
    return AWE_OK;
}

awe_status Plan::adjoint(const float* resid, float* src_adj, float* grad_phys, hipStream_t s) {
    awe_status st = adjoint_begin(resid, src_adj, grad_phys, s);
    bool done = false;
    while (!st && !done) st = adjoint_advance(1 << 30, s, &done);
    return st;
}
