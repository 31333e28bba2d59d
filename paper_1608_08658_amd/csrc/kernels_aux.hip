// Off-grid point operators, coefficient build, gradient fold and reductions.
#include "awe_internal.hpp"

namespace awe {
namespace {

constexpr int kBlock = 256;

inline unsigned blocks_for(int64_t n, int64_t cap = 65535 * 8) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

// Off-grid point operators (Sec. IV, sparse-point insertion and
// interpolation), one launch for both.  Work items [0, nrows) inject, the
// rest sample:
//   injection (the transpose of the multilinear interpolation): one item per
//     touched grid node; the node's CSR row lists (point, weight) pairs in
//     ascending point order, so the sum is deterministic and needs no atomics.
//       field[node] += C[node] * scale * sum_e w_e values[pt_e]
//       imaging:  grad[node] += usnap[node] * (that same increment)
//       save-t:   grad[node] += (that same increment)        (usnap == NULL)
//   sampling: out[r] = scale * sum_k w[r][k] probe[node[r][k]].
// The injected and the sampled arrays must not alias: the engine samples
// u[n] (or mu[n+1]) while it injects into u[n+1] (or mu[n]).
__global__ void __launch_bounds__(kBlock)
sparse_k(InjectOp a, SampleOp b) {
    const int64_t total = (int64_t)a.nrows + b.npts;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < total; j += (int64_t)gridDim.x * kBlock) {
        // explicit fused multiply-adds: the stencil launch's fused form of
        // these operators (stencil_impl.hpp) computes the same expressions
        if (j < a.nrows) {
            float s = 0.f;
            for (int e = a.rowptr[j]; e < a.rowptr[j + 1]; ++e) s = __builtin_fmaf(a.w[e], a.values[a.pt[e]], s);
            const int64_t i = a.node[j];
            const float cs = s * a.scale;
            a.field[i] = __builtin_fmaf(a.coef[i], cs, a.field[i]);
            if (a.grad) {
                a.grad[i] = a.usnap ? __builtin_fmaf(a.usnap[i], a.coef[i] * cs, a.grad[i])   // imaging: g += u inc
                                    : __builtin_fmaf(a.coef[i], cs, a.grad[i]);               // save-t:  t += inc
            }
        } else {
            const int64_t r = j - a.nrows;
            float s = 0.f;
            for (int k = 0; k < b.corners; ++k)
                s = __builtin_fmaf(b.w[r * b.corners + k], b.field[b.node[r * b.corners + k]], s);
            b.out[r] = s * b.scale;
        }
    }
}

// The sum over shots of per-shot gradients (Eq. 2 sums the misfit over
// shots, so its gradient is the sum of theirs), in a fixed order: element i
// of out is sum_{p = 0..nparts-1} parts[p][i] accumulated in FP64 from
// parts[0] up and rounded once, whatever order the parts were computed in.
struct SumParts {
    const float* p[kMaxSumParts];
};
__global__ void __launch_bounds__(kBlock)
sum_parts_k(float* out, SumParts parts, int nparts, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        double acc = 0.0;
        for (int q = 0; q < nparts; ++q) acc += (double)parts.p[q][i];
        out[i] = (float)acc;
    }
}

struct PadGeo {
    int64_t n0, n1, n2;          // padded extents
    int64_t p0, p1, p2;          // physical extents
    int64_t sy, sz, origin;
    int nbl;
};

__device__ __forceinline__ int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

// C = dt^2 / (m + eta dt / 2) on the padded grid, in FP64 then rounded once.
// The absorbing layer takes m from the nearest physical edge cell.
__global__ void __launch_bounds__(kBlock)
coef_k(float* coef, const float* m, PadGeo g, const double* ez, const double* ey, const double* ex, double dt) {
    const int64_t total = g.n0 * g.n1 * g.n2;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
        const int64_t x = i % g.n2;
        const int64_t y = (i / g.n2) % g.n1;
        const int64_t z = i / (g.n2 * g.n1);
        const int64_t pz = clampi(z - g.nbl, 0, g.p0 - 1);
        const int64_t py = g.p1 > 1 ? clampi(y - g.nbl, 0, g.p1 - 1) : 0;
        const int64_t px = clampi(x - g.nbl, 0, g.p2 - 1);
        const double mv = (double)m[(pz * g.p1 + py) * g.p2 + px];
        const double eta = ez[z] + ey[y] + ex[x];
        coef[g.origin + z * g.sz + y * g.sy + x] = (float)(dt * dt / (mv + 0.5 * eta * dt));
    }
}

// Per-block min, max and non-finite count of the model (fixed block order).
__global__ void __launch_bounds__(kBlock)
minmax_k(const float* m, int64_t n, float* partial) {
    __shared__ float smin[kBlock], smax[kBlock], sbad[kBlock];
    float lo = INFINITY, hi = -INFINITY, bad = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const float v = m[i];
        if (!isfinite(v)) bad += 1.f;
        else { lo = fminf(lo, v); hi = fmaxf(hi, v); }
    }
    smin[threadIdx.x] = lo; smax[threadIdx.x] = hi; sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + s]);
            sbad[threadIdx.x] += sbad[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[3 * blockIdx.x + 0] = smin[0];
        partial[3 * blockIdx.x + 1] = smax[0];
        partial[3 * blockIdx.x + 2] = sbad[0];
    }
}

// Adjoint of the edge-replication padding, scaled: every physical cell gets
// scale * (sum of the padded cells that copy it), summed in FP64 in a fixed
// order.  Interior cells map to one padded cell, face cells gather a line of
// the layer (nbl + 1 cells); edge and corner cells gather a square or a cube
// of it and are left to fold_wide_k, one workgroup each, so that no thread
// sums a whole corner block alone.
struct FoldCell {
    int64_t z, y, x;                 // physical indices
    int64_t z_lo, z_hi, y_lo, y_hi, x_lo, x_hi;   // padded preimage
    int wide;                        // axes whose preimage has more than one cell
};
__device__ __forceinline__ FoldCell fold_cell(const PadGeo& p, int64_t i) {
    FoldCell c;
    c.x = i % p.p2;
    c.y = (i / p.p2) % p.p1;
    c.z = i / (p.p2 * p.p1);
    c.z_lo = (c.z == 0) ? 0 : c.z + p.nbl;
    c.z_hi = (c.z == p.p0 - 1) ? p.n0 - 1 : c.z + p.nbl;
    c.y_lo = c.y_hi = 0;
    if (p.p1 > 1) {
        c.y_lo = (c.y == 0) ? 0 : c.y + p.nbl;
        c.y_hi = (c.y == p.p1 - 1) ? p.n1 - 1 : c.y + p.nbl;
    }
    c.x_lo = (c.x == 0) ? 0 : c.x + p.nbl;
    c.x_hi = (c.x == p.p2 - 1) ? p.n2 - 1 : c.x + p.nbl;
    c.wide = (c.z_hi > c.z_lo) + (c.y_hi > c.y_lo) + (c.x_hi > c.x_lo);
    return c;
}

__global__ void __launch_bounds__(kBlock)
fold_k(float* grad, const float* g, PadGeo p, float scale) {
    const int64_t total = p.p0 * p.p1 * p.p2;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
        const FoldCell c = fold_cell(p, i);
        if (c.wide >= 2) continue;                  // fold_wide_k
        double s = 0.0;
        for (int64_t zz = c.z_lo; zz <= c.z_hi; ++zz)
            for (int64_t yy = c.y_lo; yy <= c.y_hi; ++yy) {
                const float* row = g + p.origin + zz * p.sz + yy * p.sy;
                for (int64_t xx = c.x_lo; xx <= c.x_hi; ++xx) s += (double)row[xx];
            }
        grad[i] = (float)(s * (double)scale);
    }
}

// One edge or corner cell per workgroup: each thread sums a fixed strided
// part of the preimage, then a fixed-order tree adds the parts.
__global__ void __launch_bounds__(kBlock)
fold_wide_k(float* grad, const float* g, PadGeo p, float scale, const int64_t* cells) {
    __shared__ double sh[kBlock];
    const int64_t i = cells[blockIdx.x];
    const FoldCell c = fold_cell(p, i);
    const int64_t ny = c.y_hi - c.y_lo + 1, nx = c.x_hi - c.x_lo + 1;
    const int64_t count = (c.z_hi - c.z_lo + 1) * ny * nx;
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < count; k += kBlock) {
        const int64_t zz = c.z_lo + k / (ny * nx), rem = k % (ny * nx);
        s += (double)g[p.origin + zz * p.sz + (c.y_lo + rem / nx) * p.sy + c.x_lo + rem % nx];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[i] = (float)(sh[0] * (double)scale);
}

__global__ void __launch_bounds__(kBlock)
pack_k(float* dense, const float* pitched, PadGeo g, float scale) {
    const int64_t total = g.n0 * g.n1 * g.n2;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
        const int64_t x = i % g.n2;
        const int64_t y = (i / g.n2) % g.n1;
        const int64_t z = i / (g.n2 * g.n1);
        dense[i] = scale * pitched[g.origin + z * g.sz + y * g.sy + x];
    }
}

// Edge-replication padding of a physical field onto the pitched padded grid.
__global__ void __launch_bounds__(kBlock)
pad_k(float* out, const float* m, PadGeo g) {
    const int64_t total = g.n0 * g.n1 * g.n2;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
        const int64_t x = i % g.n2;
        const int64_t y = (i / g.n2) % g.n1;
        const int64_t z = i / (g.n2 * g.n1);
        const int64_t pz = clampi(z - g.nbl, 0, g.p0 - 1);
        const int64_t py = g.p1 > 1 ? clampi(y - g.nbl, 0, g.p1 - 1) : 0;
        const int64_t px = clampi(x - g.nbl, 0, g.p2 - 1);
        out[g.origin + z * g.sz + y * g.sy + x] = m[(pz * g.p1 + py) * g.p2 + px];
    }
}

__global__ void __launch_bounds__(kBlock)
unpack_k(float* pitched, const float* dense, PadGeo g) {
    const int64_t total = g.n0 * g.n1 * g.n2;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
        const int64_t x = i % g.n2;
        const int64_t y = (i / g.n2) % g.n1;
        const int64_t z = i / (g.n2 * g.n1);
        pitched[g.origin + z * g.sz + y * g.sy + x] = dense[i];
    }
}

// Residual and per-block FP64 partial sums of its square (fixed order).
__global__ void __launch_bounds__(kBlock)
misfit_k(const float* tr, const float* obs, int64_t n, float* resid, double* partial) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const float r = tr[i] - obs[i];
        if (resid) resid[i] = r;
        acc += (double)r * (double)r;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(kBlock)
sum_partials_k(const double* partial, int nparts, double* result) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kBlock) acc += partial[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *result = 0.5 * sh[0];
}

__global__ void __launch_bounds__(kBlock)
fill_k(float* p, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = v;
}

PadGeo pad_geo(const Layout& L, const int64_t phys[3], int nbl) {
    PadGeo g;
    g.n0 = L.n[0]; g.n1 = L.n[1]; g.n2 = L.n[2];
    g.p0 = phys ? phys[0] : L.n[0];
    g.p1 = phys ? phys[1] : L.n[1];
    g.p2 = phys ? phys[2] : L.n[2];
    g.sy = L.sy; g.sz = L.sz; g.origin = L.origin;
    g.nbl = nbl;
    return g;
}

}  // namespace

hipError_t launch_sparse(const InjectOp& a, const SampleOp& b, hipStream_t s) {
    const int64_t total = (int64_t)a.nrows + b.npts;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(sparse_k, dim3(blocks_for(total)), dim3(kBlock), 0, s, a, b);
    return hipGetLastError();
}

hipError_t launch_coef(float* coef, const float* m_phys, const Layout& L, const int64_t phys[3], int nbl,
                       const double* eta_z, const double* eta_y, const double* eta_x, double dt, hipStream_t s) {
    PadGeo g = pad_geo(L, phys, nbl);
    hipLaunchKernelGGL(coef_k, dim3(blocks_for(L.points(), 8192)), dim3(kBlock), 0, s, coef, m_phys, g, eta_z, eta_y,
                       eta_x, dt);
    return hipGetLastError();
}

hipError_t launch_minmax(const float* m, int64_t n, float* partial, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(minmax_k, dim3(blocks), dim3(kBlock), 0, s, m, n, partial);
    return hipGetLastError();
}

hipError_t launch_fold(float* grad_phys, const float* g, const Layout& L, const int64_t phys[3], int nbl,
                       float scale, const int64_t* wide_cells, int32_t nwide, hipStream_t s) {
    PadGeo p = pad_geo(L, phys, nbl);
    hipLaunchKernelGGL(fold_k, dim3(blocks_for(p.p0 * p.p1 * p.p2, 8192)), dim3(kBlock), 0, s, grad_phys, g, p,
                       scale);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nwide <= 0) return e;
    hipLaunchKernelGGL(fold_wide_k, dim3((unsigned)nwide), dim3(kBlock), 0, s, grad_phys, g, p, scale, wide_cells);
    return hipGetLastError();
}

hipError_t launch_pack(float* dense, const float* pitched, const Layout& L, float scale, hipStream_t s) {
    PadGeo g = pad_geo(L, nullptr, 0);
    hipLaunchKernelGGL(pack_k, dim3(blocks_for(L.points(), 8192)), dim3(kBlock), 0, s, dense, pitched, g, scale);
    return hipGetLastError();
}

hipError_t launch_pad(float* pitched, const float* m_phys, const Layout& L, const int64_t phys[3], int nbl,
                      hipStream_t s) {
    PadGeo g = pad_geo(L, phys, nbl);
    hipLaunchKernelGGL(pad_k, dim3(blocks_for(L.points(), 8192)), dim3(kBlock), 0, s, pitched, m_phys, g);
    return hipGetLastError();
}

hipError_t launch_unpack(float* pitched, const float* dense, const Layout& L, hipStream_t s) {
    PadGeo g = pad_geo(L, nullptr, 0);
    hipLaunchKernelGGL(unpack_k, dim3(blocks_for(L.points(), 8192)), dim3(kBlock), 0, s, pitched, dense, g);
    return hipGetLastError();
}

hipError_t launch_misfit(const float* tr, const float* obs, int64_t n, float* resid, double* partial, int blocks,
                         double* result, hipStream_t s) {
    hipLaunchKernelGGL(misfit_k, dim3(blocks), dim3(kBlock), 0, s, tr, obs, n, resid, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_partials_k, dim3(1), dim3(kBlock), 0, s, partial, blocks, result);
    return hipGetLastError();
}

hipError_t launch_sum_parts(float* out, const float* const* parts, int nparts, int64_t n, hipStream_t s) {
    if (nparts < 1 || nparts > kMaxSumParts) return hipErrorInvalidValue;
    if (n <= 0) return hipSuccess;
    SumParts sp{};
    for (int q = 0; q < nparts; ++q) sp.p[q] = parts[q];
    hipLaunchKernelGGL(sum_parts_k, dim3(blocks_for(n, 16384)), dim3(kBlock), 0, s, out, sp, nparts, n);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_k, dim3(blocks_for(n, 16384)), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace awe
