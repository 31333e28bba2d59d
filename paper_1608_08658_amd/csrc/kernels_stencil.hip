// One time step of the damped acoustic scheme (Sec. V.A, Eq. 1 with the
// damping of Listing 1), forward or adjoint, optionally fused with the
// zero-lag imaging condition of the adjoint-state gradient (Eq. 3).
//
//   t   = C * L_P(uc) + a * (up - uc),        a = (eta_z + eta_y + eta_x) * C / dt
//   out = 2 uc - up + t                        (= (2-a) uc - (1-a) up + C L_P uc)
//   imaging:  grad += usnap * t               (t = mu[n] - 2 mu[n+1] + mu[n+2] without
//                                               the receiver term, which the injection adds)
//
// The adjoint of the scheme is the same update run backwards in time, so one
// kernel serves both directions.  Accumulating t instead of the second time
// difference of mu avoids the cancellation of three nearly equal FP32 values.
//
// Memory access plan (HBM-bound: 16 B per point forward, 28 B with imaging):
//   * a workgroup owns a 64 (x, one wavefront wide) x TY (y) column of the grid
//     and streams through a chunk of z planes;
//   * each thread keeps its points' z-neighbourhood (2M+1 planes) in registers,
//     so every value of uc is fetched from HBM once per z-chunk;
//   * the current plane, with an M-wide x/y halo, is staged in LDS (double
//     buffered, one barrier per plane) for the x and y derivatives; the halo
//     cells are re-read from L2 / the Infinity Cache, not HBM;
//   * the loads for plane z+1 are issued before the barrier of plane z so their
//     latency hides behind the arithmetic of plane z;
//   * each thread owns RY consecutive y rows, so y-neighbours inside its own
//     rows come from registers.
// 2-D uses the same scheme with a 64-point x row in LDS and no y axis.
#include "awe_internal.hpp"

namespace awe {
namespace {

__device__ __forceinline__ void lds_barrier() {
    // Orders the LDS writes of this plane before other waves read them.  Only
    // LDS needs to be visible across the workgroup; outstanding global loads
    // (the prefetch of the next plane) are left in flight.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

struct Geo3 {
    int32_t nz, ny, nx;
    int64_t sy, sz, origin;
};

template <int M, int BY, int RY, bool IMG>
__global__ void __launch_bounds__(kTileX * BY)
step3d(StepArgs a, StencilCoef k, Geo3 g, int zchunk) {
    constexpr int TY = BY * RY;
    constexpr int LW = kTileX + 2 * M;
    constexpr int LH = TY + 2 * M;
    constexpr int NQ = 2 * M + 1;
    constexpr int NH = (2 * M + BY - 1) / BY;     // y-halo rows per thread row
    __shared__ float lds[2][LH][LW];

    const int tx = threadIdx.x;
    const int ty = threadIdx.y;
    const int x = blockIdx.x * kTileX + tx;
    const int yb = blockIdx.y * TY;
    const int y0 = yb + ty * RY;
    const int z0 = blockIdx.z * zchunk;
    const int z1 = min(z0 + zchunk, g.nz);
    if (z0 >= z1) return;                          // uniform over the workgroup

    const int64_t sy = g.sy, sz = g.sz;
    const bool xin = x < g.nx;                     // this lane owns a grid point
    const bool xld = x < g.nx + M;                 // this lane's column is in the allocation
    bool rin[RY], rld[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        rin[r] = xin && (y0 + r < g.ny);
        rld[r] = xld && (y0 + r < g.ny + M);
    }
    // x halo: lanes tx < M load the left columns, lanes tx >= 64-M the right ones.
    const bool hl = tx < M;
    const bool hr = tx >= kTileX - M;
    const int hx = hl ? (blockIdx.x * kTileX - M + tx) : (blockIdx.x * kTileX + M + tx);
    const int hlx = hl ? tx : (tx + 2 * M);        // LDS column of the halo value
    const bool hxl = (hl || hr) && (hx < g.nx + M);
    // y halo: 2M rows (M above, M below the tile), 64 columns; thread row ty
    // loads halo rows h = ty, ty + BY, ... < 2M.
    int hyrow[NH];                                 // LDS row of each halo value
    bool hyl[NH];                                  // load it (valid and in the allocation)
    int64_t hyoff[NH];                             // its offset from the thread's row y0
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        const int h = ty + i * BY;
        const int y = (h < M) ? (yb - M + h) : (yb + TY + (h - M));
        hyrow[i] = (h < M) ? h : (TY + h);
        hyl[i] = (h < 2 * M) && xld && (y < g.ny + M);
        hyoff[i] = (int64_t)(y - y0) * sy;
    }

    const int64_t base = g.origin + (int64_t)y0 * sy + x;   // (z = 0, row y0, column x)
    const float* uc = a.uc + base;
    const float* up = a.up + base;
    float* out = a.out + base;
    const float* cf = a.coef + base;
    const float* us = IMG ? a.usnap + base : nullptr;
    float* gr = IMG ? a.grad + base : nullptr;
    const float* uch = a.uc + g.origin + (int64_t)y0 * sy + hx;   // x-halo column

    const float exv = xin ? a.eta_x[x] : 0.f;
    float eyv[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) eyv[r] = (y0 + r < g.ny) ? a.eta_y[y0 + r] : 0.f;

    // register queue of the z-neighbourhood: q[r][j] = uc(z - M + j)
    float q[RY][NQ];
#pragma unroll
    for (int j = 1; j < NQ; ++j) {
        const int64_t zo = (int64_t)(z0 - M + j - 1) * sz;
#pragma unroll
        for (int r = 0; r < RY; ++r) q[r][j] = rld[r] ? uc[zo + r * sy] : 0.f;
    }

    // prefetch registers for plane z
    float fr[RY], pv[RY], cv[RY], sv[RY], gv[RY], hxv[RY], hyv[NH];
    auto fetch = [&](int z) {
        const int64_t zo = (int64_t)z * sz;
        const int64_t zf = (int64_t)(z + M) * sz;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            fr[r] = rld[r] ? uc[zf + r * sy] : 0.f;
            pv[r] = rin[r] ? up[zo + r * sy] : 0.f;
            cv[r] = rin[r] ? cf[zo + r * sy] : 0.f;
            if (IMG) {
                sv[r] = rin[r] ? us[zo + r * sy] : 0.f;
                gv[r] = rin[r] ? gr[zo + r * sy] : 0.f;
            }
            hxv[r] = (hxl && (y0 + r < g.ny + M)) ? uch[zo + r * sy] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < NH; ++i) hyv[i] = hyl[i] ? uc[zo + hyoff[i]] : 0.f;
    };
    fetch(z0);

    for (int z = z0; z < z1; ++z) {
        const int b = (z - z0) & 1;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
#pragma unroll
            for (int j = 0; j < NQ - 1; ++j) q[r][j] = q[r][j + 1];
            q[r][NQ - 1] = fr[r];
        }
        // stage plane z in LDS
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            lds[b][M + ty * RY + r][M + tx] = q[r][M];
            if (hl || hr) lds[b][M + ty * RY + r][hlx] = hxv[r];
        }
#pragma unroll
        for (int i = 0; i < NH; ++i)
            if (ty + i * BY < 2 * M) lds[b][hyrow[i]][M + tx] = hyv[i];

        float p[RY], c[RY], s[RY], gg[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            p[r] = pv[r];
            c[r] = cv[r];
            if (IMG) { s[r] = sv[r]; gg[r] = gv[r]; }
        }
        if (z + 1 < z1) fetch(z + 1);
        lds_barrier();

        const float ezv = a.eta_z[z];
        const int64_t zo = (int64_t)z * sz;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int ly = M + ty * RY + r;
            const int lx = M + tx;
            float lap = k.c0 * q[r][M];
#pragma unroll
            for (int kk = 1; kk <= M; ++kk) {
                const float yu = (r - kk >= 0) ? q[(r - kk) >= 0 ? (r - kk) : 0][M] : lds[b][ly - kk][lx];
                const float yd = (r + kk < RY) ? q[(r + kk) < RY ? (r + kk) : 0][M] : lds[b][ly + kk][lx];
                lap += k.cz[kk] * (q[r][M - kk] + q[r][M + kk]);
                lap += k.cy[kk] * (yu + yd);
                lap += k.cx[kk] * (lds[b][ly][lx - kk] + lds[b][ly][lx + kk]);
            }
            const float u0 = q[r][M];
            const float av = (ezv + eyv[r] + exv) * c[r] * k.inv_dt;
            const float t = c[r] * lap + av * (p[r] - u0);
            if (rin[r]) {
                out[zo + r * sy] = (u0 - p[r]) + u0 + t;
                if (IMG) gr[zo + r * sy] = gg[r] + s[r] * t;
            }
        }
    }
}

struct Geo2 {
    int32_t nz, nx;
    int64_t sz, origin;
};

// 2-D: block = 64 x NW threads; wave w streams z planes [z0 + w*zchunk, ...).
template <int M, int NW, bool IMG>
__global__ void __launch_bounds__(kTileX * NW)
step2d(StepArgs a, StencilCoef k, Geo2 g, int zchunk) {
    constexpr int LW = kTileX + 2 * M;
    constexpr int NQ = 2 * M + 1;
    __shared__ float lds[2][NW][LW];

    const int tx = threadIdx.x;
    const int w = threadIdx.y;
    const int x = blockIdx.x * kTileX + tx;
    const int zw = (blockIdx.y * NW + w) * zchunk;        // first plane of this wave
    const int zend = min(zw + zchunk, g.nz);              // may be <= zw for idle waves
    const int64_t sz = g.sz;
    const bool xin = x < g.nx;
    const bool xld = x < g.nx + M;
    const bool hl = tx < M;
    const bool hr = tx >= kTileX - M;
    const int hx = hl ? (blockIdx.x * kTileX - M + tx) : (blockIdx.x * kTileX + M + tx);
    const int hlx = hl ? tx : (tx + 2 * M);
    const bool hxl = (hl || hr) && (hx < g.nx + M);

    const int64_t base = g.origin + x;
    const float* uc = a.uc + base;
    const float* up = a.up + base;
    float* out = a.out + base;
    const float* cf = a.coef + base;
    const float* us = IMG ? a.usnap + base : nullptr;
    float* gr = IMG ? a.grad + base : nullptr;
    const float* uch = a.uc + g.origin + hx;
    const float exv = xin ? a.eta_x[x] : 0.f;

    // planes z in [-M, nz + M) are in the allocation
    auto inz = [&](int z) { return z >= -M && z < g.nz + M; };
    float q[NQ];
#pragma unroll
    for (int j = 1; j < NQ; ++j) {
        const int z = zw - M + j - 1;
        q[j] = (xld && inz(z) && zw < g.nz) ? uc[(int64_t)z * sz] : 0.f;
    }
    float fr, pv, cv, sv = 0.f, gv = 0.f, hv;
    auto fetch = [&](int z) {
        const bool live = z < zend;
        const int64_t zo = (int64_t)z * sz;
        fr = (live && xld) ? uc[zo + (int64_t)M * sz] : 0.f;
        pv = (live && xin) ? up[zo] : 0.f;
        cv = (live && xin) ? cf[zo] : 0.f;
        if (IMG) {
            sv = (live && xin) ? us[zo] : 0.f;
            gv = (live && xin) ? gr[zo] : 0.f;
        }
        hv = (live && hxl) ? uch[zo] : 0.f;
    };
    fetch(zw);
    for (int i = 0; i < zchunk; ++i) {
        const int z = zw + i;
        const int b = i & 1;
#pragma unroll
        for (int j = 0; j < NQ - 1; ++j) q[j] = q[j + 1];
        q[NQ - 1] = fr;
        lds[b][w][M + tx] = q[M];
        if (hl || hr) lds[b][w][hlx] = hv;
        const float p = pv, c = cv, s = sv, gg = gv;
        if (i + 1 < zchunk) fetch(z + 1);
        lds_barrier();
        if (z < zend) {
            const int lx = M + tx;
            float lap = k.c0 * q[M];
#pragma unroll
            for (int kk = 1; kk <= M; ++kk) {
                lap += k.cz[kk] * (q[M - kk] + q[M + kk]);
                lap += k.cx[kk] * (lds[b][w][lx - kk] + lds[b][w][lx + kk]);
            }
            const float ezv = a.eta_z[z];
            const float u0 = q[M];
            const float av = (ezv + exv) * c * k.inv_dt;
            const float t = c * lap + av * (p - u0);
            if (xin) {
                out[(int64_t)z * sz] = (u0 - p) + u0 + t;
                if (IMG) gr[(int64_t)z * sz] = gg + s * t;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// launch-shape tables
// 3-D configurations: (BY, RY) -> workgroup 64 x BY threads, tile 64 x BY*RY.
// 2-D configurations: NW waves per workgroup.
// ---------------------------------------------------------------------------
template <int M, bool IMG>
hipError_t launch3(int cfg, const Layout& L, const StencilCoef& k, const StepArgs& a, int zchunk, hipStream_t s) {
    Geo3 g{(int32_t)L.n[0], (int32_t)L.n[1], (int32_t)L.n[2], L.sy, L.sz, L.origin};
    const unsigned gx = (unsigned)((L.n[2] + kTileX - 1) / kTileX);
    const unsigned gz = (unsigned)((L.n[0] + zchunk - 1) / zchunk);
    switch (cfg) {
        case 0: {   // 64 x 16 tile, 256 threads, 4 rows per thread
            dim3 grid(gx, (unsigned)((L.n[1] + 15) / 16), gz);
            hipLaunchKernelGGL((step3d<M, 4, 4, IMG>), grid, dim3(kTileX, 4), 0, s, a, k, g, zchunk);
            break;
        }
        case 1: {   // 64 x 8 tile, 256 threads, 2 rows per thread
            dim3 grid(gx, (unsigned)((L.n[1] + 7) / 8), gz);
            hipLaunchKernelGGL((step3d<M, 4, 2, IMG>), grid, dim3(kTileX, 4), 0, s, a, k, g, zchunk);
            break;
        }
        case 2: {   // 64 x 32 tile, 512 threads, 4 rows per thread
            dim3 grid(gx, (unsigned)((L.n[1] + 31) / 32), gz);
            hipLaunchKernelGGL((step3d<M, 8, 4, IMG>), grid, dim3(kTileX, 8), 0, s, a, k, g, zchunk);
            break;
        }
        default: {  // 64 x 16 tile, 512 threads, 2 rows per thread
            dim3 grid(gx, (unsigned)((L.n[1] + 15) / 16), gz);
            hipLaunchKernelGGL((step3d<M, 8, 2, IMG>), grid, dim3(kTileX, 8), 0, s, a, k, g, zchunk);
            break;
        }
    }
    return hipGetLastError();
}

template <int M, bool IMG>
hipError_t launch2(int cfg, const Layout& L, const StencilCoef& k, const StepArgs& a, int zchunk, hipStream_t s) {
    Geo2 g{(int32_t)L.n[0], (int32_t)L.n[2], L.sz, L.origin};
    const unsigned gx = (unsigned)((L.n[2] + kTileX - 1) / kTileX);
    const int nw = (cfg == 0) ? 4 : 1;
    const int64_t per_block = (int64_t)nw * zchunk;
    dim3 grid(gx, (unsigned)((L.n[0] + per_block - 1) / per_block));
    if (nw == 4)
        hipLaunchKernelGGL((step2d<M, 4, IMG>), grid, dim3(kTileX, 4), 0, s, a, k, g, zchunk);
    else
        hipLaunchKernelGGL((step2d<M, 1, IMG>), grid, dim3(kTileX, 1), 0, s, a, k, g, zchunk);
    return hipGetLastError();
}

template <bool IMG>
hipError_t dispatch(const Layout& L, const StencilCoef& k, const StepArgs& a, int cfg, int zchunk, hipStream_t s) {
    const bool d3 = L.ndim == 3;
#define AWE_CASE(MM) \
    case MM: return d3 ? launch3<MM, IMG>(cfg, L, k, a, zchunk, s) : launch2<MM, IMG>(cfg, L, k, a, zchunk, s);
    switch (L.half) {
        AWE_CASE(1) AWE_CASE(2) AWE_CASE(3) AWE_CASE(4)
        AWE_CASE(5) AWE_CASE(6) AWE_CASE(7) AWE_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef AWE_CASE
}

}  // namespace

int num_tile_cfgs(int ndim) { return ndim == 3 ? 4 : 2; }

int tile_rows(int ndim, int cfg) {
    if (ndim == 3) {
        static const int rows[4] = {16, 8, 32, 16};
        return rows[cfg & 3];
    }
    return cfg == 0 ? 4 : 1;
}

hipError_t launch_step(const Layout& L, const StencilCoef& k, const StepArgs& a, bool imaging, int cfg,
                       int zchunk, hipStream_t s) {
    if (zchunk < 1 || cfg < 0 || cfg >= num_tile_cfgs(L.ndim)) return hipErrorInvalidValue;
    return imaging ? dispatch<true>(L, k, a, cfg, zchunk, s) : dispatch<false>(L, k, a, cfg, zchunk, s);
}

}  // namespace awe
