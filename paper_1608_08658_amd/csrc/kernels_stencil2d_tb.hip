// 2-D forward steps in blocks: one launch advances up to tb_steps(M) time
// steps of the damped acoustic scheme (Sec. V.A, Eq. 1 with the damping of
// Listing 1), with the point source injected and the receivers sampled at
// every step inside the launch.
//
// A small 2-D grid (a 1000^2 field is 4 MB) takes a few microseconds per
// step, so a step per launch is bound by launch latency, not memory.  Here a
// workgroup owns a 32 x 32 tile and loads u[n] and u[n-1] on the tile plus
// an H = T*M halo into LDS; each of the T steps then updates a
// region M narrower on every side than the one before (overlapped temporal
// tiling: halo points are computed by every tile that needs them), so after
// T steps the tile itself holds u[n+T] and u[n+T-1], which are written out.
// Ghost points outside the padded grid stay zero, as in memory.
//
// Every point's update, injection increment and receiver sample is the same
// expression, over the same values in the same order, as in the one-step
// kernel and the point-operator kernel, so the two paths agree bit for bit.
#include "awe_internal.hpp"

namespace awe {
namespace {

constexpr int kTbTile = 32;
constexpr int kTbRecPerThread = 2;   // receivers per tile: at most 512
constexpr int kTbGroup = 4;          // rows per thread evaluated together

// Eight steps per launch (halo H = T*M of 8 points at order 2, 16 at order
// 4).  Measured against one step per launch (the tuned one-step kernel, 201
// steps, a source and 200 receivers): order 2 is 2.4x faster on
// 121^2..400^2 grids and 1.4-1.8x on 1040^2..2500^2; order 4 1.7-1.8x on
// 121^2..400^2 and 1.15-1.25x on 1040^2..1500^2 but slower from 1800^2 (the
// plan limits blocking by grid size accordingly).  Sixteen steps at order 2
// and four at order 4 were slower (by up to 9% and 10%); order 8 (two steps,
// halo 8) gained at most 13% on small grids and lost from 640^2, so
// blocking is used for orders 2 and 4.
template <int M>
constexpr int tb_T() { return M <= 2 ? 8 : 1; }

struct TbGeo {
    int32_t nz, nx;
    int64_t sz, origin;
};

template <int M, int T>
__global__ void __launch_bounds__(256)
step2d_tb(const float* __restrict__ uc, const float* __restrict__ up, float* __restrict__ out_c,
          float* __restrict__ out_p, const float* __restrict__ coef, const float* __restrict__ eta_z,
          const float* __restrict__ eta_x, StencilCoef k, TbGeo g, TbPoints p, int n0, int nsteps) {
    constexpr int H = M * T;
    constexpr int E = kTbTile + 2 * H;   // extended tile edge
    constexpr int NR = (E + 3) / 4;      // rows per thread (every 4th)
    constexpr int NC = (E + 63) / 64;    // columns per thread (every 64th)
    __shared__ float buf[2][E * E];
    __shared__ float inj_cs[kFuseMaxNodes][T];   // source increments of this launch's steps

    const int lane = threadIdx.x, wrow = threadIdx.y;   // block 64 x 4
    const int tid = wrow * 64 + lane;
    const int zlo = (int)blockIdx.y * kTbTile - H, xlo = (int)blockIdx.x * kTbTile - H;
    auto gidx = [&](int z, int x) { return g.origin + (int64_t)z * g.sz + x; };
    auto inside = [&](int ez, int ex) {
        const int z = zlo + ez, x = xlo + ex;
        return ez < E && ex < E && z >= 0 && z < g.nz && x >= 0 && x < g.nx;
    };

    // Each thread owns the points (wrow + 4i, lane + 64j) of the extended tile
    // for the whole launch and keeps their C and damping factor in registers.
    // Every load is issued unconditionally (points off the grid read grid
    // point (0, 0) and discard it), so they all go out before the first wait.
    float cf[NR][NC], av[NR][NC];
#pragma unroll
    for (int i0 = 0; i0 < NR; i0 += kTbGroup) {
        float lu[kTbGroup][NC], lp[kTbGroup][NC];
#pragma unroll
        for (int di = 0; di < kTbGroup; ++di) {
            const int i = i0 + di < NR ? i0 + di : NR - 1;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                const int ez = wrow + 4 * i, ex = lane + 64 * j;
                const bool in = inside(ez, ex);
                const int z = in ? zlo + ez : 0, x = in ? xlo + ex : 0;
                const int64_t gi = gidx(z, x);
                const float c = coef[gi], ev = eta_z[z] + eta_x[x];
                lu[di][j] = in ? uc[gi] : 0.f;
                lp[di][j] = in ? up[gi] : 0.f;
                cf[i][j] = in ? c : 0.f;
                av[i][j] = in ? ev * c : 0.f;   // the tables hold eta / dt
            }
        }
#pragma unroll
        for (int di = 0; di < kTbGroup; ++di) {
            if (i0 + di >= NR) continue;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                const int ez = wrow + 4 * (i0 + di), ex = lane + 64 * j;
                if (ez < E && ex < E) {
                    buf[0][ez * E + ex] = lu[di][j];
                    buf[1][ez * E + ex] = lp[di][j];
                }
            }
        }
    }
    // The point operators' data, read once per launch so that the steps touch
    // only LDS: the source rows' increments for every step and the node's C,
    // and up to kTbRecPerThread receivers per thread (the host keeps tiles
    // within that).
    const bool inj = p.wavelet && tid < p.nrows;
    int inj_ez = -1, inj_ex = -1;
    float inj_c = 0.f;
    if (inj) {
        inj_ez = p.src_zyx[3 * tid] - zlo;
        inj_ex = p.src_zyx[3 * tid + 2] - xlo;
        inj_c = coef[p.src_node[tid]];
        for (int st = 0; st < nsteps; ++st) {
            const float* vals = p.wavelet + (int64_t)(n0 + st) * p.nsrc;
            float acc = 0.f;
            for (int q = p.src_rowptr[tid]; q < p.src_rowptr[tid + 1]; ++q)
                acc = __builtin_fmaf(p.src_w[q], vals[p.src_pt[q]], acc);
            inj_cs[tid][st] = acc * p.src_scale;
        }
    }
    const int tile = (int)blockIdx.y * (int)gridDim.x + (int)blockIdx.x;
    int rec_r[kTbRecPerThread], rec_e[kTbRecPerThread];
    float rec_w[kTbRecPerThread][4];
    if (p.traces) {
        const int rb = p.tile_ptr[tile], rn = p.tile_ptr[tile + 1] - rb;
#pragma unroll
        for (int q = 0; q < kTbRecPerThread; ++q) {
            const int i = tid + 256 * q;
            rec_r[q] = i < rn ? p.tile_rec[rb + i] : -1;
            const int r = rec_r[q] < 0 ? 0 : rec_r[q];
            rec_e[q] = i < rn ? (p.rec_zx[2 * r] - zlo) * E + (p.rec_zx[2 * r + 1] - xlo) : 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) rec_w[q][c] = i < rn ? p.rec_w[4 * r + c] : 0.f;
        }
    }
    __syncthreads();

    float* cur = buf[0];
    float* prv = buf[1];
    for (int s = 0; s < nsteps; ++s) {
        // receivers whose lowest node is in this tile sample u[n0 + s]
        if (p.traces && s >= p.first_row) {
            float* row = p.traces + (int64_t)(n0 + s) * p.nrec;
#pragma unroll
            for (int q = 0; q < kTbRecPerThread; ++q) {
                if (rec_r[q] < 0) continue;
                float acc = 0.f;
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc = __builtin_fmaf(rec_w[q][c], cur[rec_e[q] + ((c >> 1) & 1) * E + (c & 1)], acc);
                row[rec_r[q]] = acc * p.rec_scale;
            }
        }
        // u[n0+s+1] over the region M narrower than the last, in place of
        // u[n0+s-1].  Branch-free in groups of kTbGroup rows: each point of a
        // group is evaluated at an address clamped into the readable interior
        // (so the group's LDS reads are in flight together), then the points
        // of the region are stored.  A point reads u[n0+s-1] only at itself,
        // so the stores need no barrier before the next group.
        const int lo = (s + 1) * M, hi = E - (s + 1) * M;
#pragma unroll
        for (int i0 = 0; i0 < NR; i0 += kTbGroup) {
            float nv[kTbGroup][NC];
#pragma unroll
            for (int di = 0; di < kTbGroup; ++di) {
                const int i = i0 + di < NR ? i0 + di : NR - 1;
                const int ez = wrow + 4 * i;
                const int ezc = min(max(ez, M), E - 1 - M);
#pragma unroll
                for (int j = 0; j < NC; ++j) {
                    const int ex = lane + 64 * j;
                    const int e = ezc * E + min(max(ex, M), E - 1 - M);
                    const float u0 = cur[e];
                    float lap = k.c0 * u0;
#pragma unroll
                    for (int kk = 1; kk <= M; ++kk) {
                        lap += k.cz[kk] * (cur[e - kk * E] + cur[e + kk * E]);
                        lap += k.cx[kk] * (cur[e - kk] + cur[e + kk]);
                    }
                    const float pv = prv[e];
                    const float c = cf[i][j];
                    // the update of step2d, rounding for rounding
                    const float d = pv - u0;
                    const float t = __builtin_fmaf(c, lap, av[i][j] * d);
                    nv[di][j] = (u0 - d) + t;
                }
            }
#pragma unroll
            for (int di = 0; di < kTbGroup; ++di) {
                if (i0 + di >= NR) continue;
                const int ez = wrow + 4 * (i0 + di);
#pragma unroll
                for (int j = 0; j < NC; ++j) {
                    const int ex = lane + 64 * j;
                    if (ez >= lo && ez < hi && ex >= lo && ex < hi && inside(ez, ex)) prv[ez * E + ex] = nv[di][j];
                }
            }
        }
        __syncthreads();
        // the source's increment for step n0+s, at its nodes inside that region
        if (p.wavelet && p.nrows > 0) {
            if (inj && inj_ez >= lo && inj_ez < hi && inj_ex >= lo && inj_ex < hi) {
                const int e = inj_ez * E + inj_ex;
                prv[e] = __builtin_fmaf(inj_c, inj_cs[tid][s], prv[e]);
            }
            __syncthreads();
        }
        float* tmp = cur;
        cur = prv;
        prv = tmp;
    }

    // the tile's u[n0+nsteps] and u[n0+nsteps-1]
    for (int ez = H + wrow; ez < H + kTbTile; ez += 4) {
        const int z = zlo + ez;
        if (z >= g.nz) break;
        for (int ex = H + lane; ex < H + kTbTile; ex += 64) {
            const int x = xlo + ex;
            if (x >= g.nx) continue;
            out_c[gidx(z, x)] = cur[ez * E + ex];
            out_p[gidx(z, x)] = prv[ez * E + ex];
        }
    }
}

template <int M>
hipError_t launch_tb_m(const Layout& L, const StencilCoef& k, const float* uc, const float* up, float* out_c,
                       float* out_p, const float* coef, const float* eta_z, const float* eta_x, const TbPoints& p,
                       int n0, int nsteps, hipStream_t s) {
    if (nsteps < 1 || nsteps > tb_T<M>()) return hipErrorInvalidValue;
    const TbGeo g{(int32_t)L.n[0], (int32_t)L.n[2], L.sz, L.origin};
    const dim3 grid((unsigned)((L.n[2] + kTbTile - 1) / kTbTile), (unsigned)((L.n[0] + kTbTile - 1) / kTbTile));
    hipLaunchKernelGGL((step2d_tb<M, tb_T<M>()>), grid, dim3(64, 4), 0, s, uc, up, out_c, out_p, coef, eta_z, eta_x,
                       k, g, p, n0, nsteps);
    return hipGetLastError();
}

}  // namespace

int tb_steps(int half) {
    switch (half) {
        case 1: return tb_T<1>();
        case 2: return tb_T<2>();
        default: return 1;   // no blocking
    }
}

int tb_tile() { return kTbTile; }
int tb_max_tile_receivers() { return 256 * kTbRecPerThread; }

hipError_t launch_step2d_tb(const Layout& L, const StencilCoef& k, const float* uc, const float* up, float* out_c,
                            float* out_p, const float* coef, const float* eta_z, const float* eta_x,
                            const TbPoints& p, int n0, int nsteps, hipStream_t s) {
    if (L.ndim != 2 || p.nrows < 0 || p.nrows > kFuseMaxNodes || (p.nrows > 0 && !p.src_zyx)) return hipErrorInvalidValue;
    if (out_c == uc || out_c == up || out_p == uc || out_p == up || out_c == out_p) return hipErrorInvalidValue;
    switch (L.half) {
        case 1: return launch_tb_m<1>(L, k, uc, up, out_c, out_p, coef, eta_z, eta_x, p, n0, nsteps, s);
        case 2: return launch_tb_m<2>(L, k, uc, up, out_c, out_p, coef, eta_z, eta_x, p, n0, nsteps, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace awe
