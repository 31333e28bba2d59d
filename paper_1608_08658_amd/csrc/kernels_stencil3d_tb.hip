// Two 3-D time steps per z-sweep (temporal blocking; the paper discusses
// time tiling in Sec. VI) of the damped acoustic scheme (Sec. V.A, Eq. 1
// with the damping of Listing 1), for space orders 2-8 and no point
// operators.  It is a measured prototype: bit-identical to two launches of
// the one-step kernel, and slower than them on every grid measured (the
// one-step kernel is bound by instruction issue and latency, not only by
// bytes, and this one does more of both), so no forward path uses it.
//
//   level 1: u[n+1] on the 64 x TY region of a workgroup (its owned
//            (64 - 2M) x (TY - 2M) tile plus M on every side), z planes
//            [z0 - M, z1 + M), set to zero outside the grid (the scheme's
//            boundary), written out at owned points;
//   level 2: u[n+2] on the owned tile, z planes [z0, z1), M planes behind
//            level 1: its x and y neighbours come from a ring of M + 1
//            level-1 planes in LDS, its z neighbours from a register queue.
// Every index is clamped into the zero ghost frame of the allocation, so a
// clamped load returns the exact value (0) of a point outside the grid.
// Each point's update is the same expression over the same values in the
// same order as in step3d, hence the bitwise agreement.
#include "stencil_impl.hpp"

namespace awe {
namespace {

struct GeoTb3 {
    int32_t nz, ny, nx;
    int64_t sy, sz;
    uint32_t yx0;                // element offset of (y, x) = (0, 0) within a plane: M * sy + kXOff
    uint32_t z0off;              // element offset of plane 0: M * sz
    uint32_t gx, gy, ntiles, ngrid;
    uint32_t bytes;              // allocation size in bytes (< 2^31)
};

template <int M, int BY, int RY>
__global__ void __launch_bounds__(64 * BY)
step3d_tb2(const float* uc, const float* up, float* o1, float* o2, const float* coef, const float* eta_z,
           const float* eta_y, const float* eta_x, StencilCoef k, GeoTb3 g, int zchunk) {
    constexpr int TX = 64, TY = BY * RY;
    constexpr int OX = TX - 2 * M, OY = TY - 2 * M;
    constexpr int LW = 128, LH = TY + 2 * M;
    constexpr int NQ = 2 * M + 1, NS = M + 1;
    constexpr int NH = (2 * M + BY - 1) / BY;
    constexpr bool kHyFull = (2 * M) % BY == 0;
    static_assert(TX + 2 * M <= LW && OY > 0, "tile too small for the half-width");
    // the double-buffered staging planes of u[n], then the ring of level-1
    // planes with a row of padding on each side (level-2 reads of lanes that
    // own no point stray up to M past a ring plane; their results are dropped)
    __shared__ float smem[2 * LH * LW + TX + NS * TY * TX + TX];
    auto stg = reinterpret_cast<float (*)[LH][LW]>(smem);
    auto ring = reinterpret_cast<float (*)[TY][TX]>(smem + 2 * LH * LW + TX);

    uint32_t bx, by, bz;
    {
        const uint32_t per = g.ngrid / kXcds;
        const uint32_t lin = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
        if (lin >= g.ntiles) return;
        bx = lin % g.gx;
        by = (lin / g.gx) % g.gy;
        bz = lin / (g.gx * g.gy);
    }
    const int tx = threadIdx.x;
    const int ty = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int xo0 = bx * OX, yo0 = by * OY;
    const int x = xo0 - M + tx;                    // this lane's level-1 column
    const int yb = yo0 - M;                        // first level-1 row of the tile
    const int y0 = yb + ty * RY;                   // this thread's first row
    const int z0 = bz * zchunk;
    const int z1 = min(z0 + zchunk, g.nz);
    if (z0 >= z1) return;

    const auto r_uc = slab_rsrc(uc, g.bytes), r_up = slab_rsrc(up, g.bytes), r_cf = slab_rsrc(coef, g.bytes);
    const auto r_o1 = slab_rsrc(o1, g.bytes), r_o2 = slab_rsrc(o2, g.bytes);
    auto cz_ = [&](int z) { return min(max(z, -M), g.nz + M - 1); };
    auto cy_ = [&](int y) { return min(max(y, -M), g.ny + M - 1); };
    auto cx_ = [&](int xx) { return min(max(xx, -M), g.nx + M - 1); };
    auto soff = [&](int z) { return (uint32_t)((g.z0off + (int64_t)cz_(z) * g.sz) * 4); };
    auto voff = [&](int y, int xx) { return (uint32_t)((g.yx0 + (int64_t)cy_(y) * g.sy + cx_(xx)) * 4); };

    const bool xin = x >= 0 && x < g.nx;
    const bool xown = tx >= M && tx < M + OX && x < g.nx;
    const bool wave_owns = ty * RY + RY > M && ty * RY < TY - M;   // owned rows in this wave
    uint32_t v_u[RY], v_st[RY];
    bool yin[RY];
    float eyv[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int y = y0 + r;
        v_u[r] = voff(y, x);
        yin[r] = y >= 0 && y < g.ny;
        const bool own = xown && y >= yo0 && y < yo0 + OY && y < g.ny;
        v_st[r] = own ? voff(y, x) : kOob;
        eyv[r] = yin[r] ? eta_y[y] : 0.f;
        asm volatile("" : "+v"(v_u[r]), "+v"(v_st[r]));
    }
    const float exv = xin ? eta_x[x] : 0.f;
    // x halo of the staged plane: lanes tx < M load x - M, lanes tx >= 64 - M load x + M
    const bool hl = tx < M, hr = tx >= TX - M;
    const int hlx = hl ? tx : (tx + 2 * M);
    uint32_t v_hx[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        v_hx[r] = (hl || hr) ? voff(y0 + r, hl ? x - M : x + M) : kOob;
        asm volatile("" : "+v"(v_hx[r]));
    }
    int hyrow[NH];
    uint32_t v_hy[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        const int h = ty + i * BY;
        const int y = (h < M) ? (yb - M + h) : (yb + TY + (h - M));
        hyrow[i] = (h < M) ? h : (TY + h);
        v_hy[i] = voff(y, x);
        asm volatile("" : "+v"(v_hy[i]));
    }

    // register queues, renamed by unrolling the plane loop NQ times: u[n]
    // (planes zl - M .. zl + M), level 1 (zl - 2M .. zl), C (zl - M .. zl)
    float q[RY][NQ], q2[RY][NQ], cq[RY][NQ];
    const int zs = z0 - M;                         // first level-1 plane
#pragma unroll
    for (int j = 1; j < NQ; ++j)
#pragma unroll
        for (int r = 0; r < RY; ++r) q[r][j] = bload(r_uc, v_u[r], soff(zs - M + j - 1));
#pragma unroll
    for (int j = 0; j < NQ; ++j)
#pragma unroll
        for (int r = 0; r < RY; ++r) q2[r][j] = cq[r][j] = 0.f;
    drain_vmem();

    struct Pre {
        float fr[RY], pv[RY], cv[RY], hxv[RY], hyv[NH], ezn;
    };
    Pre P;
    auto fetch = [&](int z) {
        P.ezn = (z >= 0 && z < g.nz) ? eta_z[z] : 0.f;
        const uint32_t so = soff(z), sf = soff(z + M);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            P.fr[r] = bload(r_uc, v_u[r], sf);
            P.pv[r] = bload<AWE_CPOL_STREAM>(r_up, v_u[r], so);
            P.cv[r] = bload<AWE_CPOL_STREAM>(r_cf, v_u[r], so);
            P.hxv[r] = bload(r_uc, v_hx[r], so);
        }
#pragma unroll
        for (int i = 0; i < NH; ++i)
            if (kHyFull || ty + i * BY < 2 * M) P.hyv[i] = bload(r_uc, v_hy[i], so);
    };
    const int zend = z1 + M;                       // level-1 planes [zs, zend)
    fetch(zs);

    auto one_plane = [&](auto ph, int zl) {
        constexpr int PH = decltype(ph)::value;
        auto Q = [&](int r, int j) -> float& { return q[r][(j + PH) % NQ]; };
        auto Q2 = [&](int r, int j) -> float& { return q2[r][(j + PH) % NQ]; };
        auto CQ = [&](int r, int j) -> float& { return cq[r][(j + PH) % NQ]; };
        const int b = (zl - zs) & 1;
#pragma unroll
        for (int r = 0; r < RY; ++r) Q(r, NQ - 1) = P.fr[r];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            stg[b][M + ty * RY + r][M + tx] = Q(r, M);
            if (hl || hr) stg[b][M + ty * RY + r][hlx] = P.hxv[r];
        }
#pragma unroll
        for (int i = 0; i < NH; ++i)
            if (kHyFull || ty + i * BY < 2 * M) stg[b][hyrow[i]][M + tx] = P.hyv[i];
        float p[RY], c[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            p[r] = P.pv[r];
            c[r] = P.cv[r];
        }
        const float ezv = P.ezn;
        if (zl + 1 < zend) fetch(zl + 1);
        // one barrier per plane orders the staging writes before the reads
        // of this plane, the ring write of plane zl - 1 before level 2 reads
        // it M planes later, and the last level-2 read of a ring slot before
        // level 1 overwrites it (the slot of zl last held zl - M - 1).  Ring
        // slots count from the chunk's first level-1 plane zs, which is
        // negative in a chunk that starts less than M planes into the grid:
        // a slot taken as zl % NS would then be negative and land in the
        // staging planes that other waves are reading.
        lds_barrier();

        // level 1: u[n+1](zl) on the whole region, 0 outside the grid
        const bool zin = zl >= 0 && zl < g.nz;
        const float ezx = ezv + exv;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const float* ly = &stg[b][M + ty * RY + r][M + tx];
            float lap = k.c0 * Q(r, M);
#pragma unroll
            for (int kk = 1; kk <= M; ++kk) {
                const float yu = (r - kk >= 0) ? Q((r - kk) >= 0 ? (r - kk) : 0, M) : ly[-kk * LW];
                const float yd = (r + kk < RY) ? Q((r + kk) < RY ? (r + kk) : 0, M) : ly[kk * LW];
                lap += k.cz[kk] * (Q(r, M - kk) + Q(r, M + kk));
                lap += k.cy[kk] * (yu + yd);
                lap += k.cx[kk] * (ly[-kk] + ly[kk]);
            }
            const float u0 = Q(r, M);
            const float d = p[r] - u0;
            const float av = (ezx + eyv[r]) * c[r];
            const float t = __builtin_fmaf(c[r], lap, av * d);
            const float v = (zin && xin && yin[r]) ? (u0 - d) + t : 0.f;
            Q2(r, NQ - 1) = v;
            CQ(r, M) = c[r];
            ring[(zl - zs) % NS][ty * RY + r][tx] = v;
            if (zl >= z0 && zl < z1) bstore<AWE_CPOL_STREAM>(r_o1, v, v_st[r], soff(zl));
        }
        // level 2: u[n+2](zl - M), once level 1 is M planes ahead
        const int z2 = zl - M;
        if (z2 >= z0 && wave_owns) {
            const float ezx2 = eta_z[z2] + exv;
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                const float* ly = &ring[(z2 - zs) % NS][ty * RY + r][tx];
                float lap = k.c0 * Q2(r, M);
#pragma unroll
                for (int kk = 1; kk <= M; ++kk) {
                    const float yu = (r - kk >= 0) ? Q2((r - kk) >= 0 ? (r - kk) : 0, M) : ly[-kk * TX];
                    const float yd = (r + kk < RY) ? Q2((r + kk) < RY ? (r + kk) : 0, M) : ly[kk * TX];
                    lap += k.cz[kk] * (Q2(r, M - kk) + Q2(r, M + kk));
                    lap += k.cy[kk] * (yu + yd);
                    lap += k.cx[kk] * (ly[-kk] + ly[kk]);
                }
                const float u1 = Q2(r, M);
                const float d = Q(r, 0) - u1;      // u[n](z2) - u[n+1](z2)
                const float c2 = CQ(r, 0);
                const float av = (ezx2 + eyv[r]) * c2;
                const float t = __builtin_fmaf(c2, lap, av * d);
                bstore<AWE_CPOL_STREAM>(r_o2, (u1 - d) + t, v_st[r], soff(z2));
            }
        }
    };
    int zl = zs;
    for (;;) {
        static_for<NQ>([&](auto s_) {
            constexpr int PH = (decltype(s_)::value + 1) % NQ;
            if (zl < zend) one_plane(std::integral_constant<int, PH>{}, zl);
            ++zl;
        });
        if (zl >= zend) break;
    }
}

// 16 wavefronts of two rows: a 64 x 32 level-1 region, (64 - 2M) x (32 - 2M)
// owned points (BY = 8 with four rows per thread was slower: two waves per
// SIMD instead of four)
constexpr int kTb3Waves = 16, kTb3Rows = 2;

template <int M>
hipError_t launch_tb3_m(const Layout& L, const StencilCoef& k, const float* uc, const float* up, float* o1, float* o2,
                        const float* coef, const float* ez, const float* ey, const float* ex, int zchunk, hipStream_t s) {
    constexpr int OX = 64 - 2 * M, OY = kTb3Waves * kTb3Rows - 2 * M;
    GeoTb3 g{(int32_t)L.n[0], (int32_t)L.n[1], (int32_t)L.n[2], L.sy, L.sz, (uint32_t)(M * L.sy + kXOff),
             (uint32_t)(M * L.sz), 0, 0, 0, 0, (uint32_t)(L.total * 4)};
    g.gx = (uint32_t)((L.n[2] + OX - 1) / OX);
    g.gy = (uint32_t)((L.n[1] + OY - 1) / OY);
    g.ntiles = g.gx * g.gy * (uint32_t)((L.n[0] + zchunk - 1) / zchunk);
    g.ngrid = (g.ntiles + kXcds - 1) / kXcds * kXcds;
    hipLaunchKernelGGL((step3d_tb2<M, kTb3Waves, kTb3Rows>), dim3(g.ngrid), dim3(64, kTb3Waves), 0, s, uc, up, o1, o2,
                       coef, ez, ey, ex, k, g, zchunk);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step3d_tb2(const Layout& L, const StencilCoef& k, const float* uc, const float* up, float* o1,
                             float* o2, const float* coef, const float* ez, const float* ey, const float* ex, int zchunk,
                             hipStream_t s) {
    if (L.ndim != 3 || zchunk < 1 || L.half < 1 || L.half > kTb3MaxHalf || L.total * 4 > 0x7FFFFFF0ll)
        return hipErrorInvalidValue;
    switch (L.half) {
        case 1: return launch_tb3_m<1>(L, k, uc, up, o1, o2, coef, ez, ey, ex, zchunk, s);
        case 2: return launch_tb3_m<2>(L, k, uc, up, o1, o2, coef, ez, ey, ex, zchunk, s);
        case 3: return launch_tb3_m<3>(L, k, uc, up, o1, o2, coef, ez, ey, ex, zchunk, s);
        default: return launch_tb3_m<4>(L, k, uc, up, o1, o2, coef, ez, ey, ex, zchunk, s);
    }
}

}  // namespace awe
