// One time step of linearised (Born) modelling in 3-D as a single z-sweep:
// the background step (Sec. V.A, Eq. 1 with the damping of Listing 1) and
// the scattered step driven by its second time difference advance together.
//
//   t   = C L_P(u) + a (u[n-1] - u[n])        u[n+1]  = 2 u[n] - u[n-1] + t
//   td  = C L_P(du) + a (du[n-1] - du[n]) - (C / dt^2) dm t
//                                             du[n+1] = 2 du[n] - du[n-1] + td
//
// with the source injected into u[n+1] and t at its nodes before td uses t.
// The save-t and born modes of step3d compute the same two updates in two
// launches, t going through memory; here it stays in a register: 32
// algorithmic bytes per point-step (read u[n], u[n-1], du[n], du[n-1], C, dm;
// write u[n+1], du[n+1]) instead of 44.  Every value is the same expression
// over the same operands in the same order as in the two launches (the
// injection the same fused multiply-adds as inj_apply), so the results are
// bit for bit the same.
//
// Workgroup: 64 x 8 threads, two rows each (a 64 x 16 tile), both fields
// staged in LDS with their x/y halo, each with its register z-queue; the
// receivers sample du[n] in workgroups appended to the tile grid.
#include "stencil_impl.hpp"

namespace awe {
namespace {

constexpr int kBornWaves = 8, kBornRows = 2;

// Orders 2-8 run the z loop in whole rounds of NQ planes without a per-plane
// guard and test each plane only in the chunk's last partial round (a
// guarded plane's join merges the refilled prefetch set through register
// copies that wait for the loads just issued).  At order 8 that needs 130
// VGPRs, one wave per SIMD fewer, unless the compiler is held to four waves
// per SIMD (128 VGPRs, three values spilled, reloaded once per round): 298 ->
// 292 ms for Born modelling at 336^3 (311 ms unbounded).  Orders 10-16 keep
// the guard: whole rounds would raise their registers past the next
// occupancy step.
template <int M>
__global__ void __launch_bounds__(kTileX * kBornWaves) __attribute__((amdgpu_waves_per_eu(M == 4 ? 4 : 1)))
born3d(BornArgs a, StencilCoef k, Geo3 g, int zchunk, FusedSparse fs) {
    constexpr bool kWholeRounds = M <= 4;
    constexpr int BY = kBornWaves, RY = kBornRows;
    constexpr int TY = BY * RY, LW = 128, LH = TY + 2 * M, NQ = 2 * M + 1;
    constexpr int NH = (2 * M + BY - 1) / BY;
    constexpr bool kHyFull = (2 * M) % BY == 0;
    static_assert(kTileX + 2 * M <= LW, "halo wider than the LDS row");
    __shared__ float lu[2][LH][LW];
    __shared__ float ld[2][LH][LW];

    if (blockIdx.x >= g.ngrid) {                   // a sampling workgroup
        fused_sample(fs.smp, (int64_t)(blockIdx.x - g.ngrid) * (kTileX * BY) + threadIdx.y * kTileX + threadIdx.x);
        return;
    }
    uint32_t bx, by, bz;
    if (!xcd_tile(g, bx, by, bz)) return;
    const int tx = threadIdx.x;
    const int ty = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int x = bx * kTileX + tx, yb = by * TY, y0 = yb + ty * RY;
    const int z0 = bz * zchunk, z1 = min(z0 + zchunk, g.nz);
    if (z0 >= z1) return;

    // slab descriptors and offsets exactly as in step3d
    const int64_t sy = g.sy, sz = g.sz;
    const int64_t slab = g.origin + (int64_t)(z0 - M) * sz - (int64_t)M * sy - M;
    const uint64_t left = (uint64_t)(g.total - slab) * 4u;
    const uint32_t bytes = left > 0x7FFFFFF0ull ? 0x7FFFFFF0u : (uint32_t)left;
    const auto r_u = slab_rsrc(a.u + slab, bytes), r_up = slab_rsrc(a.up + slab, bytes);
    const auto r_du = slab_rsrc(a.du + slab, bytes), r_dup = slab_rsrc(a.dup + slab, bytes);
    const auto r_cf = slab_rsrc(a.coef + slab, bytes), r_dm = slab_rsrc(a.dm + slab, bytes);
    const auto r_o = slab_rsrc(a.out + slab, bytes), r_do = slab_rsrc(a.dout + slab, bytes);
    const uint32_t plane = (uint32_t)(sz * 4);
    auto soff = [&](int z) { return (uint32_t)(z - z0 + M) * plane; };
    auto colb = [&](int xx) { return (uint32_t)((min(xx, g.nx + M - 1) + M) * 4); };
    auto rowb = [&](int y) { return (uint32_t)((int64_t)(min(y, g.ny + M - 1) + M) * sy * 4); };
    const uint32_t v_ld = colb(x);
    const uint32_t v_st = x < g.nx ? (uint32_t)((x + M) * 4) : kOob;
    const bool hl = tx < M, hr = tx >= kTileX - M;
    const int hlx = hl ? tx : (tx + 2 * M);
    const uint32_t v_hx = (hl || hr) ? colb(hl ? x - M : x + M) : kOob;
    uint32_t v_str[RY], v_pvr[RY], v_ldr[RY], v_hxr[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const uint32_t s_row = rowb(y0 + r);
        v_str[r] = (y0 + r < g.ny && x < g.nx) ? v_st + s_row : kOob;
        v_pvr[r] = x < g.nx ? v_st + s_row : kOob;
        v_ldr[r] = v_ld + s_row;
        v_hxr[r] = (hl || hr) ? v_hx + s_row : kOob;
        asm volatile("" : "+v"(v_str[r]), "+v"(v_pvr[r]), "+v"(v_ldr[r]), "+v"(v_hxr[r]));
    }
    int hyrow[NH];
    uint32_t v_hyr[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        const int h = ty + i * BY;
        const int y = (h < M) ? (yb - M + h) : (yb + TY + (h - M));
        hyrow[i] = (h < M) ? h : (TY + h);
        v_hyr[i] = v_ld + rowb(y);
        asm volatile("" : "+v"(v_hyr[i]));
    }
    // whether a source node lies in this workgroup's tile and chunk (uniform):
    // the per-plane injection below runs in those workgroups only, so the
    // others never wait on the node table's scalar loads (a copy of the
    // sweep without the injection for them took 40% more registers)
    bool wg_inj = false;
    for (int j = 0; j < fs.inj.nrows; ++j) {
        const int zj = fs.inj_zyx[3 * j], yj = fs.inj_zyx[3 * j + 1], xj = fs.inj_zyx[3 * j + 2];
        wg_inj = wg_inj || (zj >= z0 && zj < z1 && yj >= yb && yj < yb + TY && xj >= (int)bx * kTileX &&
                            xj < (int)bx * kTileX + kTileX);
    }
    const float exv = x < g.nx ? a.eta_x[x] : 0.f;
    float eyv[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) eyv[r] = (y0 + r < g.ny) ? a.eta_y[y0 + r] : 0.f;

    float q[RY][NQ], qd[RY][NQ];
#pragma unroll
    for (int j = 1; j < NQ; ++j)
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            q[r][j] = bload(r_u, v_ldr[r], soff(z0 - M + j - 1));
            qd[r][j] = bload(r_du, v_ldr[r], soff(z0 - M + j - 1));
        }
    drain_vmem();
    struct Pre {
        float fr[RY], fd[RY], pv[RY], pd[RY], cv[RY], mv[RY], hx[RY], hxd[RY], hy[NH], hyd[NH], ezn;
    };
    Pre P;
    auto fetch = [&](int z) {
        P.ezn = a.eta_z[z];
        const uint32_t so = soff(z), sf = soff(z + M);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            P.fr[r] = bload(r_u, v_ldr[r], sf);
            P.fd[r] = bload(r_du, v_ldr[r], sf);
            P.pv[r] = bload<AWE_CPOL_STREAM>(r_up, v_pvr[r], so);
            P.pd[r] = bload<AWE_CPOL_STREAM>(r_dup, v_pvr[r], so);
            P.cv[r] = bload<AWE_CPOL_STREAM>(r_cf, v_pvr[r], so);
            P.mv[r] = bload<AWE_CPOL_STREAM>(r_dm, v_pvr[r], so);
            P.hx[r] = bload(r_u, v_hxr[r], so);
            P.hxd[r] = bload(r_du, v_hxr[r], so);
        }
#pragma unroll
        for (int i = 0; i < NH; ++i)
            if (kHyFull || ty + i * BY < 2 * M) {
                P.hy[i] = bload(r_u, v_hyr[i], so);
                P.hyd[i] = bload(r_du, v_hyr[i], so);
            }
    };
    fetch(z0);

    auto one_plane = [&](auto ph, auto whole, int z) {
        constexpr int PH = decltype(ph)::value;
        auto Q = [&](int r, int j) -> float& { return q[r][(j + PH) % NQ]; };
        auto QD = [&](int r, int j) -> float& { return qd[r][(j + PH) % NQ]; };
        const int b = (z - z0) & 1;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            Q(r, NQ - 1) = P.fr[r];
            QD(r, NQ - 1) = P.fd[r];
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            lu[b][M + ty * RY + r][M + tx] = Q(r, M);
            ld[b][M + ty * RY + r][M + tx] = QD(r, M);
            if (hl || hr) {
                lu[b][M + ty * RY + r][hlx] = P.hx[r];
                ld[b][M + ty * RY + r][hlx] = P.hxd[r];
            }
        }
#pragma unroll
        for (int i = 0; i < NH; ++i)
            if (kHyFull || ty + i * BY < 2 * M) {
                lu[b][hyrow[i]][M + tx] = P.hy[i];
                ld[b][hyrow[i]][M + tx] = P.hyd[i];
            }
        float p[RY], pd[RY], c[RY], mm[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            p[r] = P.pv[r];
            pd[r] = P.pd[r];
            c[r] = P.cv[r];
            mm[r] = P.mv[r];
        }
        const float ezv = P.ezn;
        // inside a whole round the refill takes no branch: past the chunk's
        // end it loads the last plane again, unused
        if constexpr (decltype(whole)::value) fetch(min(z + 1, z1 - 1));
        else if (z + 1 < z1) fetch(z + 1);
        lds_barrier();

        const uint32_t so = soff(z);
        const float ezx = ezv + exv;
        float ou[RY], t[RY], av[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const float* lyu = &lu[b][M + ty * RY + r][M + tx];
            float lap = k.c0 * Q(r, M);
#pragma unroll
            for (int kk = 1; kk <= M; ++kk) {
                const float yu = (r - kk >= 0) ? Q((r - kk) >= 0 ? (r - kk) : 0, M) : lyu[-kk * LW];
                const float yd = (r + kk < RY) ? Q((r + kk) < RY ? (r + kk) : 0, M) : lyu[kk * LW];
                lap += k.cz[kk] * (Q(r, M - kk) + Q(r, M + kk));
                lap += k.cy[kk] * (yu + yd);
                lap += k.cx[kk] * (lyu[-kk] + lyu[kk]);
            }
            av[r] = (ezx + eyv[r]) * c[r];
            const float u0 = Q(r, M), d = p[r] - u0;
            t[r] = __builtin_fmaf(c[r], lap, av[r] * d);
            ou[r] = (u0 - d) + t[r];
        }
        // the source into u[n+1] and t at its nodes in this plane (the
        // arithmetic of inj_apply, with C, the stored value and t in registers)
        for (int j = 0; wg_inj && j < fs.inj.nrows; ++j) {
            if (fs.inj_zyx[3 * j] != z) continue;                 // uniform
            const int yj = fs.inj_zyx[3 * j + 1], xj = fs.inj_zyx[3 * j + 2];
            if (xj != x || yj < y0 || yj >= y0 + RY) continue;
            float sv = 0.f;
            for (int e = fs.inj.rowptr[j]; e < fs.inj.rowptr[j + 1]; ++e)
                sv = __builtin_fmaf(fs.inj.w[e], fs.inj.values[fs.inj.pt[e]], sv);
            const float cs = sv * fs.inj.scale;
#pragma unroll
            for (int r = 0; r < RY; ++r)
                if (yj == y0 + r) {
                    ou[r] = __builtin_fmaf(c[r], cs, ou[r]);
                    t[r] = __builtin_fmaf(c[r], cs, t[r]);
                }
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            bstore<AWE_CPOL_STREAM>(r_o, ou[r], v_str[r], so);
            const float* lyd = &ld[b][M + ty * RY + r][M + tx];
            float lapd = k.c0 * QD(r, M);
#pragma unroll
            for (int kk = 1; kk <= M; ++kk) {
                const float yu = (r - kk >= 0) ? QD((r - kk) >= 0 ? (r - kk) : 0, M) : lyd[-kk * LW];
                const float yd = (r + kk < RY) ? QD((r + kk) < RY ? (r + kk) : 0, M) : lyd[kk * LW];
                lapd += k.cz[kk] * (QD(r, M - kk) + QD(r, M + kk));
                lapd += k.cy[kk] * (yu + yd);
                lapd += k.cx[kk] * (lyd[-kk] + lyd[kk]);
            }
            const float w0 = QD(r, M), dd = pd[r] - w0;
            float td = __builtin_fmaf(c[r], lapd, av[r] * dd);
            td -= (c[r] * k.inv_dt2) * (mm[r] * t[r]);
            bstore<AWE_CPOL_STREAM>(r_do, (w0 - dd) + td, v_str[r], so);
        }
    };
    int z = z0;
    if constexpr (kWholeRounds) {
        while (z + NQ <= z1) {
            static_for<NQ>([&](auto s_) {
                one_plane(std::integral_constant<int, (decltype(s_)::value + 1) % NQ>{}, std::true_type{}, z);
                ++z;
            });
        }
        static_for<NQ>([&](auto s_) {
            if (z < z1) one_plane(std::integral_constant<int, (decltype(s_)::value + 1) % NQ>{}, std::false_type{}, z);
            ++z;
        });
    } else {
        for (;;) {
            static_for<NQ>([&](auto s_) {
                constexpr int PH = (decltype(s_)::value + 1) % NQ;
                if (z < z1) one_plane(std::integral_constant<int, PH>{}, std::false_type{}, z);
                ++z;
            });
            if (z >= z1) break;
        }
    }
}

template <int M>
hipError_t launch_born_m(const Layout& L, const StencilCoef& k, const BornArgs& a, int zchunk, hipStream_t s,
                         const FusedSparse& fs) {
    constexpr int TY = kBornWaves * kBornRows;
    Geo3 g{(int32_t)L.n[0], (int32_t)L.n[1], (int32_t)L.n[2], L.sy, L.sz, L.origin, 0, 0, 0, 0, L.total};
    g.gx = (uint32_t)((L.n[2] + kTileX - 1) / kTileX);
    g.gy = (uint32_t)((L.n[1] + TY - 1) / TY);
    g.ntiles = g.gx * g.gy * (uint32_t)((L.n[0] + zchunk - 1) / zchunk);
    g.ngrid = (g.ntiles + kXcds - 1) / kXcds * kXcds;
    const dim3 grid(g.ngrid + sample_groups(fs.smp.npts, kTileX * kBornWaves));
    hipLaunchKernelGGL((born3d<M>), grid, dim3(kTileX, kBornWaves), 0, s, a, k, g, zchunk, fs);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_born3d(const Layout& L, const StencilCoef& k, const BornArgs& a, int zchunk, hipStream_t s,
                         const FusedSparse& fs) {
    if (L.ndim != 3 || zchunk < 1 || fs.inj.nrows > kFuseMaxNodes || (fs.inj.nrows > 0 && !fs.inj_zyx))
        return hipErrorInvalidValue;
    switch (L.half) {
        case 1: return launch_born_m<1>(L, k, a, zchunk, s, fs);
        case 2: return launch_born_m<2>(L, k, a, zchunk, s, fs);
        case 3: return launch_born_m<3>(L, k, a, zchunk, s, fs);
        case 4: return launch_born_m<4>(L, k, a, zchunk, s, fs);
        case 5: return launch_born_m<5>(L, k, a, zchunk, s, fs);
        case 6: return launch_born_m<6>(L, k, a, zchunk, s, fs);
        case 7: return launch_born_m<7>(L, k, a, zchunk, s, fs);
        case 8: return launch_born_m<8>(L, k, a, zchunk, s, fs);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace awe
