// One time step of the damped acoustic scheme (Sec. V.A, Eq. 1 with the
// damping of Listing 1), forward or adjoint, optionally fused with the
// zero-lag imaging condition of the adjoint-state gradient (Eq. 3).
//
//   t   = C * L_P(uc) + a * (up - uc),        a = (eta_z + eta_y + eta_x) * C / dt
//   out = 2 uc - up + t                        (= (2-a) uc - (1-a) up + C L_P uc)
//
// The damping tables the kernels read hold eta / dt (scaled on the host), and
// 2 uc - up is formed as uc - (up - uc) from the difference the damping term
// uses: rounding of -(a - b) and b - a is the same, so this is (uc - up) + uc.
//
// Modes (template parameter MODE, see StepMode):
//   plain    just the update above;
//   imaging  grad += usnap * t            (t = mu[n] - 2 mu[n+1] + mu[n+2] without
//                                           the receiver term, which the injection adds);
//   save-t   grad = t                      (the background's second time difference
//                                           for linearised modelling, cancellation-free);
//   born     t -= (C / dt^2) * usnap * grad (usnap = dm, grad = the background's
//                                           second time difference): the scattered
//                                           field's source of linearised (Born) modelling.
//
// The adjoint of the scheme is the same update run backwards in time, so one
// kernel serves both directions.  Accumulating t instead of the second time
// difference of mu avoids the cancellation of three nearly equal FP32 values.
//
// Memory access plan (HBM-bound: 16 B per point forward, 28 B with imaging):
//   * a workgroup owns a TX (x: one or two wavefronts of 64 points) x TY (y)
//     column of the grid and streams through a chunk of z planes;
//   * each thread keeps its points' z-neighbourhood (2M+1 planes) in registers,
//     so every value of uc is fetched from HBM once per z-chunk;
//   * the current plane, with an M-wide x/y halo, is staged in LDS (double
//     buffered, one barrier per plane) for the x and y derivatives; the halo
//     cells are re-read from L2 / the Infinity Cache;
//   * the loads for plane z+1 (z+2 in plain steps of orders 10-16) are issued
//     before the barrier of plane z so their latency hides behind the
//     arithmetic of the planes in between;
//   * each thread owns RY consecutive y rows, so y-neighbours inside its own
//     rows come from registers;
//   * a wavefront owns 64 columns of one thread row; each lane keeps one
//     column-plus-row offset per row in a vector register, set once, and a
//     load's scalar offset carries the z plane alone;
//   * steps that load one plane ahead run the z loop in whole rounds of the
//     queue's period without a per-plane guard, so the loads of a plane stay
//     in flight across the plane computed meanwhile.
// A step may also carry its time step's point operators (FusedSparse):
// workgroups appended to the tile grid sample the input, and in plain and
// save-t steps the workgroup whose tile holds a source node adds the
// injection (to t as well in save-t) after its sweep.
// 2-D uses the same scheme with a 64-point x row in LDS and no y axis.
#pragma once

#include <type_traits>
#include <utility>

#include "awe_internal.hpp"

namespace awe {
namespace {

template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
// f(integral_constant<int, 0>) ... f(integral_constant<int, N-1>), unrolled.
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// s_waitcnt vmcnt(0) (gfx9 encoding: expcnt and lgkmcnt left at their maxima).
// Used once after the queue is filled: with no load of the prologue still in
// flight when the loop starts, the compiler's wait analysis does not carry
// them into the loop, where they would force a full drain on every plane.
__device__ __forceinline__ void drain_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

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
    uint32_t gx, gy, ntiles;     // tile grid (x tiles, y tiles) and total tiles incl. z chunks
    uint32_t ngrid;              // workgroups of the tile grid (ntiles rounded up to the XCD count);
                                 // workgroups past it sample (fused point operators)
    int64_t total;               // elements in each field's allocation
};

// Fused point operators of a plain step (FusedSparse): one receiver sample
// per thread of a sampling workgroup, and one injection row, each with the
// arithmetic of sparse_k (the same explicit fused multiply-adds).
__device__ __forceinline__ void fused_sample(const SampleOp& b, int64_t r) {
    if (r >= b.npts) return;
    float s = 0.f;
    for (int k = 0; k < b.corners; ++k) s = __builtin_fmaf(b.w[r * b.corners + k], b.field[b.node[r * b.corners + k]], s);
    b.out[r] = s * b.scale;
}
// Orders the workgroup's stores of its tile before any of its threads reads
// them back: every wave waits for its stores to complete (vector-memory
// counter at zero; gfx9 counts stores there) before the barrier, and the
// reader then reads through to L2.  The fences keep the compiler from moving
// memory operations across.
__device__ __forceinline__ void tile_stores_visible() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    drain_vmem();
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}
// Injection row j added to the output after the workgroup's sweep: the
// value the sweep stored (read from L2, past this CU's L1) plus the increment,
// and for a save-t step the increment added to t as well.  Only the
// workgroup whose tile holds the node touches it.
__device__ __forceinline__ void inj_apply(const InjectOp& a, int j) {
    float s = 0.f;
    for (int e = a.rowptr[j]; e < a.rowptr[j + 1]; ++e) s = __builtin_fmaf(a.w[e], a.values[a.pt[e]], s);
    const int64_t i = a.node[j];
    const float cs = s * a.scale;
    const float v = __hip_atomic_load(a.field + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a.field[i] = __builtin_fmaf(a.coef[i], cs, v);
    if (a.grad) {
        const float t = __hip_atomic_load(a.grad + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a.grad[i] = __builtin_fmaf(a.coef[i], cs, t);
    }
}

// Workgroups are dealt to the 8 XCDs round-robin by linear id, and each XCD
// has its own L2.  Remap so that XCD k runs the contiguous logical range
// [k*per, (k+1)*per) of tiles (x fastest, then y, then z chunk): tiles that
// share halo rows and columns then run at the same time on the same L2.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ bool xcd_tile(const Geo3& g, uint32_t& bx, uint32_t& by, uint32_t& bz) {
    const uint32_t per = g.ngrid / kXcds;
    const uint32_t lin = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    if (lin >= g.ntiles) return false;
    bx = lin % g.gx;
    by = (lin / g.gx) % g.gy;
    bz = lin / (g.gx * g.gy);
    return true;
}

// Raw buffer access.  A descriptor covers one workgroup's slab of a field;
// an offset at or beyond its size reads 0 and drops a store, so lanes with
// nothing to load or store are given kOob instead of a branch.  The z-plane
// offset is wave-uniform and goes in the scalar offset.
constexpr uint32_t kOob = 0xFFFFFFF0u;
constexpr int kRsrcWord3 = 0x00020000;   // gfx9 family: 32-bit data format

__device__ __forceinline__ __amdgpu_buffer_rsrc_t slab_rsrc(const float* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0, (int)bytes, kRsrcWord3);
}
// Cache policy of the arrays that are touched once per step (u[n-1], C, the
// output, and with imaging the snapshot and gradient): the wavefield planes
// re-read as halos and z-queue warm-up keep the default policy.
#ifndef AWE_CPOL_STREAM
#define AWE_CPOL_STREAM 2   // NT: stream through L2 with early eviction
#endif
template <int CPOL = 0>
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, CPOL));
}
template <int CPOL = 0>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, float v, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, CPOL);
}

template <int M, int BX, int BY, int RY, int MODE>
__global__ void __launch_bounds__(kTileX * BX * BY)
step3d(StepArgs a, StencilCoef k, Geo3 g, int zchunk, FusedSparse fs) {
    constexpr int TX = kTileX * BX;               // tile width: BX wavefronts side by side
    constexpr int TY = BY * RY;
    // LDS row pitch, a multiple of 64 dwords (128 for one wavefront): every
    // y-neighbour pair (y-k, y+k) is then one ds_read2st64 with immediate
    // offsets, instead of an address computation per pair
    constexpr int LW = BX == 1 ? 128 : 64 * ((TX + 2 * M + 63) / 64);
    static_assert(TX + 2 * M <= LW, "halo wider than the LDS row");
    constexpr int LH = TY + 2 * M;
    constexpr int NQ = 2 * M + 1;
    constexpr int NH = (2 * M + BY - 1) / BY;     // y-halo rows per thread row
    constexpr bool kHyFull = (2 * M) % BY == 0;   // every thread row has NH halo rows
    __shared__ float lds[2][LH][LW];

    if (blockIdx.x >= g.ngrid) {                   // a sampling workgroup
        fused_sample(fs.smp, (int64_t)(blockIdx.x - g.ngrid) * (kTileX * BX * BY) + threadIdx.y * kTileX + threadIdx.x);
        return;
    }
    uint32_t bx, by, bz;
    if (!xcd_tile(g, bx, by, bz)) return;          // uniform over the workgroup
    const int tx = threadIdx.x;
    // Each wavefront (64 lanes) owns 64 columns of RY rows: wave wv is column
    // block wx and thread row ty, so everything indexed by them is
    // wave-uniform and lives in scalar registers.
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int wx = wv % BX;
    const int ty = wv / BX;
    const int lxb = wx * kTileX;                   // tile-local first column of this wave
    const int x = bx * TX + lxb + tx;
    const int yb = by * TY;
    const int y0 = yb + ty * RY;
    const int z0 = bz * zchunk;
    const int z1 = min(z0 + zchunk, g.nz);
    if (z0 >= z1) return;

    // slab base: grid point (z0 - M, -M, -M); every access of this workgroup
    // lies at a non-negative offset from it and inside the allocation
    const int64_t sy = g.sy, sz = g.sz;
    const int64_t slab = g.origin + (int64_t)(z0 - M) * sz - (int64_t)M * sy - M;
    const uint64_t left = (uint64_t)(g.total - slab) * 4u;
    const uint32_t bytes = left > 0x7FFFFFF0ull ? 0x7FFFFFF0u : (uint32_t)left;
    const auto r_uc = slab_rsrc(a.uc + slab, bytes);
    const auto r_up = slab_rsrc(a.up + slab, bytes);
    const auto r_out = slab_rsrc(a.out + slab, bytes);
    const auto r_cf = slab_rsrc(a.coef + slab, bytes);
    const auto r_us = slab_rsrc((MODE == kStepImaging || MODE == kStepBorn) ? a.usnap + slab : a.uc + slab, bytes);
    const auto r_gr = slab_rsrc(MODE != kStepPlain ? a.grad + slab : a.out + slab, bytes);
    const uint32_t plane = (uint32_t)(sz * 4);     // bytes per z plane
    auto soff = [&](int z) { return (uint32_t)(z - z0 + M) * plane; };
    // Byte offsets from the slab base: column and row go in the per-lane
    // vector offset (one register per row, set once), the plane in the
    // scalar offset, so a load needs no address arithmetic and the rows hold
    // no scalar registers (with the 3M+2 stencil coefficients in scalar
    // registers, per-row scalar offsets made the compiler spill them).
    // Loads stay inside the allocation by construction: columns and rows are
    // clamped to the last ghost column / row, and no owned point uses a value
    // loaded from beyond them.  Lanes that own no point get kOob for the
    // arrays read only at owned points (reads 0) and for stores (dropped).
    auto colb = [&](int xx) { return (uint32_t)((min(xx, g.nx + M - 1) + M) * 4); };
    auto rowb = [&](int y) { return (uint32_t)((int64_t)(min(y, g.ny + M - 1) + M) * sy * 4); };
    const uint32_t v_ld = colb(x);
    const uint32_t v_st = x < g.nx ? (uint32_t)((x + M) * 4) : kOob;
    uint32_t s_row[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) s_row[r] = rowb(y0 + r);
    // per-row offsets: stores (kOob where the row owns no point: a branch per
    // row would split the unrolled plane into blocks the scheduler cannot
    // mix), arrays read at owned points, and the wavefield.  The empty asm
    // keeps each in a vector register instead of being recomputed per load.
    uint32_t v_str[RY], v_pvr[RY], v_ldr[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        v_str[r] = (y0 + r < g.ny && x < g.nx) ? v_st + s_row[r] : kOob;
        v_pvr[r] = x < g.nx ? v_st + s_row[r] : kOob;
        v_ldr[r] = v_ld + s_row[r];
        asm volatile("" : "+v"(v_str[r]), "+v"(v_pvr[r]), "+v"(v_ldr[r]));
    }
    // x halo: lanes tx < M of the first wave column load the left columns,
    // lanes tx >= 64-M of the last the right ones.
    const bool hl = wx == 0 && tx < M;
    const bool hr = wx == BX - 1 && tx >= kTileX - M;
    // LDS column of the x-halo value.  In the order-16 plain step every lane
    // writes one: lanes without a halo value write the 0 they loaded into
    // their own column, which the plane value written next overwrites (a
    // wave's LDS writes complete in order), so the write needs no exec-mask
    // branch (0.4-0.8% in the best 480^3 shape; 9% slower at order 14).
    constexpr bool kHaloAll = M == 8 && MODE == kStepPlain;
    const int hlx = hl ? tx : (hr || !kHaloAll) ? (lxb + tx + 2 * M) : (M + lxb + tx);
    const uint32_t v_hx = (hl || hr) ? colb(hl ? x - M : x + M) : kOob;
    uint32_t v_hxr[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        v_hxr[r] = (hl || hr) ? v_hx + s_row[r] : kOob;
        asm volatile("" : "+v"(v_hxr[r]));
    }
    // y halo: 2M rows (M above, M below the tile); thread row ty loads halo
    // rows h = ty, ty + BY, ... < 2M in its wave's 64 columns.
    int hyrow[NH];
    uint32_t s_hy[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        const int h = ty + i * BY;
        const int y = (h < M) ? (yb - M + h) : (yb + TY + (h - M));
        hyrow[i] = (h < M) ? h : (TY + h);
        s_hy[i] = rowb(y);
    }
    uint32_t v_hyr[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        v_hyr[i] = v_ld + s_hy[i];
        asm volatile("" : "+v"(v_hyr[i]));
    }

    const float exv = x < g.nx ? a.eta_x[x] : 0.f;
    float eyv[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) eyv[r] = (y0 + r < g.ny) ? a.eta_y[y0 + r] : 0.f;


    // Loads run PF planes ahead of the plane computed: one plane for low
    // orders, two for plain steps of orders 10-16, where one plane of
    // arithmetic does not cover the load latency (the order-14 and order-16
    // steps wait on memory for ~40% of a wave's life with one plane).
    constexpr int PF = (M >= 5 && MODE == kStepPlain) ? 2 : 1;
    // register queue of the z-neighbourhood: logical slot j holds uc(z - M + j),
    // j = 0..2M, in NQ2 >= 2M+1 physical slots; NQ2 is a multiple of PF so that
    // the loop unrolled NQ2 times also cycles the PF prefetch register sets
    // at compile time
    constexpr int NQ2 = (NQ % PF) ? NQ + PF - NQ % PF : NQ;
    float q[RY][NQ2];
#pragma unroll
    for (int j = 1; j < NQ; ++j)
#pragma unroll
        for (int r = 0; r < RY; ++r) q[r][j] = bload(r_uc, v_ldr[r], soff(z0 - M + j - 1));
    drain_vmem();

    // what fetch(z) loads for plane z: the queue head uc(z + M), u_prev, C
    // (and snapshot and gradient), the x and y halo of uc(z), eta_z
    struct Pre {
        float fr[RY], pv[RY], cv[RY], sv[RY], gv[RY], hxv[RY], hyv[NH], ezn;
    };
    Pre pre[PF];
    auto fetch = [&](Pre& P, int z) {
        // first in the batch: vector-memory counters retire in order, so the
        // compute of earlier planes only waits for loads issued before this one
        P.ezn = a.eta_z[z];
        const uint32_t so = soff(z), sf = soff(z + M);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            P.fr[r] = bload(r_uc, v_ldr[r], sf);
            // arrays read only at owned points: lanes past the grid read
            // nothing (a clamped column can sit in a line of its own)
            P.pv[r] = bload<AWE_CPOL_STREAM>(r_up, v_pvr[r], so);
            P.cv[r] = bload<AWE_CPOL_STREAM>(r_cf, v_pvr[r], so);
            if (MODE == kStepImaging || MODE == kStepBorn) {
                P.sv[r] = bload<AWE_CPOL_STREAM>(r_us, v_pvr[r], so);
                P.gv[r] = bload<AWE_CPOL_STREAM>(r_gr, v_pvr[r], so);
            }
            P.hxv[r] = bload(r_uc, v_hxr[r], so);
        }
#pragma unroll
        for (int i = 0; i < NH; ++i)
            if (kHyFull || ty + i * BY < 2 * M) P.hyv[i] = bload(r_uc, v_hyr[i], so);
    };
#pragma unroll
    for (int i = 0; i < PF; ++i)
        if (z0 + i < z1) fetch(pre[i], z0 + i);

    // One plane.  The z-queue is never shifted: in iteration z the logical
    // slot j (plane z - M + j) lives in physical slot (j + PH) % NQ2, with PH
    // advancing by one per plane, and plane z0 + i uses prefetch set i % PF.
    // The loop is unrolled NQ2 times so PH and the set are compile-time
    // constants and no register moves are needed.
    auto one_plane = [&](auto ph, auto set, auto whole, int z) {
        constexpr int PH = decltype(ph)::value;
        Pre& P = pre[decltype(set)::value];
        auto Q = [&](int r, int j) -> float& { return q[r][(j + PH) % NQ2]; };
        const int b = (z - z0) & 1;
#pragma unroll
        for (int r = 0; r < RY; ++r) Q(r, NQ - 1) = P.fr[r];
        // stage plane z in LDS
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if constexpr (kHaloAll) {
                lds[b][M + ty * RY + r][hlx] = P.hxv[r];
                lds[b][M + ty * RY + r][M + lxb + tx] = Q(r, M);
            } else {
                lds[b][M + ty * RY + r][M + lxb + tx] = Q(r, M);
                if (hl || hr) lds[b][M + ty * RY + r][hlx] = P.hxv[r];
            }
        }
#pragma unroll
        for (int i = 0; i < NH; ++i)
            if (kHyFull || ty + i * BY < 2 * M) lds[b][hyrow[i]][M + lxb + tx] = P.hyv[i];

        float p[RY], c[RY], s[RY], gg[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            p[r] = P.pv[r];
            c[r] = P.cv[r];
            if (MODE == kStepImaging || MODE == kStepBorn) { s[r] = P.sv[r]; gg[r] = P.gv[r]; }
        }
        const float ezv = P.ezn;
        // the set is consumed: refill it with plane z + PF.  Inside a whole
        // round the refill takes no branch (past the chunk's end it loads
        // the last plane again, unused): a branch's join would merge the
        // refilled set with the old one, and the register copies that merge
        // needs wait for the loads just issued.  The order-16 plain step
        // refills without a branch in guarded planes too (404 -> 381 us per
        // 480^3 step; at orders 10-14 and with imaging that was slower).
        if constexpr (decltype(whole)::value || (M == 8 && MODE == kStepPlain)) fetch(P, min(z + PF, z1 - 1));
        else if (z + PF < z1) fetch(P, z + PF);
        lds_barrier();

        const uint32_t so = soff(z);
        // One LDS offset per thread and one per row, hidden from the optimiser
        // (the empty asm emits nothing): every neighbour is then an immediate
        // offset from them (x: 0..2M dwords, y: multiples of LW), so each pair
        // of reads is one ds_read2 / ds_read2st64 with no address arithmetic.
        int lofs = (b * LH + ty * RY) * LW + lxb + tx + M;   // (row ly - M, column lx)
        asm volatile("" : "+v"(lofs));
        int lrow[RY];                                  // (row ly, column lx - M)
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            lrow[r] = lofs + (r + M) * LW - M;
            asm volatile("" : "+v"(lrow[r]));
        }
        const float* lflat = &lds[0][0][0];
        const float ezx = ezv + exv;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const float* ly = lflat + lofs + (r + M) * LW;   // this point, y pairs
            const float* lx = lflat + lrow[r] + M;           // this point, x pairs
            float lap = k.c0 * Q(r, M);
#pragma unroll
            for (int kk = 1; kk <= M; ++kk) {
                const float yu = (r - kk >= 0) ? Q((r - kk) >= 0 ? (r - kk) : 0, M) : ly[-kk * LW];
                const float yd = (r + kk < RY) ? Q((r + kk) < RY ? (r + kk) : 0, M) : ly[kk * LW];
                lap += k.cz[kk] * (Q(r, M - kk) + Q(r, M + kk));
                lap += k.cy[kk] * (yu + yd);
                lap += k.cx[kk] * (lx[-kk] + lx[kk]);
            }
            const float u0 = Q(r, M);
            const float d = p[r] - u0;
            const float av = (ezx + eyv[r]) * c[r];
            // the Laplacian term's product is the exact one (the larger term;
            // fusing the damping product instead raised the GPU dot-test
            // error at order 16 to 1.5e-5); written out so the 2-D kernels
            // round alike
            float t = __builtin_fmaf(c[r], lap, av * d);
            if (MODE == kStepBorn) t -= (c[r] * k.inv_dt2) * (s[r] * gg[r]);
            bstore<AWE_CPOL_STREAM>(r_out, (u0 - d) + t, v_str[r], so);
            if (MODE == kStepImaging) bstore<AWE_CPOL_STREAM>(r_gr, gg[r] + s[r] * t, v_str[r], so);
            if (MODE == kStepSaveT) bstore<AWE_CPOL_STREAM>(r_gr, t, v_str[r], so);
        }
    };
    // before plane z0 the queue holds planes z0-M .. z0+M-1 in physical slots
    // 1..NQ-1, i.e. logical slot j sits in (j + 1) % NQ2: the first plane has PH = 1.
    // Steps that load one plane ahead run whole rounds of NQ2 planes
    // unguarded and test each plane only in the chunk's last partial round.
    // A guarded plane ends in a join where the refilled prefetch set meets
    // the old one, and the register copies of that merge wait for the loads
    // just issued, so no load outlived its plane (at order 8 every plane
    // drained the memory counter): 110 -> 107 us per 336^3 order-8 step,
    // 572 -> 553 us per 480^3 order-16 imaging step.  Plain steps of orders
    // 10-16, which load two planes ahead, keep the guard on every plane: with
    // whole rounds the 480^3 order-16 step took 387 against 376 us.
    // The partial round is straight-line code after the loop, not a second
    // loop: as a loop it raised the order-8 kernels' registers by a third.
    constexpr bool kWholeRounds = PF == 1;
    int z = z0;
    if constexpr (kWholeRounds) {
        while (z + NQ2 <= z1) {
            static_for<NQ2>([&](auto s_) {
                constexpr int PH = (decltype(s_)::value + 1) % NQ2;
                one_plane(std::integral_constant<int, PH>{}, std::integral_constant<int, decltype(s_)::value % PF>{},
                          std::true_type{}, z);
                ++z;
            });
        }
        static_for<NQ2>([&](auto s_) {
            constexpr int PH = (decltype(s_)::value + 1) % NQ2;
            if (z < z1)
                one_plane(std::integral_constant<int, PH>{}, std::integral_constant<int, decltype(s_)::value % PF>{},
                          std::false_type{}, z);
            ++z;
        });
    } else {
        for (;;) {
            static_for<NQ2>([&](auto s_) {
                constexpr int PH = (decltype(s_)::value + 1) % NQ2;
                if (z < z1)
                    one_plane(std::integral_constant<int, PH>{}, std::integral_constant<int, decltype(s_)::value % PF>{},
                              std::false_type{}, z);
                ++z;
            });
            if (z >= z1) break;
        }
    }

    // Fused injection: the workgroup whose tile holds a node adds its
    // increment once the whole tile is stored.
    if constexpr (MODE == kStepPlain || MODE == kStepSaveT) {
        const int xb = (int)bx * TX;
        auto in_tile = [&](int j) {
            const int zj = fs.inj_zyx[3 * j], yj = fs.inj_zyx[3 * j + 1], xj = fs.inj_zyx[3 * j + 2];
            return zj >= z0 && zj < z1 && yj >= yb && yj < yb + TY && xj >= xb && xj < xb + TX;
        };
        bool wg_inj = false;
        for (int j = 0; j < fs.inj.nrows; ++j) wg_inj = wg_inj || in_tile(j);   // uniform over the workgroup
        if (wg_inj) {
            tile_stores_visible();
            const int j = wv * kTileX + tx;
            if (j < fs.inj.nrows && in_tile(j)) inj_apply(fs.inj, j);
        }
    }
}

struct Geo2 {
    int32_t nz, nx;
    int64_t sz, origin, total;
    uint32_t gy;                 // block rows of the tile grid; rows past it sample
};

// 2-D: block = 64 x NW threads; wave w streams z planes [zw, zw + zchunk).
template <int M, int NW, int MODE>
__global__ void __launch_bounds__(kTileX * NW)
step2d(StepArgs a, StencilCoef k, Geo2 g, int zchunk, FusedSparse fs) {
    constexpr int LW = kTileX + 2 * M;
    constexpr int NQ = 2 * M + 1;
    __shared__ float lds[2][NW][LW];

    if (blockIdx.y >= g.gy) {                      // a sampling workgroup
        const int64_t blk = (int64_t)(blockIdx.y - g.gy) * gridDim.x + blockIdx.x;
        fused_sample(fs.smp, blk * (kTileX * NW) + threadIdx.y * kTileX + threadIdx.x);
        return;
    }

    const int tx = threadIdx.x;
    const int w = threadIdx.y;
    const int x = blockIdx.x * kTileX + tx;
    const int zw = (blockIdx.y * NW + w) * zchunk;        // first plane of this wave
    const int zend = min(zw + zchunk, g.nz);              // <= zw for an idle wave
    const bool live_wave = zw < g.nz;

    // slab base: grid point (zw - M, -M); an idle wave gets an empty slab
    const int64_t sz = g.sz;
    const int64_t slab = live_wave ? g.origin + (int64_t)(zw - M) * sz - M : 0;
    const uint64_t left = live_wave ? (uint64_t)(g.total - slab) * 4u : 0;
    const uint32_t bytes = left > 0x7FFFFFF0ull ? 0x7FFFFFF0u : (uint32_t)left;
    const auto r_uc = slab_rsrc(a.uc + slab, bytes);
    const auto r_up = slab_rsrc(a.up + slab, bytes);
    const auto r_out = slab_rsrc(a.out + slab, bytes);
    const auto r_cf = slab_rsrc(a.coef + slab, bytes);
    const auto r_us = slab_rsrc((MODE == kStepImaging || MODE == kStepBorn) ? a.usnap + slab : a.uc + slab, bytes);
    const auto r_gr = slab_rsrc(MODE != kStepPlain ? a.grad + slab : a.out + slab, bytes);
    const uint32_t plane = (uint32_t)(sz * 4);
    auto soff = [&](int z) { return (uint32_t)(z - zw + M) * plane; };

    const bool xin = x < g.nx;
    const bool xld = x < g.nx + M;
    const uint32_t o_in = xin ? (uint32_t)(x + M) * 4u : kOob;
    const uint32_t o_ld = xld ? (uint32_t)(x + M) * 4u : kOob;
    const bool hl = tx < M;
    const bool hr = tx >= kTileX - M;
    const int hx = hl ? ((int)blockIdx.x * kTileX - M + tx) : ((int)blockIdx.x * kTileX + M + tx);
    const int hlx = hl ? tx : (tx + 2 * M);
    const uint32_t o_hx = ((hl || hr) && hx < g.nx + M) ? (uint32_t)(hx + M) * 4u : kOob;
    const float exv = xin ? a.eta_x[x] : 0.f;


    float q[NQ];
#pragma unroll
    for (int j = 1; j < NQ; ++j) q[j] = bload(r_uc, o_ld, soff(zw - M + j - 1));
    drain_vmem();
    float fr, pv, cv, sv = 0.f, gv = 0.f, hv, ezn;
    auto fetch = [&](int z) {
        const bool live = z < zend;                   // wave-uniform
        ezn = live ? a.eta_z[z] : 0.f;                // first in the batch (in-order counters)
        const uint32_t so = soff(z);
        fr = bload(r_uc, live ? o_ld : kOob, soff(z + M));
        pv = bload<AWE_CPOL_STREAM>(r_up, live ? o_in : kOob, so);
        cv = bload<AWE_CPOL_STREAM>(r_cf, live ? o_in : kOob, so);
        if (MODE == kStepImaging || MODE == kStepBorn) {
            sv = bload<AWE_CPOL_STREAM>(r_us, live ? o_in : kOob, so);
            gv = bload<AWE_CPOL_STREAM>(r_gr, live ? o_in : kOob, so);
        }
        hv = bload(r_uc, live ? o_hx : kOob, so);
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
        const float p = pv, c = cv, s = sv, gg = gv, ezv = ezn;
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
            const float u0 = q[M];
            const float d = p - u0;
            const float av = (ezv + exv) * c;
            float t = __builtin_fmaf(c, lap, av * d);   // as in step2d_tb
            if (MODE == kStepBorn) t -= (c * k.inv_dt2) * (s * gg);
            bstore<AWE_CPOL_STREAM>(r_out, (u0 - d) + t, o_in, soff(z));
            if (MODE == kStepImaging) bstore<AWE_CPOL_STREAM>(r_gr, gg + s * t, o_in, soff(z));
            if (MODE == kStepSaveT) bstore<AWE_CPOL_STREAM>(r_gr, t, o_in, soff(z));
        }
    }

    // fused injection (see step3d): the block covers columns [xb, xb + 64)
    // and planes [zb, zb + NW * zchunk)
    if constexpr (MODE == kStepPlain || MODE == kStepSaveT) {
        const int xb = (int)blockIdx.x * kTileX, zb = (int)blockIdx.y * NW * zchunk;
        auto in_tile = [&](int j) {
            const int zj = fs.inj_zyx[3 * j], xj = fs.inj_zyx[3 * j + 2];
            return zj >= zb && zj < zb + NW * zchunk && xj >= xb && xj < xb + kTileX;
        };
        bool wg_inj = false;
        for (int j = 0; j < fs.inj.nrows; ++j) wg_inj = wg_inj || in_tile(j);   // uniform over the block
        if (wg_inj) {
            tile_stores_visible();
            const int j = w * kTileX + tx;
            if (j < fs.inj.nrows && in_tile(j)) inj_apply(fs.inj, j);
        }
    }
}

// ---------------------------------------------------------------------------
// launch-shape tables
// 3-D configurations: (BY, RY) -> workgroup 64 x BY threads, tile 64 x BY*RY.
// 2-D configurations: NW waves per workgroup.
// ---------------------------------------------------------------------------
// Workgroups that sample `npts` points, `per` threads each.
inline uint32_t sample_groups(int32_t npts, int per) { return npts > 0 ? (uint32_t)((npts + per - 1) / per) : 0u; }

template <int M, int MODE>
hipError_t launch3(int cfg, const Layout& L, const StencilCoef& k, const StepArgs& a, int zchunk, hipStream_t s,
                   const FusedSparse& fs) {
    if constexpr (MODE == kStepBorn || MODE == kStepSaveT) {
        // linearised modelling uses one shape (cfg 3) to bound the number of kernels
        if (cfg != 3) return hipErrorInvalidValue;
    }
    const int ty = tile_rows(3, cfg), tcols = tile_cols(3, cfg);
    Geo3 g{(int32_t)L.n[0], (int32_t)L.n[1], (int32_t)L.n[2], L.sy, L.sz, L.origin, 0, 0, 0, 0, L.total};
    g.gx = (uint32_t)((L.n[2] + tcols - 1) / tcols);
    g.gy = (uint32_t)((L.n[1] + ty - 1) / ty);
    const uint32_t gz = (uint32_t)((L.n[0] + zchunk - 1) / zchunk);
    g.ntiles = g.gx * g.gy * gz;
    g.ngrid = (g.ntiles + kXcds - 1) / kXcds * kXcds;          // a multiple of the XCD count
    const int waves = (cfg == 0 || cfg == 1) ? 4 : 8;
    const dim3 grid(g.ngrid + sample_groups(fs.smp.npts, kTileX * waves));
    const dim3 block(kTileX, waves);
    if constexpr (MODE == kStepBorn || MODE == kStepSaveT) {
        hipLaunchKernelGGL((step3d<M, 1, 8, 2, MODE>), grid, block, 0, s, a, k, g, zchunk, fs);
    } else {
        switch (cfg) {
            case 0:     // 64 x 16 tile, 256 threads, 4 rows per thread
                hipLaunchKernelGGL((step3d<M, 1, 4, 4, MODE>), grid, block, 0, s, a, k, g, zchunk, fs);
                break;
            case 1:     // 64 x 8 tile, 256 threads, 2 rows per thread
                hipLaunchKernelGGL((step3d<M, 1, 4, 2, MODE>), grid, block, 0, s, a, k, g, zchunk, fs);
                break;
            case 2:     // 64 x 32 tile, 512 threads, 4 rows per thread
                hipLaunchKernelGGL((step3d<M, 1, 8, 4, MODE>), grid, block, 0, s, a, k, g, zchunk, fs);
                break;
            case 4:     // 128 x 8 tile, 512 threads, 2 rows per thread
                hipLaunchKernelGGL((step3d<M, 2, 4, 2, MODE>), grid, block, 0, s, a, k, g, zchunk, fs);
                break;
            case 5:     // 128 x 16 tile, 512 threads, 4 rows per thread
                hipLaunchKernelGGL((step3d<M, 2, 4, 4, MODE>), grid, block, 0, s, a, k, g, zchunk, fs);
                break;
            default:    // 64 x 16 tile, 512 threads, 2 rows per thread
                hipLaunchKernelGGL((step3d<M, 1, 8, 2, MODE>), grid, block, 0, s, a, k, g, zchunk, fs);
                break;
        }
    }
    return hipGetLastError();
}

template <int M, int MODE>
hipError_t launch2(int cfg, const Layout& L, const StencilCoef& k, const StepArgs& a, int zchunk, hipStream_t s,
                   const FusedSparse& fs) {
    Geo2 g{(int32_t)L.n[0], (int32_t)L.n[2], L.sz, L.origin, L.total, 0};
    const unsigned gx = (unsigned)((L.n[2] + kTileX - 1) / kTileX);
    const int nw = (MODE == kStepBorn || MODE == kStepSaveT || cfg == 0) ? 4 : 1;
    const int64_t per_block = (int64_t)nw * zchunk;
    g.gy = (uint32_t)((L.n[0] + per_block - 1) / per_block);
    const uint32_t sg = sample_groups(fs.smp.npts, kTileX * nw);
    dim3 grid(gx, g.gy + (sg + gx - 1) / gx);   // sampling rows after the tile rows
    if constexpr (MODE == kStepBorn || MODE == kStepSaveT) {
        if (cfg != 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL((step2d<M, 4, MODE>), grid, dim3(kTileX, 4), 0, s, a, k, g, zchunk, fs);
    } else {
        if (nw == 4)
            hipLaunchKernelGGL((step2d<M, 4, MODE>), grid, dim3(kTileX, 4), 0, s, a, k, g, zchunk, fs);
        else
            hipLaunchKernelGGL((step2d<M, 1, MODE>), grid, dim3(kTileX, 1), 0, s, a, k, g, zchunk, fs);
    }
    return hipGetLastError();
}

// every mode for one half-width M
template <int M>
hipError_t launch_m(const Layout& L, const StencilCoef& k, const StepArgs& a, int mode, int cfg, int zchunk,
                    hipStream_t s, const FusedSparse& fs) {
    const bool d3 = L.ndim == 3;
    switch (mode) {
        case kStepPlain: return d3 ? launch3<M, kStepPlain>(cfg, L, k, a, zchunk, s, fs) : launch2<M, kStepPlain>(cfg, L, k, a, zchunk, s, fs);
        case kStepImaging: return d3 ? launch3<M, kStepImaging>(cfg, L, k, a, zchunk, s, fs) : launch2<M, kStepImaging>(cfg, L, k, a, zchunk, s, fs);
        case kStepBorn: return d3 ? launch3<M, kStepBorn>(cfg, L, k, a, zchunk, s, fs) : launch2<M, kStepBorn>(cfg, L, k, a, zchunk, s, fs);
        case kStepSaveT: return d3 ? launch3<M, kStepSaveT>(cfg, L, k, a, zchunk, s, fs) : launch2<M, kStepSaveT>(cfg, L, k, a, zchunk, s, fs);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace awe
