// Internal declarations shared by the host engine and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace awe {

constexpr int kMaxHalf = 8;      // M = P/2 for space order P <= 16
constexpr int kXOff = 32;        // interior x offset in floats (128-byte aligned rows)
constexpr int kTileX = 64;       // one wavefront spans 64 unit-stride points

// Device layout of every wavefield-sized array.  The padded computational grid
// (physical model + absorbing layer) of extents n[0] x n[1] x n[2] (z, y, x;
// n[1] = 1 in 2-D) sits inside a larger pitched allocation whose extra cells
// are zero and never written: M planes above and below, M rows on each side
// (3-D only) and kXOff / >= M columns on the left / right.  The stencil thus
// reads its zero boundary from memory instead of branching, and every row of
// the grid starts on a 128-byte boundary.
struct Layout {
    int ndim = 0;
    int half = 0;                // M
    int64_t n[3] = {1, 1, 1};    // computational extents (z, y, x)
    int64_t sy = 0, sz = 0;      // strides in elements (x stride is 1)
    int64_t origin = 0;          // element offset of grid point (0, 0, 0)
    int64_t total = 0;           // elements in the allocation
    int64_t points() const { return n[0] * n[1] * n[2]; }
    int64_t index(int64_t z, int64_t y, int64_t x) const { return origin + z * sz + y * sy + x; }
};

// FD weights pre-scaled by 1 / h_a^2, and the time-step constants.
struct StencilCoef {
    float cz[kMaxHalf + 1];
    float cy[kMaxHalf + 1];
    float cx[kMaxHalf + 1];
    float c0;                    // c_0 * sum_a 1 / h_a^2
    float inv_dt;
    float inv_dt2;
};

// What a stencil launch does besides the update (see stencil_impl.hpp).
enum StepMode { kStepPlain = 0, kStepImaging = 1, kStepBorn = 2, kStepSaveT = 3 };

// Arguments of one stencil step.  out may alias up (in-place update): every
// thread reads up at a point before it writes out at the same point, and no
// other thread touches that point.
struct StepArgs {
    const float* uc;             // u[n] (forward) / mu[n+1] (adjoint): stencil input
    const float* up;             // u[n-1] / mu[n+2]
    float* out;                  // u[n+1] / mu[n]
    const float* coef;           // C = dt^2 / (m + eta dt / 2)
    const float* eta_z;          // per-axis damping tables (eta = sum of the three)
    const float* eta_y;
    const float* eta_x;
    const float* usnap;          // imaging: forward wavefield u[n]; born: dm on the padded grid
    float* grad;                 // imaging: accumulates u[n] * (mu[n] - 2 mu[n+1] + mu[n+2]);
                                 // save-t: receives t; born: the background's t (read)
};

struct FusedSparse;

// Kernel launchers (kernels_stencil.hip, kernels_aux.hip).  All return the
// launch status; none synchronise.  A plain step may take over the point
// operators of its time step (fs, see FusedSparse).
hipError_t launch_step(const Layout& L, const StencilCoef& k, const StepArgs& a, int mode,
                       int tile_cfg, int zchunk, hipStream_t s, const FusedSparse* fs = nullptr);
int num_tile_cfgs(int ndim);
int tile_rows(int ndim, int tile_cfg);   // y rows (3-D) or z chunks per block (2-D)
int tile_cols(int ndim, int tile_cfg);   // x columns per tile (3-D; 64 in 2-D)

// One launch of the off-grid point operators (kernels_aux.hip): injection
// into one array and sampling of another.  A zero count disables either part.
struct InjectOp {
    float* field = nullptr;              // receives the injection
    const float* coef = nullptr;         // C on the padded grid
    const int64_t* node = nullptr;       // CSR by grid node: node index per row
    const int32_t* rowptr = nullptr;     // nrows + 1 row starts
    const int32_t* pt = nullptr;         // point index per entry
    const float* w = nullptr;            // multilinear weight per entry
    const float* values = nullptr;       // one value per point (this time step)
    const float* usnap = nullptr;        // imaging: forward wavefield u[n]
    float* grad = nullptr;               // imaging / save-t accumulator (or NULL)
    float scale = 1.f;
    int32_t nrows = 0;
};
struct SampleOp {
    float* out = nullptr;                // npts values
    const float* field = nullptr;        // sampled array
    const int64_t* node = nullptr;       // [npts][corners] grid nodes
    const float* w = nullptr;            // [npts][corners] weights
    float scale = 1.f;
    int32_t npts = 0;
    int32_t corners = 0;
};
hipError_t launch_sparse(const InjectOp& a, const SampleOp& b, hipStream_t s);

// The point operators of one time step carried out by the stencil launch
// itself: extra workgroups past the tile grid sample the step's input (which
// the launch only reads), and in plain and save-t steps the few workgroups
// whose tile holds an injection node add its increment to the output (and to
// t in save-t) after their sweep, with the same arithmetic as launch_sparse
// (the stored value first, then the increment added).  Injection is fused
// only for at most kFuseMaxNodes nodes.
constexpr int kFuseMaxNodes = 8;
struct FusedSparse {
    InjectOp inj;                      // inj.field is the step's output; nrows <= kFuseMaxNodes
    const int32_t* inj_zyx = nullptr;  // [nrows][3]: (z, y, x) grid indices of the nodes (y = 0 in 2-D)
    SampleOp smp;                      // smp.field is the step's input
};
// 2-D forward steps in blocks of up to tb_steps(M) per launch
// (kernels_stencil2d_tb.hip): the point operators of every step travel with
// the launch.  Injection takes the source CSR rows (at most kFuseMaxNodes
// nodes) and wavelet rows n0..; sampling takes each receiver's base node and
// weights and a list of receivers by tb_tile() x tb_tile() tile of that node.
struct TbPoints {
    const float* wavelet = nullptr;      // [nt][nsrc]; NULL: no injection
    int32_t nsrc = 0;
    int32_t nrows = 0;                   // source CSR rows (grid nodes)
    const int64_t* src_node = nullptr;
    const int32_t* src_rowptr = nullptr;
    const int32_t* src_pt = nullptr;
    const float* src_w = nullptr;
    const int32_t* src_zyx = nullptr;    // [nrows][3]
    float src_scale = 1.f;
    float* traces = nullptr;             // [nt][nrec]; NULL: no sampling
    int32_t nrec = 0;
    int32_t first_row = 0;               // steps s < first_row of the launch record nothing
    const int32_t* rec_zx = nullptr;     // [nrec][2]: (z, x) of the receiver's lowest node
    const float* rec_w = nullptr;        // [nrec][4]: weights in corner order
    const int32_t* tile_ptr = nullptr;   // [tiles + 1]
    const int32_t* tile_rec = nullptr;   // [nrec]: receivers by tile, ascending
    float rec_scale = 1.f;
};
int tb_steps(int half);
int tb_tile();
int tb_max_tile_receivers();
// (uc, up) = (u[n0], u[n0-1]) -> (out_c, out_p) = (u[n0+nsteps], u[n0+nsteps-1]);
// the outputs must be distinct from the inputs (tiles read halos of others).
// One 3-D Born time step as a single sweep (kernels_born3d.hip): the
// background u and the scattered du advance together, t = the background's
// second time difference in a register; the source (at most kFuseMaxNodes
// nodes) goes into u[n+1] and t, the receivers sample du[n].
struct BornArgs {
    const float *u, *up, *du, *dup, *coef, *dm, *eta_z, *eta_y, *eta_x;
    float *out, *dout;           // u[n+1], du[n+1]; may alias up, dup (in-place update)
};
hipError_t launch_born3d(const Layout& L, const StencilCoef& k, const BornArgs& a, int zchunk, hipStream_t s,
                         const FusedSparse& fs);

// Two 3-D plain steps per z-sweep without point operators, half-widths
// 1..kTb3MaxHalf, fields under 2 GB (kernels_stencil3d_tb.hip): o1 = u[n+1],
// o2 = u[n+2] from uc = u[n], up = u[n-1]; the outputs alias neither input.
constexpr int kTb3MaxHalf = 4;
hipError_t launch_step3d_tb2(const Layout& L, const StencilCoef& k, const float* uc, const float* up, float* o1,
                             float* o2, const float* coef, const float* ez, const float* ey, const float* ex, int zchunk,
                             hipStream_t s);
hipError_t launch_step2d_tb(const Layout& L, const StencilCoef& k, const float* uc, const float* up, float* out_c,
                            float* out_p, const float* coef, const float* eta_z, const float* eta_x,
                            const TbPoints& p, int n0, int nsteps, hipStream_t s);
hipError_t launch_coef(float* coef, const float* m_phys, const Layout& L, const int64_t phys[3], int nbl,
                       const double* eta_z, const double* eta_y, const double* eta_x, double dt, hipStream_t s);
hipError_t launch_minmax(const float* m, int64_t n, float* partial /* [3 * blocks] */, int blocks, hipStream_t s);
hipError_t launch_fold(float* grad_phys, const float* g, const Layout& L, const int64_t phys[3], int nbl,
                       float scale, const int64_t* wide_cells /* edge and corner cells (fold_wide_cells) */,
                       int32_t nwide, hipStream_t s);
std::vector<int64_t> fold_wide_cells(int ndim, const int64_t phys[3], int nbl);
hipError_t launch_pack(float* dense, const float* pitched, const Layout& L, float scale, hipStream_t s);
hipError_t launch_pad(float* pitched, const float* m_phys, const Layout& L, const int64_t phys[3], int nbl,
                      hipStream_t s);
hipError_t launch_unpack(float* pitched, const float* dense, const Layout& L, hipStream_t s);
hipError_t launch_misfit(const float* tr, const float* obs, int64_t n, float* resid, double* partial,
                         int blocks, double* result, hipStream_t s);
hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s);
constexpr int kMaxSumParts = 64;
// out[i] = sum of parts[0..nparts-1][i] in that order, FP64, one rounding
// (parts: host array of device pointers, nparts <= kMaxSumParts).
hipError_t launch_sum_parts(float* out, const float* const* parts, int nparts, int64_t n, hipStream_t s);
constexpr int kReduceBlocks = 1024;

}  // namespace awe
