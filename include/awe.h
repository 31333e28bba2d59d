/*
 * awe.h - C ABI of an acoustic wave-equation engine for AMD MI355X (gfx950).
 *
 * The operator is the explicit finite-difference scheme for
 *
 *     m u_tt + eta u_t - laplace(u) = q,      u = u_t = 0 at t = 0,
 *
 * i.e. Eq. (1) of Kukreja et al., "Devito: automated fast finite difference
 * computation" (arXiv:1608.08658, Sec. V.A) with the damping term of its
 * Listing 1: second order in time, even order P = 2..16 in space, an
 * absorbing layer of nbl points on every side of the physical model, source
 * injection and receiver interpolation at off-grid points (Sec. IV).  The
 * adjoint run backwards in time (Eq. 4, Listing 2) and the adjoint-state
 * gradient of the L2 trace misfit (Eqs. 2-3) are provided with periodic or
 * binomial wavefield checkpointing and recomputation, and the linearised
 * (Born) operator whose adjoint that gradient is.
 *
 * Conventions for every call
 *   - Layout: arrays are FP32, C order, axis 0 = depth (slowest), the last
 *     axis unit stride.  "physical" arrays have the model's shape; "padded"
 *     arrays have shape[a] + 2 nbl points on every axis.
 *   - Units: SI.  m is squared slowness (s^2/m^2), spacing in metres, dt in
 *     seconds, coordinates in metres from the first physical grid point.
 *   - Pointers named *_dev are device pointers on the plan's device; *_host
 *     are host pointers.  The caller owns every pointer it passes; the library
 *     never frees or keeps a caller pointer beyond the call, except where a
 *     call says so (the server keeps traces_host until the request is done).
 *   - Streams: awe_stream is a hipStream_t (NULL = the legacy default stream).
 *     Calls enqueue work on that stream and return without waiting for it,
 *     except where a call says it synchronises.  The caller synchronises the
 *     stream before reading results.
 *   - Errors: every call returns an awe_status; AWE_OK is 0 and errors are
 *     negative.  Nothing aborts.  awe_last_error() gives a message for the
 *     last failing call on the calling thread.  Arguments are validated
 *     before any work is enqueued.
 *   - Threading: a plan is not re-entrant; different plans may be used from
 *     different threads on different streams.
 *   - Devices: a plan or a server lives on the HIP device that is current on
 *     the calling thread when it is created (hipSetDevice); calls that
 *     enqueue work on a plan must be made with that device current
 *     (AWE_EINVAL otherwise).
 */
#ifndef AWE_H
#define AWE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t awe_status;

enum {
    AWE_OK = 0,
    AWE_EINVAL = -1,     /* invalid argument or geometry                         */
    AWE_ENOMEM = -2,     /* device allocation failed or budget exceeded           */
    AWE_EHIP = -3,       /* a HIP runtime call failed (message has HIP's text)    */
    AWE_ESTATE = -4,     /* call out of order (e.g. gradient before forward)      */
    AWE_EUNSTABLE = -5,  /* dt above the stability limit, or non-finite values    */
    AWE_EBUSY = -6,      /* server queue full or request still running            */
    AWE_ENODEV = -7      /* no usable gfx950 device                               */
};

typedef void* awe_stream;
typedef struct awe_plan_s* awe_plan;
typedef struct awe_server_s* awe_server;

/*
 * One modelling problem (everything except the model and the wavelet).
 * Sec. V.C passes model, nt, dt, h and the space order to forward() and
 * adjoint() (Listings 1-2); the generated operator also takes source and
 * receiver coordinates (Listing 3).
 */
typedef struct awe_geometry {
    int32_t ndim;            /* 2 or 3                                               */
    int32_t space_order;     /* even, 2..16                                          */
    int64_t shape[3];        /* physical points per axis (first ndim used), >= 2     */
    double spacing[3];       /* metres per axis (first ndim used), > 0               */
    int32_t nbl;             /* absorbing points added on every side, >= 0           */
    int32_t damp_power;      /* k of the layer profile eta_max (d/nbl)^k, 1..4       */
    double damp_R;           /* target round-trip reflection, 0 < R < 1              */
    double damp_vref;        /* reference speed in eta_max (m/s), > 0                */
    double dt;               /* time step (s), > 0, <= awe_dt_max of the model      */
    int32_t nt;              /* time samples; nt-1 steps are taken, >= 1             */
    int32_t nsrc;            /* >= 0                                                 */
    int32_t nrec;            /* >= 0                                                 */
    int32_t reserved;        /* must be 0                                            */
    const double* src_coords;  /* host [nsrc][ndim]; copied by awe_plan_create       */
    const double* rec_coords;  /* host [nrec][ndim]; copied by awe_plan_create       */
} awe_geometry;

/* Text for the last error on the calling thread ("" if none).  The string
 * stays valid until the next failing call on the same thread. */
const char* awe_last_error(void);

/* Library version string, e.g. "awe 0.1 gfx950". */
const char* awe_version(void);

/*
 * Weights c_0..c_M (M = order/2) of the central second derivative of even
 * order `order` on a unit grid (Sec. IV.A, derivative expressions; for order 2 they are -2, 1).
 * w_host must hold M+1 doubles.  Pure host function.
 */
awe_status awe_fd_weights(int32_t order, double* w_host);

/*
 * Stability limit of the undamped scheme for speeds <= vmax:
 * dt_max = 2 / (vmax sqrt(sum_a sum_{k=-M..M} |c_k| / h_a^2)).
 * spacing_host holds ndim values.  Pure host function.
 */
awe_status awe_dt_max(int32_t ndim, int32_t order, const double* spacing_host, double vmax, double* dt_max);

/*
 * Device bytes a plan for `g` holds: forward only (ckpt_every == 0) or
 * forward + gradient with checkpoints every ckpt_every steps.  Used for
 * admission control.  Pure host function.
 */
awe_status awe_footprint(const awe_geometry* g, int32_t ckpt_every, uint64_t* bytes);

/*
 * Binomial checkpointing (Griewank 1992; Griewank & Walther 2000, the
 * "revolve" schedule): the alternative to a stored full history of the
 * forward wavefield that the paper names as under evaluation (Sec. IV.B, memory mapping).
 * The gradient's reverse sweep (Eqs. 3-4) visits the states
 * (u[t], u[t-1]), t = nt-1 .. 0; with `snapshots` stored states the schedule
 * takes the fewest forward steps that any schedule with that many stored
 * states can.  For nt time samples, *forward_steps_host receives the forward
 * steps of the whole gradient (the first sweep's nt - 1 included) and
 * *fields_host the wavefield buffers the schedule holds at most (a stored
 * state is a pair of fields; states one step apart share one).  nt >= 1,
 * snapshots >= 0; schedules above 2^31 forward steps are AWE_EINVAL.
 * Pure host function.
 */
awe_status awe_binomial_cost(int32_t nt, int32_t snapshots, int64_t* forward_steps_host, int32_t* fields_host);

/* Device bytes a plan for `g` holds for forward + gradient with binomial
 * checkpointing over `snapshots` stored states.  Pure host function. */
awe_status awe_footprint_binomial(const awe_geometry* g, int32_t snapshots, uint64_t* bytes);

/*
 * Validate `g`, build the off-grid point tables and allocate the plan's
 * forward fields on the current HIP device.  Coordinates outside the padded
 * grid are AWE_EINVAL.  The plan owns every device buffer it allocates;
 * awe_plan_destroy frees them.  Synchronous (waits for the null stream, on
 * which its set-up runs).  For 3-D grids of 4M points and more and 2-D grids
 * of 64K points and more, the first plan of a grid size times the stencil's
 * launch shapes on its own buffers (the paper's block-size autotuning,
 * Sec. IV.B, loop blocking; tens to hundreds of launches) unless a shape for the same
 * order and size (3-D: a size within 30% in points) is already known in the
 * process;
 * the environment variables AWE_TILE=cfg,zchunk and AWE_AUTOTUNE=0 pin or
 * skip it.  Every shape gives bit-identical results.
 */
awe_status awe_plan_create(const awe_geometry* g, awe_plan* out);
awe_status awe_plan_destroy(awe_plan plan);

/* Facts about a plan: out_host[0..2] = padded points per axis (1 beyond
 * ndim), out_host[3] = device bytes currently held, out_host[4..5] = launch
 * shape (workgroup configuration, z planes per workgroup) of the forward
 * stencil and out_host[6..7] that of the adjoint stencil with imaging.
 * out_host must hold 8 values. */
awe_status awe_plan_info(awe_plan plan, int64_t* out_host);

/*
 * Launch timing for measurement: with every > 0, the plan records a HIP
 * event pair on the launching stream around every every-th stencil step
 * launch and every every-th point-operator launch of its forward, step,
 * recompute and adjoint sweeps (awe_born and launch-shape tuning are not
 * timed); every == 0 switches it off.  Each call clears what was recorded.
 * awe_plan_kernel_times waits for the recorded launches and writes
 * out_host[0..5] = (count, mean microseconds) for stencil steps without
 * imaging (forward and recompute, the point operators inside included when
 * they run in the same launch), stencil steps with imaging (the gradient's
 * adjoint), and point operators launched on their own.  The events add
 * nothing to the launches they bracket but a timestamp each.
 */
awe_status awe_plan_time_kernels(awe_plan plan, int32_t every);
awe_status awe_plan_kernel_times(awe_plan plan, double* out_host);

/*
 * Load the physical model m_dev (physical shape, squared slowness: the `m`
 * of Eq. 1 and Listing 1) and build the update coefficients on the padded
 * grid: the absorbing layer of nbl points on every side (Sec. V.D pads the
 * 201 x 201 x 70 model with 40 points per side) copies the nearest edge cell
 * of the model, and the layer's damping is the `damp` term of Listing 1
 * (profile: awe_geometry's damp_power, damp_R, damp_vref).  Checks that m is
 * finite and positive and that dt <= awe_dt_max(max speed): otherwise
 * AWE_EUNSTABLE.  Synchronises `stream` (it reads the model's extrema back
 * to the host).
 */
awe_status awe_set_model(awe_plan plan, const float* m_dev, awe_stream stream);

/*
 * Forward modelling (Eq. 1, Listing 1) from zero initial state:
 *   u[n+1] = (2-a) u[n] - (1-a) u[n-1] + C (L u[n] + S q[n]),  n = 0..nt-2,
 *   traces[n] = R u[n]  (traces[0] = 0),
 * with C = dt^2 / (m + eta dt/2), a = eta C / dt.
 * wavelet_dev: [nt][nsrc] source signatures at t = n dt (may be NULL when
 * nsrc == 0).  traces_dev: [nt][nrec] output (may be NULL when nrec == 0).
 * ckpt_every > 0 stores the state pair every ckpt_every steps (and a copy of
 * the wavelet) for a following awe_adjoint with a gradient; 0 stores
 * nothing.  The final state stays in the plan (awe_get_state).
 */
awe_status awe_forward(awe_plan plan, const float* wavelet_dev, float* traces_dev,
                       int32_t ckpt_every, awe_stream stream);

/*
 * awe_forward (same traces, bit for bit) storing the states of the binomial
 * schedule with `snapshots` stored states (awe_binomial_cost) instead of
 * periodic checkpoints, for one following awe_adjoint with a gradient, which
 * runs the rest of the schedule and consumes it: a second gradient needs a
 * new call (AWE_ESTATE otherwise).  Stored states reference the forward's
 * own buffers, so nothing is copied.  The gradient equals that of the
 * periodic checkpoints bit for bit.  The final state stays in the plan until
 * that gradient runs.
 */
awe_status awe_forward_binomial(awe_plan plan, const float* wavelet_dev, float* traces_dev,
                                int32_t snapshots, awe_stream stream);

/*
 * Adjoint modelling (Eq. 4, Listing 2) driven by receiver data resid_dev
 * [nt][nrec], run backwards in time:
 *   mu[n] = (2-a) mu[n+1] - (1-a) mu[n+2] + C (L mu[n+1] + R^T y[n]),
 * src_adj_dev (optional, [nt][nsrc]) receives F^T y: S^T mu[n+1] for
 * n <= nt-2 and 0 for n = nt-1, so that <F x, y> = <x, F^T y> (Eqs. 5-6).
 * grad_m_dev (optional, physical shape) receives the gradient of
 * 1/2 ||traces - d_obs||^2 with respect to the physical m when resid_dev =
 * traces - d_obs (Eq. 3, the exact derivative of the discrete misfit);
 * it needs the preceding awe_forward on this plan to have used
 * ckpt_every > 0, or an awe_forward_binomial not yet used by a gradient
 * (else AWE_ESTATE).  Forward states are recomputed from the stored ones
 * during the sweep.  Afterwards the plan's wavefield state (awe_get_state)
 * is the zero pair; periodic checkpoints stay valid for another gradient.
 */
awe_status awe_adjoint(awe_plan plan, const float* resid_dev, float* src_adj_dev,
                       float* grad_m_dev, awe_stream stream);

/*
 * The forward state a gradient reads is the model of awe_set_model, the
 * states stored by the last awe_forward / awe_forward_binomial and its
 * wavelet (Eq. 3 pairs the adjoint field with the forward field of the same
 * model and source).  *id_host receives an identifier of that state; it
 * changes with every awe_set_model, awe_forward, awe_forward_binomial and
 * awe_born on the plan, and when a gradient consumes binomial states.  A
 * caller that keeps a forward for a later gradient (an autograd graph) takes
 * the identifier right after that forward and passes it to
 * awe_adjoint_checked.  Pure host function.
 */
awe_status awe_forward_id(awe_plan plan, int64_t* id_host);

/*
 * awe_adjoint, after checking that the plan still holds the forward state
 * forward_id (awe_forward_id): AWE_ESTATE, before any work is enqueued, if
 * another forward, model or linearised run has replaced it since.  F^T
 * (grad_m_dev NULL) is checked too, since it depends on the model.
 */
awe_status awe_adjoint_checked(awe_plan plan, int64_t forward_id, const float* resid_dev, float* src_adj_dev,
                               float* grad_m_dev, awe_stream stream);

/*
 * Linearised (Born) modelling: traces_dev [nt][nrec] = J dm, the derivative
 * of the forward traces with respect to the physical model in the direction
 * dm_dev (physical shape).  Differentiating the scheme of awe_forward (with
 * the absorbing layer fixed) gives a scattered field du driven by the
 * background's second time difference:
 *   du[n+1] = (2-a) du[n] - (1-a) du[n-1] + C L du[n] - (C/dt^2) dm (u[n+1] - 2u[n] + u[n-1]),
 *   traces[n] = R du[n].
 * Its adjoint is the gradient of awe_adjoint: <J dm, y> = <dm, J^T y>, the
 * linear-algebra counterpart of Eq. (3).  Uses the model of awe_set_model and
 * overwrites the plan's wavefield state (and any stored checkpoints).
 */
awe_status awe_born(awe_plan plan, const float* wavelet_dev, const float* dm_dev, float* traces_dev,
                    awe_stream stream);

/* The padded gradient of the last awe_adjoint that produced one
 * (padded shape, dense).  AWE_ESTATE if there is none. */
awe_status awe_get_gradient_padded(awe_plan plan, float* g_pad_dev, awe_stream stream);

/*
 * State access for restarts and tests: the state is the pair
 * (u[n], u[n-1]) as dense padded arrays.  awe_set_state copies them in;
 * awe_step then advances `nsteps` steps from time index n0, injecting
 * wavelet rows n0..n0+nsteps-1 (wavelet_dev [nt][nsrc], may be NULL) and
 * writing traces rows n0+1..n0+nsteps (traces_dev [nt][nrec], may be NULL);
 * n0 + nsteps must be <= nt - 1.  awe_get_state copies the current pair out.
 */
awe_status awe_set_state(awe_plan plan, const float* u_dev, const float* u_prev_dev, awe_stream stream);
awe_status awe_step(awe_plan plan, int32_t n0, int32_t nsteps, const float* wavelet_dev,
                    float* traces_dev, awe_stream stream);
/*
 * Temporal blocking (Sec. VI discusses time tiling), a measured prototype:
 * advances the state by 2 * npairs steps, two steps per z-sweep of one
 * launch, with no point operators (the plan must have no sources; no traces
 * are recorded).  The result is bit for bit what awe_step gives for the same
 * steps; it is slower than awe_step on every grid measured, so no forward
 * path uses it.  3-D plans of space order <= 8 with fields under 2 GB only
 * (AWE_EINVAL otherwise; AWE_ESTATE before awe_set_model).  zchunk = z planes
 * per workgroup (0: a built-in choice).  The first call allocates two more
 * fields, not counted by awe_footprint.
 */
awe_status awe_step2_blocked(awe_plan plan, int32_t npairs, int32_t zchunk, awe_stream stream);
awe_status awe_get_state(awe_plan plan, float* u_dev, float* u_prev_dev, awe_stream stream);

/*
 * Misfit of Eq. (2): resid_dev = traces_dev - d_obs_dev (n values) and
 * *phi_host = 1/2 sum resid^2 accumulated in FP64 in a fixed order
 * (deterministic).  resid_dev may be NULL.  Synchronises `stream`.
 */
awe_status awe_misfit(const float* traces_dev, const float* d_obs_dev, int64_t n,
                      float* resid_dev, double* phi_host, awe_stream stream);

/*
 * awe_misfit for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops): the same kernels and the same FP64
 * sum in the same order, so *phi_dev equals awe_misfit's *phi_host bit for
 * bit.  It allocates nothing: the per-block partial sums live in a fixed
 * 8 KiB device array of the library (one per device, kept until the process
 * ends), enough for any n.  Φ is written to phi_dev (device, one double) and
 * nothing is synchronised.  Calls that overlap on one device (different
 * streams or threads) share that array and race; serialise them.
 */
awe_status awe_misfit_noalloc(const float* traces_dev, const float* d_obs_dev, int64_t n,
                              float* resid_dev, double* phi_dev, awe_stream stream);

/*
 * Sum over shots: out_dev[i] = sum_{p=0}^{nparts-1} parts_host[p][i] for
 * i < n, accumulated in FP64 in the order p = 0, 1, ... and rounded once to
 * FP32.  The misfit of Eq. 2 over several shots is the sum of theirs, so its
 * gradient is the sum of the per-shot gradients; summing in a fixed order
 * makes the result independent of the order in which the shots finished.
 * parts_host is a host array of nparts (1..64) device pointers to FP32
 * arrays of n values; out_dev may be one of them.
 */
awe_status awe_sum_fields(float* out_dev, const float* const* parts_host, int32_t nparts, int64_t n,
                          awe_stream stream);

/* ---------------------------------------------------------------------------
 * Serving: a shot server with continuous batching on the current device.
 * Requests (forward shots, or gradients) carry their own geometry, model
 * and wavelet (host memory, copied at submit).  An engine thread admits
 * queued requests in arrival order while the sum of their awe_footprint
 * stays within hbm_fraction of the device memory that was free at creation
 * and at most max_active run at once; while max_active run, one more request
 * may be admitted and set up ahead (plan and uploads, on a host thread of
 * its own), to start as soon as a slot frees (its state is already
 * AWE_REQ_RUNNING, its footprint counted).  Each running request advances on its
 * own stream in chunks of chunk_steps time steps, two chunks in flight,
 * independently of the others (no batch-wide barrier); a request that
 * finishes is retired and its traces copied to traces_host (host
 * [nt][nrec], kept by the server until the request is done).  While
 * requests run the engine waits for no stream but the one it is working on:
 * plans are set up on their request's stream (launch shapes are timed only
 * while no other request runs), and device memory of retired requests goes
 * to a pool (counted against the budget) from which later requests take
 * buffers of the same size, freed in one batch only when the server has no
 * work left or the queue head needs the room.  Stats' "bytes reserved"
 * counts running requests plus pooled memory; "iterations" counts passes of
 * the engine loop.
 * ------------------------------------------------------------------------- */
enum { AWE_REQ_QUEUED = 0, AWE_REQ_RUNNING = 1, AWE_REQ_DONE = 2, AWE_REQ_FAILED = 3 };

awe_status awe_server_create(double hbm_fraction, int32_t chunk_steps, int32_t max_active,
                             awe_server* out);
/* A forward request.  Copies g (and its coordinates), m_host (physical
 * shape) and wavelet_host ([nt][nsrc]).  Returns a ticket >= 0.
 * Non-blocking. */
awe_status awe_server_submit(awe_server srv, const awe_geometry* g, const float* m_host,
                             const float* wavelet_host, float* traces_host, int64_t* ticket);
/*
 * A gradient request (Eqs. 2-3): the forward with checkpoints every
 * ckpt_every steps, the misfit against d_obs_host ([nt][nrec], copied at
 * submit) and the adjoint-state gradient, each advanced in chunks among the
 * other requests' work with the arithmetic of awe_forward, awe_misfit and
 * awe_adjoint on a plan run alone (so the results equal theirs bit for bit).
 * Its footprint (awe_footprint with ckpt_every, plus inputs and traces) is
 * admitted against the budget like any request.  When the request is done,
 * grad_dev (device memory on the server's device, physical shape, kept by
 * the caller until then) holds the gradient with respect to m, *phi_host
 * the misfit and traces_host ([nt][nrec]) the modelled traces; phi_host and
 * traces_host may be NULL.  Returns a ticket >= 0.  Non-blocking.
 */
awe_status awe_server_submit_gradient(awe_server srv, const awe_geometry* g, const float* m_host,
                                      const float* wavelet_host, const float* d_obs_host, int32_t ckpt_every,
                                      float* traces_host, float* grad_dev, double* phi_host, int64_t* ticket);
/* state = AWE_REQ_*; times_host[4] = (submit, admit, start, done) in seconds
 * on the server's monotonic clock (-1 where not reached yet).  For a failed
 * request *state is AWE_REQ_FAILED and awe_last_error() holds its message. */
awe_status awe_server_poll(awe_server srv, int64_t ticket, int32_t* state, double* times_host);
/* Blocks until the request is done or failed, or timeout_s elapses (AWE_EBUSY). */
awe_status awe_server_wait(awe_server srv, int64_t ticket, double timeout_s);
/* out_host[0..7] = (submitted, admitted, completed, failed, running, queued,
 * bytes reserved, iterations). */
awe_status awe_server_stats(awe_server srv, int64_t* out_host);
/* Waits for running requests, drops queued ones (marked failed), frees all. */
awe_status awe_server_destroy(awe_server srv);

#ifdef __cplusplus
}
#endif

#endif /* AWE_H */
