#!/usr/bin/env python3
"""Throughput benchmark of the acoustic forward operator on one MI355X.

Workload: 3-D acoustic forward, 256^3 physical grid + 40-point absorbing
layer on every side (336^3 computed points), h = 10 m, space order 8,
1000 time samples (999 steps), seeded layered model (6-10 layers, 1.5-4.5
km/s increasing with depth, 2% Gaussian noise), 15 Hz Ricker at an off-grid
point near the surface, 256 x 256 receivers at 25 m depth, FP32.

One benchmark "step" is one full shot: 999 stencil updates, each followed by
the source injection and the sampling of all 65 536 receivers, with inputs
resident in HBM.  value = computed grid-point updates per second
(336^3 * 999 per step).

Also reported: the stencil kernel's average launch duration against the
8 TB/s HBM roofline at 16 algorithmic bytes per point update.  Each time step
is one launch of the stencil (source injection and receiver sampling run
inside it), so the duration is the timed region's GPU time (HIP events on the
launching stream) over its launch count.  And the FP64 CPU oracle timed on a
few steps of the same grid.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = 16.0     # read u[n], u[n-1], C; write u[n+1]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


PROFILE = os.path.join(ROOT, "profiles", "step3d_o8_336cube_forward.md")
PROFILE_O16_STEP = os.path.join(ROOT, "profiles", "step3d_o16_480cube_forward.md")
PROFILE_O16_IMAGING = os.path.join(ROOT, "profiles", "step3d_o16_480cube_gradient_imaging.md")
PROFILE_BORN = os.path.join(ROOT, "profiles", "born3d_o8_336cube_born.md")
KERNEL_SRC = os.path.join(ROOT, "paper_1608_08658_amd", "csrc", "stencil_impl.hpp")
BORN_SRC = (os.path.join(ROOT, "paper_1608_08658_amd", "csrc", "kernels_born3d.hip"), KERNEL_SRC)


def kernel_source_digest(path=KERNEL_SRC):
    """sha256 of the kernel source (one path, or several read in order)
    without its comments and blank lines: recorded counters stay valid across
    edits of the comments, not of the code."""
    import hashlib
    import re
    paths = (path,) if isinstance(path, str) else tuple(path)
    text = re.sub(r"/\*.*?\*/", "", "\n".join(open(p).read() for p in paths), flags=re.S)
    lines = [re.sub(r"//.*$", "", line).rstrip() for line in text.splitlines()]
    return hashlib.sha256("\n".join(line for line in lines if line.strip()).encode()).hexdigest()


def profiled_traffic(shape, path=PROFILE, src=KERNEL_SRC):
    """HBM bytes per launch from a committed rocprofv3 counter summary (one
    entry per launch shape that was profiled), or None when the kernel code
    (``src``) has changed since the counters were taken or this launch shape
    was not profiled."""
    try:
        digest, per_shape = None, {}
        for line in open(path):
            t = line.strip()
            if not line.startswith("    "):
                continue
            if t.startswith("source_digest:"):
                digest = t.split()[1]
            elif t.startswith("shape ") and "traffic_bytes_per_launch" in t:
                f = t.split()
                per_shape[f[1].rstrip(":")] = float(f[f.index("traffic_bytes_per_launch") + 1])
        if digest != kernel_source_digest(src):
            return None
        return per_shape.get(f"{shape[0]},{shape[1]}")
    except (OSError, ValueError, IndexError):
        return None


def cpu_baseline(shot, dt, steps):
    """The FP64 oracle, untuned, on `steps` time steps of the same grid."""
    import oracle
    prob = oracle.Problem(shot.shape, shot.spacing, shot.order, shot.nbl, dt, steps + 1, shot.src_coords,
                          shot.rec_coords, damp_power=shot.damp_power, damp_R=shot.damp_R,
                          damp_vref=shot.damp_vref)
    op = oracle.Operator(prob, shot.m)
    w = shot.wavelet(dt)[: steps + 1]
    t0 = time.perf_counter()
    op.forward(w)
    t = time.perf_counter() - t0
    npad = int(np.prod(prob.padded_shape))
    return {"value": npad * steps / t, "unit": "grid-pt updates/s", "cores": 1, "kind": "oracle",
            "host_cpus": os.cpu_count(), "host_cpus_allowed": len(os.sched_getaffinity(0)),
            "sample": f"{steps} steps (with injection and receiver sampling) of the same "
                      f"{'x'.join(map(str, prob.padded_shape))} grid, NumPy FP64, single-threaded",
            "seconds": round(t, 3)}


def bench_gradient(torch, awe, synth, n=400, nt=2000, snapshots=20):
    """FWI gradient of the L2 trace misfit: 3-D, n^3 + 40-point layer, order 16,
    h = 12.5 m, nt samples, checkpoints every 50 steps, layered model with a
    +-10% Gaussian anomaly as the true model and its smoothed copy as the start.
    Reports the gradient time against a plain forward of the same shot, and
    the same gradient with binomial checkpointing over `snapshots` stored
    states (fewer fields held, more forward steps recomputed)."""
    shot = synth.config_3d_gradient(n=n, nt=nt)
    K = shot.extra["checkpoint_every"]
    m_true = shot.extra["m_true"]
    vmax = float(np.sqrt(1.0 / min(shot.m.min(), m_true.min())))
    dt = shot.dt_factor * awe.dt_max(3, shot.order, shot.spacing, vmax)
    plan = awe.Plan(shape=shot.shape, spacing=shot.spacing, space_order=shot.order, nbl=shot.nbl, dt=dt,
                    nt=shot.nt, src_coords=shot.src_coords, rec_coords=shot.rec_coords,
                    damp_power=shot.damp_power, damp_R=shot.damp_R, damp_vref=shot.damp_vref)
    npad = int(np.prod(plan.padded))
    w = torch.tensor(shot.wavelet(dt), dtype=torch.float32, device="cuda")
    plan.set_model(torch.tensor(m_true, dtype=torch.float32, device="cuda"))
    d_obs = plan.forward(w).clone()
    plan.set_model(torch.tensor(shot.m, dtype=torch.float32, device="cuda"))

    def events():
        return [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def gradient(ev):
        ev[0].record()
        tr = plan.forward(w, ckpt_every=K)
        ev[1].record()
        phi, resid = awe.misfit(tr, d_obs)
        ev[2].record()
        _, g = plan.adjoint(resid, want_src_adj=False, want_grad=True)
        ev[3].record()
        torch.cuda.synchronize()
        return phi, g

    gradient(events())                      # warm-up (tunes the imaging kernel's launch shape)
    ev = events()
    phi, g = gradient(ev)
    t_fwd_ckpt = ev[0].elapsed_time(ev[1]) / 1e3
    t_adj = ev[2].elapsed_time(ev[3]) / 1e3
    t_grad = ev[0].elapsed_time(ev[3]) / 1e3
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f0.record()
    plan.forward(w)
    f1.record()
    torch.cuda.synchronize()
    t_fwd = f0.elapsed_time(f1) / 1e3
    # Per-kernel durations from HIP events on the launching stream around
    # every 4th launch of one more (untimed) gradient: the stencil step
    # without imaging (forward with the receivers sampled inside, and the
    # recomputation), the adjoint step with imaging, and the residual
    # injection launched on its own.
    plan.time_kernels(4)
    gradient(events())
    kt = plan.kernel_times()
    plan.time_kernels(0)
    kernels = {}
    for kind, nbytes in (("step", BYTES_PER_UPDATE), ("imaging", 28.0)):
        cnt, us = kt[kind]
        if cnt:
            gbs = nbytes * npad / (us * 1e-6) / 1e9
            kernels[kind] = {"launches_timed": cnt, "avg_launch_us": us, "bytes_per_update": nbytes,
                             "achieved_GBps": gbs, "frac": gbs / HBM_PEAK_GBS}
    if kt["points"][0]:
        kernels["points"] = {"launches_timed": kt["points"][0], "avg_launch_us": kt["points"][1]}
    info = plan.info()
    for kind, shape, path in (("step", info["forward_shape"], PROFILE_O16_STEP),
                              ("imaging", info["imaging_shape"], PROFILE_O16_IMAGING)):
        if kind in kernels:
            kernels[kind]["launch_shape"] = list(shape)
            kernels[kind]["traffic"] = profiled_traffic(tuple(shape), path)
    log("gradient kernels: " + ", ".join(f"{k} {v['avg_launch_us']:.1f} us" +
                                          (f" ({100 * v['frac']:.1f}% of peak)" if "frac" in v else "")
                                          for k, v in kernels.items()))
    info = plan.info()
    finite = bool(torch.isfinite(g).all().item())
    binomial = None
    if snapshots is not None and snapshots >= 0:
        def gradient_binomial(ev):
            ev[0].record()
            tr = plan.forward(w, snapshots=snapshots)
            ev[1].record()
            _, resid = awe.misfit(tr, d_obs)
            ev[2].record()
            _, gb = plan.adjoint(resid, want_src_adj=False, want_grad=True)
            ev[3].record()
            torch.cuda.synchronize()
            return gb

        gradient_binomial(events())         # warm-up (allocates the buffer pool)
        evb = events()
        gb = gradient_binomial(evb)
        steps, fields = awe.binomial_cost(shot.nt, snapshots)
        t_b = evb[0].elapsed_time(evb[3]) / 1e3
        binomial = {"snapshots": snapshots, "forward_steps": steps, "buffer_fields": fields,
                    "gradient_s": t_b, "forward_s": evb[0].elapsed_time(evb[1]) / 1e3,
                    "adjoint_with_recompute_s": evb[2].elapsed_time(evb[3]) / 1e3,
                    "gradient_over_forward": t_b / t_fwd, "device_bytes": plan.info()["bytes"],
                    "bitwise_equal_to_periodic": bool(torch.equal(gb, g))}
        log(f"binomial checkpointing, {snapshots} snapshots: {t_b:.3f} s, {steps} forward steps, "
            f"{binomial['device_bytes'] / 2**30:.1f} GiB held (periodic {info['bytes'] / 2**30:.1f} GiB), "
            f"bitwise equal: {binomial['bitwise_equal_to_periodic']}")
    plan.close()
    upd = npad * (shot.nt - 1)
    log(f"gradient {shot.name}: {t_grad:.3f} s (forward+checkpoints {t_fwd_ckpt:.3f} s, adjoint+recompute "
        f"{t_adj:.3f} s), plain forward {t_fwd:.3f} s, ratio {t_grad / t_fwd:.2f}, phi {phi:.4e}, finite={finite}")
    return {
        "workload": f"3-D FWI gradient, {n}^3 physical + 40-point layer ({'x'.join(map(str, plan.padded))} "
                    f"computed), order 16, {shot.nt} samples, checkpoints every {K} steps, layered model with "
                    f"a Gaussian anomaly, smoothed start, {len(shot.rec_coords)} receivers",
        "gradient_s": t_grad, "forward_with_checkpoints_s": t_fwd_ckpt, "adjoint_with_recompute_s": t_adj,
        "plain_forward_s": t_fwd, "gradient_over_forward": t_grad / t_fwd,
        "algorithmic_gradient_over_forward": 60.0 / 16.0,
        "gradient_updates_per_s": 3 * upd / t_grad,
        "gradient_algorithmic_GBps": 60.0 * upd / t_grad / 1e9,
        "device_bytes": info["bytes"], "launch_shapes": {"forward": info["forward_shape"],
                                                         "imaging": info["imaging_shape"]},
        "kernels": kernels, "finite": finite, "binomial": binomial,
    }


def bench_serve(awe, synth, count=200, scale=0.5, seed=4, max_active=16, chunk=64):
    """Continuous-batching shot server under Poisson load.  First the
    saturation rate mu (every request submitted at once), then Poisson
    arrivals at 0.5, 0.8 and 0.95 mu with p50/p99 latency (result on the
    host minus arrival, queueing included)."""
    reqs = synth.serving_requests(seed, count, scale=scale)
    prepared = []
    for r in reqs:
        dt = r.dt_factor * awe.dt_max(r.ndim, r.order, r.spacing, r.vmax)
        g = awe.make_geometry(shape=r.shape, spacing=r.spacing, space_order=r.order, nbl=r.nbl, dt=dt, nt=r.nt,
                              src_coords=r.src_coords, rec_coords=r.rec_coords, damp_power=r.damp_power,
                              damp_R=r.damp_R, damp_vref=r.damp_vref)
        npad = int(np.prod([n + 2 * r.nbl for n in r.shape]))
        prepared.append((g, r.m.astype(np.float32), r.wavelet(dt).astype(np.float32), npad * (r.nt - 1)))
    work = sum(p[3] for p in prepared)

    def run(rate):
        srv = awe.Server(hbm_fraction=0.9, chunk_steps=chunk, max_active=max_active)
        rng = np.random.default_rng(seed + 1)
        tickets = []
        t0 = time.perf_counter()
        t_next = 0.0
        for g, m, w, _ in prepared:
            if rate:
                t_next += rng.exponential(1.0 / rate)
                delay = t0 + t_next - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            tickets.append(srv.submit(g, m, w)[0])
        for t in tickets:
            srv.wait(t, timeout=600)
        times = np.array([srv.poll(t)[1] for t in tickets])
        srv.close()
        lat = times[:, 3] - times[:, 0]
        span = times[:, 3].max() - times[:, 0].min()
        return {"offered_per_s": rate, "shots_per_s": len(tickets) / span, "p50_latency_s": float(np.percentile(lat, 50)),
                "p99_latency_s": float(np.percentile(lat, 99)), "mean_latency_s": float(lat.mean()),
                "grid_pt_updates_per_s": work / span, "wall_s": span}

    sat = run(None)
    mu = sat["shots_per_s"]
    log(f"serving: saturation {mu:.2f} shots/s, {sat['grid_pt_updates_per_s'] / 1e9:.1f} Gpt/s")
    points = []
    for f in (0.5, 0.8, 0.95):
        res = run(f * mu)
        res["load"] = f
        points.append(res)
        log(f"serving at {f:.2f} mu: {res['shots_per_s']:.2f} shots/s, p50 {res['p50_latency_s'] * 1e3:.1f} ms, "
            f"p99 {res['p99_latency_s'] * 1e3:.1f} ms")
    return {"workload": f"{count} seeded shot requests (2-D n^2 and 3-D n^3 mix, orders 4/8/16, layered models, "
                        f"sizes and step counts scaled by {scale}), chunk {chunk} steps, up to {max_active} running",
            "requests": count, "saturation": sat, "poisson": points}


def bench_served_gradient(torch, awe, synth, n=300, nt=1500, nshots=32, max_active=1):
    """Served gradient requests: per-shot FWI gradients submitted to the shot
    server (awe_server_submit_gradient: forward with checkpoints, misfit and
    adjoint-state gradient, advanced in chunks), summed on the device in
    fixed shot order (awe_sum_fields), timed from the first submission to the
    summed gradient; against a plain forward of the same shot.  One shot is
    repeated through the autograd Function, which gives the same bits."""
    shots = synth.config_served_gradient(n=n, nt=nt, nshots=nshots)
    K = shots[0].extra["checkpoint_every"]
    m_true = shots[0].extra["m_true"]
    vmax = float(np.sqrt(1.0 / min(shots[0].m.min(), m_true.min())))
    dt = shots[0].dt_factor * awe.dt_max(3, shots[0].order, shots[0].spacing, vmax)
    mt = torch.tensor(m_true, dtype=torch.float32, device="cuda")
    m0_host = shots[0].m.astype(np.float32)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    geoms, wavelets, observed, t_fwd = [], [], [], []
    for i, sh in enumerate(shots):
        g = awe.make_geometry(shape=sh.shape, spacing=sh.spacing, space_order=sh.order, nbl=sh.nbl, dt=dt, nt=sh.nt,
                              src_coords=sh.src_coords, rec_coords=sh.rec_coords, damp_power=sh.damp_power,
                              damp_R=sh.damp_R, damp_vref=sh.damp_vref)
        w = sh.wavelet(dt).astype(np.float32)
        plan = awe.Plan(shape=sh.shape, spacing=sh.spacing, space_order=sh.order, nbl=sh.nbl, dt=dt, nt=sh.nt,
                        src_coords=sh.src_coords, rec_coords=sh.rec_coords, damp_power=sh.damp_power,
                        damp_R=sh.damp_R, damp_vref=sh.damp_vref)
        plan.set_model(mt)
        wd = torch.tensor(w, device="cuda")
        ev[0].record()
        d_obs = plan.forward(wd)
        ev[1].record()
        torch.cuda.synchronize()
        t_fwd.append(ev[0].elapsed_time(ev[1]) / 1e3)
        geoms.append(g)
        wavelets.append(w)
        observed.append(d_obs.cpu().numpy())
        if i < len(shots) - 1:     # the last shot's plan serves the autograd check
            plan.close()
    log(f"served gradients: {len(shots)} observed shots modelled, forward {np.median(t_fwd):.3f} s per shot")
    grads = [torch.empty(shots[0].shape, dtype=torch.float32, device="cuda") for _ in shots]
    srv = awe.Server(hbm_fraction=0.9, chunk_steps=64, max_active=max_active)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    subs = [srv.submit_gradient(geoms[i], m0_host, wavelets[i], observed[i], K, grads[i], want_traces=False)
            for i in range(len(shots))]
    for t, _, _ in subs:
        srv.wait(t, timeout=900)
    times = np.array([srv.poll(t)[1] for t, _, _ in subs])
    total = awe.sum_fields(grads)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    srv.close()
    lat = times[:, 3] - times[:, 0]
    svc = times[:, 3] - times[:, 2]
    phi = float(sum(p[0] for _, _, p in subs))
    # the autograd path on the last shot: the same gradient bit for bit
    sh = shots[-1]
    m = torch.tensor(m0_host, device="cuda").requires_grad_(True)
    tr = awe.Gradient.apply(m, torch.tensor(wavelets[-1], device="cuda"), plan, K)
    loss = 0.5 * ((tr - torch.tensor(observed[-1], device="cuda")) ** 2).sum()
    loss.backward()
    same = bool(torch.equal(m.grad, grads[-1]))
    plan.close()
    npad = (n + 80) ** 3
    tf = float(np.median(t_fwd))
    per_shot = wall / len(shots)
    log(f"served gradients: {len(shots)} requests in {wall:.2f} s ({per_shot:.3f} s per shot, "
        f"{per_shot / tf:.2f}x the forward), p50 latency {np.percentile(lat, 50):.2f} s, "
        f"autograd path bitwise equal: {same}")
    return {"workload": f"{nshots} gradient requests on one {n}^3 layered model with an anomaly (+40-point layer), "
                        f"order 8, {nt} samples, checkpoints every {K} steps, 4x8 surface sources, "
                        f"{len(shots[0].rec_coords)} receivers, served (up to {max_active} running), "
                        f"gradients summed on device in shot order",
            "shots": nshots, "max_active": max_active, "total_gradient_s": wall, "gradient_s_per_shot": per_shot,
            "median_service_s": float(np.median(svc)), "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)), "median_forward_s": tf,
            "gradient_over_forward": per_shot / tf, "algorithmic_gradient_over_forward": 3.75,
            "gradient_algorithmic_GBps": 60.0 * npad * (nt - 1) / per_shot / 1e9,
            "total_misfit": phi, "autograd_equals_served": same,
            "gradient_finite": bool(torch.isfinite(total).all().item())}


def bench_born(torch, awe, synth, n=256, nt=1000):
    """Linearised (Born) modelling J dm on the forward workload's grid: the
    background and the scattered field advance together in one sweep per
    step, 32 algorithmic bytes per point-step (read u[n], u[n-1], du[n],
    du[n-1], C, dm; write u[n+1], du[n+1]; the background's second time
    difference stays in a register; as two launches it went through memory,
    44 bytes)."""
    shot = synth.config_3d_forward(n=n, nt=nt)
    dt = shot.dt_factor * awe.dt_max(3, shot.order, shot.spacing, shot.vmax)
    plan = awe.Plan(shape=shot.shape, spacing=shot.spacing, space_order=shot.order, nbl=shot.nbl, dt=dt, nt=shot.nt,
                    src_coords=shot.src_coords, rec_coords=shot.rec_coords, damp_power=shot.damp_power,
                    damp_R=shot.damp_R, damp_vref=shot.damp_vref)
    plan.set_model(torch.tensor(shot.m, dtype=torch.float32, device="cuda"))
    w = torch.tensor(shot.wavelet(dt), dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(9)
    dm = torch.tensor((0.05 * shot.m * synth.random_state(rng, shot.shape, 4.0)).astype(np.float32), device="cuda")
    plan.born(w, dm)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    tr = plan.born(w, dm)
    ev[1].record()
    torch.cuda.synchronize()
    t = ev[0].elapsed_time(ev[1]) / 1e3
    npad = int(np.prod(plan.padded))
    finite = bool(torch.isfinite(tr).all().item())
    plan.close()
    gbs = 32.0 * npad * (shot.nt - 1) / t / 1e9
    log(f"Born modelling: {t * 1e3:.1f} ms, {npad * (shot.nt - 1) / t / 1e9:.1f} G updates/s of the pair, "
        f"{gbs:.0f} GB/s algorithmic ({100 * gbs / HBM_PEAK_GBS:.1f}%)")
    # HBM bytes per launch from the committed counters of the one-sweep kernel
    # on this grid (None if its code changed since or the grid differs)
    traffic = profiled_traffic(("born", shot.shape[0] + 2 * shot.nbl), PROFILE_BORN, BORN_SRC)
    return {"workload": f"J dm on the {n}^3 order-8 forward workload ({'x'.join(map(str, shot.shape))} physical, "
                        f"{shot.nt} samples, {len(shot.rec_coords)} receivers), smooth 5% dm",
            "born_s": t, "pair_updates_per_s": npad * (shot.nt - 1) / t, "bytes_per_update": 32.0,
            "algorithmic_GBps": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS, "finite": finite,
            "kernel": "born3d<M=4> (both fields in one sweep per step)", "traffic": traffic,
            "algorithmic_bytes_per_launch": 32.0 * npad}


def bench_small_2d(torch, awe, synth, reps=5):
    """The small 2-D shot (101 x 101 + 10-point layer = 121 x 121 computed,
    order 4, 500 samples): 57 KiB per field, so each step is bound by launch
    latency, not HBM; reported as time per step, not against the roofline."""
    shot = synth.config_2d_small()
    dt = shot.dt_factor * awe.dt_max(2, shot.order, shot.spacing, 1500.0)
    plan = awe.Plan(shape=shot.shape, spacing=shot.spacing, space_order=shot.order, nbl=shot.nbl, dt=dt, nt=shot.nt,
                    src_coords=shot.src_coords, rec_coords=shot.rec_coords, damp_power=shot.damp_power,
                    damp_R=shot.damp_R, damp_vref=shot.damp_vref)
    plan.set_model(torch.tensor(shot.m, dtype=torch.float32, device="cuda"))
    w = torch.tensor(shot.wavelet(dt), dtype=torch.float32, device="cuda")
    plan.forward(w)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    times = []
    for _ in range(reps):
        ev[0].record()
        tr = plan.forward(w)
        ev[1].record()
        torch.cuda.synchronize()
        times.append(ev[0].elapsed_time(ev[1]) / 1e3)
    t = float(np.median(times))
    npad = int(np.prod(plan.padded))
    finite = bool(torch.isfinite(tr).all().item())
    plan.close()
    log(f"small 2-D: {shot.nt} samples in {t * 1e3:.2f} ms, {t / (shot.nt - 1) * 1e6:.2f} us per step")
    return {"workload": "2-D 101x101 + 10-point layer (121x121 computed), h = 10 m, v = 1500 m/s, order 4, "
                        "500 samples, 10 Hz Ricker at the centre, 101 receivers",
            "nt": shot.nt, "forward_s": t, "us_per_step": t / (shot.nt - 1) * 1e6,
            "grid_pt_updates_per_s": npad * (shot.nt - 1) / t, "finite": finite}


def bench_two_steps_per_sweep(torch, awe, synth, pairs=20):
    """The temporal-blocking prototype (two order-8 steps per z-sweep, no
    point operators) against single steps on the 336^3 forward grid, from the
    same seeded state; results are bit-identical (tested)."""
    shot = synth.config_3d_forward(nt=2 * pairs + 1)
    dt = shot.dt_factor * awe.dt_max(3, shot.order, shot.spacing, float(np.sqrt(1.0 / shot.m.min())))
    plan = awe.Plan(shape=shot.shape, spacing=shot.spacing, space_order=shot.order, nbl=shot.nbl, dt=dt,
                    nt=shot.nt, src_coords=np.zeros((0, 3)), rec_coords=np.zeros((0, 3)), damp_power=shot.damp_power,
                    damp_R=shot.damp_R, damp_vref=shot.damp_vref)
    plan.set_model(torch.tensor(shot.m, dtype=torch.float32, device="cuda"))
    P = plan.padded
    u0 = torch.tensor(synth.random_state(np.random.default_rng(9), P, 3.0), dtype=torch.float32, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    times = {}
    for name, run in (("single", lambda: plan.step(0, 2 * pairs)), ("blocked", lambda: plan.step2_blocked(pairs))):
        plan.set_state(u0, u0 * 0.999)
        run()                                   # warm-up (the first blocked call allocates two fields)
        plan.set_state(u0, u0 * 0.999)
        ev[0].record()
        run()
        ev[1].record()
        torch.cuda.synchronize()
        times[name] = ev[0].elapsed_time(ev[1]) * 1e3 / (2 * pairs)
    plan.close()
    npad = int(np.prod(P))
    log(f"two steps per sweep (prototype): {times['blocked']:.1f} us per step against {times['single']:.1f} us "
        f"for single steps")
    return {"workload": f"{2 * pairs} order-8 steps without point operators on the 336^3 forward grid, seeded state",
            "single_step_us": times["single"], "two_per_sweep_us_per_step": times["blocked"],
            "speedup": times["single"] / times["blocked"],
            "single_frac": 16.0 * npad / (times["single"] * 1e-6) / 8e12,
            "two_per_sweep_frac": 16.0 * npad / (times["blocked"] * 1e-6) / 8e12}


def bench_paper_example(torch, awe, synth):
    """The paper's 3-D run (Sec. V.D): 281 x 281 x 150 computed points,
    h = 15 m, order 14, 10 Hz Ricker, 1 s modelled, synthetic layered model."""
    shot = synth.config_paper_example()
    dt = shot.dt_factor * awe.dt_max(3, shot.order, shot.spacing, shot.vmax)
    shot.nt = int(round(shot.extra["t_end"] / dt)) + 1
    plan = awe.Plan(shape=shot.shape, spacing=shot.spacing, space_order=shot.order, nbl=shot.nbl, dt=dt, nt=shot.nt,
                    src_coords=shot.src_coords, rec_coords=shot.rec_coords, damp_power=shot.damp_power,
                    damp_R=shot.damp_R, damp_vref=shot.damp_vref)
    plan.set_model(torch.tensor(shot.m, dtype=torch.float32, device="cuda"))
    w = torch.tensor(shot.wavelet(dt), dtype=torch.float32, device="cuda")
    plan.forward(w)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    tr = plan.forward(w)
    ev[1].record()
    torch.cuda.synchronize()
    t = ev[0].elapsed_time(ev[1]) / 1e3
    npad = int(np.prod(plan.padded))
    finite = bool(torch.isfinite(tr).all().item())
    # the step kernel's own time (HIP events around every 4th launch, on an extra run)
    plan.time_kernels(4)
    plan.forward(w)
    torch.cuda.synchronize()
    n_timed, step_us = plan.kernel_times()["step"]
    plan.time_kernels(0)
    shape = plan.info()["forward_shape"]
    plan.close()
    log(f"paper example: {shot.nt} samples in {t * 1e3:.1f} ms, {npad * (shot.nt - 1) / t / 1e9:.1f} Gpt/s; "
        f"step kernel {step_us:.1f} us in shape {shape}")
    return {"workload": "the paper's 3-D run: 201x201x70 + 40-point layer (150x281x281 computed), h = 15 m, "
                        "order 14, 10 Hz Ricker, 1 s modelled, synthetic layered model (the paper gives none)",
            "nt": shot.nt, "dt": dt, "forward_s": t, "grid_pt_updates_per_s": npad * (shot.nt - 1) / t,
            "algorithmic_GBps": 16.0 * npad * (shot.nt - 1) / t / 1e9,
            "step_kernel": {"avg_launch_us": step_us, "launches_timed": n_timed,
                            "frac": 16.0 * npad / (step_us * 1e-6) / 8e12,
                            "launch_shape": {"workgroup_cfg": shape[0], "zchunk": shape[1]}},
            "finite": finite}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-steps", type=int, default=4, help="oracle time steps for the CPU baseline (0 = skip)")
    ap.add_argument("--n", type=int, default=256, help="physical grid points per axis")
    ap.add_argument("--nt", type=int, default=1000)
    ap.add_argument("--gradient-n", type=int, default=400,
                    help="physical points per axis of the gradient workload (0 = skip it)")
    ap.add_argument("--gradient-nt", type=int, default=2000, help="time samples of the gradient workload")
    ap.add_argument("--binomial-snapshots", type=int, default=20,
                    help="stored states of the binomial-checkpointing gradient (-1 = skip it)")
    ap.add_argument("--paper-example", type=int, default=1, help="run the paper's 3-D example workload (0 = skip)")
    ap.add_argument("--born", type=int, default=1, help="time Born modelling on the forward grid (0 = skip)")
    ap.add_argument("--small-2d", type=int, default=1, help="time the small 2-D shot (0 = skip)")
    ap.add_argument("--two-steps-per-sweep", type=int, default=1,
                    help="time the temporal-blocking prototype against single steps (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=200, help="requests per serving point (0 = skip)")
    ap.add_argument("--serve-scale", type=float, default=1.0,
                    help="size/step scale of the serving mix (1 = the full mix; < 1 shrinks it for quick runs)")
    ap.add_argument("--served-gradient-shots", type=int, default=32,
                    help="shots of the 300^3 served-gradient workload (0 = skip; 32 is the full workload)")
    ap.add_argument("--copy-ref-mb", type=int, default=0,
                    help="also run a plain device-to-device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (independent shots would shard "
              "one per GPU, one process each); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1608_08658_amd as awe
    import synth

    torch.cuda.set_device(0)
    shot = synth.config_3d_forward(n=args.n, nt=args.nt)
    dt = shot.dt_factor * awe.dt_max(3, shot.order, shot.spacing, shot.vmax)
    log(f"workload {shot.name}: padded {[n + 2 * shot.nbl for n in shot.shape]}, dt {dt:.4e} s")
    plan = awe.Plan(shape=shot.shape, spacing=shot.spacing, space_order=shot.order, nbl=shot.nbl, dt=dt,
                    nt=shot.nt, src_coords=shot.src_coords, rec_coords=shot.rec_coords,
                    damp_power=shot.damp_power, damp_R=shot.damp_R, damp_vref=shot.damp_vref)
    npad = int(np.prod(plan.padded))
    shape_cfg, shape_zc = plan.info()["forward_shape"]
    log(f"stencil launch shape: workgroup configuration {shape_cfg}, {shape_zc} z planes per workgroup")
    m = torch.tensor(shot.m, dtype=torch.float32, device="cuda")
    w = torch.tensor(shot.wavelet(dt), dtype=torch.float32, device="cuda")
    traces = torch.empty((shot.nt, len(shot.rec_coords)), dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    plan.set_model(m)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0

    for i in range(args.warmup):
        plan.forward(w, traces=traces)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for i in range(args.steps):
        plan.forward(w, traces=traces)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    updates = npad * (shot.nt - 1)
    value = updates * args.steps / (gpu_ms / 1e3)
    finite = bool(torch.isfinite(traces).all().item())
    log(f"timed {args.steps} shots: {gpu_ms:.1f} ms GPU ({wall:.2f} s wall), {value / 1e9:.1f} Gpt/s, finite={finite}")

    # The dominant kernel is the stencil, launched once per time step with the
    # injection and receiver sampling inside; its average launch duration over
    # the timed region (each shot's two zero fills and final sample launch,
    # < 0.1% of the time, are counted against it).
    nk = shot.nt - 1
    kern_s = gpu_ms / 1e3 / (args.steps * nk)
    achieved = BYTES_PER_UPDATE * npad / kern_s / 1e9
    log(f"stencil kernel: {kern_s * 1e6:.1f} us/launch, {achieved:.0f} GB/s algorithmic "
        f"({100 * achieved / HBM_PEAK_GBS:.1f}% of {HBM_PEAK_GBS:.0f} GB/s)")
    # reference: the same stencil without the point operators, back to back
    k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    k0.record()
    plan.step(0, nk)
    k1.record()
    torch.cuda.synchronize()
    plain_s = k0.elapsed_time(k1) / 1e3 / nk
    log(f"plain stencil launches (no point operators): {plain_s * 1e6:.1f} us/launch")
    plan.close()

    if args.copy_ref_mb > 0:
        # a plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE per
        # dispatch calibrate the counters against bytes actually moved
        nel = args.copy_ref_mb * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"reference copy: {args.copy_ref_mb} MiB read + written, 3 times")
        del src, dst

    grad = None
    if args.gradient_n > 0:
        log("gradient workload ...")
        grad = bench_gradient(torch, awe, synth, n=args.gradient_n, nt=args.gradient_nt,
                              snapshots=args.binomial_snapshots)

    paper = None
    if args.paper_example:
        log("paper example workload ...")
        paper = bench_paper_example(torch, awe, synth)

    small = None
    if args.small_2d:
        log("small 2-D workload ...")
        small = bench_small_2d(torch, awe, synth)

    tb3 = None
    if args.two_steps_per_sweep:
        log("two steps per sweep (temporal-blocking prototype) ...")
        tb3 = bench_two_steps_per_sweep(torch, awe, synth)

    born = None
    if args.born:
        log("Born modelling ...")
        born = bench_born(torch, awe, synth, n=args.n, nt=args.nt)

    serve = None
    if args.serve_requests > 0:
        log("serving workload ...")
        serve = bench_serve(awe, synth, count=args.serve_requests, scale=args.serve_scale)

    shots = None
    if args.served_gradient_shots > 0:
        log("served-gradient workload ...")
        shots = bench_served_gradient(torch, awe, synth, nshots=args.served_gradient_shots)

    base = None
    if args.cpu_steps > 0:
        log(f"CPU oracle baseline: {args.cpu_steps} steps ...")
        base = cpu_baseline(shot, dt, args.cpu_steps)
        log(f"  {base['value'] / 1e6:.2f} Mpt/s in {base['seconds']} s")

    traffic = profiled_traffic((shape_cfg, shape_zc))
    out = {
        "metric": "grid-pt updates/s",
        "value": value,
        "unit": "grid-pt updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"3-D acoustic forward shot, {args.n}^3 physical + 40-point layer "
                        f"({'x'.join(map(str, plan.padded))} computed), order 8, {shot.nt} samples, "
                        f"layered model, 15 Hz Ricker, {len(shot.rec_coords)} receivers",
            "grid": list(plan.padded), "space_order": shot.order, "nt": shot.nt,
            "nrec": len(shot.rec_coords), "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": BYTES_PER_UPDATE * npad,
            "kernel": "step3d<M=4> (forward stencil; source injection and receiver sampling inside the launch)",
            "avg_launch_us": kern_s * 1e6, "plain_stencil_avg_launch_us": plain_s * 1e6,
            "launch_shape": {"workgroup_cfg": shape_cfg, "zchunk": shape_zc},
            "bytes_per_update": BYTES_PER_UPDATE, "updates_per_launch": npad,
        },
        "cpu_baseline": base,
        "gradient": grad,
        "paper_example": paper,
        "small_2d": small,
        "two_steps_per_sweep": tb3,
        "born": born,
        "serving": serve,
        "served_gradients": shots,
        "setup_s": round(setup_s, 3),
        "traces_finite": finite,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
