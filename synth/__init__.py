"""Seeded synthetic inputs for the acoustic operator: velocity models, source
signatures, acquisition geometry and random test vectors.

This module holds no arithmetic of the method itself (no FD weights, no
damping, no time stepping, no interpolation, no stability limit): it only
draws and shapes the inputs that both the GPU library and the CPU oracle are
fed.  The paper's own experiment (Sec. V.D) names no velocity model or data
set, so these generators stand in for it.

Conventions: SI units; axis 0 is depth; coordinates are metres from the first
physical grid point; m = 1 / v^2 (squared slowness, s^2/m^2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "ricker", "ricker_fn", "layered_velocity", "gaussian_anomaly", "smooth",
    "Shot", "config_2d_small", "config_3d_forward", "config_3d_gradient",
    "config_3d_gradient_crop", "config_served_gradient", "config_paper_example", "serving_requests",
    "random_traces", "random_state",
]


# --------------------------------------------------------------------------
# source signature
# --------------------------------------------------------------------------
def ricker_fn(f0: float, t0: float | None = None):
    """Ricker wavelet s(t) = (1 - 2 pi^2 f0^2 (t-t0)^2) exp(-pi^2 f0^2 (t-t0)^2),
    peak amplitude 1, delayed by t0 (default 1/f0)."""
    t0 = 1.0 / f0 if t0 is None else t0

    def s(t):
        a = (math.pi * f0 * (np.asarray(t, dtype=np.float64) - t0)) ** 2
        return (1.0 - 2.0 * a) * np.exp(-a)
    return s


def ricker(f0: float, dt: float, nt: int, t0: float | None = None) -> np.ndarray:
    """The Ricker wavelet sampled at t = n dt, n = 0..nt-1 (FP64)."""
    return ricker_fn(f0, t0)(np.arange(nt) * dt)


# --------------------------------------------------------------------------
# velocity models
# --------------------------------------------------------------------------
def layered_velocity(shape, rng: np.random.Generator, nlayers=(6, 10), vrange=(1500.0, 4500.0)) -> np.ndarray:
    """Flat layers stacked along axis 0 with velocities drawn uniformly in
    ``vrange`` and sorted to increase with depth; interfaces at sorted,
    distinct random depths.  Returns v (FP64, m/s)."""
    nz = int(shape[0])
    lo, hi = nlayers
    nl = int(rng.integers(lo, hi + 1))
    nl = max(1, min(nl, nz))
    tops = np.sort(rng.choice(np.arange(1, nz), size=nl - 1, replace=False)) if nl > 1 else np.array([], int)
    vel = np.sort(rng.uniform(vrange[0], vrange[1], size=nl))
    prof = np.empty(nz)
    edges = np.concatenate([[0], tops, [nz]])
    for i in range(nl):
        prof[edges[i]:edges[i + 1]] = vel[i]
    view = [nz] + [1] * (len(shape) - 1)
    return np.broadcast_to(prof.reshape(view), tuple(int(n) for n in shape)).copy()


def multiplicative_noise(v: np.ndarray, rng: np.random.Generator, rel: float) -> np.ndarray:
    """v * (1 + rel * N(0,1)), i.i.d. per point."""
    return v * (1.0 + rel * rng.standard_normal(v.shape))


def gaussian_anomaly(v: np.ndarray, rng: np.random.Generator, amplitude=0.10, sigma_pts=40.0,
                     centre_frac=(0.6, 0.5, 0.5)) -> np.ndarray:
    """v * (1 +- amplitude exp(-r^2 / 2 sigma^2)) with a seeded sign, centred at
    the given fraction of each axis (depth first)."""
    sign = 1.0 if rng.random() < 0.5 else -1.0
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in v.shape], indexing="ij")
    r2 = sum((g - centre_frac[a] * (v.shape[a] - 1)) ** 2 for a, g in enumerate(grids))
    return v * (1.0 + sign * amplitude * np.exp(-r2 / (2.0 * sigma_pts ** 2)))


def smooth(v: np.ndarray, sigma_pts: float) -> np.ndarray:
    """Gaussian-smoothed copy (the starting model of an inversion)."""
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(v, sigma_pts, mode="nearest")


# --------------------------------------------------------------------------
# shot descriptions
# --------------------------------------------------------------------------
@dataclass
class Shot:
    """Inputs of one modelling job.  ``dt`` is left to each side: it is a
    fraction ``dt_factor`` of the stability limit computed from the model."""
    name: str
    shape: tuple
    spacing: tuple
    order: int
    nbl: int
    nt: int
    m: np.ndarray                      # physical squared slowness, FP64
    src_coords: np.ndarray             # [nsrc, ndim] metres
    rec_coords: np.ndarray             # [nrec, ndim] metres
    f0: float                          # Ricker peak frequency (Hz)
    dt_factor: float = 0.5
    damp_power: int = 1
    damp_R: float = 1e-3
    damp_vref: float = 1500.0
    extra: dict = field(default_factory=dict)

    @property
    def ndim(self):
        return len(self.shape)

    @property
    def vmax(self):
        return float(np.sqrt(1.0 / self.m.min()))

    def wavelet(self, dt: float) -> np.ndarray:
        """[nt, nsrc] source signatures sampled at n dt."""
        s = ricker(self.f0, dt, self.nt)
        return np.repeat(s[:, None], len(self.src_coords), axis=1)


def _line_receivers(n, h, depth):
    x = np.arange(n) * h
    return np.stack([np.full(n, depth), x], axis=1)


def _plane_receivers(ny, nx, hy, hx, depth):
    yy, xx = np.meshgrid(np.arange(ny) * hy, np.arange(nx) * hx, indexing="ij")
    return np.stack([np.full(yy.size, depth), yy.ravel(), xx.ravel()], axis=1)


def config_2d_small(seed: int = 1) -> Shot:
    """2-D, 101 x 101, h = 10 m, v = 1500 m/s, order 4, 500 steps, 10-point
    linear layer, 10 Hz Ricker at the grid centre, 101 receivers on a line
    20 m below the top."""
    shape = (101, 101)
    h = 10.0
    m = np.full(shape, 1.0 / 1500.0 ** 2)
    src = np.array([[500.0, 500.0]])
    rec = _line_receivers(101, h, 20.0)
    return Shot("2d-101x101-o4-nt500", shape, (h, h), 4, 10, 500, m, src, rec, 10.0,
                damp_power=1, damp_vref=1500.0)


def _layered_m(shape, rng, noise=0.0):
    v = layered_velocity(shape, rng)
    if noise:
        v = multiplicative_noise(v, rng, noise)
    return v


def config_3d_forward(seed: int = 2, n: int = 256, nbl: int = 40, nt: int = 1000) -> Shot:
    """3-D forward: n^3, h = 10 m, order 8, layered model (6-10 layers,
    1.5-4.5 km/s increasing with depth, 2% Gaussian noise), 40-point layer,
    15 Hz Ricker at an off-grid point near the surface, an n x n receiver
    plane at 25 m depth."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    h = 10.0
    v = _layered_m(shape, rng, noise=0.02)
    phi = rng.uniform(0.1, 0.9, size=3)
    c = (n - 1) / 2.0
    src = np.array([[(2.0 + phi[0]) * h, (c + phi[1]) * h, (c + phi[2]) * h]])
    rec = _plane_receivers(n, n, h, h, 25.0)
    return Shot(f"3d-{n}^3-o8-nt{nt}", shape, (h, h, h), 8, nbl, nt, 1.0 / v ** 2, src, rec, 15.0,
                damp_vref=float(v.min()), extra={"v": v})


def _true_and_start(shape, rng, sigma_pts, smooth_pts):
    v = layered_velocity(shape, rng)
    vt = gaussian_anomaly(v, rng, amplitude=0.10, sigma_pts=sigma_pts)
    v0 = smooth(vt, smooth_pts)
    return vt, v0


def config_3d_gradient(seed: int = 3, n: int = 400, nbl: int = 40, nt: int = 2000,
                       sigma_pts: float = 40.0, smooth_pts: float = 10.0, nrec_side: int | None = None) -> Shot:
    """3-D FWI gradient: n^3, h = 12.5 m, order 16, layered true model with a
    +-10% Gaussian anomaly, smoothed starting model, 10 Hz Ricker near the
    surface at an off-grid point, receivers on an n x n plane at depth 2.5 h,
    checkpoints every 50 steps.  ``m`` is the starting model; the true model
    is in ``extra['m_true']``."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    h = 12.5
    vt, v0 = _true_and_start(shape, rng, sigma_pts, smooth_pts)
    phi = rng.uniform(0.1, 0.9, size=3)
    c = (n - 1) / 2.0
    src = np.array([[(2.0 + phi[0]) * h, (c + phi[1]) * h, (c + phi[2]) * h]])
    k = n if nrec_side is None else nrec_side
    stride = (n - 1) / max(k - 1, 1)
    rec = _plane_receivers(k, k, stride * h, stride * h, 2.5 * h)
    return Shot(f"3d-{n}^3-o16-nt{nt}-grad", shape, (h, h, h), 16, nbl, nt, 1.0 / v0 ** 2, src, rec, 10.0,
                damp_vref=float(min(vt.min(), v0.min())),
                extra={"m_true": 1.0 / vt ** 2, "checkpoint_every": 50})


def config_3d_gradient_crop(seed: int = 3, nt: int = 2000) -> Shot:
    """The 64^3 crop of the 3-D gradient problem (10-point layer, same h, dt
    rule and nt) that the FP64 oracle can run in full."""
    return config_3d_gradient(seed=seed, n=64, nbl=10, nt=nt, sigma_pts=6.4, smooth_pts=1.6, nrec_side=16)


def config_served_gradient(seed: int = 5, n: int = 300, nbl: int = 40, nt: int = 1500, nshots: int = 32,
                           nrec_side: int = 200) -> list[Shot]:
    """32 shots on one n^3 layered model with an anomaly (h = 10 m, order 8),
    sources on a 4 x 8 surface grid at depth 2.5 h, an nrec_side^2 receiver
    plane evenly spanning the surface, checkpoints every 30 steps.  All shots
    share ``m`` (the smoothed start) and ``extra['m_true']``."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    h = 10.0
    vt, v0 = _true_and_start(shape, rng, sigma_pts=0.1 * n, smooth_pts=0.025 * n)
    L = (n - 1) * h
    span = np.linspace(0.0, L, nrec_side)
    yy, xx = np.meshgrid(span, span, indexing="ij")
    rec = np.stack([np.full(yy.size, 2.5 * h), yy.ravel(), xx.ravel()], axis=1)
    shots = []
    rows, cols = 4, 8
    for s in range(nshots):
        i, j = divmod(s % (rows * cols), cols)
        src = np.array([[2.5 * h, (i + 0.5) * L / rows, (j + 0.5) * L / cols]])
        shots.append(Shot(f"3d-{n}^3-o8-nt{nt}-shot{s}", shape, (h, h, h), 8, nbl, nt, 1.0 / v0 ** 2, src, rec,
                          10.0, damp_vref=float(min(vt.min(), v0.min())),
                          extra={"m_true": 1.0 / vt ** 2, "checkpoint_every": 30}))
    return shots


def config_paper_example(seed: int = 6, t_end: float = 1.0) -> Shot:
    """The paper's own 3-D modelling run (Sec. V.D): 201 x 201 x 70 points
    (70 in depth) with a 40-point layer on every side (281 x 281 x 150
    computed), h = 15 m, 10 Hz Ricker, 1 s modelled, space order 14.  The paper
    gives no velocity model; a seeded layered model (1.5-4.5 km/s) stands in.
    201 receivers on a line across the centre at depth 2h.  ``nt`` is set from
    the modelled time once dt is known (see ``extra['t_end']``)."""
    rng = np.random.default_rng(seed)
    shape = (70, 201, 201)
    h = 15.0
    v = layered_velocity(shape, rng)
    src = np.array([[2.5 * h, 100.3 * h, 100.6 * h]])
    rec = np.stack([np.full(201, 2.0 * h), np.full(201, 100.0 * h), np.arange(201) * h], axis=1)
    return Shot("paper-3d-201x201x70-o14", shape, (h, h, h), 14, 40, 0, 1.0 / v ** 2, src, rec, 10.0,
                damp_vref=float(v.min()), extra={"t_end": t_end})


def serving_requests(seed: int, count: int, scale: float = 1.0) -> list[Shot]:
    """A seeded mix of forward shot requests: 2-D (n^2, n in 500..2000) or 3-D
    (n^3, n in 128..384) with equal probability, space order in {4, 8, 16},
    500-3000 steps, layered model, one 10 Hz Ricker and 10^U(2,4) receivers on
    a line (2-D) or a near-square plane (3-D) at depth 2.5 h; h = 10 m,
    40-point layer.  ``scale`` < 1 shrinks grid sizes and step counts
    proportionally for small functional tests."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        ndim = 2 if rng.random() < 0.5 else 3
        if ndim == 2:
            n = int(rng.integers(500, 2001))
        else:
            n = int(rng.integers(128, 385))
        order = int(rng.choice([4, 8, 16]))
        nt = int(rng.integers(500, 3001))
        nrec = int(round(10 ** rng.uniform(2, 4)))
        n = max(16, int(round(n * scale)))
        nt = max(8, int(round(nt * scale)))
        nrec = max(1, min(nrec, n ** (ndim - 1)))
        h = 10.0
        shape = (n,) * ndim
        v = layered_velocity(shape, rng)
        L = (n - 1) * h
        if ndim == 2:
            x = np.linspace(0.0, L, nrec)
            rec = np.stack([np.full(nrec, 2.5 * h), x], axis=1)
            src = np.array([[2.5 * h + 0.3 * h, 0.5 * L + 0.37 * h]])
        else:
            side = int(math.ceil(math.sqrt(nrec)))
            span = np.linspace(0.0, L, side)
            yy, xx = np.meshgrid(span, span, indexing="ij")
            rec = np.stack([np.full(yy.size, 2.5 * h), yy.ravel(), xx.ravel()], axis=1)[:nrec]
            src = np.array([[2.5 * h + 0.3 * h, 0.5 * L + 0.41 * h, 0.5 * L + 0.37 * h]])
        out.append(Shot(f"req{i}-{ndim}d-{n}-o{order}-nt{nt}", shape, (h,) * ndim, order, 40 if scale >= 1 else max(4, int(40 * scale)),
                        nt, 1.0 / v ** 2, src, rec, 10.0, damp_vref=float(v.min())))
    return out


# --------------------------------------------------------------------------
# random test vectors
# --------------------------------------------------------------------------
def random_traces(rng: np.random.Generator, nt: int, npts: int, f0: float, dt: float) -> np.ndarray:
    """Gaussian noise band-limited by convolving each column with a Ricker
    wavelet (for dot-product tests)."""
    w = ricker(f0, dt, nt)
    x = rng.standard_normal((nt, npts))
    out = np.empty_like(x)
    for j in range(npts):
        out[:, j] = np.convolve(x[:, j], w)[:nt]
    return out


def random_state(rng: np.random.Generator, shape, smooth_pts: float = 2.0) -> np.ndarray:
    """A smooth random field (Gaussian noise, Gaussian-filtered) of unit RMS."""
    from scipy.ndimage import gaussian_filter
    f = gaussian_filter(rng.standard_normal(shape), smooth_pts, mode="wrap")
    return f / np.sqrt(np.mean(f * f))
