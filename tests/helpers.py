"""Shared helpers for the GPU parity tests: run one seeded shot through the
oracle and through the library on identical inputs."""
import sys

import numpy as np

import oracle
import synth


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def shot_dt(shot):
    """dt = dt_factor * stability limit, from the oracle (an input to both sides)."""
    return shot.dt_factor * oracle.dt_max(shot.order, shot.spacing, shot.vmax)


def oracle_problem(shot, dt, nt=None, src=None, rec=None):
    return oracle.Problem(shot.shape, shot.spacing, shot.order, shot.nbl, dt, nt or shot.nt,
                          shot.src_coords if src is None else src, shot.rec_coords if rec is None else rec,
                          damp_power=shot.damp_power, damp_R=shot.damp_R, damp_vref=shot.damp_vref)


def gpu_plan(shot, dt, nt=None, src=None, rec=None):
    import paper_1608_08658_amd as awe
    return awe.Plan(shape=shot.shape, spacing=shot.spacing, space_order=shot.order, nbl=shot.nbl, dt=dt,
                    nt=nt or shot.nt, src_coords=shot.src_coords if src is None else src,
                    rec_coords=shot.rec_coords if rec is None else rec, damp_power=shot.damp_power,
                    damp_R=shot.damp_R, damp_vref=shot.damp_vref)


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def small_3d_shot(seed, order, shape=(40, 46, 90), nbl=6, nt=120, nrec=37, f0=25.0):
    """A small layered 3-D shot that spans several tiles in x and y, several
    z chunks and ragged tails on every axis; off-grid source and receivers."""
    rng = np.random.default_rng(seed)
    h = (10.0, 9.0, 11.0)
    v = synth.multiplicative_noise(synth.layered_velocity(shape, rng, nlayers=(3, 5), vrange=(1500.0, 3000.0)),
                                   rng, 0.02)
    span = np.array([(n - 1) * hh for n, hh in zip(shape, h)])
    src = np.array([[0.21, 0.47, 0.53]]) * span
    rec = np.column_stack([np.full(nrec, 0.1 * span[0] + 3.3),
                           rng.uniform(0, span[1], nrec), rng.uniform(0, span[2], nrec)])
    return synth.Shot(f"small3d-o{order}", shape, h, order, nbl, nt, 1.0 / v ** 2, src, rec, f0,
                      dt_factor=0.5, damp_power=2, damp_vref=float(v.min()))


def small_2d_shot(seed, order, shape=(150, 170), nbl=10, nt=300, nrec=41, f0=15.0):
    rng = np.random.default_rng(seed)
    h = (10.0, 12.0)
    v = synth.multiplicative_noise(synth.layered_velocity(shape, rng, nlayers=(4, 7)), rng, 0.02)
    span = np.array([(n - 1) * hh for n, hh in zip(shape, h)])
    src = np.array([[0.31 * span[0] + 2.7, 0.52 * span[1] + 3.1]])
    rec = np.column_stack([np.full(nrec, 25.0), np.linspace(0, span[1], nrec)])
    return synth.Shot(f"small2d-o{order}", shape, h, order, nbl, nt, 1.0 / v ** 2, src, rec, f0,
                      dt_factor=0.5, damp_power=1, damp_vref=float(v.min()))


def oracle_block(op, lo, hi, nt=None, backend="numpy"):
    """The oracle operator ``op`` restricted to the padded-grid block
    [lo, hi): update coefficients sliced, node indices shifted, and only the
    sources and receivers whose nodes all lie inside the block kept.  Returns
    (block operator, kept source indices, kept receiver indices).

    Its fields equal the full operator's wherever nothing outside the block
    reaches them: callers place every source and receiver that can influence
    the block inside it and size the block so that no field reaches its
    faces within nt steps (the stencil spreads M points per step).  backend
    "c" takes the oracle's C time step (bit-identical to NumPy, faster)."""
    import copy
    sl = tuple(slice(a, b) for a, b in zip(lo, hi))
    p = copy.copy(op.p)
    p.padded_shape = tuple(b - a for a, b in zip(lo, hi))
    if nt is not None:
        p.nt = int(nt)
    sub = object.__new__(oracle.Operator)
    sub.p = p
    sub.backend = backend
    sub.A, sub.B, sub.C = op.A[sl], op.B[sl], op.C[sl]
    sub.vol = op.vol
    lo_a, hi_a = np.asarray(lo), np.asarray(hi)

    def restrict(table):
        if table is None:
            return None, np.zeros(0, dtype=np.int64)
        nodes, w = table
        inside = np.all((nodes >= lo_a) & (nodes < hi_a), axis=(1, 2))
        idx = np.nonzero(inside)[0]
        if idx.size == 0:
            return None, idx
        return (nodes[idx] - lo_a, w[idx]), idx

    sub.src, src_idx = restrict(op.src)
    sub.rec, rec_idx = restrict(op.rec)
    return sub, src_idx, rec_idx
