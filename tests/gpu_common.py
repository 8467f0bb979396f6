"""Shared helpers of the GPU parity tests: run one workload through the HIP library (C ABI) and
through the CPU oracle from the same seeded inputs, and compare."""
import numpy as np
import torch

import oracle as O
from paper_1710_07073_amd import lbm as L
from paper_1710_07073_amd import sim as S


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a))


def gpu_sim(w, flags=0, bubbles=True):
    sim = S.Simulation(w.shape, w.omega, precision=w.dtype, bc=w.bc, flags=flags)
    if bubbles and w.nb:
        sim.add_bubbles(w.pos, w.d, S.bubble_params(**w.params), vel=w.vel)
    return sim


def oracle_state(w):
    lat = O.Lattice(*w.shape, w.omega, w.bc)
    bub = O.Bubbles(pos=w.pos.copy(), d=w.d.copy(), vel=None if w.vel is None else w.vel.copy())
    return lat, bub, O.bubble_params(**w.params)


def state_index(sim):
    """Which of the two torch population tensors holds the current state."""
    p = L.lbm_state_buffer(sim.ctx)
    return 0 if p == sim.pops[0].data_ptr() else 1


def to_buffer_layout(sim, R):
    """R (19, nz, ny, nx) in the context's population layout: plane-blocked (nz, 19, ny, nx)
    unless the plain structure-of-arrays flag is set."""
    R = np.asarray(R)
    if not (sim.flags & L.LBM_FLAG_PLAIN_SOA):
        R = R.transpose(1, 0, 2, 3)
    return np.ascontiguousarray(R)


def set_post_collision_state(sim, R):
    """Overwrite the GPU's current (post-collision) buffer with R (19, nz, ny, nx)."""
    k = state_index(sim)
    buf = torch.from_numpy(to_buffer_layout(sim, R)).to(sim.dtype)
    sim.pops[k].view(-1).copy_(buf.view(-1))
    torch.cuda.synchronize()


def gpu_u(sim):
    _, u, sums = sim.moments(fields=True)
    return u.double().cpu().numpy(), sums
