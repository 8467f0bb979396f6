"""Checkpoint and resume through the C ABI: the state a method step leaves (the post-collision
buffer, the velocity field of the last collision, the bubble arrays) is all a run needs to
continue, so a lattice restored from it reproduces the uninterrupted run bit for bit, through
lbm_checkpoint / lbm_restore or by copying the buffer lbm_state_buffer names (the route
adjoint.py's checkpoints take)."""
import ctypes as ct

import numpy as np
import pytest
import torch

import workloads as W
from paper_1710_07073_amd import lbm as L
from paper_1710_07073_amd import sim as S

_FIELDS = ("x", "y", "z", "ux", "uy", "uz", "ulx", "uly", "ulz", "state")


def _state_tensor(sim):
    ptr = L.lbm_state_buffer(sim.ctx)
    return sim.pops[0] if sim.pops[0].data_ptr() == ptr else sim.pops[1]


def _new_sim(w, prec):
    sim = S.Simulation(w.shape, w.omega, precision=prec, bc=w.bc)
    sim.add_bubbles(w.pos, w.d, S.bubble_params(**w.params))
    return sim


@pytest.mark.gpu
@pytest.mark.parametrize("route", ["abi", "buffers"])
@pytest.mark.parametrize("prec,shape,steps", [("f64", (32, 32, 64), (40, 30)),
                                              ("f32", (128, 128, 256), (24, 16))])
def test_resume_from_checkpoint_is_bitwise_the_uninterrupted_run(prec, shape, steps, route):
    """The second case is large enough for the overlapped step (2^22 sites). route abi:
    lbm_checkpoint / lbm_restore; buffers: the state buffer lbm_state_buffer names, copied by
    the caller."""
    nx, ny, nz = shape
    pos = np.array([[nx / 2, nx / 2 + 3.2, nx / 2 - 2.7], [ny / 2, ny / 2 - 1.4, ny / 2 + 2.9],
                    [6.0, 8.5, 11.0]])
    w = W.Workload("resume", shape, 1.3, (0,) * 6, pos, np.array([3.0, 2.6, 3.4]),
                   W.params(g=1e-4, sigma=1e-4), sum(steps), prec)
    print(f"[case] resume {prec} {shape} after {steps[0]} of {sum(steps)} steps", flush=True)
    a = _new_sim(w, prec)
    a.run(steps[0])
    if route == "abi":
        snap = a.checkpoint()
    else:
        snap = dict(state=_state_tensor(a).clone(), vel=a.vel.clone(),
                    bubbles={k: a.bubbles.t[k].clone() for k in _FIELDS})
    a.run(steps[1])
    ref_pops, ref_x, ref_u = a.populations(), a.bubbles.positions(), a.bubbles.velocities()
    a.check()
    a.close()
    b = _new_sim(w, prec)
    b.run(3)  # the restored lattice need not be fresh
    if route == "abi":
        b.restore(snap)
    else:
        _state_tensor(b).copy_(snap["state"])
        b.vel.copy_(snap["vel"])
        for k, v in snap["bubbles"].items():
            b.bubbles.t[k].copy_(v)
    b.run(steps[1])
    assert torch.equal(b.populations(), ref_pops)
    assert np.array_equal(b.bubbles.positions(), ref_x)
    assert np.array_equal(b.bubbles.velocities(), ref_u)
    b.check()
    b.close()
