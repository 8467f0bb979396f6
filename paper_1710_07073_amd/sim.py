"""A simulation object over the C ABI: allocates the device buffers with PyTorch (memory and
streams only) and calls the library for every step of Algorithm 1."""
from __future__ import annotations

import ctypes as ct

import numpy as np
import torch

from . import lbm as L

_BUBBLE_FIELDS = ("x", "y", "z", "ux", "uy", "uz", "d", "ulx", "uly", "ulz")


def _ptr(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else None


class Bubbles:
    """Device bubble state (double precision structure of arrays) for the C ABI."""

    def __init__(self, pos, d, vel=None, device="cuda"):
        pos = np.asarray(pos, np.float64).reshape(3, -1)
        nb = pos.shape[1]
        self.nb = nb
        self.t = {}
        vel = np.zeros((3, nb)) if vel is None else np.asarray(vel, np.float64).reshape(3, nb)
        init = dict(x=pos[0], y=pos[1], z=pos[2], ux=vel[0], uy=vel[1], uz=vel[2],
                    d=np.asarray(d, np.float64).reshape(nb), ulx=np.zeros(nb), uly=np.zeros(nb),
                    ulz=np.zeros(nb))
        for k in _BUBBLE_FIELDS:
            self.t[k] = torch.tensor(init[k], dtype=torch.float64, device=device)
        self.t["state"] = torch.ones(max(nb, 1), dtype=torch.int32, device=device)[:nb]
        for k in ("psix", "psiy", "psiz"):
            self.t[k] = torch.zeros(max(nb, 1), dtype=torch.float64, device=device)[:nb]
        self.t["work"] = torch.empty(max(nb, 1) * L.LBM_BUBBLE_WORK, dtype=torch.float64,
                                     device=device)
        self.soa = L.BubbleSoA(*[ct.c_void_p(self.t[k].data_ptr()) for k in
                                 _BUBBLE_FIELDS + ("state", "psix", "psiy", "psiz", "work")])

    def positions(self):
        return torch.stack([self.t["x"], self.t["y"], self.t["z"]]).cpu().numpy()

    def velocities(self):
        return torch.stack([self.t["ux"], self.t["uy"], self.t["uz"]]).cpu().numpy()

    def reactions(self):
        return torch.stack([self.t["psix"], self.t["psiy"], self.t["psiz"]]).cpu().numpy()

    def state(self):
        return self.t["state"].cpu().numpy()

    def liquid_velocity(self):
        return torch.stack([self.t["ulx"], self.t["uly"], self.t["ulz"]]).cpu().numpy()


def bubble_params(g=1e-5, rho_l=1.0, rho_b=1e-3, sigma=4.19e-5, c_a=0.5, drag_scale=1.0,
                  lift_scale=1.0, kernel_factor=1.5, cd_k=0.15, lift_f0=0.474, n_sub=10,
                  coupling=0):
    """coupling: 0 or LBM_REACTION_* | LBM_COUPLING_* bits (lbm.py)."""
    return L.BubbleParams(g, rho_l, rho_b, sigma, c_a, drag_scale, lift_scale, kernel_factor, cd_k,
                          lift_f0, int(n_sub), int(coupling))


class Simulation:
    """Liquid lattice plus optional bubbles on one GPU."""

    def __init__(self, shape, omega, precision="f64", bc=(0,) * 6, flags=0, device="cuda",
                 stream=None):
        self.shape = tuple(int(s) for s in shape)
        nx, ny, nz = self.shape
        self.precision = L.LBM_FP64_SHIFTED if precision in ("f64", "fp64", L.LBM_FP64_SHIFTED) \
            else L.LBM_FP32_SHIFTED
        self.dtype = torch.float64 if self.precision == L.LBM_FP64_SHIFTED else torch.float32
        self.desc = L.make_desc(self.shape, omega, self.precision, bc, flags)
        pop_b, field_b, scratch_b = L.lbm_bytes_required(self.desc)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        n = nx * ny * nz
        self.cells = n
        self.flags = int(flags)
        # population buffers in the library's layout: plane-blocked (nz, 19, ny, nx) by default
        pshape = (19, nz, ny, nx) if self.flags & L.LBM_FLAG_PLAIN_SOA else (nz, 19, ny, nx)
        self.pops = [torch.empty(pshape, dtype=self.dtype, device=self.device) for _ in range(2)]
        self.force = torch.empty((3, nz, ny, nx), dtype=self.dtype, device=self.device)
        self.vel = torch.empty((3, nz, ny, nx), dtype=self.dtype, device=self.device)
        self.scratch = torch.empty(scratch_b, dtype=torch.uint8, device=self.device)
        assert self.pops[0].numel() * self.pops[0].element_size() == pop_b
        self.ctx = L.lbm_init(self.desc, _ptr(self.pops[0]), _ptr(self.pops[1]), _ptr(self.force),
                              _ptr(self.vel), _ptr(self.scratch),
                              ct.c_void_p(self.stream.cuda_stream))
        self.bubbles = None
        self.params = None

    def close(self):
        if self.ctx:
            L.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- bubbles ----
    def add_bubbles(self, pos, d, params, vel=None):
        self.bubbles = Bubbles(pos, d, vel, device=self.device)
        self.params = params
        return self.bubbles

    # ---- stepping ----
    def step(self, nsteps=1):
        """nsteps method steps (bubble half then liquid step) of Algorithm 1."""
        for _ in range(nsteps):
            if self.bubbles is not None and self.bubbles.nb > 0:
                L.bubbles_step(self.ctx, self.params, self.bubbles.soa, self.bubbles.nb)
            L.lbm_step(self.ctx, 1)

    def run(self, nsteps, graph_steps=0):
        """nsteps method steps through lbm_run (graph replay when graph_steps > 0)."""
        if self.bubbles is not None and self.bubbles.nb > 0:
            L.lbm_run(self.ctx, self.params, self.bubbles.soa, self.bubbles.nb, nsteps, graph_steps)
        else:
            empty = Bubbles(np.zeros((3, 0)), np.zeros(0), device=self.device)
            L.lbm_run(self.ctx, self.params or bubble_params(), empty.soa, 0, nsteps, graph_steps)

    def liquid_steps(self, nsteps=1):
        L.lbm_step(self.ctx, nsteps)

    # ---- observables ----
    def populations(self):
        nx, ny, nz = self.shape
        out = torch.empty((19, nz, ny, nx), dtype=self.dtype, device=self.device)
        L.lbm_populations(self.ctx, _ptr(out))
        return out

    def moments(self, fields=True):
        nx, ny, nz = self.shape
        rho = u = None
        if fields:
            rho = torch.empty((nz, ny, nx), dtype=self.dtype, device=self.device)
            u = torch.empty((3, nz, ny, nx), dtype=self.dtype, device=self.device)
        sums = L.moments(self.ctx, _ptr(rho), _ptr(u), True)
        return rho, u, sums

    def check(self):
        L.lbm_check(self.ctx)

    # ---- checkpoint and resume ----
    _SAVED = ("x", "y", "z", "ux", "uy", "uz", "ulx", "uly", "ulz", "state")

    def checkpoint(self):
        """Device copies of what the next step needs: the post-collision buffer, the velocity
        field of the last collision (lbm_checkpoint) and the bubble arrays."""
        state = torch.empty_like(self.pops[0])
        vel = torch.empty_like(self.vel)
        L.lbm_checkpoint(self.ctx, _ptr(state), _ptr(vel))
        bub = None
        if self.bubbles is not None:
            bub = {k: self.bubbles.t[k].clone() for k in self._SAVED}
        return dict(state=state, vel=vel, bubbles=bub)

    def restore(self, ckpt):
        """Continue from a checkpoint of a lattice of the same description (lbm_restore)."""
        L.lbm_restore(self.ctx, _ptr(ckpt["state"]), _ptr(ckpt["vel"]))
        if ckpt["bubbles"] is not None:
            for k, v in ckpt["bubbles"].items():
                self.bubbles.t[k].copy_(v)


class Batch:
    """Many columns (each a Workload-like spec) stepped together through the batched C ABI."""

    def __init__(self, columns, params, precision="f32", flags=0, device="cuda", stream=None):
        """columns: list of dicts with shape, omega, bc, pos (3, nb), d (nb), and optionally g
        and sigma (the column's bubbles' gravity and surface tension; default: params')."""
        self.columns = columns
        self.precision = L.LBM_FP64_SHIFTED if precision in ("f64", "fp64") else L.LBM_FP32_SHIFTED
        self.dtype = torch.float64 if self.precision == L.LBM_FP64_SHIFTED else torch.float32
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.cols = L.make_columns([(c["shape"], c["omega"], c["bc"], np.asarray(c["d"]).size,
                                     c.get("g", 0.0), c.get("sigma", 0.0)) for c in columns])
        pool_b, scratch_b = L.lbm_batch_bytes_required(self.cols, self.precision)
        self.pool = torch.empty(pool_b, dtype=torch.uint8, device=self.device)
        self.scratch = torch.empty(scratch_b, dtype=torch.uint8, device=self.device)
        self.handle = L.lbm_batch_init(self.cols, self.precision, flags, _ptr(self.pool),
                                       _ptr(self.scratch), ct.c_void_p(self.stream.cuda_stream))
        pos = np.concatenate([np.asarray(c["pos"], np.float64).reshape(3, -1) for c in columns], axis=1)
        d = np.concatenate([np.asarray(c["d"], np.float64).reshape(-1) for c in columns])
        vel = None
        if any(c.get("vel") is not None for c in columns):
            vel = np.concatenate([np.zeros((3, np.asarray(c["d"]).size)) if c.get("vel") is None
                                  else np.asarray(c["vel"], np.float64).reshape(3, -1) for c in columns],
                                 axis=1)
        self.bubbles = Bubbles(pos, d, vel, device=self.device)
        self.params = params
        self.ncols = len(columns)
        self.cells = sum(int(np.prod(c["shape"])) for c in columns)

    def close(self):
        if self.handle:
            L.lbm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, nsteps=1):
        L.lbm_batch_step(self.handle, self.params, self.bubbles.soa, self.bubbles.nb, nsteps)

    def run(self, nsteps, graph_steps=0):
        L.lbm_batch_run(self.handle, self.params, self.bubbles.soa, self.bubbles.nb, nsteps,
                        graph_steps)

    def populations(self, col):
        nx, ny, nz = self.columns[col]["shape"]
        out = torch.empty((19, nz, ny, nx), dtype=self.dtype, device=self.device)
        L.lbm_batch_populations(self.handle, col, _ptr(out))
        return out

    def bubble_range(self, col):
        c = self.cols[col]
        return c.bubble_begin, c.bubble_begin + c.nb

    def check(self):
        L.lbm_batch_check(self.handle)

    def sums(self):
        """(ncols, 4) per-column (sum rho, sum rho u) and a mask of the columns whose sums are not
        finite (diverged)."""
        sums, _ = L.lbm_batch_sums(self.handle, self.ncols)
        return sums, ~np.isfinite(sums).all(axis=1)
