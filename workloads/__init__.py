"""Seeded synthetic inputs for the bubble-column workloads.

This module only draws and lays out inputs (lattice shapes, relaxation rates, bubble positions
and diameters, property constants). It holds none of the method's arithmetic, and both the CPU
oracle tests and the GPU library's tests/benchmark read their inputs from here.

The columns stand in for the paper's rectangular bubble columns (Table 2: 30 x 30 x 90; Table 5
and Table 6: up to 120 x 120 x 360) at larger sizes; all values are in lattice units
(dx = dt_l = 1, rho_l = 1), gravity along -z, bubble sub-step dt_b = dt_l / 10 (Table 2).
Surface tension is chosen so that the Eotvos number at the workload's median diameter is 2.148,
the value of the paper's 4 mm air bubble in water (Table 3).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

SEED = 1710
BB, FS, PER = 0, 1, 2
EO_4MM = 2.148  # (rho_l - rho_b) g d^2 / sigma of a 4 mm air bubble in water (Table 3)


def sigma_for(g, d_median, rho_ratio=1e-3):
    """Surface tension giving Eo = 2.148 at the median diameter."""
    return (1.0 - rho_ratio) * g * d_median ** 2 / EO_4MM


@dataclass
class Workload:
    name: str
    shape: tuple            # (nx, ny, nz)
    omega: float
    bc: tuple               # (-x, +x, -y, +y, -z, +z)
    pos: np.ndarray         # (3, nb) bubble centres, cell centres at integer coordinates
    d: np.ndarray           # (nb,) diameters
    params: dict            # bubble-phase constants
    steps: int
    dtype: str              # "f64" or "f32" population storage
    vel: np.ndarray = None  # (3, nb) initial bubble velocities (zero if None)
    meta: dict = field(default_factory=dict)

    @property
    def nb(self):
        return int(self.pos.shape[1])

    @property
    def cells(self):
        nx, ny, nz = self.shape
        return nx * ny * nz


def params(g=1e-5, rho_b=1e-3, sigma=4.19e-5, drag_scale=1.0, lift_scale=1.0, c_a=0.5,
           kernel_factor=1.5, cd_k=0.15, lift_f0=0.474, n_sub=10, coupling=0):
    """Bubble constants; coupling selects a coupling variant (the same bit values on both sides:
    1, 2 reaction as sub-step mean or net force, 4 point-sampled weights, 8 exact time)."""
    return dict(g=g, rho_l=1.0, rho_b=rho_b, sigma=sigma, c_a=c_a, drag_scale=drag_scale,
                lift_scale=lift_scale, kernel_factor=kernel_factor, cd_k=cd_k, lift_f0=lift_f0,
                n_sub=n_sub, coupling=coupling)


def plain_fp64(steps=500):
    """32 x 32 x 64 column of liquid at rest, omega = 1, bounce-back walls, one bubble of
    diameter 3 at (16, 16, 8), g = 1e-5, density ratio 1e-3."""
    return Workload("plain_fp64_32x32x64", (32, 32, 64), 1.0, (BB,) * 6,
                    np.array([[16.0], [16.0], [8.0]]), np.array([3.0]),
                    params(g=1e-5, sigma=sigma_for(1e-5, 3.0)), steps, "f64")


def single_fp32(steps=5000):
    """128 x 128 x 512 column (8.4 M sites), omega = 1.6, bounce-back walls, one bubble of
    diameter 4 released at the bottom centre."""
    return Workload("single_fp32_128x128x512", (128, 128, 512), 1.6, (BB,) * 6,
                    np.array([[63.5], [63.5], [8.0]]), np.array([4.0]),
                    params(g=1e-5, sigma=sigma_for(1e-5, 4.0)), steps, "f32")


def morton_order(pos):
    """Permutation listing bubbles along a Z-order (Morton) curve of their cells, so that bubbles
    adjacent in the list are adjacent in space."""
    c = np.floor(np.asarray(pos)).astype(np.int64).clip(0, (1 << 16) - 1)
    key = np.zeros(c.shape[1], dtype=np.int64)
    for bit in range(16):
        for a in range(3):
            key |= ((c[a] >> bit) & 1) << (3 * bit + a)
    return np.argsort(key, kind="stable")


def dense(steps=2000, shape=(256, 256, 768), nb=20000, seed=SEED):
    """Dense dispersed flow: omega drawn in [1.2, 1.8]; nb bubbles uniformly in the bottom 20 %,
    ln d ~ N(ln 3, 0.25^2), kept a window half-width away from the side and bottom walls. The
    bubbles are listed in Morton order of their positions."""
    rng = np.random.default_rng(seed)
    omega = float(rng.uniform(1.2, 1.8))
    nx, ny, nz = shape
    d = np.exp(rng.normal(np.log(3.0), 0.25, nb))
    n = 1.5 * d
    x = rng.uniform(n, nx - 1 - n)
    y = rng.uniform(n, ny - 1 - n)
    z = rng.uniform(n, 0.2 * nz)
    pos = np.stack([x, y, z])
    order = morton_order(pos)
    return Workload(f"dense_{nx}x{ny}x{nz}_{nb}b", shape, omega, (BB,) * 6,
                    np.ascontiguousarray(pos[:, order]), np.ascontiguousarray(d[order]),
                    params(g=1e-5, sigma=sigma_for(1e-5, 3.0)), steps, "f32")


def batched(ncol=64, steps=3000, seed=SEED, lo=24, hi=96):
    """Uneven columns for the batched sweep: cross-section n_x, n_y uniform in {lo..hi}, height
    2-4 times n_x, omega_k = 0.6 + 1.3 k / (ncol - 1), 1-8 bubbles of diameter 2-5 in the bottom
    20 % away from the walls. Returns a list of Workloads."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(ncol):
        nx = int(rng.integers(lo, hi + 1))
        ny = int(rng.integers(lo, hi + 1))
        h = rng.uniform(2.0, 4.0)
        nz = int(round(h * nx))
        omega = 0.6 + 1.3 * k / max(ncol - 1, 1)
        nb = int(rng.integers(1, 9))
        d = rng.uniform(2.0, 5.0, nb)
        n = 1.5 * d
        x = rng.uniform(n, nx - 1 - n)
        y = rng.uniform(n, ny - 1 - n)
        z = rng.uniform(n, np.maximum(n + 1.0, 0.2 * nz))
        out.append(Workload(f"column{k}_{nx}x{ny}x{nz}", (nx, ny, nz), float(omega), (BB,) * 6,
                            np.stack([x, y, z]), d, params(g=1e-5, sigma=sigma_for(1e-5, 3.5)),
                            steps, "f32"))
    return out


def adjoint(steps=2000, drag_scale=1.0, lift_scale=1.0, omega=1.4):
    """64 x 64 x 192 column with 4 bubbles of diameter 3; g = 1e-4, sigma = 1e-4."""
    pos = np.array([[26.0, 38.0, 26.0, 38.0], [26.0, 26.0, 38.0, 38.0], [20.0, 24.0, 28.0, 32.0]])
    return Workload("adjoint_64x64x192_4b", (64, 64, 192), float(omega), (BB,) * 6, pos,
                    np.full(4, 3.0), params(g=1e-4, sigma=1e-4, drag_scale=drag_scale,
                                            lift_scale=lift_scale), steps, "f32",
                    meta=dict(target=(1.15, 0.8, 1.5), theta0=(1.0, 1.0, 1.4), checkpoint=100))


STABILITY_OMEGAS = (1.90, 1.92, 1.94, 1.95, 1.96, 1.965, 1.97, 1.975, 1.98, 1.985, 1.99, 1.995,
                    1.998, 1.999, 1.9995, 1.9999)


# Air bubble in water (Table 3) and standard gravity, SI units
WATER_NU, WATER_RHO, AIR_RHO, WATER_SIGMA, GRAVITY = 1e-6, 1000.0, 1.0, 0.073, 9.81


@dataclass(frozen=True)
class _Column:
    """The paper's tank (App. A: 0.15 x 0.15 m, water level 0.45 m) resolving a bubble of d_b
    metres at grid spacing dx = aspect d_b, liquid step dt = 1e-4 s, water at 1000 kg/m^3 and 1 in
    lattice units. The conversion factors (lattice over physical) are LCF = 1/dx, TCF = 1/dt and
    MCF = LCF^3 / 1000 (App. A); the columns' inputs are converted here, independently of the
    package's own units module."""
    d_b: float
    aspect: float
    dt: float = 1e-4

    @property
    def lcf(self):
        return 1.0 / (self.aspect * self.d_b)

    @property
    def tcf(self):
        return 1.0 / self.dt

    @property
    def mcf(self):
        return self.lcf ** 3 / WATER_RHO

    def cells(self, metres):
        return round(metres * self.lcf)

    @property
    def shape(self):
        return (self.cells(0.15), self.cells(0.15), self.cells(0.45))

    @property
    def d_lu(self):
        return self.d_b * self.lcf

    @property
    def g(self):
        return GRAVITY * self.lcf / self.tcf ** 2

    @property
    def sigma(self):
        return WATER_SIGMA * self.mcf / self.tcf ** 2

    @property
    def omega(self):
        # nu = (1/omega - 1/2) / 3 in lattice units (eq. (9))
        return 1.0 / (3.0 * WATER_NU * self.lcf ** 2 / self.tcf + 0.5)


def stability(steps=20000, omegas=STABILITY_OMEGAS):
    """The stability sweep (Sec. 4.3): the App. A column (0.15 x 0.15 x 0.45 m tank at aspect ratio
    1.25 for a 4 mm bubble: 30 x 30 x 90 cells, d = 0.8) with g and sigma of air in water converted
    to lattice units (g = 9.81 m/s^2, sigma = 0.073 N/m, dt = 1e-4 s), bounce-back walls and bottom,
    free-slip top, the bubble released at the bottom centre; one column per omega."""
    col = _Column(0.004, 1.25)
    nx, ny, nz = col.shape
    pos = np.array([[nx / 2 - 0.5], [ny / 2 - 0.5], [3.0]])
    bc = (BB, BB, BB, BB, BB, FS)
    return [Workload(f"stability_omega{om}", (nx, ny, nz), float(om), bc, pos.copy(),
                     np.array([col.d_lu]), params(g=col.g, sigma=col.sigma), steps, "f32")
            for om in omegas]


# gravity (lattice units) of the bubble swarms that drive the liquid hard enough for the BGK step
# to go unstable near omega = 2: 32 swarm bubbles in 16 x 16 x 48 raise a plume of |u| ~ 0.25
SWARM_G = 3e-2


def swarm(nb=32, omega=1.995, shape=(16, 16, 48), g=SWARM_G, seed=5, bc=(BB,) * 6, steps=1000,
          dtype="f64"):
    """A swarm of nb bubbles, diameters uniform in [2, 3], placed uniformly in the lower 5/12 of
    the column at least 3 cells from the side walls and the bottom. With g = 3e-2 their buoyancy
    drives a plume fast enough (|u| ~ 0.2-0.4) that the BGK liquid loses stability as omega
    approaches 2: the stability test of Sec. 4.3 with the forcing made strong."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    d = rng.uniform(2.0, 3.0, nb)
    pos = np.stack([rng.uniform(3, nx - 4, nb), rng.uniform(3, ny - 4, nb),
                    rng.uniform(3, nz * 5 / 12, nb)])
    return Workload(f"swarm_{nx}x{ny}x{nz}_{nb}b_omega{omega}", tuple(shape), float(omega), tuple(bc),
                    pos, d, params(g=g, sigma=sigma_for(g, 2.5)), steps, dtype,
                    meta=dict(nb=nb))


SWARM_OMEGAS = (1.90, 1.93, 1.95, 1.96, 1.97, 1.98, 1.99, 1.995)
SWARM_COUNTS = (16, 64, 256, 320, 384, 448, 512, 768)


def stability_swarm(steps=3000, omegas=SWARM_OMEGAS, counts=SWARM_COUNTS):
    """The stability map (Sec. 4.3) over omega and forcing: the App. A column (30 x 30 x 90,
    bounce-back walls and bottom, free-slip top) holding a swarm of 16 to 768 bubbles (the forcing
    axis: one batch shares g, so the swarm size varies), one column per (omega, swarm size)."""
    return [swarm(nb=n, omega=om, shape=(30, 30, 90), bc=(BB, BB, BB, BB, BB, FS), steps=steps,
                  dtype="f32", seed=SEED + n)
            for n in counts for om in omegas]


GRID_CASES = ((0.004, 1.25), (0.004, 0.625), (0.004, 0.3125),
              (0.008, 1.25), (0.008, 0.625), (0.008, 0.3125),
              (0.010, 1.25), (0.010, 0.625), (0.010, 0.3125))


TERMINAL_DIAMETERS_MM = (2, 3, 4, 5, 6, 7, 8, 9, 10)


def terminal_sweep(steps=10000, aspect=1.25, diameters_mm=TERMINAL_DIAMETERS_MM):
    """The terminal-velocity sweep of Sec. 4.1 (Table 4): air bubbles of 2 to 10 mm in the
    0.15 x 0.15 x 0.45 m water tank at one aspect ratio dx / d_b (1.25, App. A), built as the
    grid-independence columns (the tank rounded to whole cells)."""
    return grid_independence(steps, cases=tuple((d * 1e-3, aspect) for d in diameters_mm))


def grid_independence(steps=10000, cases=GRID_CASES, release=0.02):
    """The grid-independence study (Sec. 4.2, Tables 5 and 6): the 0.15 x 0.15 x 0.45 m tank for
    bubbles of 4, 8 and 10 mm at aspect ratios dx / d_b of 1.25, 0.625 and 0.3125, the Table 3
    properties (water: nu = 1e-6 m^2/s, so omega is 1.9992 to 1.99999; air at 1 kg/m^3;
    sigma = 0.073 N/m; g = 9.81 m/s^2) converted to lattice units per App. A with dt = 1e-4 s;
    bounce-back walls and bottom, free-slip top; the bubble released at rest `release` metres
    above the bottom on the axis. 10000 steps are 1 s of rise."""
    out = []
    for d_b, aspect in cases:
        col = _Column(d_b, aspect)
        nx, ny, nz = col.shape
        pos = np.array([[nx / 2 - 0.5], [ny / 2 - 0.5], [release * col.lcf]])
        p = params(g=col.g, sigma=col.sigma, rho_b=AIR_RHO / WATER_RHO)
        out.append(Workload(f"grid_{int(d_b * 1000)}mm_ar{aspect}", (nx, ny, nz), float(col.omega),
                            (BB, BB, BB, BB, BB, FS), pos, np.array([col.d_lu]), p, steps, "f32",
                            meta=dict(d_mm=d_b * 1000, aspect=aspect, lcf=col.lcf, tcf=col.tcf)))
    return out


def with_steps(w: Workload, steps: int) -> Workload:
    return replace(w, steps=steps)


def random_populations(shape, amp, seed=SEED, dtype=np.float64):
    """Random shifted populations g = f - w of amplitude amp, layout (19, nz, ny, nx)."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, (19, nz, ny, nx)).astype(dtype)


def random_field(shape, amp, seed=SEED, dtype=np.float64):
    """Random vector field, layout (3, nz, ny, nx)."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, (3, nz, ny, nx)).astype(dtype)
