"""Plain FP64 CPU oracle of the arXiv 1710.07073 bubble-column method (LBGK + LPT, two-way).

TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked against. Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it. It shares no
code with the GPU library (``paper_1710_07073_amd``) and never imports it.

The arithmetic lives in ``lbm_oracle.cpp`` (plain loops, double precision, built with
``-O2 -ffp-contract=off``); this module only marshals numpy arrays through ctypes and loops
over steps. Section / equation / table / algorithm citations are to the paper:

* ``lattice``, ``equilibrium``, ``guo_source``, ``collide_node``: Sec. 2.2, eq. (5)-(15)
* ``lbm_step``, ``stream``: Sec. 2.2, eq. (16) + Sec. 3.3 boundary conditions
* ``moments``: eq. (10)
* ``kernel_Z``, ``kernel_P``, ``axis_weights``, ``interpolate``, ``spread``: Sec. 3.2, eq. (18)-(21)
* ``closures``, ``drag_lift``, ``bubble_ode``: Sec. 2.1, eq. (1)-(4), Table 1
* ``method_step``, ``run``: Algorithm 1
* coupling variants (``bubble_params(coupling=...)``, bits ``REACTION_SUBSTEP_MEAN``,
  ``REACTION_NET_FORCE``, ``POINT_KERNEL``, ``EXACT_TIME``): the reaction of Sec. 3.2 against that
  of Algorithm 1, point-sampled instead of cell-integral weights (eq. (18)-(19)), and the time
  level of the forward coupling

Populations are stored shifted, g = f - w, structure-of-arrays ``g[q, z, y, x]`` in the
paper's velocity order (axis directions, face diagonals, rest).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
import time
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.cpp")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

BC_BOUNCE_BACK, BC_FREE_SLIP, BC_PERIODIC = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (plain C++17, no GPU code)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
               _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class BubbleParams(ct.Structure):
    """Bubble-phase constants (Table 1, Table 3; readings for the garbled constants)."""
    _fields_ = [("g", ct.c_double), ("rho_l", ct.c_double), ("rho_b", ct.c_double),
                ("sigma", ct.c_double), ("c_a", ct.c_double), ("drag_scale", ct.c_double),
                ("lift_scale", ct.c_double), ("kernel_factor", ct.c_double), ("cd_k", ct.c_double),
                ("lift_f0", ct.c_double), ("n_sub", ct.c_int32), ("coupling", ct.c_int32)]

# coupling variant bits (lbm_oracle.cpp, ORC_*)
REACTION_SUBSTEP_MEAN = 1
REACTION_NET_FORCE = 2
POINT_KERNEL = 4
EXACT_TIME = 8


def bubble_params(g=1e-5, rho_l=1.0, rho_b=1e-3, sigma=4.19e-5, c_a=0.5, drag_scale=1.0,
                  lift_scale=1.0, kernel_factor=1.5, cd_k=0.15, lift_f0=0.474, n_sub=10,
                  coupling=0):
    return BubbleParams(g, rho_l, rho_b, sigma, c_a, drag_scale, lift_scale, kernel_factor, cd_k,
                        lift_f0, n_sub, int(coupling))


_lib = None
_D = ct.POINTER(ct.c_double)
_I = ct.POINTER(ct.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ct.CDLL(_LIB)
        L.orc_lattice.argtypes = [_I, _D, _I]
        L.orc_equilibrium.argtypes = [ct.c_double, _D, _D]
        L.orc_equilibrium.restype = None
        L.orc_guo_source.argtypes = [ct.c_double, _D, _D, _D]
        L.orc_guo_source.restype = None
        L.orc_collide_node.argtypes = [ct.c_double, _D, _D, _D, _D, _D]
        L.orc_collide_node.restype = None
        L.orc_kernel_Z.argtypes = [ct.c_double, ct.c_double]
        L.orc_kernel_Z.restype = ct.c_double
        L.orc_kernel_P.argtypes = [ct.c_double]
        L.orc_kernel_P.restype = ct.c_double
        L.orc_axis_weights.argtypes = [ct.c_double, ct.c_double, ct.c_int, ct.c_int, _I, _D, ct.c_int,
                                       ct.c_int]
        L.orc_lbm_step.argtypes = [ct.c_int, ct.c_int, ct.c_int, _I, ct.c_double, _D, _D, _D, _D,
                                   ct.c_int]
        L.orc_stream.argtypes = [ct.c_int, ct.c_int, ct.c_int, _I, _D, _D]
        L.orc_moments.argtypes = [ct.c_int, ct.c_int, ct.c_int, _D, _D, _D, _D]
        L.orc_curl.argtypes = [ct.c_int, ct.c_int, ct.c_int, _I, _D, _D]
        L.orc_closures.argtypes = [ct.POINTER(BubbleParams), ct.c_double, ct.c_double, ct.c_double,
                                   _D, _D, _D]
        L.orc_closures.restype = None
        L.orc_drag_lift.argtypes = [ct.POINTER(BubbleParams), ct.c_double, ct.c_double, _D, _D, _D,
                                    _D, _D]
        L.orc_drag_lift.restype = None
        L.orc_bubble_ode.argtypes = [ct.POINTER(BubbleParams), ct.c_double, ct.c_double, ct.c_int,
                                     ct.c_double, _D, _D, _D, _D, _D, _D, _D, _I, _I, _D, _D]
        L.orc_bubble_ode.restype = None
        L.orc_interpolate.argtypes = [ct.c_int, ct.c_int, ct.c_int, _I, _D, _D, ct.c_double, _D, _D,
                                      ct.c_int]
        L.orc_spread.argtypes = [ct.c_int, ct.c_int, ct.c_int, _I, _D, ct.c_double, _D, _D, ct.c_int]
        L.orc_method_step.argtypes = [ct.c_int, ct.c_int, ct.c_int, _I, ct.c_double,
                                      ct.POINTER(BubbleParams), ct.c_int, _D, _D, _D, _D, _I, _D, _D,
                                      _D, _D, _D, ct.c_int]
        _lib = L
    return _lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _i(a):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_I)


def _vec(x, n=3):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(n))


def _bc(bc):
    return np.ascontiguousarray(np.asarray(bc, dtype=np.int32).reshape(6))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


# ------------------------------------------------------------------------------------------
# Lattice and node-level arithmetic (eq. (5)-(15))
# ------------------------------------------------------------------------------------------
def lattice():
    """D3Q19 velocities (19x3 int), weights (19) and opposite index (19), eq. (7)-(8)."""
    c = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, np.int32)
    lib().orc_lattice(_i(c), _d(w), _i(opp))
    return c, w, opp


def equilibrium(rho, u):
    """Unshifted equilibrium f_eq of eq. (6)."""
    out = np.zeros(19)
    lib().orc_equilibrium(float(rho), _d(_vec(u)), _d(out))
    return out


def guo_source(omega, u, F):
    """Discrete force term of eq. (12)."""
    out = np.zeros(19)
    lib().orc_guo_source(float(omega), _d(_vec(u)), _d(_vec(F)), _d(out))
    return out


def collide_node(omega, g, F):
    """Shifted pre-collision populations -> shifted post-collision (eq. (13)-(15)), rho, u."""
    out = np.zeros(19)
    rho = np.zeros(1)
    u = np.zeros(3)
    lib().orc_collide_node(float(omega), _d(_vec(g, 19)), _d(_vec(F)), _d(out), _d(rho), _d(u))
    return out, float(rho[0]), u


# ------------------------------------------------------------------------------------------
# Lattice fields
# ------------------------------------------------------------------------------------------
@dataclass
class Lattice:
    """A liquid lattice: shape (nx, ny, nz), faces (-x,+x,-y,+y,-z,+z), relaxation omega."""
    nx: int
    ny: int
    nz: int
    omega: float
    bc: tuple = (0, 0, 0, 0, 0, 0)
    g: np.ndarray = field(default=None, repr=False)
    tmp: np.ndarray = field(default=None, repr=False)
    U: np.ndarray = field(default=None, repr=False)
    F: np.ndarray = field(default=None, repr=False)

    def __post_init__(self):
        shp = (self.nz, self.ny, self.nx)
        if self.g is None:
            self.g = np.zeros((19,) + shp)  # fluid at rest, rho = 1 (Algorithm 1 initialisation)
        self.tmp = np.zeros((19,) + shp)
        if self.U is None:
            self.U = np.zeros((3,) + shp)
        if self.F is None:
            self.F = np.zeros((3,) + shp)
        self._bc = _bc(self.bc)

    @property
    def shape(self):
        return (self.nx, self.ny, self.nz)

    @property
    def cells(self):
        return self.nx * self.ny * self.nz

    def step(self, F=None, nthreads=0):
        """One liquid step with force field F (3, nz, ny, nx) or none; updates g and U."""
        Fp = None if F is None else np.ascontiguousarray(F, dtype=np.float64)
        _check(lib().orc_lbm_step(self.nx, self.ny, self.nz, _i(self._bc), float(self.omega),
                                  _d(self.g), _d(self.tmp), _d(Fp), _d(self.U), int(nthreads)),
               "lbm_step")

    def moments(self):
        N = self.cells
        rho = np.zeros((self.nz, self.ny, self.nx))
        u = np.zeros((3, self.nz, self.ny, self.nx))
        sums = np.zeros(4)
        _check(lib().orc_moments(self.nx, self.ny, self.nz, _d(self.g), _d(rho), _d(u), _d(sums)),
               "moments")
        del N
        return rho, u, sums


def stream(post, bc):
    """Streaming eq. (16) with the boundary rules, post-collision -> pre-collision populations."""
    post = np.ascontiguousarray(post, dtype=np.float64)
    _, nz, ny, nx = post.shape
    pre = np.zeros_like(post)
    _check(lib().orc_stream(nx, ny, nz, _i(_bc(bc)), _d(post), _d(pre)), "stream")
    return pre


def curl(U, bc):
    U = np.ascontiguousarray(U, dtype=np.float64)
    _, nz, ny, nx = U.shape
    out = np.zeros_like(U)
    _check(lib().orc_curl(nx, ny, nz, _i(_bc(bc)), _d(U), _d(out)), "curl")
    return out


# ------------------------------------------------------------------------------------------
# Mapping kernel (eq. (18)-(21))
# ------------------------------------------------------------------------------------------
def kernel_Z(r, n):
    return lib().orc_kernel_Z(float(r), float(n))


def kernel_P(s):
    return lib().orc_kernel_P(float(s))


def axis_weights(xb, n, N, periodic=False, point=False):
    cap = 4 * int(np.ceil(n)) + 8
    idx = np.zeros(cap, np.int32)
    w = np.zeros(cap)
    k = lib().orc_axis_weights(float(xb), float(n), int(N), int(bool(periodic)), _i(idx), _d(w), cap,
                               int(bool(point)))
    if k < 0:
        raise ValueError("axis_weights capacity or empty point-sampled window")
    return idx[:k].copy(), w[:k].copy()


def interpolate(U, bc, xb, n, point=False):
    U = np.ascontiguousarray(U, dtype=np.float64)
    _, nz, ny, nx = U.shape
    ul = np.zeros(3)
    wl = np.zeros(3)
    _check(lib().orc_interpolate(nx, ny, nz, _i(_bc(bc)), _d(U), _d(_vec(xb)), float(n), _d(ul),
                                 _d(wl), int(bool(point))), "interpolate")
    return ul, wl


def spread(F, bc, xb, n, psi, point=False):
    """F (3, nz, ny, nx) += psi * W, in place."""
    assert F.dtype == np.float64 and F.flags.c_contiguous
    _, nz, ny, nx = F.shape
    _check(lib().orc_spread(nx, ny, nz, _i(_bc(bc)), _d(_vec(xb)), float(n), _d(_vec(psi)), _d(F),
                            int(bool(point))), "spread")
    return F


# ------------------------------------------------------------------------------------------
# Bubble dynamics (eq. (1)-(4), Table 1)
# ------------------------------------------------------------------------------------------
def closures(P, nu, d, ur_mag):
    """(C_D |u_r|, C_L, Re) of Table 1 / eq. (3)."""
    cdu, cl, re = np.zeros(1), np.zeros(1), np.zeros(1)
    lib().orc_closures(ct.byref(P), float(nu), float(d), float(ur_mag), _d(cdu), _d(cl), _d(re))
    return float(cdu[0]), float(cl[0]), float(re[0])


def drag_lift(P, nu, d, ub, ul, wl):
    FD, FL = np.zeros(3), np.zeros(3)
    lib().orc_drag_lift(ct.byref(P), float(nu), float(d), _d(_vec(ub)), _d(_vec(ul)), _d(_vec(wl)),
                        _d(FD), _d(FL))
    return FD, FL


def bubble_ode(P, nu, dt_b, n_sub, d, ul, wl, dul, ub, xb):
    """n_sub explicit sub-steps of eq. (4) in an unbounded liquid; returns (ub, xb, psi)."""
    ub = _vec(ub).copy()
    xb = _vec(xb).copy()
    psi = np.zeros(3)
    lib().orc_bubble_ode(ct.byref(P), float(nu), float(dt_b), int(n_sub), float(d), _d(_vec(ul)),
                         _d(_vec(wl)), _d(_vec(dul)), _d(ub), _d(xb), None, None, None, None, None,
                         _d(psi))
    return ub, xb, psi


# ------------------------------------------------------------------------------------------
# The coupled method (Algorithm 1)
# ------------------------------------------------------------------------------------------
@dataclass
class Bubbles:
    """Bubble state, structure of arrays: pos/vel/ulp (3, nb), d (nb), state (nb)."""
    pos: np.ndarray
    d: np.ndarray
    vel: np.ndarray = None
    ulp: np.ndarray = None
    state: np.ndarray = None

    def __post_init__(self):
        self.pos = np.ascontiguousarray(np.asarray(self.pos, np.float64).reshape(3, -1))
        nb = self.pos.shape[1]
        self.d = np.ascontiguousarray(np.asarray(self.d, np.float64).reshape(nb))
        self.vel = np.zeros((3, nb)) if self.vel is None else np.ascontiguousarray(self.vel, np.float64)
        self.ulp = np.zeros((3, nb)) if self.ulp is None else np.ascontiguousarray(self.ulp, np.float64)
        self.state = (np.ones(nb, np.int32) if self.state is None
                      else np.ascontiguousarray(self.state, np.int32))

    @property
    def nb(self):
        return self.pos.shape[1]


def method_step(lat: Lattice, P, bub: Bubbles, nthreads=0):
    """One step of Algorithm 1; returns the reactions psi (3, nb) spread in this step."""
    psi = np.zeros((3, max(bub.nb, 1)))
    _check(lib().orc_method_step(lat.nx, lat.ny, lat.nz, _i(lat._bc), float(lat.omega), ct.byref(P),
                                 bub.nb, _d(bub.pos), _d(bub.vel), _d(bub.d), _d(bub.ulp),
                                 _i(bub.state), _d(lat.g), _d(lat.tmp), _d(lat.F), _d(lat.U),
                                 _d(psi), int(nthreads)), "method_step")
    return psi[:, :bub.nb]


def run(lat: Lattice, P, bub: Bubbles, nsteps, record=False, nthreads=0):
    """nsteps of Algorithm 1; with record=True returns positions after every step (n, 3, nb)."""
    traj = np.zeros((nsteps, 3, bub.nb)) if record else None
    for n in range(nsteps):
        method_step(lat, P, bub, nthreads)
        if record:
            traj[n] = bub.pos
    return traj


def time_lbm(nx, ny, nz, omega, bc, nsteps, nthreads=0, nb=0, P=None, bub=None):
    """Wall time of nsteps oracle steps (for the CPU baseline); returns (seconds, cells)."""
    lat = Lattice(nx, ny, nz, omega, bc)
    if bub is not None:
        method_step(lat, P, bub, nthreads)  # warm-up
        t0 = time.perf_counter()
        for _ in range(nsteps):
            method_step(lat, P, bub, nthreads)
    else:
        lat.step(None, nthreads)
        t0 = time.perf_counter()
        for _ in range(nsteps):
            lat.step(None, nthreads)
    return time.perf_counter() - t0, lat.cells
