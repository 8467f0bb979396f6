"""Pins of the oracle's liquid step (Sec. 2.2 eq. (13)-(16), Sec. 3.3 boundary conditions):
streaming rules on single populations, exact conservation, the periodic momentum balance and the
body-force Poiseuille closed form with bounce-back walls and with a free-slip face."""
import numpy as np
import pytest

import oracle as O

BB, FS, PER = O.BC_BOUNCE_BACK, O.BC_FREE_SLIP, O.BC_PERIODIC


def _q(c, v):
    return int(np.where((c == np.array(v)).all(axis=1))[0][0])


def _single(nx, ny, nz, q, x, y, z, val=1.0):
    post = np.zeros((19, nz, ny, nx))
    post[q, z, y, x] = val
    return post


def test_stream_interior_moves_along_c():
    c, _, _ = O.lattice()
    for q in range(19):
        post = _single(5, 6, 7, q, 2, 3, 3)
        pre = O.stream(post, (BB,) * 6)
        x, y, z = 2 + c[q, 0], 3 + c[q, 1], 3 + c[q, 2]
        assert pre[q, z, y, x] == 1.0 and pre.sum() == 1.0


def test_stream_bounce_back_returns_reversed_in_place():
    c, _, opp = O.lattice()
    nx, ny, nz = 4, 4, 4
    for q in range(18):
        # start next to the wall the population points at
        x = 0 if c[q, 0] < 0 else (nx - 1 if c[q, 0] > 0 else 1)
        y = 0 if c[q, 1] < 0 else (ny - 1 if c[q, 1] > 0 else 1)
        z = 0 if c[q, 2] < 0 else (nz - 1 if c[q, 2] > 0 else 1)
        pre = O.stream(_single(nx, ny, nz, q, x, y, z), (BB,) * 6)
        assert pre[opp[q], z, y, x] == 1.0 and pre.sum() == 1.0


def test_stream_free_slip_top_reflects_specularly():
    c, _, opp = O.lattice()
    nx, ny, nz = 5, 5, 4
    bc = (BB, BB, BB, BB, BB, FS)
    for q in range(18):
        if c[q, 2] != 1:
            continue
        pre = O.stream(_single(nx, ny, nz, q, 2, 2, nz - 1), bc)
        qm = _q(c, (c[q, 0], c[q, 1], -1))
        assert pre[qm, nz - 1, 2 + c[q, 1], 2 + c[q, 0]] == 1.0 and pre.sum() == 1.0
    # at an edge where the mirrored source leaves the domain sideways: bounce-back
    q = _q(c, (1, 0, 1))
    pre = O.stream(_single(nx, ny, nz, q, nx - 1, 2, nz - 1), bc)
    assert pre[opp[q], nz - 1, 2, nx - 1] == 1.0 and pre.sum() == 1.0


def test_stream_periodic_wraps():
    c, _, _ = O.lattice()
    q = _q(c, (-1, 1, 0))
    pre = O.stream(_single(3, 4, 5, q, 0, 3, 0), (PER,) * 6)
    assert pre[q, 0, 0, 2] == 1.0 and pre.sum() == 1.0
    q = _q(c, (0, -1, -1))
    pre = O.stream(_single(3, 4, 5, q, 1, 0, 0), (PER,) * 6)
    assert pre[q, 4, 3, 1] == 1.0 and pre.sum() == 1.0


def _random_state(rng, shape, amp=1e-3):
    nx, ny, nz = shape
    return rng.uniform(-amp, amp, (19, nz, ny, nx))


@pytest.mark.parametrize("bc", [(BB,) * 6, (BB, BB, BB, BB, BB, FS), (PER,) * 6,
                                (PER, PER, BB, BB, FS, FS), (FS,) * 6])
def test_mass_conservation(bc):
    rng = np.random.default_rng(10)
    lat = O.Lattice(7, 6, 9, 1.7, bc, g=_random_state(rng, (7, 6, 9)))
    m0 = lat.g.sum()
    for _ in range(40):
        F = rng.uniform(-1e-4, 1e-4, (3, 9, 6, 7))
        lat.step(F)
        assert abs(lat.g.sum() - m0) < 1e-15
    assert np.isfinite(lat.g).all()


def test_periodic_momentum_balance():
    """Fully periodic box: the total momentum grows by exactly the total body force per step."""
    c, _, _ = O.lattice()
    c = c.astype(float)
    rng = np.random.default_rng(11)
    lat = O.Lattice(6, 5, 7, 1.2, (PER,) * 6, g=_random_state(rng, (6, 5, 7)))
    for _ in range(30):
        P0 = np.einsum("qa,qzyx->a", c, lat.g)
        F = rng.uniform(-1e-4, 1e-4, (3, 7, 5, 6))
        lat.step(F)
        P1 = np.einsum("qa,qzyx->a", c, lat.g)
        assert np.allclose(P1 - P0, F.sum(axis=(1, 2, 3)), rtol=0, atol=5e-16)


def _poiseuille(N, omega, F, width):
    """Steady body-force channel flow with half-way bounce-back walls at x = -1/2 and
    x = width - 1/2 under BGK with Guo forcing: the exact parabola plus the known slip of the
    half-way bounce-back wall, F/rho [(2 tau - 1)^2 - 3/4] / (2 tau - 1) (zero at
    tau = 1/2 + sqrt(3)/4)."""
    tau = 1 / omega
    nu = (2 * tau - 1) / 6
    x = np.arange(N)
    return F / (2 * nu) * (x + 0.5) * (width - 0.5 - x) + F * ((2 * tau - 1) ** 2 - 0.75) / (2 * tau - 1)


@pytest.mark.parametrize("omega,steps", [(0.6, 6000), (1.0, 8000), (1.6, 40000)])
def test_poiseuille_bounce_back(omega, steps):
    N, Fz = 12, 1e-6
    lat = O.Lattice(N, 1, 1, omega, (BB, BB, PER, PER, PER, PER))
    F = np.zeros((3, 1, 1, N))
    F[2] = Fz
    for _ in range(steps):
        lat.step(F)
    ex = _poiseuille(N, omega, Fz, N)
    assert np.max(np.abs(lat.U[2, 0, 0] - ex)) / ex.max() < 1e-12
    assert np.abs(lat.U[:2]).max() < 1e-18 * ex.max() / 1e-5


def test_poiseuille_magic_tau_is_exact_parabola():
    omega = 1 / (0.5 + np.sqrt(3) / 4)
    N, Fz = 10, 1e-6
    lat = O.Lattice(N, 1, 1, omega, (BB, BB, PER, PER, PER, PER))
    F = np.zeros((3, 1, 1, N))
    F[2] = Fz
    for _ in range(8000):
        lat.step(F)
    tau = 1 / omega
    nu = (2 * tau - 1) / 6
    x = np.arange(N)
    ex = Fz / (2 * nu) * (x + 0.5) * (N - 0.5 - x)
    assert np.max(np.abs(lat.U[2, 0, 0] - ex)) / ex.max() < 1e-12


def test_free_slip_half_channel_is_mirror_of_full_channel():
    """Bounce-back at the bottom, free slip at the top (Sec. 3.3): the flow equals the lower half
    of a channel twice as wide."""
    N, Fx, omega = 10, 1e-6, 0.8
    lat = O.Lattice(3, 2, N, omega, (PER, PER, PER, PER, BB, FS))
    F = np.zeros((3, N, 2, 3))
    F[0] = Fx
    for _ in range(30000):
        lat.step(F)
    ex = _poiseuille(N, omega, Fx, 2 * N)
    assert np.max(np.abs(lat.U[0, :, 1, 1] - ex)) / ex.max() < 1e-12


def test_moments_of_rest_state():
    lat = O.Lattice(4, 3, 5, 1.0)
    rho, u, sums = lat.moments()
    assert np.all(rho == 1.0) and np.all(u == 0.0)
    assert sums[0] == 60.0 and np.all(sums[1:] == 0.0)


def test_uniform_shear_vorticity():
    """Central-difference curl of a linear field is exact; bounce-back ghosts keep it exact for a
    shear that vanishes on the wall plane (zero velocity at z = -1/2)."""
    nx, ny, nz = 6, 7, 8
    gam = 1e-3
    z = np.arange(nz)[:, None, None] * np.ones((nz, ny, nx))
    U = np.zeros((3, nz, ny, nx))
    U[0] = gam * (z + 0.5)
    w = O.curl(U, (PER, PER, PER, PER, BB, BB))
    assert np.allclose(w[1, :-1], gam, rtol=1e-13, atol=0)  # top wall is at nz - 1/2, U != 0 there
    assert np.abs(w[0]).max() == 0 and np.abs(w[2]).max() == 0
    # each component and each direction: U_z = gam x gives w_y = -gam; U_y = gam x gives w_z = gam
    x = np.arange(nx)[None, None, :] * np.ones((nz, ny, nx))
    U = np.zeros((3, nz, ny, nx))
    U[2] = gam * x
    w = O.curl(U, (FS, FS, PER, PER, PER, PER))
    assert np.allclose(w[1, :, :, 1:-1], -gam, rtol=1e-13, atol=0)
    U = np.zeros((3, nz, ny, nx))
    U[1] = gam * x
    w = O.curl(U, (PER,) * 6)
    assert np.allclose(w[2, :, :, 1:-1], gam, rtol=1e-13, atol=0)
    y = np.arange(ny)[None, :, None] * np.ones((nz, ny, nx))
    U = np.zeros((3, nz, ny, nx))
    U[2] = gam * y
    w = O.curl(U, (PER,) * 6)
    assert np.allclose(w[0, :, 1:-1, :], gam, rtol=1e-13, atol=0)


def test_free_slip_ghost_keeps_tangential_velocity():
    nx, ny, nz = 4, 4, 5
    U = np.zeros((3, nz, ny, nx))
    U[0] = 2e-3  # uniform tangential flow along a free-slip top and bottom
    w = O.curl(U, (PER, PER, PER, PER, FS, FS))
    assert np.abs(w).max() == 0
    w = O.curl(U, (PER, PER, PER, PER, BB, BB))  # no-slip walls: shear at the wall rows
    assert np.allclose(w[1, 0], 2e-3) and np.allclose(w[1, -1], -2e-3)
