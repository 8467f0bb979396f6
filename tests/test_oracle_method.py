"""Pins of the oracle's coupled step (Algorithm 1): conservation laws that hold for the whole
two-way coupled update, and the qualitative rise of the single-bubble column."""
import numpy as np
import pytest

import oracle as O

BB, FS, PER = O.BC_BOUNCE_BACK, O.BC_FREE_SLIP, O.BC_PERIODIC


def _params(**kw):
    base = dict(g=1e-4, rho_l=1.0, rho_b=1e-3, sigma=1e-4, c_a=0.5)
    base.update(kw)
    return O.bubble_params(**base)


def test_periodic_box_momentum_equals_sum_of_reactions():
    """Periodic box: the liquid gains exactly the reactions -(F_D + F_L) of all bubbles."""
    c, _, _ = O.lattice()
    c = c.astype(float)
    lat = O.Lattice(20, 18, 24, 1.4, (PER,) * 6)
    bub = O.Bubbles(pos=[[5.2, 12.7, 3.1], [4.4, 9.0, 17.5], [10.0, 11.3, 23.6]], d=[3.0, 2.0, 2.5])
    P = _params()
    for _ in range(60):
        P0 = np.einsum("qa,qzyx->a", c, lat.g)
        psi = O.method_step(lat, P, bub)
        P1 = np.einsum("qa,qzyx->a", c, lat.g)
        scale = np.abs(psi).sum() + 1e-30
        assert np.allclose(P1 - P0, psi.sum(axis=1), rtol=0, atol=1e-12 * scale)
    assert np.all(bub.state == 2) and np.all(bub.vel[2] > 0)


def test_walls_conserve_mass_with_bubbles():
    lat = O.Lattice(16, 16, 32, 1.0, (BB, BB, BB, BB, BB, FS))
    bub = O.Bubbles(pos=[[8.0, 8.0, 6.0], [0.6, 15.2, 3.0]], d=[3.0, 2.0])
    P = _params()
    m0 = lat.g.sum()
    for _ in range(50):
        O.method_step(lat, P, bub)
    assert abs(lat.g.sum() - m0) < 1e-15
    assert np.isfinite(lat.g).all()


def test_single_bubble_column_rises_and_drives_the_liquid():
    """Plain FP64 single-bubble column (32 x 32 x 64, omega = 1, bounce-back walls, d = 3 at
    (16, 16, 8), g = 1e-5, density ratio 1e-3): the bubble rises and drags the liquid up."""
    lat = O.Lattice(32, 32, 64, 1.0, (BB,) * 6)
    bub = O.Bubbles(pos=[[16.0], [16.0], [8.0]], d=[3.0])
    P = O.bubble_params(g=1e-5, rho_l=1.0, rho_b=1e-3, sigma=4.19e-5)
    traj = O.run(lat, P, bub, 40, record=True)
    assert np.all(np.diff(traj[:, 2, 0]) > 0)
    # (16, 16) is half a cell off the column axis (15.5, 15.5): a tiny lateral drift is physical,
    # but the start is symmetric under the exchange of x and y
    assert abs(traj[-1, 0, 0] - 16.0) < 1e-6 and traj[-1, 0, 0] == pytest.approx(traj[-1, 1, 0], abs=1e-14)
    assert lat.U[2, 8, 16, 16] > 0


def test_bubble_deactivates_at_top_and_stops_forcing():
    lat = O.Lattice(12, 12, 16, 1.0, (BB,) * 6)
    bub = O.Bubbles(pos=[[6.0], [6.0], [14.99]], d=[2.0], vel=[[0.0], [0.0], [0.05]])
    P = _params()
    psi = O.method_step(lat, P, bub)
    assert bub.state[0] == 0 and np.abs(psi).sum() > 0
    z_stop = bub.pos[2, 0]
    psi2 = O.method_step(lat, P, bub)
    assert np.all(psi2 == 0) and bub.pos[2, 0] == z_stop


def test_neutrally_buoyant_bubble_follows_a_uniformly_accelerating_liquid():
    """Pins the fluid-acceleration terms of the bubble ODE in the coupled step (readings R7, R9): a
    neutrally buoyant bubble (rho_b = rho_l) without drag in a liquid whose velocity grows by the
    same vector a every step accelerates exactly with the liquid, since the stress-gradient and
    added-mass force (1 + C_A) rho_l V D_t u_l equals m_eff a with m_eff = (rho_b + C_A rho_l) V.
    The liquid velocity of each step is prescribed (the field the previous collision leaves,
    uniform in a periodic box, so the interpolated vorticity is exactly 0); D_t u_l is the change
    of the interpolated velocity since the previous step and 0 on the bubble's first step. So after
    step n the bubble moves at (n - 1) a, and its position gains dt_b sum of its sub-step
    velocities."""
    a = np.array([2e-4, -1e-4, 3e-4])
    lat = O.Lattice(8, 8, 8, 1.2, (PER,) * 6)
    x0 = np.array([3.3, 4.1, 2.7])
    bub = O.Bubbles(pos=x0.reshape(3, 1), d=[2.0])
    P = _params(rho_b=1.0, drag_scale=0.0, g=1e-3, sigma=1e-3)
    x = x0.copy()
    for n in range(1, 13):
        lat.U[:] = (a * n)[:, None, None, None]  # the liquid velocity this step's bubble half reads
        O.method_step(lat, P, bub)
        v_expect = (n - 1) * a
        assert np.allclose(bub.vel[:, 0], v_expect, rtol=0, atol=1e-15)
        # ten sub-steps of dt_b = 0.1, each moving the bubble by dt_b times its new velocity, which
        # gains a / 10 per sub-step from (n - 2) a: sum_k 0.1 ((n - 2) a + k a / 10) over k = 1..10
        # is (n - 1) a - 0.45 a (no motion on the first step)
        if n > 1:
            x = x + v_expect - 0.45 * a
        assert np.allclose(bub.pos[:, 0], np.mod(x, 8.0), rtol=0, atol=1e-12)
        assert np.allclose(bub.ulp[:, 0], a * n, rtol=0, atol=1e-16)


def test_lateral_wall_clamp_stops_only_the_normal_motion():
    """Pins the lateral clamp (reading R14): a bubble driven into the x = 0 wall ends the step at
    x = 0 exactly with u_x = 0, while its y and z motion is that of the same bubble without the
    lateral velocity. In quiescent liquid (the first step: U = 0, so u_l = w_l = 0 and no lift)
    with the Stokes drag alone (cd_k = 0, |u_r| d / nu small, so C_D |u_r| = 24 nu / d) every
    force on the bubble is linear and acts per component, so the clamped x motion cannot reach y
    or z; an error that zeroed the wrong component, clamped to the wrong cell or moved the bubble
    back by another rule fails one of the equalities."""
    lat_a = O.Lattice(16, 16, 24, 1.0)
    lat_b = O.Lattice(16, 16, 24, 1.0)
    P = _params(cd_k=0.0, g=1e-5, sigma=1e-5)
    pos = [[0.02], [7.4], [8.2]]
    a = O.Bubbles(pos=pos, d=[2.0], vel=[[-0.1], [0.003], [0.002]])
    b = O.Bubbles(pos=pos, d=[2.0], vel=[[0.0], [0.003], [0.002]])
    O.method_step(lat_a, P, a)
    O.method_step(lat_b, P, b)
    assert a.pos[0, 0] == 0.0 and a.vel[0, 0] == 0.0
    assert b.pos[0, 0] == 0.02 and b.vel[0, 0] == 0.0
    assert np.array_equal(a.pos[1:], b.pos[1:]) and np.array_equal(a.vel[1:], b.vel[1:])
    assert a.pos[1, 0] != 7.4 and a.pos[2, 0] != 8.2  # the other components moved
    # the same at the far wall, x = nx - 1
    c = O.Bubbles(pos=[[14.98], [7.4], [8.2]], d=[2.0], vel=[[0.1], [0.003], [0.002]])
    O.method_step(O.Lattice(16, 16, 24, 1.0), P, c)
    assert c.pos[0, 0] == 15.0 and c.vel[0, 0] == 0.0
    assert np.array_equal(c.pos[1:], b.pos[1:]) and np.array_equal(c.vel[1:], b.vel[1:])
