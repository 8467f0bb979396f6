"""Pins of the oracle's coupling variants (the alternatives to readings R3, R13 and R16).

* Reaction: the sub-step mean of -(F_D + F_L) is the impulse those forces gave the bubble over
  the liquid step, and minus the mean net force is minus the bubble's momentum change; both are
  checked through the momentum balance of the explicit sub-steps, not by re-evaluating the
  forces. At the terminal velocity the default and the sub-step mean agree and the net force
  vanishes.
* Point-sampled weights: a partition of unity on every axis, symmetric about a cell centre, and
  converging to the cell-integral weights of eq. (19) as the window widens (midpoint rule).
* Exact time: with no force in the liquid, the default coupling (the velocity of the previous
  collision) reads at step n + 1 what the exact-time variant reads at step n.
"""
import numpy as np
import pytest

import oracle as O

RHO_L, C_A = 1.0, 0.5


def _params(**kw):
    base = dict(g=1e-4, rho_l=RHO_L, rho_b=1e-3, sigma=1e-4, c_a=C_A)
    base.update(kw)
    return O.bubble_params(**base)


def _mass(P, d):
    V = np.pi * d ** 3 / 6.0
    return P.rho_b * V, P.rho_b * V + P.c_a * P.rho_l * V, (1.0 + P.c_a) * P.rho_l * V, \
        (P.rho_l - P.rho_b) * V * P.g


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_substep_mean_reaction_is_the_drag_and_lift_impulse(seed):
    rng = np.random.default_rng(seed)
    d, nu = 3.0, 0.02
    ul, wl, dul = rng.normal(0, 1e-3, 3), rng.normal(0, 1e-3, 3), rng.normal(0, 1e-5, 3)
    ub0 = rng.normal(0, 2e-3, 3)
    P = _params(coupling=O.REACTION_SUBSTEP_MEAN)
    ub, _, psi = O.bubble_ode(P, nu, 0.1, 10, d, ul, wl, dul, ub0, np.zeros(3))
    _, m_eff, va, fb = _mass(P, d)
    # m_eff (u1 - u0) = sum_k dt_b (F_D + F_L + va dul + F_B e_z) over dt_l = 1
    impulse = m_eff * (ub - ub0) - va * dul - np.array([0.0, 0.0, fb])
    assert np.allclose(psi, -impulse, rtol=1e-10, atol=1e-18)
    # the default reaction differs (forces at the final velocity only)
    _, _, psi_final = O.bubble_ode(_params(), nu, 0.1, 10, d, ul, wl, dul, ub0, np.zeros(3))
    assert np.abs(psi_final - psi).max() > 1e-3 * np.abs(psi).max()


@pytest.mark.parametrize("seed", [0, 1])
def test_net_force_reaction_is_minus_the_bubble_momentum_change(seed):
    rng = np.random.default_rng(10 + seed)
    d, nu = 2.5, 0.01
    ul, wl, dul = rng.normal(0, 1e-3, 3), rng.normal(0, 1e-3, 3), rng.normal(0, 1e-5, 3)
    ub0 = rng.normal(0, 2e-3, 3)
    P = _params(coupling=O.REACTION_NET_FORCE, rho_b=0.05)
    ub, _, psi = O.bubble_ode(P, nu, 0.1, 10, d, ul, wl, dul, ub0, np.zeros(3))
    m_b, _, _, _ = _mass(P, d)
    assert np.allclose(psi, -m_b * (ub - ub0), rtol=1e-10, atol=1e-18)


def test_reactions_at_the_terminal_velocity():
    """In a quiescent liquid at the terminal velocity drag balances buoyancy: the default and the
    sub-step mean are both F_B e_z, and the net force on the bubble is zero."""
    d, nu = 3.0, 0.02
    z3 = np.zeros(3)
    P = _params()
    ub = np.zeros(3)
    for _ in range(400):
        ub, _, _ = O.bubble_ode(P, nu, 0.1, 10000, d, z3, z3, z3, ub, z3)
    _, _, _, fb = _mass(P, d)
    for mode, expect in ((0, fb), (O.REACTION_SUBSTEP_MEAN, fb), (O.REACTION_NET_FORCE, 0.0)):
        _, _, psi = O.bubble_ode(_params(coupling=mode), nu, 0.1, 10, d, z3, z3, z3, ub, z3)
        assert abs(psi[2] - expect) <= 1e-9 * fb, (mode, psi)
        assert abs(psi[0]) == 0 and abs(psi[1]) == 0


@pytest.mark.parametrize("periodic", [False, True])
def test_point_weights_are_a_partition_of_unity(periodic):
    for xb, n, N in ((5.3, 1.2, 12), (0.2, 2.4, 10), (9.9, 4.5, 11), (3.0, 1.8, 7)):
        idx, w = O.axis_weights(xb, n, N, periodic=periodic, point=True)
        assert abs(w.sum() - 1.0) <= 1e-14
        assert np.all(w >= 0.0)
        assert idx.min() >= 0 and idx.max() < N


def test_point_weights_are_symmetric_about_a_cell_centre():
    idx, w = O.axis_weights(10.0, 2.7, 40, point=True)
    k = len(idx) // 2
    assert np.array_equal(idx, np.arange(10 - k, 11 + k))
    assert np.allclose(w, w[::-1], rtol=0, atol=1e-16)
    assert idx[np.argmax(w)] == 10


def test_point_weights_converge_to_cell_integrals():
    """The midpoint rule on the cell [i - 1/2, i + 1/2]: the difference to the cell integral shrinks
    like 1/n^3 as the window widens (Z'' ~ 1/n^3)."""
    errs = []
    for n in (2.0, 4.0, 8.0, 16.0):
        xb = 50.37
        _, wp = O.axis_weights(xb, n, 200, point=True)
        _, wi = O.axis_weights(xb, n, 200)
        errs.append(np.abs(wp - wi).max())
    for a, b in zip(errs, errs[1:]):
        assert b < a / 5.0, errs


def test_point_spreading_is_the_transpose_of_point_interpolation():
    rng = np.random.default_rng(3)
    shape = (3, 14, 13, 12)
    bc = (1, 1, 2, 2, 0, 0)
    U = rng.normal(0, 1, shape)
    xb, n, psi = np.array([5.2, 6.7, 3.1]), 2.7, rng.normal(0, 1, 3)
    F = np.zeros(shape)
    O.spread(F, bc, xb, n, psi, point=True)
    ul, _ = O.interpolate(U, bc, xb, n, point=True)
    assert abs(np.sum(F * U) - psi @ ul) <= 1e-12 * np.abs(F * U).sum()
    assert np.allclose(F.reshape(3, -1).sum(axis=1), psi, rtol=1e-13, atol=0)  # equal and opposite


def _shear_lattice(shape, omega, A=2e-3):
    """Periodic box with a shear wave u_x = A sin(2 pi z / nz) at equilibrium."""
    nx, ny, nz = shape
    lat = O.Lattice(nx, ny, nz, omega, (2,) * 6)
    _, w, _ = O.lattice()
    for z in range(nz):
        f = O.equilibrium(1.0, [A * np.sin(2 * np.pi * z / nz), 0.0, 0.0])
        lat.g[:, z, :, :] = (f - w)[:, None, None]
    return lat


def test_exact_time_reads_one_step_ahead_of_the_default():
    """No force in the liquid and a bubble that cannot move (no drag, lift, buoyancy, and
    (1 + C_A) = 0 so the liquid acceleration does not push it): the velocity the default coupling
    interpolates at step n + 1 (that of collision n) is the velocity of f^n, which the exact-time
    variant interpolates at step n."""
    shape, omega = (8, 6, 24), 1.3
    kw = dict(g=0.0, drag_scale=0.0, lift_scale=0.0, c_a=-1.0)
    seen = {}
    for mode in (0, O.EXACT_TIME):
        lat = _shear_lattice(shape, omega)
        bub = O.Bubbles(pos=np.array([[3.4], [2.2], [7.6]]), d=np.array([2.0]))
        P = _params(coupling=mode, **kw)
        ul = []
        for _ in range(6):
            O.method_step(lat, P, bub)
            ul.append(bub.ulp[:, 0].copy())
        assert np.array_equal(bub.pos, np.array([[3.4], [2.2], [7.6]]))
        seen[mode] = np.array(ul)
    default, exact = seen[0], seen[O.EXACT_TIME]
    assert np.abs(exact[0]).max() > 1e-4  # the shear wave, read at once
    assert np.abs(default[0]).max() == 0.0  # no collision before the first step
    assert np.allclose(default[1:], exact[:-1], rtol=1e-12, atol=1e-18)
    assert np.abs(exact[1:] - exact[:-1]).max() > 1e-9  # the wave decays: the shift is visible
