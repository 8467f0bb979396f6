"""Pins of the oracle's lattice arithmetic (Sec. 2.2, eq. (5)-(15)) against identities that the
D3Q19 BGK model and the Guo forcing scheme must satisfy. A dropped term, wrong weight, wrong sign
or transposed index in the oracle fails at least one of these."""
import itertools

import numpy as np
import pytest

import oracle as O


def test_velocity_set_is_d3q19():
    c, w, opp = O.lattice()
    vecs = {tuple(v) for v in c}
    assert len(vecs) == 19
    expect = {(0, 0, 0)}
    for v in itertools.product((-1, 0, 1), repeat=3):
        if 1 <= sum(abs(t) for t in v) <= 2:
            expect.add(v)
    assert vecs == expect
    # paper order: axis directions first, then face diagonals, then the rest particle (eq. (7))
    assert all(np.abs(c[q]).sum() == 1 for q in range(6))
    assert all(np.abs(c[q]).sum() == 2 for q in range(6, 18))
    assert tuple(c[18]) == (0, 0, 0)
    for q in range(19):
        assert tuple(c[opp[q]]) == tuple(-c[q])


def test_weight_moments_isotropy():
    c, w, _ = O.lattice()
    c = c.astype(float)
    assert w.sum() == pytest.approx(1.0, abs=1e-16)
    assert np.abs(w @ c).max() < 1e-17
    M2 = np.einsum("q,qa,qb->ab", w, c, c)
    assert np.allclose(M2, np.eye(3) / 3, atol=1e-16)
    M3 = np.einsum("q,qa,qb,qc->abc", w, c, c, c)
    assert np.abs(M3).max() < 1e-17
    M4 = np.einsum("q,qa,qb,qc,qd->abcd", w, c, c, c, c)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(M4, iso, atol=1e-16)


def test_equilibrium_moments():
    """eq. (6) reproduces rho, rho u and the momentum flux rho/3 I + rho u u (eq. (10))."""
    c, w, _ = O.lattice()
    c = c.astype(float)
    rng = np.random.default_rng(1)
    for _ in range(50):
        rho = rng.uniform(0.8, 1.2)
        u = rng.uniform(-0.1, 0.1, 3)
        feq = O.equilibrium(rho, u)
        assert feq.sum() == pytest.approx(rho, rel=1e-15, abs=1e-15)
        assert np.allclose(feq @ c, rho * u, rtol=0, atol=1e-16)
        Pi = np.einsum("q,qa,qb->ab", feq, c, c)
        assert np.allclose(Pi, rho / 3 * np.eye(3) + rho * np.outer(u, u), rtol=0, atol=2e-16)
    # at rest the equilibrium is the weight vector itself (Algorithm 1 initialisation)
    assert np.allclose(O.equilibrium(1.0, [0, 0, 0]), w, rtol=0, atol=0)


def test_guo_source_moments():
    """eq. (12): sum F_q = 0, sum c F_q = (1 - omega/2) F, sum c c F_q = (1 - omega/2)(uF + Fu)."""
    c, _, _ = O.lattice()
    c = c.astype(float)
    rng = np.random.default_rng(2)
    for _ in range(50):
        omega = rng.uniform(0.5, 1.95)
        u = rng.uniform(-0.1, 0.1, 3)
        F = rng.uniform(-1e-3, 1e-3, 3)
        S = O.guo_source(omega, u, F)
        pre = 1 - omega / 2
        assert abs(S.sum()) < 1e-18
        assert np.allclose(S @ c, pre * F, rtol=1e-14, atol=1e-19)
        M2 = np.einsum("q,qa,qb->ab", S, c, c)
        assert np.allclose(M2, pre * (np.outer(u, F) + np.outer(F, u)), rtol=1e-12, atol=1e-19)


def test_collision_conserves_mass_and_adds_force():
    """First forcing + BGK + second forcing: mass unchanged, raw momentum sum c f grows by F."""
    c, _, _ = O.lattice()
    c = c.astype(float)
    rng = np.random.default_rng(3)
    for _ in range(50):
        omega = rng.uniform(0.5, 1.95)
        g = rng.uniform(-1e-3, 1e-3, 19)
        F = rng.uniform(-1e-4, 1e-4, 3)
        out, rho, u = O.collide_node(omega, g, F)
        assert out.sum() == pytest.approx(g.sum(), abs=1e-17)
        assert np.allclose(out @ c, g @ c + F, rtol=0, atol=1e-16)
        # eq. (13): rho u = sum c f + F/2
        assert rho == pytest.approx(1 + g.sum(), abs=1e-16)
        assert np.allclose(rho * u, g @ c + F / 2, rtol=1e-14, atol=2e-18)


def test_collision_relaxes_towards_equilibrium():
    """Without force, the non-equilibrium part is scaled by (1 - omega) (eq. (5), tau = 1/omega)."""
    _, w, _ = O.lattice()
    rng = np.random.default_rng(4)
    omega = 1.3
    g = rng.uniform(-1e-3, 1e-3, 19)
    out, rho, u = O.collide_node(omega, g, [0, 0, 0])
    geq = O.equilibrium(rho, u) - w
    assert np.allclose(out - geq, (1 - omega) * (g - geq), rtol=0, atol=5e-17)
    # omega = 1 lands exactly on the equilibrium
    out1, rho1, u1 = O.collide_node(1.0, g, [0, 0, 0])
    assert np.allclose(out1, O.equilibrium(rho1, u1) - w, rtol=0, atol=5e-17)
