"""CPU checks of the adjoint arithmetic the GPU kernels run (evaluated through the library's host
entry points): each transposed Jacobian against central finite differences of its own forward,
and each forward against the oracle."""
import numpy as np
import pytest

import oracle as O
from paper_1710_07073_amd import lbm as L
from paper_1710_07073_amd import sim as S


def _fd(fun, x, h):
    """Central-difference gradient of a scalar function."""
    x = np.asarray(x, np.float64)
    g = np.zeros_like(x)
    for i in range(x.size):
        e = np.zeros_like(x)
        e.flat[i] = h
        g.flat[i] = (fun(x + e) - fun(x - e)) / (2 * h)
    return g


def test_host_collision_matches_oracle():
    rng = np.random.default_rng(30)
    for _ in range(20):
        p = rng.uniform(-1e-3, 1e-3, 19)
        F = rng.uniform(-1e-4, 1e-4, 3)
        om = rng.uniform(0.5, 1.95)
        out, u = L.host_collide(p, F, om)
        ref, _, u_ref = O.collide_node(om, p, F)
        assert np.allclose(out, ref, rtol=0, atol=1e-17) and np.allclose(u, u_ref, rtol=1e-14)


def test_collision_adjoint_is_the_transposed_jacobian():
    rng = np.random.default_rng(31)
    for _ in range(10):
        p = rng.uniform(-2e-2, 2e-2, 19)
        F = rng.uniform(-1e-3, 1e-3, 3)
        om = rng.uniform(0.6, 1.9)
        lam = rng.normal(size=19)
        lam_u = rng.normal(size=3)

        def loss(pp, FF=F, oo=om):
            out, u = L.host_collide(pp, FF, oo)
            return lam @ out + lam_u @ u

        _, _, mu, lf, dom = L.host_collide(p, F, om, lam, lam_u)
        assert np.allclose(mu, _fd(loss, p, 1e-6), rtol=1e-7, atol=1e-9)
        assert np.allclose(lf, _fd(lambda FF: loss(p, FF), F, 1e-6), rtol=1e-7, atol=1e-9)
        g_om = (loss(p, F, om + 1e-6) - loss(p, F, om - 1e-6)) / 2e-6
        assert dom == pytest.approx(g_om, rel=1e-7, abs=1e-10)


@pytest.mark.parametrize("periodic", [False, True])
def test_host_weights_match_oracle_and_differentiate(periodic):
    n, N = 4.5, 40
    for x in (12.37, 0.6, 39.2, 3.9):
        lo, w, dw, wx, dwx = L.host_axis_weights(x, n, N, periodic)
        idx, w_o = O.axis_weights(x, n, N, periodic)
        # the oracle lists only cells inside the domain (or wrapped); compare by cell
        cells = lo - 1 + np.arange(w.size)
        got = {}
        for c, v in zip(cells, w):
            if v != 0.0:
                key = c % N if periodic else c
                got[key] = got.get(key, 0.0) + v
        for i, v in zip(idx, w_o):
            assert got.get(int(i), 0.0) == pytest.approx(v, abs=1e-15)
        h = 1e-6
        lp, wp, dwp, _, _ = L.host_axis_weights(x + h, n, N, periodic)
        lm, wm, dwm, _, _ = L.host_axis_weights(x - h, n, N, periodic)
        if lp == lo == lm:
            assert np.allclose(wx, (wp - wm) / (2 * h), rtol=1e-6, atol=1e-9)
            assert np.allclose(dwx, (dwp - dwm) / (2 * h), rtol=1e-6, atol=1e-9)


def test_curl_weights_fold_the_bounce_back_ghost():
    """Summation by parts: sum_j w_j (U_{j+1} - U_{j-1})/2 with the wall ghost U_{-1} = -U_0
    equals sum_j dw_j U_j."""
    rng = np.random.default_rng(32)
    N, n = 30, 4.5
    for x in (0.3, 2.2, 29.0, 14.1):
        for s_lo, s_hi in ((-1.0, -1.0), (1.0, -1.0), (-1.0, 1.0)):
            lo, w, dw, _, _ = L.host_axis_weights(x, n, N, False, s_lo, s_hi)
            U = rng.normal(size=N)
            Ug = lambda j: (s_lo * U[0] if j < 0 else (s_hi * U[N - 1] if j >= N else U[j]))
            direct = sum(w[i] * 0.5 * (Ug(lo - 1 + i + 1) - Ug(lo - 1 + i - 1))
                         for i in range(w.size) if w[i] != 0.0)
            folded = sum(dw[i] * U[lo - 1 + i] for i in range(w.size) if 0 <= lo - 1 + i < N)
            assert folded == pytest.approx(direct, rel=1e-13, abs=1e-15)


def _ode_case(rng, cd_k=0.15):
    P = S.bubble_params(g=1e-4, sigma=1e-4, drag_scale=1.1, lift_scale=0.9, cd_k=cd_k)
    nu = (1 / 1.4 - 0.5) / 3
    d = 3.0
    x0 = np.array([12.3, 10.1, 20.7])
    ub0 = rng.normal(scale=2e-3, size=3)
    ul = rng.normal(scale=1e-3, size=3)
    wl = rng.normal(scale=1e-3, size=3)
    dul = rng.normal(scale=1e-5, size=3)
    return P, nu, d, x0, ub0, ul, wl, dul


def test_host_ode_matches_oracle():
    rng = np.random.default_rng(33)
    for _ in range(5):
        P, nu, d, x0, ub0, ul, wl, dul = _ode_case(rng)
        x, ub, psi = L.host_bubble_ode(P, nu, d, x0, ub0, ul, wl, dul, (40, 40, 80))
        Po = O.bubble_params(g=1e-4, sigma=1e-4, drag_scale=1.1, lift_scale=0.9)
        ub_o, x_o, psi_o = O.bubble_ode(Po, nu, 0.1, 10, d, ul, wl, dul, ub0, x0)
        assert np.allclose(x, x_o, rtol=1e-14) and np.allclose(ub, ub_o, rtol=1e-12, atol=1e-20)
        assert np.allclose(psi, psi_o, rtol=1e-12, atol=1e-22)


@pytest.mark.parametrize("cd_k", [0.15, 0.0])
def test_ode_adjoint_matches_finite_differences(cd_k):
    rng = np.random.default_rng(34)
    for _ in range(4):
        P, nu, d, x0, ub0, ul, wl, dul = _ode_case(rng, cd_k)
        lx, lub, lpsi = rng.normal(size=3), rng.normal(size=3) * 1e3, rng.normal(size=3) * 1e2
        ext, per = (40, 40, 80), (0, 0, 0)

        def loss(x0_=x0, ub0_=ub0, ul_=ul, wl_=wl, dul_=dul, nu_=nu, sD=1.1, sL=0.9):
            Pp = S.bubble_params(g=1e-4, sigma=1e-4, drag_scale=sD, lift_scale=sL, cd_k=cd_k)
            x, ub, psi = L.host_bubble_ode(Pp, nu_, d, x0_, ub0_, ul_, wl_, dul_, ext, per)
            return lx @ x + lub @ ub + lpsi @ psi

        g = L.host_bubble_ode_adjoint(P, nu, d, x0, ub0, ul, wl, dul, ext, per, lx, lub, lpsi)
        h = 1e-7
        assert np.allclose(g[0:3], _fd(lambda v: loss(x0_=v), x0, 1e-4), rtol=1e-6, atol=1e-8)
        assert np.allclose(g[3:6], _fd(lambda v: loss(ub0_=v), ub0, h), rtol=1e-5, atol=1e-6)
        assert np.allclose(g[6:9], _fd(lambda v: loss(ul_=v), ul, h), rtol=1e-5, atol=1e-6)
        assert np.allclose(g[9:12], _fd(lambda v: loss(wl_=v), wl, h), rtol=1e-5, atol=1e-6)
        assert np.allclose(g[12:15], _fd(lambda v: loss(dul_=v), dul, h), rtol=1e-5, atol=1e-6)
        for i, (kw, v0) in enumerate((("sD", 1.1), ("sL", 0.9), ("nu_", nu))):
            hh = 1e-3 * v0  # smooth in the scales; a larger step keeps round-off out
            fd = (loss(**{kw: v0 + hh}) - loss(**{kw: v0 - hh})) / (2 * hh)
            assert g[15 + i] == pytest.approx(fd, rel=1e-6, abs=1e-10), kw


def test_ode_adjoint_through_wall_clamps():
    """A bubble pushed into the side wall: the clamped components carry no derivative."""
    P = S.bubble_params(g=1e-4, sigma=1e-4)
    nu, d = (1 / 1.2 - 0.5) / 3, 3.0
    x0 = np.array([0.01, 5.0, 3.0])
    ub0 = np.array([-0.05, 0.0, 0.0])
    args = (np.zeros(3), np.zeros(3), np.zeros(3))
    x, ub, _ = L.host_bubble_ode(P, nu, d, x0, ub0, *args, (16, 16, 32))
    assert x[0] == 0.0
    g = L.host_bubble_ode_adjoint(P, nu, d, x0, ub0, *args, (16, 16, 32), (0, 0, 0),
                                  np.ones(3), np.ones(3), np.zeros(3))
    assert np.isfinite(g).all()
