"""Pins of the oracle's coupling kernel (Sec. 3.2, eq. (18)-(21)): the four design criteria the
paper states for the mapping function, the cell-integral weights against numerical quadrature of
Z, the partition of unity with clipping and wrapping, and the equal-and-opposite force transfer
(spreading is the transpose of interpolation)."""
import numpy as np
import pytest
from scipy import integrate

import oracle as O

BB, FS, PER = O.BC_BOUNCE_BACK, O.BC_FREE_SLIP, O.BC_PERIODIC


@pytest.mark.parametrize("n", [1.2, 2.4, 4.5, 7.5])
def test_mapping_function_design_criteria(n):
    """Smooth (continuous first derivative), maximum at the bubble, zero at the window edge,
    unit integral (the four criteria listed in Sec. 3.2)."""
    Z = lambda r: O.kernel_Z(r, n)
    integral, _ = integrate.quad(Z, -n, n, epsabs=1e-13, epsrel=1e-13)
    assert integral == pytest.approx(1.0, abs=1e-13)
    assert Z(n) == pytest.approx(0.0, abs=1e-15) and Z(-n) == pytest.approx(0.0, abs=1e-15)
    assert Z(1.01 * n) == 0.0 and Z(-1.01 * n) == 0.0
    h = 1e-6 * n
    for edge in (-n, n):  # one-sided slopes vanish at the edges: C1 across the support boundary
        slope_in = (Z(edge) - Z(edge - np.sign(edge) * h)) / h
        assert abs(slope_in) < 1e-5 / n
    r = np.linspace(-n, n, 2001)
    vals = np.array([Z(t) for t in r])
    assert np.argmax(vals) == 1000 and np.all(vals >= 0)
    assert np.all(np.diff(vals[:1001]) >= 0) and np.all(np.diff(vals[1000:]) <= 0)


@pytest.mark.parametrize("d", [0.8, 1.6, 3.0, 3.2, 5.0])
def test_cell_weights_are_cell_integrals_of_Z(d):
    n = 1.5 * d
    rng = np.random.default_rng(int(d * 10))
    for xb in rng.uniform(20, 21, 4):
        idx, w = O.axis_weights(xb, n, 64, periodic=False)
        for i, wi in zip(idx, w):
            q, _ = integrate.quad(lambda x: O.kernel_Z(x - xb, n), i - 0.5, i + 0.5,
                                  epsabs=1e-15, epsrel=1e-13)
            assert wi == pytest.approx(q, abs=2e-14)
        # every cell overlapping the window is present
        assert idx[0] <= xb - n + 0.5 and idx[-1] >= xb + n - 0.5


@pytest.mark.parametrize("d", [0.8, 1.6, 2.0, 3.0, 3.2, 5.0])
def test_partition_of_unity(d):
    n = 1.5 * d
    rng = np.random.default_rng(7)
    for xb in rng.uniform(0.0, 31.0, 25):
        for periodic in (False, True):
            idx, w = O.axis_weights(xb, n, 32, periodic)
            assert w.sum() == pytest.approx(1.0, abs=1e-15)
            assert np.all(w >= 0) and np.all((idx >= 0) & (idx < 32))


def test_clipping_renormalises_only_at_walls():
    n = 4.5
    idx, w = O.axis_weights(16.3, n, 32, False)
    idx_p, w_p = O.axis_weights(16.3, n, 32, True)
    assert np.array_equal(idx, idx_p) and np.allclose(w, w_p, rtol=0, atol=0)
    idx, w = O.axis_weights(0.7, n, 32, False)  # wall at -1/2 cuts the window
    assert idx.min() == 0
    raw = np.array([O.kernel_P((i + 0.5 - 0.7) / n) - O.kernel_P((i - 0.5 - 0.7) / n) for i in idx])
    assert np.allclose(w, raw / raw.sum(), rtol=1e-15)
    idx_p, w_p = O.axis_weights(0.7, n, 32, True)  # periodic: the cut-off mass wraps to the far end
    assert idx_p.max() == 31 and w_p.sum() == pytest.approx(1.0, abs=1e-15)


def _fields(rng, shape):
    nx, ny, nz = shape
    return rng.uniform(-1e-3, 1e-3, (3, nz, ny, nx))


@pytest.mark.parametrize("bc", [(BB,) * 6, (PER,) * 6, (BB, BB, BB, BB, BB, FS)])
def test_spread_is_equal_and_opposite(bc):
    rng = np.random.default_rng(5)
    shape = (16, 14, 20)
    for xb, d in [((7.3, 6.1, 9.9), 3.0), ((0.4, 13.2, 0.2), 2.0), ((15.0, 0.0, 19.6), 4.0)]:
        psi = rng.uniform(-1, 1, 3)
        F = np.zeros((3, 20, 14, 16))
        O.spread(F, bc, xb, 1.5 * d, psi)
        assert np.allclose(F.sum(axis=(1, 2, 3)), psi, rtol=1e-14, atol=0)


@pytest.mark.parametrize("bc", [(BB,) * 6, (PER,) * 6])
def test_spread_is_transpose_of_interpolation(bc):
    """<spread(psi), U> = psi . interp(U): the same weights serve both directions (eq. (20),
    eq. (21))."""
    rng = np.random.default_rng(6)
    U = _fields(rng, (16, 14, 20))
    for xb, d in [((7.3, 6.1, 9.9), 3.0), ((0.4, 13.2, 0.2), 2.0)]:
        psi = rng.uniform(-1, 1, 3)
        F = np.zeros_like(U)
        O.spread(F, bc, xb, 1.5 * d, psi)
        ul, _ = O.interpolate(U, bc, xb, 1.5 * d)
        assert np.sum(F * U) == pytest.approx(psi @ ul, rel=1e-13)


def test_interpolation_of_constant_and_shear_fields():
    """Partition of unity returns a uniform field exactly; with exact central differences the
    interpolated vorticity of a uniform shear is exact (away from walls)."""
    nx, ny, nz = 24, 24, 24
    U = np.zeros((3, nz, ny, nx))
    U[:] = np.array([1e-3, -2e-3, 5e-4])[:, None, None, None]
    ul, wl = O.interpolate(U, (BB,) * 6, (11.2, 12.7, 10.4), 4.5)
    assert np.allclose(ul, [1e-3, -2e-3, 5e-4], rtol=1e-14) and np.abs(wl).max() < 1e-18
    z = np.arange(nz)[:, None, None] * np.ones((nz, ny, nx))
    U = np.zeros((3, nz, ny, nx))
    U[0] = 1e-3 * z
    ul, wl = O.interpolate(U, (BB,) * 6, (11.2, 12.7, 10.4), 4.5)
    assert np.allclose(wl, [0, 1e-3, 0], rtol=1e-13, atol=1e-19)
