"""Physical <-> lattice conversion (App. A) against the values Table 5 and App. A print."""
import os

import numpy as np
import pytest

from paper_1710_07073_amd import units as U

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table5_conversion.txt")


def _rows():
    return np.loadtxt(GOLDEN, comments="#")


def test_appendix_a_worked_example():
    """4 mm bubble at aspect ratio 1.25: dx = 5 mm, LCF = 200, TCF = 1e4, MCF = 8000, and the
    0.15 x 0.15 x 0.45 m tank is 30 x 30 x 90 cells with d_b = 0.8 (App. A)."""
    u = U.column_units(0.004, 1.25)
    assert u.dx == pytest.approx(0.005)
    assert u.lcf == pytest.approx(200.0)
    assert u.tcf == pytest.approx(1e4)
    assert u.mcf == pytest.approx(8000.0)
    c = U.column(u, 0.004)
    assert (c.nx, c.ny, c.nz) == (30, 30, 90)
    assert c.d_b == pytest.approx(0.8)
    assert u.density(1000.0) == pytest.approx(1.0)


@pytest.mark.parametrize("row", range(9))
def test_table5_rows(row):
    aspect, lcf, mcf, tcf, dx, w, dep, h, d_mm, d_lu = _rows()[row]
    u = U.column_units(d_mm * 1e-3, aspect)
    c = U.column(u, d_mm * 1e-3)
    assert u.dx == pytest.approx(dx)
    assert u.lcf == pytest.approx(lcf)
    assert u.tcf == pytest.approx(tcf)
    assert (c.nx, c.ny, c.nz) == (w, dep, h)
    assert c.d_b == pytest.approx(d_lu)
    if row == 5:
        # the printed MCF is ten times the value of the density relation (misprint)
        assert mcf == pytest.approx(10 * u.mcf)
    else:
        assert u.mcf == pytest.approx(mcf)


def test_conversions_are_consistent():
    """Dimensional checks: a velocity is length / time, an acceleration length / time^2, a kinematic
    viscosity length^2 / time, a surface tension mass / time^2, and velocity round-trips."""
    u = U.column_units(0.004, 0.625)
    assert u.velocity(1.0) == pytest.approx(u.length(1.0) / u.time(1.0))
    assert u.acceleration(1.0) == pytest.approx(u.length(1.0) / u.time(1.0) ** 2)
    assert u.viscosity(1.0) == pytest.approx(u.length(1.0) ** 2 / u.time(1.0))
    assert u.surface_tension(1.0) == pytest.approx(u.mcf / u.time(1.0) ** 2)
    assert u.velocity_pu(u.velocity(0.2383)) == pytest.approx(0.2383)
    # Eotvos number is unit-free
    g, d, sig, drho = 9.81, 0.004, 0.0728, 999.0
    eo_pu = drho * g * d * d / sig
    eo_lu = u.density(drho) * u.acceleration(g) * u.length(d) ** 2 / u.surface_tension(sig)
    assert eo_lu == pytest.approx(eo_pu, rel=1e-12)


def test_water_viscosity_gives_omega_near_two():
    """Water (nu = 1e-6 m^2/s) on the App. A grid: nu_lu = 4e-6 and omega = 1.99995, beyond the
    stability limit 1.97 the paper reports (Sec. 4.3) — the paper's own runs cannot have used it."""
    u = U.column_units(0.004, 1.25)
    nu = u.viscosity(1e-6)
    assert nu == pytest.approx(4e-6)
    assert U.omega_of(nu) == pytest.approx(1.0 / (1.2e-5 + 0.5))
    assert U.omega_of(nu) > 1.9999


def test_input_generator_converts_like_the_units_module():
    """The synthetic physical-unit columns convert App. A units on their own (the input generator
    imports nothing from the package): shapes, diameters, omega, g and sigma equal what the
    package's units module gives for every grid case, bit for bit."""
    import workloads as W
    for w in W.grid_independence(steps=1):
        d_b, aspect = w.meta["d_mm"] * 1e-3, w.meta["aspect"]
        u = U.column_units(d_b, aspect)
        col = U.column(u, d_b)
        assert w.shape == (col.nx, col.ny, col.nz)
        assert w.d[0] == col.d_b
        assert w.omega == U.omega_of(u.viscosity(W.WATER_NU))
        assert w.params["g"] == u.acceleration(W.GRAVITY)
        assert w.params["sigma"] == u.surface_tension(W.WATER_SIGMA)
        assert w.pos[2, 0] == u.length(0.02)
    s = W.stability(steps=1, omegas=(1.9,))[0]
    u = U.column_units(0.004, 1.25)
    assert s.params["g"] == u.acceleration(W.GRAVITY) and s.d[0] == U.column(u, 0.004).d_b
