"""Physical <-> lattice units of the bubble column (App. A, Table 5).

Conversion factors are lattice over physical: LCF = dx_lu / dx_pu with dx_lu = 1, TCF = dt_lu /
dt_pu with dt_lu = 1, and MCF fixed by the densities, rho_pu = rho_lu LCF^3 / MCF (App. A). The
grid spacing follows the aspect ratio dx_pu / d_b,pu of the column (1.25, 0.625, 0.3125 in
Table 5), the liquid time step is 1e-4 s, and the liquid density is 1 in lattice units and
1000 kg/m^3 in physical units.
"""
from __future__ import annotations

from dataclasses import dataclass


@dataclass(frozen=True)
class Units:
    dx: float               # grid spacing, m
    dt: float = 1e-4        # liquid time step, s
    rho_pu: float = 1000.0  # liquid density, kg/m^3
    rho_lu: float = 1.0

    @property
    def lcf(self) -> float:
        return 1.0 / self.dx

    @property
    def tcf(self) -> float:
        return 1.0 / self.dt

    @property
    def mcf(self) -> float:
        return self.lcf ** 3 * self.rho_lu / self.rho_pu

    # physical -> lattice
    def length(self, x_m: float) -> float:
        return x_m * self.lcf

    def time(self, t_s: float) -> float:
        return t_s * self.tcf

    def velocity(self, v_ms: float) -> float:
        return v_ms * self.lcf / self.tcf

    def acceleration(self, a_ms2: float) -> float:
        return a_ms2 * self.lcf / self.tcf ** 2

    def viscosity(self, nu_m2s: float) -> float:
        """Kinematic viscosity."""
        return nu_m2s * self.lcf ** 2 / self.tcf

    def density(self, rho_kgm3: float) -> float:
        """Mass over length cubed: rho_lu = rho_pu MCF / LCF^3."""
        return rho_kgm3 * self.mcf / self.lcf ** 3

    def surface_tension(self, sigma_nm: float) -> float:
        """Surface tension (N/m = kg/s^2)."""
        return sigma_nm * self.mcf / self.tcf ** 2

    # lattice -> physical
    def velocity_pu(self, v_lu: float) -> float:
        return v_lu * self.tcf / self.lcf


def column_units(d_b: float, aspect: float, dt: float = 1e-4, rho_pu: float = 1000.0) -> Units:
    """Units of a column resolving a bubble of diameter d_b (m) at aspect ratio dx / d_b (App. A)."""
    return Units(dx=aspect * d_b, dt=dt, rho_pu=rho_pu)


def omega_of(nu_lu: float) -> float:
    """BGK relaxation rate for a lattice kinematic viscosity, nu = (1/omega - 1/2) / 3 (eq. (9))."""
    return 1.0 / (3.0 * nu_lu + 0.5)


@dataclass(frozen=True)
class Column:
    """Lattice column of App. A: width x depth x water level (cells) and the bubble diameter."""
    nx: int
    ny: int
    nz: int
    d_b: float


def column(units: Units, d_b: float, width: float = 0.15, depth: float = 0.15,
           level: float = 0.45) -> Column:
    """The paper's rectangular tank (App. A: 0.15 x 0.15 m, water level 0.45 m) in lattice cells."""
    return Column(round(units.length(width)), round(units.length(depth)), round(units.length(level)),
                  units.length(d_b))
