"""Physical parameters of the nozzle study and their lattice counterparts
(Sec. 2.2, Eqs. (5), (10)-(11), (13)-(14); Table 2).

The study's fluid is Newtonian with density 1056 kg/m^3 and dynamic
viscosity 3.5 mPa s; the domain is 0.012 x 0.012 x 0.24 m^3; the Reynolds
number is taken on the throat diameter with the mean throat velocity,
which is (d0 / d_thr)^2 times the mean inlet velocity; the time step fixes
the largest convective CFL number, 2 u_thr dt / dr.  The throat and inlet
diameters, 4 mm and 12 mm, are the FDA nozzle's (the paper's geometry
figure is not available here; the inlet Reynolds numbers it prints, about a
third of the throat's, agree).

Everything here is host arithmetic for setting up runs: lattice tau and
velocities from physical inputs.  The solver itself works in lattice units
throughout.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

RHO = 1056.0             # kg/m^3
MU = 3.5e-3              # Pa s
D_THROAT = 4.0e-3        # m
D_INLET = 12.0e-3        # m
DOMAIN = (0.24, 0.012, 0.012)  # m: axial x, then y, z

# Table 2: (Re, dr [m], dt [s]) of the resolutions R1..R4
TABLE2 = {
    ("R1", 500): (2.3e-4, 49.03e-6), ("R2", 500): (1.725e-4, 36.75e-6), ("R3", 500): (1.15e-4, 24.5e-6),
    ("R1", 3500): (2.3e-4, 9.86e-6), ("R2", 3500): (1.725e-4, 7.38e-6), ("R3", 3500): (1.15e-4, 4.93e-6),
    ("R1", 6500): (2.3e-4, 5.31e-6), ("R2", 6500): (1.725e-4, 3.98e-6), ("R3", 6500): (1.15e-4, 2.65e-6),
    ("R4", 6500): (0.776e-4, 1.7e-6),
}


def kinematic_viscosity(rho: float = RHO, mu: float = MU) -> float:
    return mu / rho


def throat_velocity(re: float, rho: float = RHO, mu: float = MU, d_thr: float = D_THROAT) -> float:
    """Mean throat velocity of a throat Reynolds number (Eq. (10))."""
    return re * mu / (rho * d_thr)


def inlet_velocity(re: float, **kw) -> float:
    """Mean inlet velocity: the throat velocity times (d_thr / d0)^2 (Eq. (11))."""
    return throat_velocity(re, **kw) * (D_THROAT / D_INLET) ** 2


def inlet_reynolds(re: float) -> float:
    """Reynolds number on the inlet diameter and mean inlet velocity."""
    return re * D_THROAT / D_INLET


def time_step(re: float, dr: float, cfl: float, rho: float = RHO, mu: float = MU, d_thr: float = D_THROAT) -> float:
    """Time step fixing the convective CFL number 2 u_thr dt / dr (Eqs. (13)-(14))."""
    return rho * d_thr * dr * cfl / (2.0 * mu * re)


def cfl(re: float, dr: float, dt: float, **kw) -> float:
    """The CFL number 2 u_thr dt / dr of a resolution (Eq. (13))."""
    return 2.0 * throat_velocity(re, **kw) * dt / dr


def lattice_tau(dr: float, dt: float, rho: float = RHO, mu: float = MU) -> float:
    """Relaxation time in time steps: tau = nu / (theta0 dt) + 1/2 with
    theta0 = dr^2 / (3 dt^2) (Eq. (5)), i.e. 3 nu dt / dr^2 + 1/2."""
    return 3.0 * kinematic_viscosity(rho, mu) * dt / dr ** 2 + 0.5


def grid(dr: float) -> tuple[int, int, int]:
    """Cells of the domain at spacing dr, as (nz, ny, nx) with x axial."""
    nx, ny, nz = (int(round(L / dr)) for L in DOMAIN)
    return nz, ny, nx


@dataclass(frozen=True)
class Resolution:
    name: str
    re: float
    dr: float
    dt: float

    @property
    def tau(self) -> float:
        return lattice_tau(self.dr, self.dt)

    @property
    def cfl(self) -> float:
        return cfl(self.re, self.dr, self.dt)

    @property
    def lattice_throat_velocity(self) -> float:
        """Mean throat velocity in cells per step (half the CFL number)."""
        return throat_velocity(self.re) * self.dt / self.dr

    @property
    def cells(self) -> tuple[int, int, int]:
        return grid(self.dr)


def resolution(name: str, re: int) -> Resolution:
    """A resolution of Table 2, e.g. resolution("R4", 6500)."""
    dr, dt = TABLE2[(name, re)]
    return Resolution(name, float(re), dr, dt)
