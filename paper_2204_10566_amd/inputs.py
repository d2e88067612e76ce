"""Seeded synthetic inputs: voxel flag fields, initial velocity fields, inlet
velocity profiles, relaxation parameters and request traces.

This module holds none of the lattice Boltzmann arithmetic: it produces the
geometry, the boundary data and the initial macroscopic fields that both the
GPU library and the FP64 oracle take as inputs, so that the two sides see
identical inputs.  Everything random is drawn from numpy's PCG64 with an
explicit seed.

Array conventions (shared with the C ABI):
  flags[nz, ny, nx] uint8 with 0 fluid, 1 solid, 2 inlet, 3 outlet;
  velocity fields u[3, nz, ny, nx] (x fastest); x is the axial direction.

The synthetic nozzle stands in for the FDA nozzle of the paper (Sec. 2.2,
"Cases description"), whose geometry file is not available here: an inlet
pipe, a conical contraction of 20 degrees total angle, a straight throat and a
sudden expansion back to the pipe radius.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FLUID, SOLID, INLET, OUTLET = 0, 1, 2, 3
CS = 1.0 / math.sqrt(3.0)  # lattice speed of sound, sqrt(theta0) with theta0 = 1/3

PERIODIC_X, PERIODIC_Y, PERIODIC_Z = 1, 2, 4


def tau_from_viscosity(nu: float) -> float:
    """Lattice relaxation time for a lattice kinematic viscosity (Sec. 2.1,
    Eq. (5), with delta t = 1 and theta0 = 1/3)."""
    return 3.0 * nu + 0.5


# ---------------------------------------------------------------------------
# Periodic box with a 3-D Taylor-Green vortex
# ---------------------------------------------------------------------------
def periodic_box(nx: int, ny: int | None = None, nz: int | None = None) -> np.ndarray:
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return np.zeros((nz, ny, nx), dtype=np.uint8)


def taylor_green_velocity(nx: int, ny: int, nz: int, u0: float) -> np.ndarray:
    """u_x = u0 sin(kx x) cos(ky y) cos(kz z), u_y = -u0 cos sin cos, u_z = 0,
    k = 2 pi / N per axis, at integer cell coordinates."""
    kx, ky, kz = 2 * math.pi / nx, 2 * math.pi / ny, 2 * math.pi / nz
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u = np.zeros((3, nz, ny, nx))
    u[0] = u0 * np.sin(kx * x) * np.cos(ky * y) * np.cos(kz * z)
    u[1] = -u0 * np.cos(kx * x) * np.sin(ky * y) * np.cos(kz * z)
    return u


def double_shear_layer_velocity(n: int, u0: float, kappa: float = 80.0, delta: float = 0.05) -> np.ndarray:
    """Periodic double shear layer on an n x n x n box (a standard stability
    stress case): u_x = u0 tanh(kappa (y' - 1/4)) for y' <= 1/2 and
    u0 tanh(kappa (3/4 - y')) above, u_y = delta u0 sin(2 pi (x' + 1/4)),
    u_z = 0, with x' = x / n, y' = y / n at integer cell coordinates."""
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    yp, xp = y / n, x / n
    u = np.zeros((3, n, n, n))
    u[0] = np.where(yp <= 0.5, u0 * np.tanh(kappa * (yp - 0.25)), u0 * np.tanh(kappa * (0.75 - yp)))
    u[1] = delta * u0 * np.sin(2 * math.pi * (xp + 0.25))
    return u


def taylor_green_2d_velocity(nx: int, ny: int, u0: float) -> np.ndarray:
    """z-independent Taylor-Green vortex on an nx x ny x 1 box."""
    kx, ky = 2 * math.pi / nx, 2 * math.pi / ny
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    u = np.zeros((3, 1, ny, nx))
    u[0, 0] = u0 * np.sin(kx * x) * np.cos(ky * y)
    u[1, 0] = -u0 * (kx / ky) * np.cos(kx * x) * np.sin(ky * y)
    return u


def random_populations(shape, seed: int, drift: float = 0.05, noise: float = 0.02) -> np.ndarray:
    """A positive random population field [27, nz, ny, nx]: the lattice
    weights w_i times (1 + 3 c_i . v) for a random drift v per cell, times
    (1 + noise U(-1, 1)) per population.  An arbitrary test state, not an
    equilibrium."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = np.array([(i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1) for i in range(27)], dtype=np.float64)
    w1 = {-1: 1.0 / 6.0, 0: 2.0 / 3.0, 1: 1.0 / 6.0}
    w = np.array([w1[a] * w1[b] * w1[g] for a, b, g in c.astype(int)])
    v = drift * rng.uniform(-1.0, 1.0, (3,) + tuple(shape))
    cv = np.tensordot(c, v, axes=(1, 0))
    f = w.reshape((27,) + (1,) * len(shape)) * (1.0 + 3.0 * cv)
    f *= 1.0 + noise * rng.uniform(-1.0, 1.0, f.shape)
    return f


# ---------------------------------------------------------------------------
# Channel between two walls normal to y (periodic in x and z)
# ---------------------------------------------------------------------------
def channel_flags(nx: int, ny: int, nz: int) -> np.ndarray:
    """Solid rows at y = 0 and y = ny - 1; the halfway walls sit at y = 0.5
    and y = ny - 1.5, so the fluid gap is H = ny - 2."""
    fl = np.zeros((nz, ny, nx), dtype=np.uint8)
    fl[:, 0, :] = SOLID
    fl[:, ny - 1, :] = SOLID
    return fl


def shear_wave_velocity(nx: int, ny: int, nz: int, u0: float) -> np.ndarray:
    """u_x = u0 sin(pi (y - 0.5) / H) between the walls of channel_flags."""
    H = ny - 2
    y = np.arange(ny)
    prof = u0 * np.sin(math.pi * (y - 0.5) / H)
    prof[0] = prof[-1] = 0.0
    u = np.zeros((3, nz, ny, nx))
    u[0] = prof[None, :, None]
    return u


def inflow_channel(nx: int, ny: int, nz: int, u_mean: float):
    """Channel with walls normal to y, periodic in z, a plane-Poiseuille
    velocity inlet at x = 0 and an outlet at x = nx - 1.  Returns
    (flags, u_in[3,nz,ny,nx], periodic_mask)."""
    fl = channel_flags(nx, ny, nz)
    fl[:, 1:ny - 1, 0] = INLET
    fl[:, 1:ny - 1, nx - 1] = OUTLET
    H = ny - 2
    y = np.arange(ny) - 0.5
    prof = 6.0 * u_mean * (y / H) * (1.0 - y / H)
    uin = np.zeros((3, nz, ny, nx))
    uin[0, :, 1:ny - 1, 0] = prof[None, 1:ny - 1]
    return fl, uin, PERIODIC_Z


# ---------------------------------------------------------------------------
# Synthetic sudden-expansion nozzle
# ---------------------------------------------------------------------------
@dataclass
class Nozzle:
    """Axisymmetric nozzle on an n x n x length voxel grid, axis along x at
    the cross-section centre.  Radii and lengths in cells."""
    n: int = 96
    length: int = 768
    R: float = 24.0                 # pipe radius (inlet and outlet pipe)
    r_throat: float = 8.0
    inlet_len: float | None = None  # default 4 R
    throat_len: float | None = None  # default 8 R
    half_angle_deg: float = 10.0    # 20 degrees total cone angle

    def profile(self) -> np.ndarray:
        """R(x) at the cell centres x + 0.5."""
        L_in = 4 * self.R if self.inlet_len is None else self.inlet_len
        L_th = 8 * self.R if self.throat_len is None else self.throat_len
        L_cone = (self.R - self.r_throat) / math.tan(math.radians(self.half_angle_deg))
        xc = np.arange(self.length) + 0.5
        r = np.full(self.length, self.R)
        cone = (xc >= L_in) & (xc < L_in + L_cone)
        r[cone] = self.R - (xc[cone] - L_in) * (self.R - self.r_throat) / L_cone
        throat = (xc >= L_in + L_cone) & (xc < L_in + L_cone + L_th)
        r[throat] = self.r_throat
        return r

    def radius_grid(self) -> np.ndarray:
        """Distance of each (z, y) cell centre from the axis."""
        c = self.n / 2.0
        z, y = np.meshgrid(np.arange(self.n) + 0.5, np.arange(self.n) + 0.5, indexing="ij")
        return np.sqrt((y - c) ** 2 + (z - c) ** 2)

    def flags(self) -> np.ndarray:
        rr = self.radius_grid()
        prof = self.profile()
        inside = rr[:, :, None] < prof[None, None, :]
        fl = np.where(inside, FLUID, SOLID).astype(np.uint8)
        fl[:, :, 0] = np.where(inside[:, :, 0], INLET, SOLID)
        fl[:, :, -1] = np.where(inside[:, :, -1], OUTLET, SOLID)
        return fl

    def radius_at(self, x: np.ndarray) -> np.ndarray:
        """R at any axial position x (cells, x = i + 0.5 at the centre of
        plane i); continuous except at the sudden expansion."""
        L_in = 4 * self.R if self.inlet_len is None else self.inlet_len
        L_th = 8 * self.R if self.throat_len is None else self.throat_len
        L_cone = (self.R - self.r_throat) / math.tan(math.radians(self.half_angle_deg))
        x = np.asarray(x, dtype=np.float64)
        r = np.full(x.shape, self.R)
        cone = (x >= L_in) & (x < L_in + L_cone)
        r = np.where(cone, self.R - (x - L_in) * (self.R - self.r_throat) / L_cone, r)
        throat = (x >= L_in + L_cone) & (x < L_in + L_cone + L_th)
        return np.where(throat, self.r_throat, r)

    def wall_distances(self, flags: np.ndarray | None = None, iters: int = 40) -> np.ndarray:
        """q[27, n, n, length]: for each link i of an updated cell x whose
        neighbour x - c_i is solid, the fraction of the link from x at
        which it crosses the nozzle surface r = R(x) (bisection of the
        inside/outside test along the link); 0.5 everywhere else."""
        fl = self.flags() if flags is None else flags
        nz_, ny_, nx_ = fl.shape
        q = np.full((27,) + fl.shape, 0.5)
        upd = (fl == FLUID) | (fl == OUTLET)
        c = self.n / 2.0
        zz, yy, xx = np.nonzero(upd)
        for i in range(27):
            cxi, cyi, czi = i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1
            if cxi == cyi == czi == 0:
                continue
            sx, sy, sz = xx - cxi, yy - cyi, zz - czi
            ok = (sx >= 0) & (sx < nx_) & (sy >= 0) & (sy < ny_) & (sz >= 0) & (sz < nz_)
            sel = np.flatnonzero(ok)
            sel = sel[fl[sz[sel], sy[sel], sx[sel]] == SOLID]
            if sel.size == 0:
                continue
            px, py, pz = xx[sel] + 0.5, yy[sel] + 0.5, zz[sel] + 0.5

            def outside(t):
                ax = px - t * cxi
                rr = np.hypot(py - t * cyi - c, pz - t * czi - c)
                return rr >= self.radius_at(ax)

            lo, hi = np.zeros(sel.size), np.ones(sel.size)
            for _ in range(iters):
                mid = 0.5 * (lo + hi)
                out = outside(mid)
                hi = np.where(out, mid, hi)
                lo = np.where(out, lo, mid)
            q[i, zz[sel], yy[sel], xx[sel]] = hi
        return q

    def mean_inlet_velocity(self, u_throat_mean: float) -> float:
        """u0 = u_thr (d_thr / d0)^2 (Sec. 2.2, Eq. (11))."""
        return u_throat_mean * (self.r_throat / self.R) ** 2

    def inlet_velocity(self, u_throat_mean: float, noise: float = 0.0, seed: int = 0) -> np.ndarray:
        """Parabolic inlet profile u(r) = 2 u0 (1 - 4 r^2 / d0^2) (Sec. 2.2,
        Eq. (12)) on the inlet cells, plus optional frozen uniform noise of
        relative amplitude `noise` (times u0) on all three components."""
        u0 = self.mean_inlet_velocity(u_throat_mean)
        d0 = 2.0 * self.R
        rr = self.radius_grid()
        fl = self.flags()
        uin = np.zeros((3, self.n, self.n, self.length))
        prof = 2.0 * u0 * (1.0 - 4.0 * rr ** 2 / d0 ** 2)
        mask = fl[:, :, 0] == INLET
        uin[0, :, :, 0] = np.where(mask, prof, 0.0)
        if noise > 0.0:
            rng = np.random.Generator(np.random.PCG64(seed))
            pert = rng.uniform(-1.0, 1.0, size=(3, self.n, self.n))
            for a in range(3):
                uin[a, :, :, 0] += np.where(mask, noise * u0 * pert[a], 0.0)
        return uin

    def inlet_velocity_cells(self, u_throat_mean: float, flags: np.ndarray | None = None) -> np.ndarray:
        """The parabolic inlet profile on the inlet cells only: [3, n_inlet]
        in ascending cell order (the layout of lbm_set_inlet_cells)."""
        fl = self.flags() if flags is None else flags
        u0 = self.mean_inlet_velocity(u_throat_mean)
        d0 = 2.0 * self.R
        cells = np.flatnonzero(fl.ravel() == INLET)
        z = cells // (self.n * self.length)
        y = (cells // self.length) % self.n
        c = self.n / 2.0
        r2 = (y + 0.5 - c) ** 2 + (z + 0.5 - c) ** 2
        out = np.zeros((3, cells.size))
        out[0] = 2.0 * u0 * (1.0 - 4.0 * r2 / d0 ** 2)
        return out

    def initial_velocity(self, u_throat_mean: float) -> np.ndarray:
        """Plug flow u_x = u0 (R / R(x))^2 on fluid cells (mass consistent)."""
        u0 = self.mean_inlet_velocity(u_throat_mean)
        fl = self.flags()
        prof = self.profile()
        u = np.zeros((3, self.n, self.n, self.length))
        ux = u0 * (self.R / prof) ** 2
        u[0] = np.where((fl == FLUID) | (fl == OUTLET), ux[None, None, :], 0.0)
        return u


def nozzle_tau(nz: Nozzle, Re: float, mach: float = 0.1) -> tuple[float, float]:
    """(tau, mean throat velocity) for a Reynolds number on the throat
    diameter (Sec. 2.2, Eq. (10)) with the peak throat velocity
    2 u_thr = mach * c_s."""
    u_thr = 0.5 * mach * CS
    nu = u_thr * (2.0 * nz.r_throat) / Re
    return tau_from_viscosity(nu), u_thr


def nozzle_config(which: str = "re500") -> dict:
    """The nozzle workloads: 96x96x768 at Re 500, 128x128x1536 at Re 6500
    with 1 % inlet noise, and that one at a quarter of its linear size."""
    if which == "re500":
        nz = Nozzle(n=96, length=768, R=24.0, r_throat=8.0)
        Re, noise = 500.0, 0.0
    elif which == "re6500":
        s = 4.0 / 3.0
        nz = Nozzle(n=128, length=1536, R=24.0 * s, r_throat=8.0 * s)
        Re, noise = 6500.0, 0.01
    elif which == "re6500_quarter":
        # the 128 x 128 x 1536 Re 6500 nozzle at a quarter of its linear size
        # (same shape, Reynolds number, Mach number and inlet noise), small
        # enough for the FP64 oracle over a 2000-step window
        nz = Nozzle(n=32, length=384, R=8.0, r_throat=8.0 / 3.0)
        Re, noise = 6500.0, 0.01
    else:
        raise ValueError(which)
    tau, u_thr = nozzle_tau(nz, Re)
    return {
        "nozzle": nz,
        "flags": nz.flags(),
        "uin": nz.inlet_velocity(u_thr, noise=noise, seed=0),
        "u0": nz.initial_velocity(u_thr),
        "tau": tau,
        "u_thr": u_thr,
        "Re": Re,
        "periodic": 0,
    }


def paper_nozzle(name: str, re: int) -> dict:
    """The synthetic nozzle on one of the paper's resolutions in that run's
    own lattice parameters (Table 2 through paper_2204_10566_amd.units): the
    pipe fills the 12 mm cross-section (radius n/2 - 1/2 cells), the throat
    is a third of it, tau = 3 nu dt / dr^2 + 1/2 and the mean throat velocity
    is half the CFL number of the run (in cells per step)."""
    from . import units

    r = units.resolution(name, re)
    nz_, ny_, nx_ = r.cells
    R = ny_ / 2.0 - 0.5
    noz = Nozzle(n=ny_, length=nx_, R=R, r_throat=R / 3.0)
    fl = noz.flags()
    u_thr = r.lattice_throat_velocity
    return {"nozzle": noz, "flags": fl, "uin_cells": noz.inlet_velocity_cells(u_thr, fl),
            "u0": noz.initial_velocity(u_thr), "tau": r.tau, "u_thr": u_thr, "Re": float(re), "resolution": r,
            "periodic": 0}


def small_nozzle(n: int = 24, length: int = 160, R: float = 8.0, r_throat: float = 3.0, Re: float = 100.0):
    """A scaled-down nozzle for tests the oracle can run in full."""
    nz = Nozzle(n=n, length=length, R=R, r_throat=r_throat, inlet_len=2 * R, throat_len=3 * R)
    tau, u_thr = nozzle_tau(nz, Re)
    return {
        "nozzle": nz,
        "flags": nz.flags(),
        "uin": nz.inlet_velocity(u_thr, noise=0.01, seed=1),
        "u0": nz.initial_velocity(u_thr),
        "tau": tau,
        "u_thr": u_thr,
        "Re": Re,
        "periodic": 0,
    }


# ---------------------------------------------------------------------------
# Batched and serving workloads
# ---------------------------------------------------------------------------
@dataclass
class DomainSpec:
    kind: str                 # "tgv" (periodic box) or "channel"
    nx: int
    ny: int
    nz: int
    tau: float
    steps: int
    u0: float = 0.02
    periodic: int = PERIODIC_X | PERIODIC_Y | PERIODIC_Z
    flags: np.ndarray | None = field(default=None, repr=False)
    u: np.ndarray | None = field(default=None, repr=False)
    uin: np.ndarray | None = field(default=None, repr=False)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    def materialise(self) -> "DomainSpec":
        if self.kind == "tgv":
            self.flags = periodic_box(self.nx, self.ny, self.nz)
            self.u = taylor_green_velocity(self.nx, self.ny, self.nz, self.u0)
            self.periodic = PERIODIC_X | PERIODIC_Y | PERIODIC_Z
        elif self.kind == "channel":
            self.flags = channel_flags(self.nx, self.ny, self.nz)
            self.u = shear_wave_velocity(self.nx, self.ny, self.nz, self.u0)
            self.periodic = PERIODIC_X | PERIODIC_Z
        else:
            raise ValueError(self.kind)
        return self


def batched_domains(count: int = 64, seed: int = 0, lo: int = 16, hi: int = 128, steps: int = 500,
                    materialise: bool = False) -> list[DomainSpec]:
    """Independent periodic-TGV or channel domains: edge n uniform in
    {lo..hi}, cube n^3 or 2n x n x n box (coin flip), tau uniform in
    [0.51, 0.8]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        n = int(rng.integers(lo, hi + 1))
        box = bool(rng.integers(0, 2))
        kind = "tgv" if rng.integers(0, 2) == 0 else "channel"
        tau = float(rng.uniform(0.51, 0.8))
        nx = 2 * n if box else n
        d = DomainSpec(kind=kind, nx=nx, ny=n, nz=n, tau=tau, steps=steps)
        out.append(d.materialise() if materialise else d)
    return out


@dataclass
class Request:
    rid: int
    arrival: float           # seconds after the start of the trace
    nozzle: Nozzle
    Re: float
    steps: int

    def build(self):
        """Flags, inlet velocity on the inlet cells only, and tau.  A served
        solve starts from rest (rho = 1, u = 0)."""
        tau, u_thr = nozzle_tau(self.nozzle, self.Re)
        fl = self.nozzle.flags()
        return {
            "flags": fl,
            "uin_cells": self.nozzle.inlet_velocity_cells(u_thr, fl),
            "tau": tau,
        }

    @property
    def ncells(self) -> int:
        return self.nozzle.n * self.nozzle.n * self.nozzle.length


def serving_trace(count: int = 200, rate: float = 20.0, seed: int = 0, steps_lo: int = 1000,
                  steps_hi: int = 5000) -> list[Request]:
    """Poisson arrivals (mean `rate` per second) of nozzle-like solves:
    cross-section n in {64, 80, 96, 112, 128}, length k n with k in {4..8},
    pipe radius n/4, throat/pipe radius ratio uniform in [0.25, 0.5], Re
    uniform in [500, 6500], step count uniform in {steps_lo..steps_hi}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for rid in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(rng.choice([64, 80, 96, 112, 128]))
        k = int(rng.integers(4, 9))
        R = n / 4.0
        ratio = float(rng.uniform(0.25, 0.5))
        Re = float(rng.uniform(500.0, 6500.0))
        steps = int(rng.integers(steps_lo, steps_hi + 1))
        nz = Nozzle(n=n, length=k * n, R=R, r_throat=R * ratio, inlet_len=2 * R,
                    throat_len=min(8 * R, k * n / 4.0))
        out.append(Request(rid=rid, arrival=t, nozzle=nz, Re=Re, steps=steps))
    return out
