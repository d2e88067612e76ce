"""FP64 CPU oracle for the D3Q27 CHM-MRT lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: this package checks the GPU library and is never
part of it.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The arithmetic lives in
``lbm_oracle.c`` (plain C, FP64, no blocking or fusion); this module only
marshals numpy arrays.  It shares no code with ``paper_2204_10566_amd``.

Every function names the passage of the paper (Huang, Noel, Berg, Hosseini,
"Simulation of the FDA Nozzle Benchmark: A Lattice Boltzmann Study") that it
follows; see the header of ``lbm_oracle.c`` for the readings taken where the
paper is silent or garbled.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
# LBM_ORACLE_LIBRARY selects another build of the same source (the
# sanitizer test loads an AddressSanitizer/UBSan build through it)
_LIB = os.environ.get("LBM_ORACLE_LIBRARY") or os.path.join(_HERE, "liblbm_oracle.so")

NQ = 27
THETA0 = 1.0 / 3.0
FLUID, SOLID, INLET, OUTLET = 0, 1, 2, 3
OK, ERR_ARG, ERR_OOM, ERR_UNSTABLE = 0, -1, -2, -4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        lp = ctypes.POINTER(ctypes.c_long)
        L.oracle_velocity_set.argtypes = [ip, dp]
        L.oracle_hermite.argtypes = [ctypes.c_int, ip, dp]
        L.oracle_hermite.restype = ctypes.c_double
        L.oracle_num_tuples.restype = ctypes.c_int
        L.oracle_feq.argtypes = [ctypes.c_double, dp, ctypes.c_int, dp]
        L.oracle_transform.argtypes = [dp, dp]
        L.oracle_relaxation.argtypes = [dp, dp]
        L.oracle_cell_moments.argtypes = [dp, dp, dp]
        L.oracle_collide.argtypes = [dp, dp, dp]
        L.oracle_collide.restype = ctypes.c_int
        L.oracle_stream.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint, dp, dp, dp]
        L.oracle_collide_field.argtypes = [u8p, ctypes.c_long, dp, dp]
        L.oracle_collide_field.restype = ctypes.c_int
        L.oracle_init_fields.argtypes = [u8p, ctypes.c_long, dp, dp, dp]
        L.oracle_step.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint, dp, dp,
                                  ctypes.c_int, dp, dp]
        L.oracle_step.restype = ctypes.c_int
        L.oracle_moments.argtypes = [u8p, ctypes.c_long, dp, dp, dp]
        L.oracle_stress.argtypes = [u8p, ctypes.c_long, dp, ctypes.c_double, dp]
        L.oracle_set_outlet.argtypes = [ctypes.c_int, ctypes.c_double]
        L.oracle_set_wall_distances.argtypes = [dp]
        L.oracle_set_equilibrium_order.argtypes = [ctypes.c_int]
        L.oracle_set_equilibrium_order.restype = ctypes.c_int
        L.oracle_run_cells.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint, dp, dp, dp,
                                       dp, ctypes.c_int, ctypes.c_long, lp, dp]
        L.oracle_run_cells.restype = ctypes.c_int
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def rates_vector(omega, omega_bulk=None, omega_high=1.0, order_rates=None):
    """Relaxation rates [omega, omega_bulk, omega_3..omega_6] (Sec. 2.1,
    text after Eq. (8); App. A after Eq. (A.6)).  The paper sets
    omega_bulk = omega and every rate of order >= 3 to one."""
    if omega_bulk is None:
        omega_bulk = omega
    high = list(order_rates) if order_rates is not None else [omega_high] * 4
    return np.array([omega, omega_bulk] + high, dtype=np.float64)


def velocity_set():
    """App. A, Eqs. (A.1)-(A.2): (c[27,3] int, w[27])."""
    c = np.zeros((NQ, 3), dtype=np.int32)
    w = np.zeros(NQ)
    lib().oracle_velocity_set(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w))
    return c, w


def hermite(idx, xi):
    """App. A, Eq. (A.3): Hermite tensor component for index tuple idx."""
    idx_a = np.ascontiguousarray(idx, dtype=np.int32)
    xi_a = _f64(xi)
    return lib().oracle_hermite(len(idx_a), idx_a.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(xi_a))


def num_tuples():
    return lib().oracle_num_tuples()


def feq(rho, u, order=6):
    """Sec. 2.1, Eq. (4) with App. A, Eq. (A.4); order 6 is the paper's."""
    out = np.zeros(NQ)
    lib().oracle_feq(float(rho), _dp(_f64(u)), int(order), _dp(out))
    return out


def transform(u):
    """Sec. 2.1, Eqs. (7)-(8): T[k, i] = H_k(c_i - u), k = p + 3q + 9r."""
    T = np.zeros((NQ, NQ))
    lib().oracle_transform(_dp(_f64(u)), _dp(T))
    return T


def relaxation(rates):
    S = np.zeros((NQ, NQ))
    lib().oracle_relaxation(_dp(_f64(rates)), _dp(S))
    return S


def cell_moments(f):
    rho = np.zeros(1)
    u = np.zeros(3)
    lib().oracle_cell_moments(_dp(_f64(f)), _dp(rho), _dp(u))
    return float(rho[0]), u


def collide(f, rates, feq_order=6):
    """Sec. 2.1, Eq. (6) for one cell, relaxing towards the equilibrium of
    Eq. (4) truncated at feq_order (6: the paper's full expansion).
    Returns (status, f*)."""
    out = np.zeros(NQ)
    with _equilibrium(feq_order):
        st = lib().oracle_collide(_dp(_f64(f)), _dp(_f64(rates)), _dp(out))
    return st, out


def _u8(flags):
    a = np.ascontiguousarray(flags, dtype=np.uint8)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def init_fields(flags, rho=None, u=None):
    """f = f^eq(rho, u) (Eq. (4)) on updatable cells.  flags: [nz, ny, nx];
    rho: same shape or None (=1); u: [3, nz, ny, nx] or None (=0).
    Returns f: [27, nz, ny, nx]."""
    fl, flp = _u8(flags)
    n = fl.size
    f = np.zeros((NQ,) + fl.shape)
    r = _f64(rho)
    uu = _f64(u)
    lib().oracle_init_fields(flp, n, _dp(r), _dp(uu), _dp(f))
    return f


def stream(flags, f, periodic=0, uin=None, outlet=None, q=None):
    """Pull streaming pass with the boundary rules of Sec. 2.2."""
    fl, flp = _u8(flags)
    nz, ny, nx = fl.shape
    fa = _f64(f)
    g = np.zeros_like(fa)
    with _boundary(flags, outlet, q):
        lib().oracle_stream(flp, nx, ny, nz, periodic, _dp(_f64(uin)), _dp(fa), _dp(g))
    return g


def collide_field(flags, f, rates, feq_order=6):
    fl, flp = _u8(flags)
    fa = _f64(f).copy()
    with _equilibrium(feq_order):
        st = lib().oracle_collide_field(flp, fl.size, _dp(_f64(rates)), _dp(fa))
    return st, fa


def step(flags, f, rates, nsteps=1, periodic=0, uin=None, outlet=None, q=None, feq_order=6):
    """nsteps of stream + collide (feq_order: truncation of the equilibrium
    the collision relaxes to, 6 the paper's).  Returns (status, f_new)."""
    fl, flp = _u8(flags)
    nz, ny, nx = fl.shape
    fa = _f64(f).copy()
    work = np.empty_like(fa)
    uin_a = _f64(uin)
    with _boundary(flags, outlet, q), _equilibrium(feq_order):
        st = lib().oracle_step(flp, nx, ny, nz, periodic, _dp(uin_a), _dp(_f64(rates)), int(nsteps), _dp(fa),
                               _dp(work))
    return st, fa


def moments(flags, f):
    """(rho[nz,ny,nx], u[3,nz,ny,nx]) of a population field."""
    fl, flp = _u8(flags)
    fa = _f64(f)
    rho = np.zeros(fl.shape)
    u = np.zeros((3,) + fl.shape)
    lib().oracle_moments(flp, fl.size, _dp(fa), _dp(rho), _dp(u))
    return rho, u


OUTLETS = {"zero_gradient": 0, "pressure": 1}


class _boundary:
    """Selects the boundary options of Sec. 2.2 for the duration of one
    call.  outlet: None or "zero_gradient" copies the last plane;
    ("pressure", rho_out) holds the outlet pressure at rho_out / 3 by
    non-equilibrium extrapolation.  q: None (halfway bounce-back) or the
    wall fraction of every link, [27, nz, ny, nx], read at wall links."""

    def __init__(self, flags, outlet=None, q=None):
        kind, rho = ("zero_gradient", 1.0) if outlet in (None, "zero_gradient") else outlet
        self.args = (OUTLETS[kind], float(rho))
        self.q = None
        if q is not None:
            self.q = np.ascontiguousarray(q, dtype=np.float64).reshape(NQ, -1)
            if self.q.shape[1] != np.asarray(flags).size:
                raise ValueError("q must hold 27 values per cell")

    def __enter__(self):
        lib().oracle_set_outlet(*self.args)
        lib().oracle_set_wall_distances(_dp(self.q))

    def __exit__(self, *exc):
        lib().oracle_set_outlet(0, 1.0)
        lib().oracle_set_wall_distances(None)


class _equilibrium:
    """Selects the truncation order of the equilibrium the collision relaxes
    to (Sec. 2.1, Eq. (4)) for the duration of one call; 6 is the paper's
    full expansion and the default."""

    def __init__(self, order):
        self.order = int(order)

    def __enter__(self):
        if lib().oracle_set_equilibrium_order(self.order) != OK:
            raise ValueError(f"equilibrium order {self.order} outside 2..6")

    def __exit__(self, *exc):
        lib().oracle_set_equilibrium_order(6)


def stress(flags, f, omega):
    """Viscous stress sigma[6, nz, ny, nx] (xx, yy, zz, xy, xz, yz) of a
    pre-collision state (Sec. 2.2, Eq. (19); App. A, Eqs. (A.7)-(A.8)):
    sigma = -(1 - omega/2) times the central second-order Hermite moment."""
    fl, flp = _u8(flags)
    fa = _f64(f)
    sig = np.zeros((6,) + fl.shape)
    lib().oracle_stress(flp, fl.size, _dp(fa), float(omega), _dp(sig))
    return sig


def run_cells(flags, cells, rates, nsteps, periodic=0, uin=None, rho0=None, u0=None, outlet=None, q=None,
              feq_order=6):
    """Populations after nsteps at the listed linear cell indices, starting
    from f^eq(rho0, u0); only the dependency cone is computed.  Returns
    (status, f[27, len(cells)])."""
    fl, flp = _u8(flags)
    nz, ny, nx = fl.shape
    cl = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((NQ, cl.size))
    with _boundary(flags, outlet, q), _equilibrium(feq_order):
        st = lib().oracle_run_cells(flp, nx, ny, nz, periodic, _dp(_f64(uin)), _dp(_f64(rho0)), _dp(_f64(u0)),
                                    _dp(_f64(rates)), int(nsteps), cl.size,
                                    cl.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dp(out))
    return st, out


def max_threads():
    return lib().oracle_max_threads()


def set_threads(n: int):
    """Threads of the following oracle calls (n <= 0: one per processor)."""
    lib().oracle_set_threads(int(n))
