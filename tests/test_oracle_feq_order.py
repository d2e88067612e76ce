"""Pins of the oracle's collision with an explicit, truncated equilibrium
(Sec. 2.1, Eq. (4) summed to an order N below the full expansion; App. A
after Eq. (A.6): only the full expansion gives central equilibrium moments
(rho, 0, ..., 0)).

Closed forms written here, not taken from the oracle: the textbook
second-order equilibrium; the third-order one on D3Q27, which adds the
Hermite terms xxy, xyy, ..., xyz (each axis at most twice); the missing
third-order central moment of the second-order equilibrium,
H_xxy(c - u) -> -rho u_x^2 u_y.  Collision pins: fixed point, the
reduction to BGK with the truncated equilibrium, conservation.  Physical
pin of the paper's remark that third-order terms remove the Galilean error
of the shear stress: a shear wave advected by a uniform stream U decays at
nu (1 - U^2 / theta0) k^2 with the second-order equilibrium and at nu k^2
from the third order on."""
import numpy as np
import pytest

THETA0 = 1.0 / 3.0
C = np.array([(i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1) for i in range(27)], dtype=np.float64)
W1 = {0: 2.0 / 3.0, 1: 1.0 / 6.0}
W = np.array([W1[abs(int(c[0]))] * W1[abs(int(c[1]))] * W1[abs(int(c[2]))] for c in C])


def feq2(rho, u):
    cu = C @ u
    return W * rho * (1.0 + cu / THETA0 + cu ** 2 / (2 * THETA0 ** 2) - (u @ u) / (2 * THETA0))


def feq3(rho, u):
    """Second order plus every third-order Hermite term the stencil carries
    (coefficient 1/(3! theta0^3), a tuple with axis a twice and b once
    appears 3 times, xyz 6 times)."""
    t = 0.0
    for a in range(3):
        for b in range(3):
            if a != b:
                t = t + 3.0 * u[a] ** 2 * u[b] * (C[:, a] ** 2 - THETA0) * C[:, b]
    t = t + 6.0 * u[0] * u[1] * u[2] * C[:, 0] * C[:, 1] * C[:, 2]
    return feq2(rho, u) + W * rho * t / (6.0 * THETA0 ** 3)


def random_state(seed):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.05 * rng.uniform(-1, 1)
    u = 0.08 * rng.uniform(-1, 1, 3)
    return rho, u, rng


@pytest.mark.parametrize("seed", range(4))
def test_truncated_equilibria_closed_forms(orc, seed):
    rho, u, _ = random_state(seed)
    assert np.abs(orc.feq(rho, u, 2) - feq2(rho, u)).max() < 1e-15
    assert np.abs(orc.feq(rho, u, 3) - feq3(rho, u)).max() < 1e-15


@pytest.mark.parametrize("seed", range(4))
def test_missing_third_order_central_moment(orc, seed):
    """Central moments (k = p + 3 q + 9 r for x^p y^q z^r) of the truncated
    equilibria: the second order lacks the rho u_a^2 u_b third moments, so
    its central H_{aab} moment is -rho u_a^2 u_b; from the third order on it
    vanishes, and so does H_xyz."""
    rho, u, _ = random_state(seed)
    T = orc.transform(u)
    m2 = T @ orc.feq(rho, u, 2)
    m3 = T @ orc.feq(rho, u, 3)
    for a in range(3):
        for b in range(3):
            if a == b:
                continue
            p = [0, 0, 0]
            p[a], p[b] = 2, 1
            k = p[0] + 3 * p[1] + 9 * p[2]
            assert abs(m2[k] - (-rho * u[a] ** 2 * u[b])) < 1e-16
            assert abs(m3[k]) < 1e-16
    assert abs(m3[1 + 3 + 9]) < 1e-16
    # orders 0..2 are exact for every truncation
    for N in (2, 3, 4, 5):
        m = T @ orc.feq(rho, u, N)
        assert abs(m[0] - rho) < 4e-15
        for k in (1, 3, 9, 2, 6, 18, 4, 10, 12):
            assert abs(m[k]) < 1e-15


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_truncated_equilibrium_is_fixed_point(orc, N):
    rho, u, rng = random_state(10 + N)
    rates = np.concatenate([rng.uniform(0.2, 1.9, 2), rng.uniform(0.2, 2.0, 4)])
    fe = orc.feq(rho, u, N)
    st, out = orc.collide(fe, rates, feq_order=N)
    assert st == 0
    assert np.abs(out - fe).max() < 1e-15


@pytest.mark.parametrize("N,ref", [(2, feq2), (3, feq3)])
def test_equal_rates_is_bgk_with_truncated_equilibrium(orc, N, ref):
    rho, u, rng = random_state(20 + N)
    f = orc.feq(rho, u, 6) * (1.0 + 0.03 * rng.uniform(-1, 1, 27))
    r, uu = orc.cell_moments(f)
    om = 1.3
    st, out = orc.collide(f, orc.rates_vector(om, om, om), feq_order=N)
    assert st == 0
    assert np.abs(out - (f + om * (ref(r, uu) - f))).max() < 1e-15


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_truncated_collision_conserves(orc, N):
    rho, u, rng = random_state(30 + N)
    f = orc.feq(rho, u, 6) * (1.0 + 0.03 * rng.uniform(-1, 1, 27))
    rates = np.concatenate([rng.uniform(0.2, 1.9, 2), rng.uniform(0.2, 2.0, 4)])
    st, out = orc.collide(f, rates, feq_order=N)
    assert st == 0
    assert abs(out.sum() - f.sum()) < 1e-15
    assert np.abs(C.T @ out - C.T @ f).max() < 1e-15


def test_bad_order_rejected(orc):
    with pytest.raises(ValueError):
        orc.collide(orc.feq(1.0, np.zeros(3)), orc.rates_vector(1.0), feq_order=1)
    with pytest.raises(ValueError):
        orc.collide(orc.feq(1.0, np.zeros(3)), orc.rates_vector(1.0), feq_order=7)


def shear_wave_rate(orc, N, U, nx=32, tau=0.8, amp=0.005, steps=100):
    """Decay rate of the mode u_y = amp sin(k (x - U t)) on a periodic line,
    per step, from its Fourier amplitude after `steps` steps."""
    k = 2 * np.pi / nx
    x = np.arange(nx)
    fl = np.zeros((1, 1, nx), np.uint8)
    u = np.zeros((3, 1, 1, nx))
    u[0] = U
    u[1, 0, 0] = amp * np.sin(k * x)
    f = orc.init_fields(fl, None, u)
    st, g = orc.step(fl, f, orc.rates_vector(1.0 / tau), steps, periodic=7, feq_order=N)
    assert st == 0
    _, uu = orc.moments(fl, g)
    a = np.abs(np.sum(uu[1, 0, 0] * np.exp(-1j * k * x))) * 2 / nx
    return -np.log(a / amp) / steps, (tau - 0.5) * THETA0 * k * k


def test_third_order_terms_restore_galilean_shear_viscosity(orc):
    U = 0.15
    r2, nuk2 = shear_wave_rate(orc, 2, U)
    r3, _ = shear_wave_rate(orc, 3, U)
    r6, _ = shear_wave_rate(orc, 6, U)
    # third order on: the viscosity of Eq. (5), independent of the stream
    assert abs(r3 / nuk2 - 1.0) < 0.01
    assert abs(r6 / r3 - 1.0) < 1e-9
    # second order: the missing rho u_x^2 u_y moment lowers the shear
    # viscosity by the factor 1 - U^2 / theta0
    assert abs((r2 / r3) / (1.0 - U * U / THETA0) - 1.0) < 0.002
