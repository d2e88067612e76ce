"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against an independent source: the weights the
paper prints (App. A), numpy's Gauss-Hermite quadrature and Hermite
polynomials (library routines), closed-form moments of the Maxwellian, the
textbook second-order equilibrium, and identities of the collision operator
(Sec. 2.1, Eqs. (3), (6)-(8); App. A, Eqs. (A.3)-(A.6)).
"""
import itertools
import math
import os

import numpy as np
import pytest
from numpy.polynomial import hermite_e as He

THETA0 = 1.0 / 3.0
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def he_scaled(n, x):
    """theta0^(n/2) He_n(x / sqrt(theta0)) from numpy's probabilists' Hermite
    polynomials: the 1-D Hermite polynomial for weight exp(-x^2/(2 theta0))."""
    coef = np.zeros(n + 1)
    coef[n] = 1.0
    s = math.sqrt(THETA0)
    return s ** n * He.hermeval(np.asarray(x) / s, coef)


def lattice():
    """Velocity set in the library's documented order, built independently."""
    c = np.array([(i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1) for i in range(27)])
    return c


# --------------------------------------------------------------------------
# velocity set and weights
# --------------------------------------------------------------------------
def test_weights_match_paper_table(orc):
    c, w = orc.velocity_set()
    assert np.array_equal(c, lattice())
    rows = [l.split() for l in open(os.path.join(GOLDEN, "d3q27_weights.txt")) if l.strip() and l[0] != "#"]
    for nnz, count, num, den in rows:
        sel = np.abs(c).sum(axis=1) == int(nnz)
        assert sel.sum() == int(count)
        assert np.allclose(w[sel], int(num) / int(den), rtol=0, atol=1e-16)


def test_weights_are_gauss_hermite_quadrature(orc):
    # numpy's 3-point Gauss-Hermite (probabilists') rule, nodes scaled by
    # sqrt(theta0) = 1/sqrt(3): the nodes become -1, 0, 1.
    x, wq = He.hermegauss(3)
    wq = wq / wq.sum()
    assert np.allclose(x / math.sqrt(3.0), [-1, 0, 1], atol=1e-14)
    c, w = orc.velocity_set()
    w1 = dict(zip([-1, 0, 1], wq))
    ref = np.array([w1[a] * w1[b] * w1[g] for a, b, g in c])
    assert np.allclose(w, ref, atol=1e-15)


def test_lattice_isotropy(orc):
    c, w = orc.velocity_set()
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), THETA0 * np.eye(3), atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib,ig->abg", w, c, c, c), 0, atol=1e-16)
    d = np.eye(3)
    iso4 = THETA0 ** 2 * (np.einsum("ab,gd->abgd", d, d) + np.einsum("ag,bd->abgd", d, d)
                          + np.einsum("ad,bg->abgd", d, d))
    assert np.allclose(np.einsum("i,ia,ib,ig,id->abgd", w, c, c, c, c), iso4, atol=1e-16)
    # opposite direction of i is 26 - i
    assert np.array_equal(c[::-1], -c)


# --------------------------------------------------------------------------
# Hermite polynomials (App. A, Eq. (A.3)), dimensional reading
# --------------------------------------------------------------------------
def test_hermite_matches_numpy_product(orc):
    rng = np.random.default_rng(3)
    for n in range(0, 7):
        for idx in itertools.product(range(3), repeat=n):
            xi = rng.uniform(-1.5, 1.5, 3)
            cnt = [idx.count(a) for a in range(3)]
            ref = np.prod([he_scaled(cnt[a], xi[a]) for a in range(3)])
            got = orc.hermite(list(idx), xi)
            assert abs(got - ref) < 1e-13 * max(1.0, abs(ref)), (idx, got, ref)


def test_hermite_second_order_paper_form(orc):
    xi = np.array([0.3, -0.7, 0.2])
    for a in range(3):
        for b in range(3):
            ref = xi[a] * xi[b] - (THETA0 if a == b else 0.0)
            assert abs(orc.hermite([a, b], xi) - ref) < 1e-15


# --------------------------------------------------------------------------
# equilibrium (Sec. 2.1, Eq. (4); App. A, Eqs. (A.4)-(A.6))
# --------------------------------------------------------------------------
def test_tuple_count(orc):
    # index tuples of length <= 6 with no axis more than twice
    assert orc.num_tuples() == sum(math.factorial(a + b + g) // (math.factorial(a) * math.factorial(b)
                                                                  * math.factorial(g))
                                   for a in range(3) for b in range(3) for g in range(3))


@pytest.mark.parametrize("rho,u", [(1.0, [0.0, 0.0, 0.0]), (1.03, [0.05, -0.02, 0.03]),
                                   (0.97, [0.2, 0.1, -0.15]), (1.2, [-0.3, 0.25, 0.05])])
def test_feq_raw_moments_are_maxwellian(orc, rho, u):
    """Every raw moment sum_i f_i c_x^p c_y^q c_z^r with p,q,r <= 2 equals
    the Maxwellian's rho m_p(u_x) m_q(u_y) m_r(u_z), m0 = 1, m1 = u,
    m2 = u^2 + theta0.  These 27 moments determine the 27 populations."""
    c = lattice()
    f = orc.feq(rho, u, 6)
    m = lambda p, v: [1.0, v, v * v + THETA0][p]
    for p, q, r in itertools.product(range(3), repeat=3):
        got = np.sum(f * c[:, 0] ** p * c[:, 1] ** q * c[:, 2] ** r)
        ref = rho * m(p, u[0]) * m(q, u[1]) * m(r, u[2])
        assert abs(got - ref) < 1e-15 * 10, (p, q, r, got, ref)


def test_feq_second_order_is_textbook(orc):
    c, w = lattice(), orc.velocity_set()[1]
    rho, u = 1.04, np.array([0.07, -0.05, 0.02])
    cu = c @ u
    ref = w * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * (u @ u))
    assert np.allclose(orc.feq(rho, u, 2), ref, atol=1e-16)


def test_feq_is_central_moment_fixed_point(orc):
    """App. A, Eqs. (A.5)-(A.6): T f^eq = (rho, 0, ..., 0) with the full
    expansion, and not with the second-order truncation."""
    rho, u = 1.1, np.array([0.12, -0.08, 0.05])
    T = orc.transform(u)
    m6 = T @ orc.feq(rho, u, 6)
    assert abs(m6[0] - rho) < 1e-14 and np.abs(m6[1:]).max() < 1e-14
    m2 = T @ orc.feq(rho, u, 2)
    assert np.abs(m2[1:]).max() > 1e-4


# --------------------------------------------------------------------------
# central-Hermite-moment transform (Sec. 2.1, Eqs. (7)-(8))
# --------------------------------------------------------------------------
def T1_numpy(u):
    cs = np.array([-1.0, 0.0, 1.0])
    return np.array([he_scaled(a, cs - u) for a in range(3)])


def test_transform_is_kronecker_of_numpy_hermite(orc):
    rng = np.random.default_rng(5)
    for _ in range(5):
        u = rng.uniform(-0.3, 0.3, 3)
        ref = np.kron(T1_numpy(u[2]), np.kron(T1_numpy(u[1]), T1_numpy(u[0])))
        assert np.allclose(orc.transform(u), ref, atol=1e-14)


def test_transform_invertible_and_orthogonal_at_rest(orc):
    for uu in [-0.4, 0.0, 0.17]:
        assert abs(np.linalg.det(T1_numpy(uu)) - 2.0) < 1e-13
    _, w = orc.velocity_set()
    T0 = orc.transform(np.zeros(3))
    G = (T0 * w) @ T0.T
    assert np.allclose(G - np.diag(np.diag(G)), 0, atol=1e-15)


# --------------------------------------------------------------------------
# collision (Sec. 2.1, Eq. (6)); pins independent of the oracle's T
# --------------------------------------------------------------------------
def random_state(orc, rng, amp=0.02):
    rho = 1 + rng.uniform(-0.05, 0.05)
    u = rng.uniform(-0.1, 0.1, 3)
    f = orc.feq(rho, u, 6)
    return f * (1 + amp * rng.uniform(-1, 1, 27))


def test_collision_fixed_point(orc):
    rng = np.random.default_rng(0)
    for _ in range(5):
        f = orc.feq(1 + 0.1 * rng.uniform(-1, 1), rng.uniform(-0.2, 0.2, 3), 6)
        st, fs = orc.collide(f, orc.rates_vector(1 / 0.53, 1.3, 1.0))
        assert st == 0 and np.abs(fs - f).max() < 1e-15


def test_collision_equal_rates_is_bgk(orc):
    """With every rate equal to omega, CHM-MRT reduces to the BGK update
    of Eq. (3): f* = f + omega (f^eq - f)."""
    rng = np.random.default_rng(1)
    for omega in [0.3, 1.0, 1.7]:
        f = random_state(orc, rng)
        rho, u = f.sum(), lattice().T @ f / f.sum()
        st, fs = orc.collide(f, orc.rates_vector(omega, omega, order_rates=[omega] * 4))
        assert st == 0
        assert np.abs(fs - (f + omega * (orc.feq(rho, u, 6) - f))).max() < 2e-16 * 10


def test_collision_unit_rates_gives_equilibrium(orc):
    rng = np.random.default_rng(2)
    f = random_state(orc, rng)
    rho, u = f.sum(), lattice().T @ f / f.sum()
    st, fs = orc.collide(f, orc.rates_vector(1.0, 1.0, 1.0))
    assert np.abs(fs - orc.feq(rho, u, 6)).max() < 1e-15


def test_collision_conserves_mass_momentum(orc):
    rng = np.random.default_rng(4)
    c = lattice()
    for _ in range(5):
        f = random_state(orc, rng, 0.05)
        st, fs = orc.collide(f, orc.rates_vector(1 / 0.51, 0.7, 1.2))
        assert abs(fs.sum() - f.sum()) < 1e-15 * 4
        assert np.abs(c.T @ fs - c.T @ f).max() < 1e-15 * 4


def test_collision_relaxes_each_central_moment(orc):
    """Central moments built with numpy (Kronecker of 1-D Hermite rows):
    off-diagonal 2nd order x(1-omega), diagonal trace x(1-omega_b),
    deviator x(1-omega), order n >= 3 x(1-omega_n), orders 0-1 kept."""
    rng = np.random.default_rng(6)
    omega, omb = 1 / 0.55, 0.8
    high = [1.1, 0.9, 1.3, 0.6]
    for _ in range(3):
        f = random_state(orc, rng, 0.05)
        rho, u = f.sum(), lattice().T @ f / f.sum()
        T = np.kron(T1_numpy(u[2]), np.kron(T1_numpy(u[1]), T1_numpy(u[0])))
        m, ms = T @ f, T @ orc.collide(f, orc.rates_vector(omega, omb, order_rates=high))[1]
        ks = [(k % 3, (k // 3) % 3, k // 9) for k in range(27)]
        diag = [k for k, (p, q, r) in enumerate(ks) if p + q + r == 2 and 2 in (p, q, r)]
        tr, trs = m[diag].mean(), ms[diag].mean()
        assert abs(trs - (1 - omb) * tr) < 1e-14
        for k, (p, q, r) in enumerate(ks):
            n = p + q + r
            if n <= 1:
                ref = m[k]
            elif n == 2 and k in diag:
                ref = (1 - omega) * (m[k] - tr) + (1 - omb) * tr
            elif n == 2:
                ref = (1 - omega) * m[k]
            else:
                ref = (1 - high[n - 3]) * m[k]
            assert abs(ms[k] - ref) < 1e-14, (k, ms[k], ref)


def test_cell_moments_brute_force(orc):
    """Density and velocity of a population set (Sec. 2.1): the plain sums
    over the lattice, built here from the documented velocity order."""
    rng = np.random.default_rng(8)
    c = lattice()
    for _ in range(5):
        f = random_state(orc, rng, 0.05)
        rho, u = orc.cell_moments(f)
        assert abs(rho - f.sum()) < 1e-15
        assert np.abs(u - (c.T @ f) / f.sum()).max() < 1e-15


def test_collide_field_is_per_cell_collision(orc):
    """The field collision applies the one-cell collision to every updated
    cell (fluid, outlet) and leaves solid and inlet cells as they are."""
    rng = np.random.default_rng(9)
    fl = np.zeros((2, 3, 4), np.uint8)
    fl[0, 1, 2] = 1  # solid
    fl[1, 0, 0] = 2  # inlet
    fl[1, 2, 3] = 3  # outlet
    f = np.stack([random_state(orc, rng, 0.05) for _ in range(fl.size)], axis=1).reshape((27,) + fl.shape)
    rates = orc.rates_vector(1 / 0.6, 0.9, order_rates=[1.1, 1.2, 0.8, 1.3])
    st, fo = orc.collide_field(fl, f, rates)
    assert st == 0
    f2, fo2 = f.reshape(27, -1), fo.reshape(27, -1)
    for cell, flag in enumerate(fl.ravel()):
        if flag in (0, 3):
            st1, ref = orc.collide(f2[:, cell], rates)
            assert st1 == 0
            assert np.array_equal(fo2[:, cell], ref)
        else:
            assert np.array_equal(fo2[:, cell], f2[:, cell])
