"""Exact pin of the outlet's transverse source shift (Sec. 2.2, "Simulation
details": the outlet condition of the last axial plane).

A population with c_x = -1 that an outlet cell (nx - 1, y, z) pulls from
beyond the box comes, for the zero-gradient outlet, from the last-plane cell
s = (nx - 1, y - c_y, z - c_z) that faces it, and the constant-pressure
outlet shifts that same value to the outlet density.  On a state that does
not vary along x this is exactly what an x-periodic box gives: there the
source is (0, y - c_y, z - c_z), which holds the same values as s.  The
tests below take an x-invariant state that does vary across y and z (walls
at y = 0 and y = ny - 1, periodic z), step it through the outlet and through
an x-periodic box, and require the two to agree bit for bit at every cell
the x = 0 face cannot have reached yet.  A source clamped to (nx - 1, y, z)
instead gives a different answer; the first test checks that the state is
such that it would."""
import numpy as np
import pytest

NX, NY, NZ = 9, 7, 5
C = np.array([(i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1) for i in range(27)])


def flags(outlet: bool):
    fl = np.zeros((NZ, NY, NX), np.uint8)
    fl[:, 0, :] = 1
    fl[:, NY - 1, :] = 1
    if outlet:
        fl[:, 1:NY - 1, NX - 1] = 3
    return fl


def x_invariant_state(orc, seed, uniform_density):
    """Populations that depend on (y, z) only; with uniform_density the
    perturbation of each cell sums to zero over i, so rho = 1 everywhere."""
    rng = np.random.default_rng(seed)
    rho = np.ones((NZ, NY, 1)) if uniform_density else 1.0 + 0.02 * rng.uniform(-1, 1, (NZ, NY, 1))
    u = 0.04 * rng.uniform(-1, 1, (3, NZ, NY, 1))
    f = orc.init_fields(np.zeros((NZ, NY, 1), np.uint8), rho, u)
    p = 0.01 * rng.uniform(-1, 1, f.shape) * f
    if uniform_density:
        p -= p.mean(axis=0, keepdims=True)
    return np.ascontiguousarray(np.broadcast_to(f + p, (27, NZ, NY, NX)))


def step_both(orc, f, rates, nsteps, outlet):
    st_o, g_o = orc.step(flags(True), f, rates, nsteps, periodic=4, outlet=outlet)
    st_p, g_p = orc.step(flags(False), f, rates, nsteps, periodic=5)
    assert st_o == 0 and st_p == 0
    return g_o, g_p


def test_state_distinguishes_the_shifted_source(orc):
    """At the outlet plane, the c_x = -1 population of the shifted source
    (nx - 1, y - c_y, z - c_z) differs from that of (nx - 1, y, z) for every
    direction with a transverse component, so an unshifted clamp fails the
    tests below."""
    f = x_invariant_state(orc, 0, False)
    for i in range(27):
        if C[i, 0] != -1 or (C[i, 1] == 0 and C[i, 2] == 0):
            continue
        for z in range(NZ):
            for y in range(2, NY - 2):
                s = f[i, (z - C[i, 2]) % NZ, y - C[i, 1], NX - 1]
                assert s != f[i, z, y, NX - 1]


@pytest.mark.parametrize("nsteps", [1, 3])
def test_zero_gradient_outlet_equals_periodic_continuation(orc, nsteps):
    """All rates 0 (pure streaming): the outlet plane receives exactly what
    an x-periodic box gives, bit for bit, and so does every cell with
    x >= nsteps."""
    f = x_invariant_state(orc, 1, False)
    g_o, g_p = step_both(orc, f, orc.rates_vector(0.0, 0.0, 0.0), nsteps, None)
    upd = flags(True)[:, :, nsteps:] != 1
    assert np.array_equal(g_o[:, :, :, nsteps:][:, upd], g_p[:, :, :, nsteps:][:, upd])


def test_pressure_outlet_at_local_density_equals_periodic_continuation(orc):
    """Constant-pressure outlet with rho_out equal to the (uniform) density:
    the extrapolated ghost value is f*(s) itself, so again the periodic
    continuation, to the rounding of rho_s."""
    f = x_invariant_state(orc, 2, True)
    rho, _ = orc.moments(np.zeros((NZ, NY, NX), np.uint8), f)
    assert np.abs(rho - 1.0).max() < 1e-14
    g_o, g_p = step_both(orc, f, orc.rates_vector(0.0, 0.0, 0.0), 1, ("pressure", 1.0))
    upd = flags(True)[:, :, 1:] != 1
    # the ghost shift (rho_out - rho_s) f^eq is zero only up to the rounding
    # of rho_s; compare to that rounding
    assert np.abs(g_o[:, :, :, 1:][:, upd] - g_p[:, :, :, 1:][:, upd]).max() < 1e-14


@pytest.mark.parametrize("outlet,nsteps", [(None, 2), (("pressure", 1.0), 1)])
def test_outlet_plane_with_collision_equals_periodic_continuation(orc, outlet, nsteps):
    """With the paper's collision (tau 0.6, higher orders at rate 1), which
    is local, the outlet plane and every cell with x >= nsteps still match
    the x-periodic run: bit for bit for the zero-gradient outlet over two
    steps; for the pressure outlet over the one step in which the faced
    density still equals rho_out (streaming then makes it vary), to the
    rounding of rho_s."""
    f = x_invariant_state(orc, 3, outlet is not None)
    g_o, g_p = step_both(orc, f, orc.rates_vector(1.0 / 0.6), nsteps, outlet)
    upd = flags(True)[:, :, nsteps:] != 1
    d = np.abs(g_o[:, :, :, nsteps:][:, upd] - g_p[:, :, :, nsteps:][:, upd]).max()
    if outlet is None:
        assert d == 0.0
    else:
        assert d < 1e-14
