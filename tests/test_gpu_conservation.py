"""Mass and momentum of a long FP32 run on a periodic box (Sec. 2.1: the
collision of Eq. (6) conserves both; streaming on a periodic box moves
them).  Every FP32 rounding changes them by about 2^-24 relative, with no
preferred sign, so over n steps of N cells the totals drift like a random
walk: about sqrt(n / N) * 6e-8, 5e-7 for 20000 steps of 256 cells.  The
bound, 5e-6, leaves a factor of ten; an error of one sign per step (such as
a velocity formed with a reciprocal that errs to one side) would add up to
about n * 6e-8 = 1e-3."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def capi():
    from paper_2204_10566_amd import capi

    return capi


def totals(d):
    rho, u = d.moments()
    r = rho.astype(np.float64)
    return r.sum(), (u.astype(np.float64) * r).reshape(3, -1).sum(axis=1)


@pytest.mark.parametrize("order", [6, 2])
def test_long_run_conserves_mass_and_momentum(capi, order):
    shape = (2, 16, 8)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u0 = np.zeros((3,) + shape)
    u0[0] = 0.05 + 0.01 * np.sin(2 * np.pi * y / ny)
    u0[1] = 0.004 * np.sin(2 * np.pi * x / nx)
    u0[2] = 0.006 * np.cos(2 * np.pi * y / ny)
    d = capi.Domain(np.zeros(shape, np.uint8), periodic=7, storage="fp32")
    d.set_params(0.5015)
    d.set_equilibrium_order(order)
    d.init_fields(None, u0.astype(np.float32))
    m0, j0 = totals(d)
    d.step(20000)
    m1, j1 = totals(d)
    d.destroy()
    em = abs(m1 - m0) / m0
    ej = float(np.abs(j1 - j0).max() / np.abs(j0).max())
    say(f"equilibrium order {order}: mass drift {em:.2e}, momentum drift {ej:.2e} over 20000 steps")
    assert em <= 5e-6 and ej <= 5e-6
