"""Constant-pressure outlet (non-equilibrium extrapolation, Sec. 2.2) on the
GPU against the oracle: random states on geometries with every boundary
kind, state access after odd step counts and a change of the outlet
density, the full-size nozzle at sampled cells, and packed execution."""
import sys

import numpy as np
import pytest

from paper_2204_10566_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def capi():
    from paper_2204_10566_amd import capi

    return capi


def updated(fl):
    return (fl == I.FLUID) | (fl == I.OUTLET)


def random_pops(fl, seed):
    # FP32-representable, so both sides start from identical values
    return I.random_populations(fl.shape, seed).astype(np.float32).astype(np.float64)


def channel(nx, ny, nz, obstacle=True):
    """Inlet plane, outlet plane, walls in y, z periodic, an obstacle."""
    fl = np.zeros((nz, ny, nx), np.uint8)
    fl[:, 0, :] = I.SOLID
    fl[:, -1, :] = I.SOLID
    fl[:, 1:-1, 0] = I.INLET
    fl[:, 1:-1, -1] = I.OUTLET
    if obstacle:
        fl[min(2, nz - 1), 3:5, nx // 3:nx // 3 + 3] = I.SOLID
    # a solid cell on the outlet plane: links of its neighbours bounce back
    fl[0, ny // 2, -1] = I.SOLID
    return fl


def inlet_velocity(fl, seed, amp=0.03):
    rng = np.random.default_rng(seed)
    uin = np.zeros((3,) + fl.shape, np.float32)
    uin[:, fl == I.INLET] = amp * rng.uniform(-1, 1, (3, int((fl == I.INLET).sum())))
    return uin


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
@pytest.mark.parametrize("shape", [(23, 9, 5), (128, 10, 6)])
def test_pressure_outlet_random_states(capi, orc, storage, shape):
    """1 and 6 steps from random populations with rho_out away from the
    state's density, on a ragged and on a row-aligned channel."""
    fl = channel(*shape)
    uin = inlet_velocity(fl, 3)
    f0 = random_pops(fl, 5)
    rates = (1 / 0.57, 1.2, 1.0)
    upd = updated(fl)
    tol = 4e-7 if storage == "fp32" else 5e-5  # per step; FP16S: 2^-11 |f - w| per store
    for steps in (1, 6):
        say(f"pressure outlet {shape} {storage} steps={steps}")
        d = capi.Domain(fl, periodic=4, storage=storage)
        d.set_rates(*rates)
        d.set_outlet("pressure", 1.03)
        d.set_inlet(uin)
        d.set_populations(f0)
        fs = d.populations().astype(np.float64)
        d.step(steps)
        st, fo = orc.step(fl, fs, orc.rates_vector(*rates), steps, periodic=4, uin=uin, outlet=("pressure", 1.03))
        assert st == 0
        err = np.abs(d.populations()[:, upd] - fo[:, upd]).max()
        say(f"  max abs err {err:.3e}")
        assert err <= tol * steps
        d.destroy()


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_pressure_outlet_state_access_and_change(capi, orc, storage):
    """3 steps, export (odd count), 1 step, new outlet density, 3 steps, new
    outlet density after the odd count, 2 steps, then the zero-gradient
    outlet for 2 steps: each segment equals the oracle's pull update."""
    fl = channel(23, 9, 5)
    uin = inlet_velocity(fl, 21)
    f0 = random_pops(fl, 13)
    rates = (1 / 0.6, 1.1, 1.0)
    rv = orc.rates_vector(*rates)
    upd = updated(fl)
    tol = 4e-7 if storage == "fp32" else 5e-5  # per step; FP16S: 2^-11 |f - w| per store
    say(f"pressure outlet state access {storage}")
    d = capi.Domain(fl, periodic=4, storage=storage)
    d.set_rates(*rates)
    d.set_outlet("pressure", 0.98)
    d.set_inlet(uin)
    d.set_populations(f0)
    fo = d.populations().astype(np.float64)
    segments = [(3, ("pressure", 0.98)), (1, ("pressure", 0.98)), (3, ("pressure", 1.02)), (2, ("pressure", 1.05)),
                (2, None)]
    total = 0
    for k, (n, outlet) in enumerate(segments):
        if k and outlet != segments[k - 1][1]:
            d.set_outlet(*(outlet or ("zero_gradient", 1.0)))
        d.step(n)
        total += n
        st, fo = orc.step(fl, fo, rv, n, periodic=4, uin=uin, outlet=outlet)
        assert st == 0
        err = np.abs(d.populations()[:, upd] - fo[:, upd]).max()
        say(f"  after {total} steps ({outlet}): max abs err {err:.3e}")
        assert err <= tol * total


def test_pressure_outlet_full_size_nozzle_sampled(capi, orc):
    """Full-size nozzle (96x96x768) with the pressure outlet, 3 steps in the
    benchmark's launch configuration; sampled cells (outlet plane and the
    plane before it, random) against the oracle's dependency-cone run."""
    cfg = I.nozzle_config("re500")
    fl, tau = cfg["flags"], cfg["tau"]
    u0 = cfg["u0"].astype(np.float32)
    uin = cfg["uin"].astype(np.float32)
    say(f"nozzle re500 {fl.shape} pressure outlet 3 steps")
    d = capi.Domain(fl, periodic=0)
    d.set_params(tau, 1.0 / tau, 1.0)
    d.set_outlet("pressure", 1.002)
    d.set_inlet(uin)
    d.init_fields(None, u0)
    d.step(3)
    fg = d.populations().reshape(27, -1)
    upd = np.flatnonzero(updated(fl).ravel())
    nx_ = fl.shape[2]
    xs = upd % nx_
    rng = np.random.default_rng(1)
    cells = np.unique(np.concatenate([rng.choice(upd[xs == nx_ - 1], 80, replace=False),
                                      rng.choice(upd[xs == nx_ - 2], 40, replace=False),
                                      rng.choice(upd, 60, replace=False)]))
    st, fo = orc.run_cells(fl, cells, orc.rates_vector(1 / tau), 3, periodic=0, uin=uin, u0=u0,
                           outlet=("pressure", 1.002))
    assert st == 0
    err = np.abs(fg[:, cells] - fo).max()
    say(f"  {cells.size} cells, max abs err {err:.3e}")
    assert err <= 1e-6


def test_pressure_outlet_in_batch_equals_alone(capi):
    """A pressure-outlet domain and a zero-gradient domain advanced in one
    packed launch end exactly where each ends alone."""
    shapes = [((23, 9, 5), ("pressure", 1.01)), ((40, 12, 7), None), ((31, 10, 4), ("pressure", 0.99))]
    say("pressure outlet packed vs alone")

    def make(k):
        shape, outlet = shapes[k]
        fl = channel(*shape)
        d = capi.Domain(fl, periodic=4, storage="fp16s")
        d.set_rates(1 / 0.6, 1 / 0.6, 1.0)
        if outlet:
            d.set_outlet(*outlet)
        d.set_inlet(inlet_velocity(fl, 50 + k, 0.02))
        d.init_fields(None, None)
        return d

    steps = [17, 24, 9]
    alone = []
    for k in range(3):
        d = make(k)
        d.step(steps[k])
        alone.append(d.populations())
        d.destroy()
    doms = [make(k) for k in range(3)]
    b = capi.Batch(1 << 32, "fp16s")
    slots = [b.admit(d, n) for d, n in zip(doms, steps)]
    b.step(max(steps))
    done = b.poll(wait=True)
    assert sorted(done) == sorted(slots)
    for k, s in enumerate(slots):
        b.release(s)
        assert np.array_equal(doms[k].populations(), alone[k]), f"domain {k} differs"
        doms[k].destroy()
    b.destroy()


def test_set_outlet_rejects_bad_arguments(capi):
    fl = channel(23, 9, 5)
    d = capi.Domain(fl, periodic=4)
    for kind, rho in [(7, 1.0), (1, 0.0), (1, -1.0), (1, float("nan"))]:
        assert capi.lbm_set_outlet(d.h, kind, rho) == capi.ERR_ARG
    assert capi.lbm_set_outlet(d.h, 1, 1.01) == capi.OK
    d.destroy()
