"""The explicit truncated equilibrium (Sec. 2.1, Eq. (4) summed to an order
N = 2..5; App. A after Eq. (A.6)) on the GPU against the oracle's collision
with the same truncation.

Random configurations of every boundary option (those of
test_gpu_random_configs) with N = 2..5, from random populations, 1..8
steps: the same per-step bounds as with the full equilibrium (FP32 4e-7,
FP16S 5e-5 max abs): forming f^eq_N and transforming f - f^eq_N adds a few
FP32 roundings of values the size of f, as the implicit form does.  Packed
with domains of the full equilibrium (reduced and general rates), each
domain ends bit for bit where it ends alone.  The advected shear wave
decays at nu (1 - U^2 / theta0) k^2 with N = 2 and at nu k^2 with N = 3, as
the oracle's pin states."""
import numpy as np
import pytest

from paper_2204_10566_amd import inputs as I

from test_gpu_random_configs import TOL_PER_STEP, build_domain, make_case

pytestmark = pytest.mark.gpu

THETA0 = 1.0 / 3.0


def say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def capi():
    from paper_2204_10566_amd import capi

    return capi


@pytest.mark.parametrize("k", range(16))
def test_random_configuration_truncated_equilibrium(capi, orc, k):
    c = make_case(100 + k)
    N = 2 + k % 4
    fl = c["fl"]
    say(f"case {k}: order {N} shape {fl.shape} periodic {c['periodic']} {c['storage']} steps {c['steps']} "
        f"outlet {c['outlet']} curved {c['q'] is not None} orders {np.round(c['order'], 3).tolist()}")
    d = build_domain(capi, c, c["storage"])
    d.set_equilibrium_order(N)
    fs = d.populations().astype(np.float64)
    d.step(c["steps"])
    fg = d.populations()
    d.destroy()
    rates = orc.rates_vector(c["omega"], c["omega_b"], order_rates=c["order"])
    st, fo = orc.step(fl, fs, rates, c["steps"], periodic=c["periodic"], uin=c["uin"], outlet=c["outlet"],
                      q=c["q"], feq_order=N)
    assert st == 0
    upd = (fl == I.FLUID) | (fl == I.OUTLET)
    err = float(np.abs(fg[:, upd] - fo[:, upd]).max()) if upd.any() else 0.0
    tol = TOL_PER_STEP[c["storage"]] * c["steps"]
    say(f"  max abs err {err:.3e} (bound {tol:.1e})")
    assert err <= tol


def test_order_six_is_the_implicit_form(capi):
    """Order 6 selects the implicit full equilibrium: the same bits as a
    domain that never set an order."""
    c = make_case(7)
    out = []
    for order in (None, 6):
        d = build_domain(capi, c, "fp32")
        if order is not None:
            d.set_equilibrium_order(order)
        d.step(c["steps"])
        out.append(d.populations())
        d.destroy()
    assert np.array_equal(out[0], out[1])


def test_bad_order_rejected(capi):
    d = capi.Domain(I.periodic_box(4), periodic=7)
    for bad in (1, 7):
        with pytest.raises(capi.LbmError) as e:
            d.set_equilibrium_order(bad)
        assert e.value.code == capi.ERR_ARG
    d.destroy()


def test_packed_truncated_equals_alone(capi):
    """A batch mixing truncated equilibria (N = 2, 3) with the full one
    (reduced and general higher-order rates): every domain ends bit for bit
    where it ends alone."""
    cases = [make_case(k, "fp16s") for k in range(6)]
    orders = [2, 6, 3, 6, 5, 6]
    steps = [3 * c["steps"] + k for k, c in enumerate(cases)]
    say(f"packed mix: orders {orders}, steps {steps}")
    alone = []
    for c, N, n in zip(cases, orders, steps):
        d = build_domain(capi, c, "fp16s")
        d.set_equilibrium_order(N)
        d.step(n)
        alone.append(d.populations())
        d.destroy()
    doms = []
    for c, N in zip(cases, orders):
        d = build_domain(capi, c, "fp16s")
        d.set_equilibrium_order(N)
        doms.append(d)
    b = capi.Batch(1 << 32, "fp16s")
    slots = [b.admit(d, n) for d, n in zip(doms, steps)]
    b.step(max(steps))
    assert sorted(b.poll(wait=True)) == sorted(slots)
    for k, s in enumerate(slots):
        b.release(s)
        assert np.array_equal(doms[k].populations(), alone[k]), f"case {k} differs"
        doms[k].destroy()
    b.destroy()


def shear_wave_rate(capi, N, U, nx=32, tau=0.8, amp=0.005, steps=100):
    k = 2 * np.pi / nx
    x = np.arange(nx)
    u = np.zeros((3, 1, 1, nx), np.float32)
    u[0] = U
    u[1, 0, 0] = amp * np.sin(k * x)
    d = capi.Domain(np.zeros((1, 1, nx), np.uint8), periodic=7)
    d.set_params(tau)
    d.set_equilibrium_order(N)
    d.init_fields(None, u)
    d.step(steps)
    _, uu = d.moments()
    d.destroy()
    a = np.abs(np.sum(uu[1, 0, 0].astype(np.float64) * np.exp(-1j * k * x))) * 2 / nx
    return -np.log(a / amp) / steps, (tau - 0.5) * THETA0 * k * k


def test_galilean_shear_viscosity(capi):
    U = 0.15
    r2, nuk2 = shear_wave_rate(capi, 2, U)
    r3, _ = shear_wave_rate(capi, 3, U)
    say(f"advected shear wave: rate/nu k^2 = {r2 / nuk2:.4f} (order 2), {r3 / nuk2:.4f} (order 3)")
    assert abs(r3 / nuk2 - 1.0) < 0.01
    assert abs((r2 / r3) / (1.0 - U * U / THETA0) - 1.0) < 0.002
