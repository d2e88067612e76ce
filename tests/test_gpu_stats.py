"""Device-side statistics (Sec. 2.2, Eqs. (15)-(19); App. A, Eqs. (A.7)-
(A.8)) against the same statistics formed by the oracle: every second step
(the library's local-phase steps) samples u, u_a u_b and the viscous stress
of the pre-collision state; the oracle forms the pre-collision state of
step k by streaming its post-collision state of step k - 1."""
import numpy as np
import pytest

from paper_2204_10566_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def capi():
    from paper_2204_10566_amd import capi

    return capi


def say(msg):
    print(f"[gpu] {msg}", flush=True)


def geometry():
    nz, ny, nx = 5, 9, 23
    fl = np.zeros((nz, ny, nx), np.uint8)
    fl[:, 0, :] = I.SOLID
    fl[:, -1, :] = I.SOLID
    fl[:, 1:-1, 0] = I.INLET
    fl[:, 1:-1, -1] = I.OUTLET
    fl[2, 3:5, 8:11] = I.SOLID
    return fl


def oracle_stats(orc, fl, f0, rates, steps, sampled, uin):
    """Means over the steps in `sampled` (1-based) of u, u_a u_b, sigma."""
    rv = orc.rates_vector(*rates)
    su = np.zeros((3,) + fl.shape)
    suu = np.zeros((6,) + fl.shape)
    ss = np.zeros((6,) + fl.shape)
    f = f0
    pa, pb = [0, 1, 2, 0, 0, 1], [0, 1, 2, 1, 2, 2]
    for k in range(1, steps + 1):
        if k in sampled:
            pre = orc.stream(fl, f, periodic=4, uin=uin)
            _, u = orc.moments(fl, pre)
            su += u
            for c in range(6):
                suu[c] += u[pa[c]] * u[pb[c]]
            ss += orc.stress(fl, pre, rates[0])
        st, f = orc.step(fl, f, rv, 1, periodic=4, uin=uin)
        assert st == 0
    n = len(sampled)
    return su / n, suu / n, ss / n


@pytest.mark.parametrize("rates", [(1 / 0.6, 1 / 0.6, 1.0), (1 / 0.53, 1.2, 1.4)])
def test_stats_match_oracle(capi, orc, rates):
    fl = geometry()
    rng = np.random.default_rng(51)
    uin = np.zeros((3,) + fl.shape, np.float32)
    uin[:, fl == I.INLET] = 0.03 * rng.uniform(-1, 1, (3, int((fl == I.INLET).sum())))
    f0 = I.random_populations(fl.shape, 53).astype(np.float32).astype(np.float64)
    say(f"statistics rates={rates}")
    d = capi.Domain(fl, periodic=4)
    d.set_rates(*rates)
    d.set_inlet(uin)
    d.set_populations(f0)
    d.stats_enable(True)
    d.step(3)
    d.step(4)  # phases continue across calls: samples at steps 2, 4, 6
    mu, muu, ms, n = d.stats()
    d.destroy()
    assert n == 3
    ou, ouu, os_ = oracle_stats(orc, fl, f0, rates, 7, {2, 4, 6}, uin)
    upd = (fl == I.FLUID) | (fl == I.OUTLET)
    eu = np.abs(mu - ou)[:, upd].max()
    euu = np.abs(muu - ouu)[:, upd].max()
    es = np.abs(ms - os_)[:, upd].max()
    say(f"  max abs err u {eu:.2e}, uu {euu:.2e}, sigma {es:.2e} (sigma scale {np.abs(os_).max():.2e})")
    assert eu <= 3e-6 and euu <= 1e-6 and es <= 3e-6
    assert np.all(mu[:, ~upd] == 0)


def test_stats_in_batch_equal_alone(capi):
    """Statistics gathered while the domain runs in a packed batch equal
    those of the same domain stepped alone."""
    spec = I.batched_domains(count=1, seed=3, lo=12, hi=20, materialise=True)[0]
    out = []
    for packed in (False, True):
        d = capi.Domain(spec.flags, periodic=spec.periodic, storage="fp32")
        d.set_params(spec.tau)
        d.init_fields(None, spec.u.astype(np.float32))
        d.stats_enable(True)
        if packed:
            b = capi.Batch(1 << 33, "fp32")
            s = b.admit(d, 9)
            while not b.poll(wait=True):
                b.step(3)
            b.release(s)
            b.destroy()
        else:
            d.step(9)
        out.append(d.stats())
        d.destroy()
    say(f"statistics alone vs batch: samples {out[0][3]} / {out[1][3]}")
    assert out[0][3] == out[1][3] == 4
    for a, b_ in zip(out[0][:3], out[1][:3]):
        assert np.array_equal(a, b_)
