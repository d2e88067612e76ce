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


def stream_waves_velocity(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u0 = np.zeros((3,) + shape)
    u0[0] = 0.05 + 0.01 * np.sin(2 * np.pi * y / ny)
    u0[1] = 0.004 * np.sin(2 * np.pi * x / nx)
    u0[2] = 0.006 * np.cos(2 * np.pi * y / ny)
    return u0.astype(np.float32)


def reynolds(mu, muu):
    pa, pb = [0, 1, 2, 0, 0, 1], [0, 1, 2, 1, 2, 2]
    return np.stack([muu[c] - mu[pa[c]] * mu[pb[c]] for c in range(6)])


def test_long_window_statistics_match_oracle(capi):
    """20000 steps (10000 samples) of a periodic box holding a uniform stream
    with decaying shear waves on it, against the oracle's FP64 means over
    the same sampled pre-collision states (tests/golden/
    make_stats_reference.py).  The mean velocity agrees to 1e-5 relative.
    The Reynolds stress <u_a u_b> - <u_a><u_b> is the variance of the waves
    (1e-6 .. 1e-5, against <u_x u_x> = 2.5e-3): an FP32 run carries its own
    waves, which after 20000 steps differ from the FP64 run's by a relative
    e_w (measured here on the final fields), and a variance differs by about
    twice that; the bound is 3 e_w.  Summing in FP32 instead would add an
    error of order 1e-7 of <u_x u_x>, 2.5e-10, i.e. 5e-5 of the stress."""
    import os

    ref = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "stats_stream_waves_20000.npz"))
    shape = ref["mean_u"].shape[1:]
    d = capi.Domain(np.zeros(shape, np.uint8), periodic=7, storage="fp32")
    d.set_params(float(ref["tau"]))
    d.init_fields(None, stream_waves_velocity(shape))
    d.stats_enable(True)
    d.step(int(ref["steps"]))
    mu, muu, ms, n = d.stats()
    _, u_end = d.moments()
    d.destroy()
    assert n == int(ref["samples"])
    ou, ouu = ref["mean_u"], ref["mean_uu"]
    rg, ro = reynolds(mu, muu), reynolds(ou, ouu)
    e_u = float(np.linalg.norm(mu - ou) / np.linalg.norm(ou))
    e_r = float(np.linalg.norm(rg - ro) / np.linalg.norm(ro))
    e_s = float(np.linalg.norm(ms - ref["mean_sigma"]) / np.linalg.norm(ref["mean_sigma"]))
    wg = u_end.astype(np.float64) - u_end.astype(np.float64).mean(axis=(1, 2, 3), keepdims=True)
    wo = ref["u_end"] - ref["u_end"].mean(axis=(1, 2, 3), keepdims=True)
    e_w = float(np.linalg.norm(wg - wo) / np.linalg.norm(wo))
    say(f"long window: {n} samples, rel. err mean u {e_u:.2e}, Reynolds stress {e_r:.2e}, sigma {e_s:.2e}; "
        f"final waves differ by {e_w:.2e} (|R| {np.abs(ro).max():.2e}, <uu>_xx {np.abs(ouu[0]).max():.2e})")
    assert e_u <= 1e-5
    assert e_r <= 3.0 * e_w


def test_statistics_sums_keep_their_digits(capi):
    """A steady uniform stream (f^eq of a periodic box, which the collision
    keeps and streaming moves onto itself): over 10000 samples the mean
    velocity is the velocity (the stream itself drifts by a few FP32 ulps
    over the run, 2e-8 measured; bound 1e-7) and the Reynolds stress
    vanishes to the FP64 rounding of the sums (<= 1e-12 of U^2, measured
    4e-16 absolute); a sequential FP32 sum of 10000 samples rounds by up to
    an ulp of the running sum per add, which leaves about 1e-7 of U^2."""
    shape = (2, 8, 8)
    U = np.array([0.05, -0.02, 0.03], np.float32)
    u0 = np.broadcast_to(U[:, None, None, None], (3,) + shape).astype(np.float32)
    d = capi.Domain(np.zeros(shape, np.uint8), periodic=7, storage="fp32")
    d.set_params(0.6)
    d.init_fields(None, u0)
    d.step(2)
    _, u_now = d.moments()
    d.stats_enable(True)
    d.step(20000)
    mu, muu, _, n = d.stats()
    _, u_end = d.moments()
    d.destroy()
    assert n == 10000
    drift = float(np.abs(u_end.astype(np.float64) - u_now).max())
    R = reynolds(mu, muu)
    say(f"steady stream: velocity drift over the run {drift:.1e}, |<u> - u| {np.abs(mu - u_now).max():.1e}, "
        f"max |R| {np.abs(R).max():.1e}")
    assert np.abs(mu - u_now).max() <= 1e-7
    assert np.abs(R).max() <= 1e-12 * float(U @ U)
