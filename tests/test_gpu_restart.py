"""Checkpoint and restart, on random configurations of every boundary option
(curved walls, both outlets, inlet cells, per-order rates), stopped after an
even or an odd number of steps.

State images (lbm_save_state / lbm_load_state) carry the device state as it
is held, so the restarted run is the uninterrupted one bit for bit, in every
storage; saving leaves the running domain untouched.

Populations (lbm_get_populations / lbm_set_populations) carry only f_i; the
library rebuilds the rest, and a restart from them differs from the
uninterrupted run by rounding alone:
  - the pressure outlet's shift of the clamped values is formed from the
    moments of the stored post-collision state, where a step forms it from
    the pre-collision moments (equal up to rounding: the collision keeps
    rho and j);
  - after an odd number of steps, the export removes the inlet term that a
    bounce-back slot carries into the next step and the next step adds it
    again, (f + t) - t + t;
  - in shifted storage the import rounds (f - w) times the scale again
    after f was formed in FP32.
With the zero-gradient outlet, in FP32 and after an even number of steps,
none of these applies and the restart is exact."""
import numpy as np
import pytest

from paper_2204_10566_amd import inputs as I

from test_gpu_random_configs import TOL_PER_STEP, build_domain, make_case

pytestmark = pytest.mark.gpu

STORAGES = ("fp32", "fp16s", "bf16s")


def say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def capi():
    from paper_2204_10566_amd import capi

    return capi


def describe(k, c, storage, n1, n2):
    say(f"case {k}: shape {c['fl'].shape} periodic {c['periodic']} {storage} steps {n1} + {n2} "
        f"outlet {c['outlet']} curved {c['q'] is not None}")


def final(d):
    out = [d.populations(), *d.moments()]
    d.destroy()
    return out


@pytest.mark.parametrize("k", range(12))
def test_state_image_restart_is_bitwise(capi, k):
    c = make_case(700 + k)  # pressure outlets in all three storages, curved walls in FP32 and BF16S
    storage = STORAGES[k % 3]
    n1, n2 = 2 * c["steps"] + (k % 2), 3 + k
    describe(k, c, storage, n1, n2)
    d = build_domain(capi, c, storage)
    d.step(n1 + n2)
    ref = final(d)

    d = build_domain(capi, c, storage)
    d.step(n1)
    image = d.save_state()
    d.step(n2)  # the saved domain runs on as if nothing happened
    cont = final(d)
    r = build_domain(capi, c, storage)
    r.load_state(image)
    r.step(n2)
    got = final(r)
    for a, b, g in zip(ref, cont, got):
        assert np.array_equal(a, b)
        assert np.array_equal(a, g)


@pytest.mark.parametrize("k", range(12))
def test_population_restart_within_rounding(capi, k):
    c = make_case(700 + k)
    storage = "fp32" if k < 8 else "fp16s"
    n1, n2 = 2 * c["steps"] + (k % 2), 3 + k
    describe(k, c, storage, n1, n2)
    d = build_domain(capi, c, storage)
    d.step(n1 + n2)
    ref = d.populations()
    d.destroy()

    d = build_domain(capi, c, storage)
    d.step(n1)
    checkpoint = d.populations()
    d.destroy()
    r = build_domain(capi, c, storage)
    r.set_populations(checkpoint)
    r.step(n2)
    got = r.populations()
    r.destroy()
    upd = (c["fl"] == I.FLUID) | (c["fl"] == I.OUTLET)
    err = float(np.abs(got[:, upd] - ref[:, upd]).max()) if upd.any() else 0.0
    say(f"  max abs difference {err:.3e}")
    exact = storage == "fp32" and n1 % 2 == 0 and (c["outlet"] is None or c["outlet"][0] != "pressure")
    if exact:
        assert np.array_equal(got, ref)
    assert err <= TOL_PER_STEP[storage] * n2


def test_state_image_rejections(capi):
    c = make_case(703)  # curved walls, no outlet
    d = build_domain(capi, c, "fp32")
    d.step(3)
    image = d.save_state()
    d.destroy()

    def code(fn):
        with pytest.raises(capi.LbmError) as e:
            fn()
        return e.value.code

    # another storage: another array size in the header
    other = build_domain(capi, c, "fp16s")
    assert code(lambda: other.load_state(image)) == capi.ERR_ARG
    other.destroy()
    # the same grid with one cell's flag changed
    c2 = dict(c)
    fl = c["fl"].copy()
    z, y, x = np.argwhere(fl == I.FLUID)[0]
    fl[z, y, x] = I.SOLID
    c2["fl"] = fl
    other = build_domain(capi, c2, "fp32")
    assert code(lambda: other.load_state(image)) == capi.ERR_STATE
    other.destroy()
    # curved walls on one side only
    c3 = dict(c, q=None)
    other = build_domain(capi, c3, "fp32")
    assert code(lambda: other.load_state(image)) == capi.ERR_STATE
    other.destroy()
    # truncated, or not an image
    same = build_domain(capi, c, "fp32")
    before = same.populations()
    assert code(lambda: same.load_state(image[:-4])) == capi.ERR_ARG
    bad = image.copy()
    bad[0] ^= 1
    assert code(lambda: same.load_state(bad)) == capi.ERR_ARG
    assert np.array_equal(same.populations(), before)
    same.load_state(image)
    same.destroy()


def fnv1a64(data: bytes) -> int:
    h = 0xCBF29CE484222325
    for b in data:
        h = ((h ^ b) * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def test_state_image_layout(capi):
    """The image's header holds what the header file documents: the tag, the
    grid, periodicity and storage, the array and kept-value sizes, the FNV-1a
    hash of the flags, the phase and instability flag; the array follows."""
    c = make_case(701)  # curved walls, pressure outlet
    for storage in ("fp32", "fp16s"):
        d = build_domain(capi, c, storage)
        d.step(5)  # odd: the image keeps phase 1
        img = d.save_state()
        nz, ny, nx = c["fl"].shape
        h = np.frombuffer(img[:64].tobytes(), "<u8")
        st = capi.STORAGE[storage]
        assert h[0] == int.from_bytes(b"LBMSTAT1", "little")
        assert h[1] == nx | ny << 16 | nz << 32 | c["periodic"] << 48 | st << 56
        assert h[2] == capi.lbm_array_bytes(nx, ny, nz, st)
        assert h[3] == d.info().n_wall_tiles * 27 * 64 * 4
        assert h[4] == fnv1a64(np.ascontiguousarray(c["fl"]).tobytes())
        assert h[5] == 1 and h[6] == 0 and h[7] == 0
        assert img.nbytes == 64 + int(h[2]) + int(h[3])
        d.destroy()


def test_state_image_between_addressing_modes(capi):
    """An image taken with the 64-bit addressing kernels restarts under the
    32-bit ones (and back) bit for bit: the image is the array as stored,
    whichever kernels stepped it."""
    c = make_case(706)
    for storage in ("fp32", "bf16s"):
        d = build_domain(capi, c, storage)
        d.step(9)
        ref_img = d.save_state()
        d.step(6)
        ref = d.populations()
        d.destroy()
        for wide_first in (True, False):
            d = build_domain(capi, c, storage)
            d.debug_wide_addressing(wide_first)
            d.step(9)
            img = d.save_state()
            assert np.array_equal(img, ref_img)
            d.destroy()
            r = build_domain(capi, c, storage)
            r.debug_wide_addressing(not wide_first)
            r.load_state(img)
            r.step(6)
            assert np.array_equal(r.populations(), ref)
            r.destroy()
