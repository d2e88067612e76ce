"""Population arrays past 4 GiB.

Buffer instructions form their byte offsets in 32 bits, so arrays larger
than 4 GiB - 64 KiB step with kernels that take 64-bit global addresses.
Those kernels run the same arithmetic in the same order: on the random
configurations of every boundary option (test_gpu_random_configs) and on
each storage, equilibrium order and statistics, forcing them onto a small
domain gives the same bits as the 32-bit kernels.  Then genuine 4.8 GB
domains (FP32, and FP16S with twice the cells), periodic in z, whose flags
and initial fields repeat a small block K times along z: by translation
invariance every block of it must end bit for bit equal to the small block
stepped alone, which exercises slots, side rows and the periodic wrap
across the whole array.  Last, the
nozzle on the paper's finest grid (8.0 GB in FP32) against the oracle at
sampled cells."""
import numpy as np
import pytest

from paper_2204_10566_amd import inputs as I

from test_gpu_random_configs import build_domain, make_case

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def capi():
    from paper_2204_10566_amd import capi

    return capi


def run_case(capi, c, storage, wide, steps, feq=6, stats=False):
    d = build_domain(capi, c, storage)
    if feq != 6:
        d.set_equilibrium_order(feq)
    if wide:
        d.debug_wide_addressing(True)
    assert d.is_wide() == wide
    if stats:
        d.stats_enable(True)
    d.step(steps)
    out = [d.populations(), *d.moments()]
    if stats:
        out += list(d.stats()[:3])
    d.destroy()
    return out


@pytest.mark.parametrize("k", range(24))
def test_wide_kernels_give_the_same_bits(capi, k):
    c = make_case(300 + k)
    storage = ("fp32", "fp16s", "bf16s")[k % 3]
    feq = (6, 6, 3, 6, 2, 6)[k % 6]
    steps = 2 * c["steps"] + 1  # odd: ends in the local phase
    stats = k % 4 == 1
    say(f"case {k}: shape {c['fl'].shape} periodic {c['periodic']} {storage} order {feq} steps {steps} "
        f"outlet {c['outlet']} curved {c['q'] is not None} stats {stats}")
    narrow = run_case(capi, c, storage, False, steps, feq, stats)
    wide = run_case(capi, c, storage, True, steps, feq, stats)
    for a, b in zip(narrow, wide):
        assert np.array_equal(a, b)


def test_graphs_and_phase_switch(capi):
    """Switching to the wide kernels mid-run, with graph replays on both
    sides of the switch, continues the same trajectory."""
    c = make_case(11, "fp32")
    ref = run_case(capi, c, "fp32", False, 75)[0]
    d = build_domain(capi, c, "fp32")
    d.step(33)
    d.debug_wide_addressing(True)
    d.step(40)
    d.debug_wide_addressing(False)
    d.step(2)
    f = d.populations()
    d.destroy()
    assert np.array_equal(f, ref)


def block_fields(shape, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    rho = (1.0 + 0.02 * rng.uniform(-1, 1, shape)).astype(np.float32)
    u = (0.04 * rng.uniform(-1, 1, (3,) + shape)).astype(np.float32)
    return rho, u


def tiled_case(general, storage="fp32"):
    """A block repeated along a periodic z axis: y walls, an inlet plane, an
    outlet plane and a few solid cells per block; nx = 128 (row-aligned
    addressing) or 100 (general addressing); in FP16 twice as many blocks
    (the array holds half the bytes per cell)."""
    if general:
        nx, ny, nz0, K = 100, 40, 5, 2200
    else:
        nx, ny, nz0, K = 128, 48, 6, 1200
    if storage != "fp32":
        K *= 2
    fl = np.zeros((nz0, ny, nx), np.uint8)
    fl[:, 0, :] = I.SOLID
    fl[:, -1, :] = I.SOLID
    fl[:, 1:-1, 0] = I.INLET
    fl[:, 1:-1, -1] = I.OUTLET
    fl[1:3, 10:14, 30:33] = I.SOLID
    uin = np.zeros((3,) + fl.shape, np.float32)
    uin[0][fl == I.INLET] = 0.05
    return fl, uin, K


@pytest.mark.parametrize("general,outlet,storage", [(False, None, "fp32"), (True, ("pressure", 0.995), "fp32"),
                                                    (False, ("pressure", 1.002), "fp16s")])
def test_domain_past_4_gib(capi, general, outlet, storage):
    fl0, uin0, K = tiled_case(general, storage)
    nz0, ny, nx = fl0.shape
    rho0, u0 = block_fields(fl0.shape, 7)
    steps = 7
    say(f"block {fl0.shape} x {K} along z, outlet {outlet}, {storage}: small run")
    small = capi.Domain(fl0, periodic=4, storage=storage)
    small.set_params(0.56)
    if outlet:
        small.set_outlet(*outlet)
    small.set_inlet(uin0)
    small.init_fields(rho0, u0)
    small.step(steps)
    fs = small.populations()
    small.destroy()

    fl = np.tile(fl0, (K, 1, 1))
    nbytes = capi.lbm_array_bytes(nx, ny, nz0 * K, 0 if storage == "fp32" else 1)
    say(f"  big domain {fl.shape}: {fl.size} cells, {nbytes / 1e9:.2f} GB of populations")
    assert nbytes > 1 << 32
    big = capi.Domain(fl, periodic=4, storage=storage)
    assert big.is_wide()
    big.set_params(0.56)
    if outlet:
        big.set_outlet(*outlet)
    big.set_inlet(np.tile(uin0, (1, K, 1, 1)))
    big.init_fields(np.tile(rho0, (K, 1, 1)), np.tile(u0, (1, K, 1, 1)))
    b = capi.Batch(1 << 36, storage)
    with pytest.raises(capi.LbmError) as e:
        b.admit(big, 1)
    assert e.value.code == capi.ERR_ARG
    b.destroy()
    big.step(steps)
    say("  stepped; comparing every block")
    fb = big.populations().reshape(27, K, nz0, ny, nx)
    big.destroy()
    bad = [j for j in range(K) if not np.array_equal(fb[:, j], fs)]
    say(f"  blocks differing from the small run: {len(bad)} of {K}")
    assert not bad


def test_finest_grid_sampled(capi, orc):
    """The synthetic nozzle on the paper's finest grid (Table 2, R4: 155 x
    155 x 3093 = 74.3 M cells, Re 6500): an 8.0 GB FP32 array, stepped by the
    64-bit kernels with general addressing (nx = 3093).  After 3 steps from
    the plug-flow start, density and velocity at sampled cells (next to the
    inlet, on the outlet plane, next to a wall, anywhere, and at cells whose
    slots lie past 4 GiB into the array) against the oracle's
    dependency-cone run.  Bound: 27 populations of 3 steps at the per-step
    FP32 bound 4e-7 each, 3.3e-5."""
    n, length = 155, 3093
    nz = I.Nozzle(n=n, length=length, R=n / 4.0, r_throat=n / 12.0)
    tau, u_thr = I.nozzle_tau(nz, 6500.0)
    fl = nz.flags()
    uin = nz.inlet_velocity(u_thr).astype(np.float32)
    u0 = nz.initial_velocity(u_thr).astype(np.float32)
    say(f"finest grid {fl.shape}: {fl.size} cells, 3 steps")
    d = capi.Domain(fl, periodic=0, storage="fp32")
    assert d.is_wide()
    d.set_params(tau, 1.0 / tau, 1.0)
    d.set_inlet(uin)
    d.init_fields(None, u0)
    d.step(3)
    rg, ug = d.moments()
    d.destroy()
    upd = np.flatnonzero(((fl == I.FLUID) | (fl == I.OUTLET)).ravel())
    x = upd % length
    solid = fl.ravel() == I.SOLID
    near = upd[solid[np.clip(upd + length, 0, fl.size - 1)] | solid[np.clip(upd - length, 0, fl.size - 1)]]
    rng = np.random.default_rng(74)
    cells = np.unique(np.concatenate([rng.choice(upd[x == 1], 8, replace=False),
                                      rng.choice(upd[x == length - 1], 8, replace=False),
                                      rng.choice(near, 8, replace=False), rng.choice(upd, 8, replace=False),
                                      rng.choice(upd[upd * 27 * 4 > 1 << 32], 8, replace=False)]))
    st, fo = orc.run_cells(fl, cells, orc.rates_vector(1.0 / tau), 3, periodic=0, uin=uin, u0=u0)
    assert st == 0
    err = 0.0
    for k, c in enumerate(cells):
        ro, uo = orc.cell_moments(fo[:, k])
        err = max(err, abs(float(rg.ravel()[c]) - ro), float(np.abs(ug.reshape(3, -1)[:, c] - uo).max()))
    say(f"  {cells.size} cells: max abs err of rho and u {err:.3e}")
    assert err <= 27 * 3 * 4e-7
