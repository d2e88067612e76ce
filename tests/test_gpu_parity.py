"""GPU parity: the HIP library against the FP64 oracle, through the C ABI.

Tolerances (FP32 storage and arithmetic against FP64):
  - Taylor-Green 32^3, u0 = 0.05, tau = 0.6, 100 steps: velocity relative L2
    <= 1e-5 (the stated target);
  - one step from random populations: max |f_gpu - f_oracle| <= 4e-7, about
    ten FP32 ulps of the largest population (8/27), which bounds the rounding
    of the ~600 FP32 operations of one update;
  - nozzle geometries: velocity error relative to the peak velocity;
  - FP16 shifted storage: velocity relative L2 <= 1e-3; from random
    populations, max abs <= 5e-5 per step (each store rounds 2^14 (f - w)
    to 11 significant bits, at most 2^-11 |f - w|, and these states keep
    |f - w| near 0.01).
"""
import os
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


def rel_l2(a, b, mask=None):
    if mask is not None:
        a = a[..., mask]
        b = b[..., mask]
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def updated(fl):
    return (fl == I.FLUID) | (fl == I.OUTLET)


def run_gpu(capi, fl, periodic, steps, tau=None, rates=None, u0=None, rho0=None, uin=None, storage="fp32",
            pops=None):
    d = capi.Domain(fl, periodic=periodic, storage=storage)
    if rates is not None:
        d.set_rates(*rates)
    else:
        d.set_params(tau, 1.0 / tau, 1.0)
    if uin is not None:
        d.set_inlet(uin)
    d.init_fields(rho0, u0)
    if pops is not None:
        d.set_populations(pops)
    if steps:
        d.step(steps)
    return d


def test_init_equilibrium_matches_oracle(capi, orc):
    """GPU product-form equilibrium == oracle Hermite-sum equilibrium."""
    say("init equilibrium 12x10x8")
    fl = np.zeros((8, 10, 12), np.uint8)
    rng = np.random.default_rng(11)
    rho = 1 + 0.05 * rng.uniform(-1, 1, fl.shape)
    u = 0.15 * rng.uniform(-1, 1, (3,) + fl.shape)
    d = run_gpu(capi, fl, 7, 0, tau=0.6, u0=u, rho0=rho)
    fg = d.populations()
    fo = orc.init_fields(fl, rho.astype(np.float32), u.astype(np.float32))
    assert np.abs(fg - fo).max() < 1e-7


@pytest.mark.parametrize("storage", ["fp32"])
def test_tgv32_100_steps(capi, orc, storage):
    """32^3 periodic Taylor-Green vortex, u0 = 0.05, rho = 1, tau = 0.6,
    paper's rates (omega_bulk = 1/tau, omega_high = 1), 100 steps."""
    n, tau = 32, 0.6
    fl = I.periodic_box(n)
    u0 = I.taylor_green_velocity(n, n, n, 0.05)
    say(f"tgv32 {storage} 100 steps")
    d = run_gpu(capi, fl, 7, 100, tau=tau, u0=u0, storage=storage)
    rg, ug = d.moments()
    f = orc.init_fields(fl, None, u0.astype(np.float32))
    st, f = orc.step(fl, f, orc.rates_vector(1 / tau), 100, periodic=7)
    assert st == 0
    ro, uo = orc.moments(fl, f)
    e_u = rel_l2(ug, uo)
    e_p = float(np.linalg.norm(rg - ro) / np.linalg.norm(ro - ro.mean()))
    say(f"tgv32 {storage}: e_u={e_u:.3e} e_p={e_p:.3e}")
    assert e_u <= 1e-5
    # global mass and momentum drift of the FP32 state
    assert abs(rg.sum() / ro.sum() - 1) < 1e-6
    assert np.abs((rg * ug).sum(axis=(1, 2, 3))).max() < 1e-3 * 1e-3 * rg.size


def random_pops(orc, fl, seed):
    # FP32-representable, so both sides start from identical values
    return I.random_populations(fl.shape, seed).astype(np.float32).astype(np.float64)


def mixed_geometry():
    """x: inlet plane, fluid, outlet plane; y: walls; z periodic; a solid
    obstacle and a ragged cell count (not a multiple of 64)."""
    nz, ny, nx = 5, 9, 23
    fl = np.zeros((nz, ny, nx), np.uint8)
    fl[:, 0, :] = I.SOLID
    fl[:, -1, :] = I.SOLID
    fl[:, 1:-1, 0] = I.INLET
    fl[:, 1:-1, -1] = I.OUTLET
    fl[2, 3:5, 8:11] = I.SOLID
    return fl


@pytest.mark.parametrize("rates", [(1 / 0.6, 1 / 0.6, 1.0), (1 / 0.51, 0.7, 1.3), (1.9, 1.2, 0.4)])
def test_one_step_random_populations(capi, orc, rates):
    """Populations after one and after five steps from random states on a
    geometry with every boundary kind, with general rates."""
    fl = mixed_geometry()
    rng = np.random.default_rng(3)
    uin = np.zeros((3,) + fl.shape)
    uin[:, fl == I.INLET] = 0.02 * rng.uniform(-1, 1, (3, int((fl == I.INLET).sum())))
    uin = uin.astype(np.float32)
    f0 = random_pops(orc, fl, 5)
    upd = updated(fl)
    for steps in (1, 5):
        say(f"random pops rates={rates} steps={steps}")
        d = run_gpu(capi, fl, 4, steps, rates=rates, uin=uin, pops=f0)
        fg = d.populations()
        st, fo = orc.step(fl, f0, orc.rates_vector(rates[0], rates[1], rates[2]), steps, periodic=4, uin=uin)
        assert st == 0
        err = np.abs(fg[:, upd] - fo[:, upd]).max()
        say(f"  max abs err {err:.3e}")
        assert err <= 4e-7 * steps


def test_small_nozzle_run(capi, orc):
    """A scaled-down nozzle (inlet, cone, throat, sudden expansion, outlet)
    run 200 steps from the plug-flow start; velocity error relative to the
    peak velocity."""
    cfg = I.small_nozzle(n=24, length=160, R=8.0, r_throat=3.0, Re=100.0)
    fl, tau = cfg["flags"], cfg["tau"]
    say(f"small nozzle 24x24x160 tau={tau:.5f} 200 steps")
    d = run_gpu(capi, fl, 0, 200, tau=tau, u0=cfg["u0"].astype(np.float32), uin=cfg["uin"].astype(np.float32))
    rg, ug = d.moments()
    f = orc.init_fields(fl, None, cfg["u0"].astype(np.float32))
    st, f = orc.step(fl, f, orc.rates_vector(1 / tau), 200, periodic=0, uin=cfg["uin"].astype(np.float32))
    assert st == 0
    ro, uo = orc.moments(fl, f)
    upd = updated(fl)
    e_u = rel_l2(ug, uo, upd)
    e_max = float(np.abs(ug - uo)[:, upd].max() / np.abs(uo[:, upd]).max())
    say(f"small nozzle: e_u={e_u:.3e} max/peak={e_max:.3e}")
    assert e_u <= 1e-4 and e_max <= 1e-4


@pytest.mark.parametrize("which,storage", [("re500", "fp32"), ("re500", "fp16s"), ("re6500", "fp32"),
                                           ("re6500", "fp16s")])
def test_full_size_nozzle_sampled(capi, orc, which, storage):
    """Full-size nozzles (96x96x768 at Re 500, 128x128x1536 at Re 6500 with
    inlet noise), 3 steps in the benchmark's launch configuration;
    populations compared at sampled cells (inlet-adjacent, outlet,
    wall-adjacent, throat, random) against the oracle's dependency-cone run
    from the same initial fields.  FP16-shifted storage rounds each stored
    value to 2^-11 of 2^14 (f - w), a few 1e-6 on these states (measured
    2.4e-6 after 3 steps); the bound is 2e-5."""
    cfg = I.nozzle_config(which)
    fl, tau = cfg["flags"], cfg["tau"]
    u0 = cfg["u0"].astype(np.float32)
    uin = cfg["uin"].astype(np.float32)
    say(f"nozzle {which} {fl.shape} {storage} 3 steps")
    d = run_gpu(capi, fl, 0, 3, tau=tau, u0=u0, uin=uin, storage=storage)
    fg = d.populations().reshape(27, -1)
    upd = np.flatnonzero(updated(fl).ravel())
    nz_, ny_, nx_ = fl.shape
    xs = upd % nx_
    rng = np.random.default_rng(0)
    picks = [upd[xs == 1][:40], upd[xs == nx_ - 1][:40], rng.choice(upd, 120, replace=False)]
    # cells next to a wall
    solid = fl.ravel() == I.SOLID
    near = upd[solid[np.clip(upd + nx_, 0, fl.size - 1)] | solid[np.clip(upd - nx_, 0, fl.size - 1)]]
    picks.append(rng.choice(near, 60, replace=False))
    cells = np.unique(np.concatenate(picks))
    st, fo = orc.run_cells(fl, cells, orc.rates_vector(1 / tau), 3, periodic=0, uin=uin, u0=u0)
    assert st == 0
    err = np.abs(fg[:, cells] - fo).max()
    say(f"nozzle {which} {storage}: {cells.size} cells, max abs err {err:.3e}")
    assert err <= (1e-6 if storage == "fp32" else 2e-5)
    d.destroy()


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_full_size_nozzle_sampled_12_steps(capi, orc, storage):
    """The benchmark nozzle (96x96x768, Re 500) 12 steps deep, replayed from
    the step graphs of 8 and 4 steps as a timed run replays them, at 40
    sampled cells (inlet-adjacent, outlet, wall-adjacent, random) against
    the oracle's dependency-cone run.  Bounds four times those of 3 steps
    (the per-step rounding adds up): FP32 4e-6, FP16S 8e-5 max abs.  The
    200-step full-size comparison with FP64 is in test_gpu_precision."""
    cfg = I.nozzle_config("re500")
    fl, tau = cfg["flags"], cfg["tau"]
    u0 = cfg["u0"].astype(np.float32)
    uin = cfg["uin"].astype(np.float32)
    steps = 12
    say(f"nozzle re500 {fl.shape} {storage} {steps} steps")
    d = run_gpu(capi, fl, 0, steps, tau=tau, u0=u0, uin=uin, storage=storage)
    fg = d.populations().reshape(27, -1)
    d.destroy()
    upd = np.flatnonzero(updated(fl).ravel())
    nx_ = fl.shape[2]
    xs = upd % nx_
    rng = np.random.default_rng(12)
    solid = fl.ravel() == I.SOLID
    near = upd[solid[np.clip(upd + nx_, 0, fl.size - 1)] | solid[np.clip(upd - nx_, 0, fl.size - 1)]]
    picks = [rng.choice(upd[xs == 1], 10, replace=False), rng.choice(upd[xs == nx_ - 1], 10, replace=False),
             rng.choice(upd, 10, replace=False), rng.choice(near, 10, replace=False)]
    cells = np.unique(np.concatenate(picks))
    st, fo = orc.run_cells(fl, cells, orc.rates_vector(1 / tau), steps, periodic=0, uin=uin, u0=u0)
    assert st == 0
    err = np.abs(fg[:, cells] - fo).max()
    say(f"nozzle re500 {storage} {steps} steps: {cells.size} cells, max abs err {err:.3e}")
    assert err <= (4e-6 if storage == "fp32" else 8e-5)


NOZZLE_REF = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "nozzle_re500_200_sampled.npz")


@pytest.mark.parametrize("storage", ["fp32", "fp16s", "bf16s"])
def test_bench_nozzle_200_steps_against_oracle(capi, storage):
    """The benchmark nozzle (96x96x768, Re 500) over its first 200 steps
    from the plug-flow start, stepped as the benchmark steps it (graph
    replays), against the oracle's full FP64 run of the same window
    (tests/golden/make_nozzle_reference.py): the 27 populations at 2048
    sampled cells (next to the inlet, on the outlet plane, next to a wall,
    in the throat and the expansion, anywhere) and the velocity at 16384.
    The population bound is the per-step bound of the random configurations
    times the steps (FP32 4e-7, FP16S 5e-5, BF16S 2e-4 per step); the
    velocity error e_u (relative L2) is held to the bounds of the precision
    comparison (FP32 1e-4, FP16S 1e-3, BF16S 1e-2)."""
    ref = np.load(NOZZLE_REF)
    steps = int(ref["steps"])
    cfg = I.nozzle_config("re500")
    fl, tau = cfg["flags"], cfg["tau"]
    assert abs(tau - float(ref["tau"])) < 1e-15
    say(f"nozzle re500 {fl.shape} {storage} {steps} steps against the FP64 oracle")
    d = run_gpu(capi, fl, 0, steps, tau=tau, u0=cfg["u0"].astype(np.float32), uin=cfg["uin"].astype(np.float32),
                storage=storage)
    fg = d.populations().reshape(27, -1)
    _, ug = d.moments()
    d.destroy()
    err = float(np.abs(fg[:, ref["pop_cells"]] - ref["f"]).max())
    uo = ref["u"]
    e_u = float(np.linalg.norm(ug.reshape(3, -1)[:, ref["moment_cells"]] - uo) / np.linalg.norm(uo))
    per_step = {"fp32": 4e-7, "fp16s": 5e-5, "bf16s": 2e-4}[storage]
    say(f"  populations at {ref['pop_cells'].size} cells: max abs err {err:.3e} (bound {per_step * steps:.1e}); "
        f"e_u {e_u:.3e} at {ref['moment_cells'].size} cells")
    assert err <= per_step * steps
    assert e_u <= {"fp32": 1e-4, "fp16s": 1e-3, "bf16s": 1e-2}[storage]


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_tgv320_probe_sampled(capi, orc, storage):
    """The benchmark's bandwidth probe: the periodic Taylor-Green vortex on
    320^3 cells (3.5 GB of FP32 populations, the largest array of the tests,
    with byte offsets up to 3.5e9 of the 4 GiB the buffer instructions
    address), 3 steps in the benchmark's launch configuration.  Sampled
    cells (the last tiles of the array, the periodic faces, random) against
    the oracle's dependency-cone run, and the total mass of all cells
    against its initial value (conserved by the update up to rounding)."""
    n, tau = 320, 0.6
    fl = I.periodic_box(n)
    u0 = I.taylor_green_velocity(n, n, n, 0.05).astype(np.float32)
    say(f"tgv {n}^3 {storage} 3 steps")
    d = run_gpu(capi, fl, 7, 0, tau=tau, u0=u0, storage=storage)
    rho, _ = d.moments()
    m0 = float(rho.astype(np.float64).sum())
    d.step(3)
    rho, _ = d.moments()
    m1 = float(rho.astype(np.float64).sum())
    fg = d.populations().reshape(27, -1)
    d.destroy()
    ncells = fl.size
    rng = np.random.default_rng(3)
    cells = np.unique(np.concatenate([
        np.arange(ncells - 130, ncells),  # the last two tiles and a bit
        np.arange(0, 70),  # the first tile, periodic neighbour of the last
        rng.integers(0, n, 40) * n * n + rng.integers(0, n, 40) * n,  # x = 0
        rng.integers(0, n, 40) * n * n + rng.integers(0, n, 40) * n + (n - 1),  # x = n - 1
        rng.choice(ncells, 100, replace=False),
    ]))
    st, fo = orc.run_cells(fl, cells, orc.rates_vector(1 / tau), 3, periodic=7, u0=u0)
    assert st == 0
    err = float(np.abs(fg[:, cells] - fo).max())
    drift = abs(m1 - m0) / m0
    say(f"tgv {n}^3 {storage}: {cells.size} cells, max abs err {err:.3e}, mass drift {drift:.2e}")
    assert err <= (1e-6 if storage == "fp32" else 2e-5)
    assert drift <= 1e-6


def test_fp16_shifted_tgv32(capi, orc):
    n, tau = 32, 0.6
    fl = I.periodic_box(n)
    u0 = I.taylor_green_velocity(n, n, n, 0.05)
    say("tgv32 fp16s / bf16s 100 steps")
    f = orc.init_fields(fl, None, u0.astype(np.float32))
    st, f = orc.step(fl, f, orc.rates_vector(1 / tau), 100, periodic=7)
    ro, uo = orc.moments(fl, f)
    res = {}
    for storage in ("fp16s", "bf16s"):
        d = run_gpu(capi, fl, 7, 100, tau=tau, u0=u0, storage=storage)
        rg, ug = d.moments()
        res[storage] = (rel_l2(ug, uo), float(np.linalg.norm(rg - ro) / np.linalg.norm(ro - ro.mean())))
        say(f"tgv32 {storage}: e_u={res[storage][0]:.3e} e_p={res[storage][1]:.3e}")
    assert res["fp16s"][0] <= 1e-3
    assert res["bf16s"][0] <= 2e-2


def test_empty_and_degenerate_domains(capi, orc):
    """All-solid domain (no tiles), one-cell-thick periodic slab, a 1x1x1
    periodic cell, and a ragged 7x5x3 box."""
    say("degenerate domains")
    d = capi.Domain(np.ones((3, 4, 5), np.uint8), periodic=0)
    d.set_params(0.7)
    d.step(10)
    assert d.info().n_tiles == 0
    for shape in [(1, 6, 10), (1, 1, 1), (3, 5, 7)]:
        fl = np.zeros(shape, np.uint8)
        f0 = random_pops(orc, fl, 9)
        dd = run_gpu(capi, fl, 7, 4, rates=(1 / 0.55, 1.1, 1.0), pops=f0)
        st, fo = orc.step(fl, f0, orc.rates_vector(1 / 0.55, 1.1, 1.0), 4, periodic=7)
        assert np.abs(dd.populations() - fo).max() <= 2e-6


def test_unstable_run_reports_error(capi):
    """A state with negative density is reported as LBM_ERR_UNSTABLE and the
    error stays until the fields are re-initialised."""
    say("unstable detection")
    fl = np.zeros((4, 4, 4), np.uint8)
    d = capi.Domain(fl, periodic=7)
    d.set_params(0.6)
    f = -np.ones((27,) + fl.shape, np.float32) * 0.01
    d.set_populations(f)
    assert d.step_status(1) == capi.ERR_UNSTABLE
    assert d.step_status(1) == capi.ERR_UNSTABLE
    d.init_fields()
    assert d.step_status(3) == capi.OK


def test_async_steps_equal_synchronous_steps(capi):
    """lbm_step_async followed by lbm_step_wait gives the same bits as
    lbm_step, across graph replays and odd counts, and the wait reports an
    unstable step as lbm_step does."""
    say("async steps")
    fl = I.periodic_box(12)
    u0 = I.taylor_green_velocity(12, 12, 12, 0.04).astype(np.float32)
    out = []
    for use_async in (False, True):
        d = capi.Domain(fl, periodic=7)
        d.set_params(0.57)
        d.init_fields(None, u0)
        for n in (1, 70, 3, 0, 129):
            if use_async:
                d.step_async(n)
                assert d.wait_status() == capi.OK
            else:
                d.step(n)
        out.append(d.populations())
        d.destroy()
    assert np.array_equal(out[0], out[1])
    d = capi.Domain(fl, periodic=7)
    d.set_params(0.6)
    d.set_populations(-np.ones((27,) + fl.shape, np.float32) * 0.01)
    d.step_async(2)
    assert d.wait_status() == capi.ERR_UNSTABLE
    assert d.step_status(1) == capi.ERR_UNSTABLE
    d.destroy()


def test_adopted_torch_array_and_stream(capi, orc):
    """The population array and the stream come from torch."""
    import torch

    n = 16
    fl = I.periodic_box(n)
    u0 = I.taylor_green_velocity(n, n, n, 0.03).astype(np.float32)
    nbytes = int(capi.lbm_array_bytes(n, n, n, capi.FP32))
    assert nbytes >= 27 * 4 * fl.size and nbytes % 256 == 0
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    say("torch-adopted array 16^3")
    d = capi.Domain(fl, periodic=7, storage="fp32", stream=s.cuda_stream, array=a.data_ptr())
    d.set_params(0.7)
    d.init_fields(None, u0)
    d.step(20)
    rho = torch.empty(fl.size, dtype=torch.float32, device="cuda")
    u = torch.empty(3 * fl.size, dtype=torch.float32, device="cuda")
    d.moments_device(rho.data_ptr(), u.data_ptr())
    ug = u.cpu().numpy().reshape((3,) + fl.shape)
    f = orc.init_fields(fl, None, u0)
    st, f = orc.step(fl, f, orc.rates_vector(1 / 0.7), 20, periodic=7)
    _, uo = orc.moments(fl, f)
    assert rel_l2(ug, uo) <= 1e-5
    d.destroy()


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_state_access_between_odd_and_even_steps(capi, orc, storage):
    """The library runs steps in place, alternating two phases.  Reading the
    state after an odd number of steps, changing the inlet velocity there
    and stepping on must equal the pull update of the oracle: 3 steps,
    export, 1 step, new inlet velocity, 3 steps, export."""
    fl = mixed_geometry()
    rng = np.random.default_rng(21)
    n_in = int((fl == I.INLET).sum())
    uin1 = np.zeros((3,) + fl.shape, np.float32)
    uin1[:, fl == I.INLET] = 0.03 * rng.uniform(-1, 1, (3, n_in))
    uin2 = np.zeros((3,) + fl.shape, np.float32)
    uin2[:, fl == I.INLET] = 0.03 * rng.uniform(-1, 1, (3, n_in))
    f0 = random_pops(orc, fl, 13)
    rates = (1 / 0.57, 1.1, 1.2)
    rv = orc.rates_vector(*rates)
    upd = updated(fl)
    tol = 4e-7 if storage == "fp32" else 5e-5  # per step; FP16S: 2^-11 |f - w| per store
    say(f"odd/even state access {storage}")
    d = capi.Domain(fl, periodic=4, storage=storage)
    d.set_rates(*rates)
    d.set_inlet(uin1)
    d.set_populations(f0)
    f0 = d.populations().astype(np.float64)  # the stored (rounded) start
    d.step(3)
    st, fo = orc.step(fl, f0, rv, 3, periodic=4, uin=uin1)
    assert st == 0
    assert np.abs(d.populations()[:, upd] - fo[:, upd]).max() <= 3 * tol
    d.step(1)
    d.set_inlet(uin2)
    d.step(3)
    st, fo = orc.step(fl, fo, rv, 1, periodic=4, uin=uin1)
    st, fo = orc.step(fl, fo, rv, 3, periodic=4, uin=uin2)
    err = np.abs(d.populations()[:, upd] - fo[:, upd]).max()
    say(f"  max abs err {err:.3e}")
    assert err <= 7 * tol
    rg, ug = d.moments()
    ro, uo = orc.moments(fl, fo)
    assert np.abs(ug - uo)[:, upd].max() <= 7 * tol * 30


def row_aligned_channel():
    """nx = 128 (rows of whole 64-cell tiles; y and z neighbours keep the lane
    alignment): inlet plane, outlet plane, walls in y, z periodic, two
    obstacles."""
    nz, ny, nx = 6, 10, 128
    fl = np.zeros((nz, ny, nx), np.uint8)
    fl[:, 0, :] = I.SOLID
    fl[:, -1, :] = I.SOLID
    fl[:, 1:-1, 0] = I.INLET
    fl[:, 1:-1, -1] = I.OUTLET
    fl[1:4, 3:6, 40:44] = I.SOLID
    fl[:, 6, 90:93] = I.SOLID
    return fl


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_row_aligned_domain(capi, orc, storage):
    """Random populations on a row-aligned channel: 1 and 6 steps against the
    oracle."""
    fl = row_aligned_channel()
    rng = np.random.default_rng(31)
    n_in = int((fl == I.INLET).sum())
    uin = np.zeros((3,) + fl.shape, np.float32)
    uin[:, fl == I.INLET] = 0.03 * rng.uniform(-1, 1, (3, n_in))
    f0 = random_pops(orc, fl, 17)
    rates = (1 / 0.56, 1.3, 1.0)
    upd = updated(fl)
    tol = 4e-7 if storage == "fp32" else 5e-5  # per step; FP16S: 2^-11 |f - w| per store
    for steps in (1, 6):
        say(f"row-aligned channel {storage} steps={steps}")
        d = capi.Domain(fl, periodic=4, storage=storage)
        d.set_rates(*rates)
        d.set_inlet(uin)
        d.set_populations(f0)
        fs = d.populations().astype(np.float64)
        d.step(steps)
        st, fo = orc.step(fl, fs, orc.rates_vector(*rates), steps, periodic=4, uin=uin)
        assert st == 0
        err = np.abs(d.populations()[:, upd] - fo[:, upd]).max()
        say(f"  max abs err {err:.3e}")
        assert err <= tol * steps
        d.destroy()


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
@pytest.mark.parametrize("periodic", [7, 5])
def test_row_aligned_periodic_x(capi, orc, storage, periodic):
    """nx = 128 with x periodic: the first and last tile of each row take
    their boundary elements across the wrap.  Solid blocks (one touching
    x = 0 and x = nx - 1) make wall tiles at the wrap; with y closed the
    rows at y = 0 and y = ny - 1 bounce back every y link."""
    nz, ny, nx = 5, 7, 128
    fl = np.zeros((nz, ny, nx), np.uint8)
    fl[1:3, 2:4, 0:2] = I.SOLID
    fl[2:4, 4:6, nx - 2:] = I.SOLID
    fl[0, 3, 60:66] = I.SOLID
    f0 = random_pops(orc, fl, 61)
    rates = (1 / 0.59, 1.2, 1.0)
    upd = updated(fl)
    tol = 4e-7 if storage == "fp32" else 5e-5  # per step; FP16S: 2^-11 |f - w| per store
    for steps in (1, 4):
        say(f"row-aligned periodic x {storage} periodic={periodic} steps={steps}")
        d = capi.Domain(fl, periodic=periodic, storage=storage)
        d.set_rates(*rates)
        d.set_populations(f0)
        fs = d.populations().astype(np.float64)
        d.step(steps)
        st, fo = orc.step(fl, fs, orc.rates_vector(*rates), steps, periodic=periodic)
        assert st == 0
        err = np.abs(d.populations()[:, upd] - fo[:, upd]).max()
        say(f"  max abs err {err:.3e}")
        assert err <= tol * steps
        d.destroy()


@pytest.mark.parametrize("order_rates", [(1.3, 0.8, 1.6, 0.5), (1.0, 1.0, 1.0, 1.2)])
def test_per_order_rates(capi, orc, order_rates):
    """A separate rate for each order 3..6 of the higher central moments:
    one and four steps from random populations on the geometry with every
    boundary kind."""
    fl = mixed_geometry()
    rng = np.random.default_rng(41)
    uin = np.zeros((3,) + fl.shape, np.float32)
    uin[:, fl == I.INLET] = 0.02 * rng.uniform(-1, 1, (3, int((fl == I.INLET).sum())))
    f0 = random_pops(orc, fl, 43)
    upd = updated(fl)
    for steps in (1, 4):
        say(f"order rates {order_rates} steps={steps}")
        d = capi.Domain(fl, periodic=4)
        d.set_rates(1 / 0.58, 1.1, 1.0)
        d.set_order_rates(*order_rates)
        d.set_inlet(uin)
        d.set_populations(f0)
        d.step(steps)
        st, fo = orc.step(fl, f0, orc.rates_vector(1 / 0.58, 1.1, order_rates=order_rates), steps, periodic=4, uin=uin)
        assert st == 0
        err = np.abs(d.populations()[:, upd] - fo[:, upd]).max()
        say(f"  max abs err {err:.3e}")
        assert err <= 4e-7 * steps
        d.destroy()
