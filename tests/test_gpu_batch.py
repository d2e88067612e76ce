"""Packed multi-domain execution and the serving loop on the GPU.

Each domain advanced inside a packed launch must end in exactly the state it
reaches when advanced alone (same per-cell arithmetic, same kernels), so the
comparisons here are bitwise.  The graph-replay test checks that replaying a
captured graph several times, with eager work in between, gives the same
state as eager launches."""
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


def build(capi, spec, storage):
    d = capi.Domain(spec.flags, periodic=spec.periodic, storage=storage)
    d.set_params(spec.tau, 1.0 / spec.tau, 1.0)
    d.init_fields(None, spec.u.astype(np.float32))
    return d


def small_specs(count, seed, lo=10, hi=26):
    specs = I.batched_domains(count=count, seed=seed, lo=lo, hi=hi, materialise=True)
    rng = np.random.default_rng(seed)
    for s in specs:
        s.steps = int(rng.integers(5, 40))
    return specs


# cache blocks (group bytes, window steps): the default, one group per
# class, and groups of a few small domains with short and odd windows
CACHE_BLOCKS = [None, (0, 8), (200_000, 5), (1, 3), (600_000, 1)]


@pytest.mark.parametrize("storage", ["fp16s", "fp32"])
@pytest.mark.parametrize("cache", CACHE_BLOCKS)
def test_alone_equals_mix_staggered(capi, storage, cache):
    """Domains admitted at even and odd steps (both parity classes), with
    different step counts so that some finish inside a window, each end bit
    for bit where they end alone, whatever the cache blocking."""
    specs = small_specs(6, 1)
    say(f"alone vs mix {storage} cache {cache}: " + ", ".join(f"{s.kind}{s.nx}x{s.ny}x{s.nz}/{s.steps}" for s in specs))
    alone = []
    for s in specs:
        d = build(capi, s, storage)
        d.step(s.steps)
        alone.append(d.populations())
        d.destroy()
    doms = [build(capi, s, storage) for s in specs]
    b = capi.Batch(1 << 34, storage)
    if cache:
        b.set_cache_block(*cache)
    slots = {}
    order = [[0, 1, 2], [3], [4, 5]]
    pending = set()
    for group in order:
        for k in group:
            slots[k] = b.admit(doms[k], specs[k].steps)
            pending.add(slots[k])
        b.step(3)
    while pending:
        b.step(4)
        for s in b.poll():
            pending.discard(s)
    for k, s in slots.items():
        b.release(s)
        got = doms[k].populations()
        assert np.array_equal(got, alone[k]), f"domain {k} differs"
        doms[k].destroy()
    b.destroy()


def test_budget_limits_admission(capi):
    spec = I.DomainSpec(kind="tgv", nx=20, ny=20, nz=20, tau=0.6, steps=5).materialise()
    doms = [build(capi, spec, "fp16s") for _ in range(3)]
    size = int(doms[0].info().device_bytes)
    say(f"budget admission, {size} bytes per domain")
    b = capi.Batch(2 * size, "fp16s")
    s0 = b.admit(doms[0], 5)
    s1 = b.admit(doms[1], 5)
    assert s0 is not None and s1 is not None
    assert b.admit(doms[2], 5) is None  # over budget: the caller queues it
    b.step(5)
    assert sorted(b.poll(wait=True)) == sorted([s0, s1])
    b.release(s0)
    s2 = b.admit(doms[2], 5)
    assert s2 is not None
    b.release(s1)
    b.step(5)
    assert b.poll(wait=True) == [s2]
    b.release(s2)
    # all three took the same 5 steps from the same start
    p = [d.populations() for d in doms]
    assert np.array_equal(p[0], p[1]) and np.array_equal(p[0], p[2])
    for d in doms:
        d.destroy()
    b.destroy()


@pytest.mark.parametrize("cache", [None, (500_000, 3)])
def test_release_churn_and_compaction(capi, cache):
    """Admit and release many domains so that the packed table is compacted
    while a long-running domain stays resident; every result still equals
    its stand-alone run (also with groups of a few domains)."""
    long_spec = I.DomainSpec(kind="tgv", nx=40, ny=40, nz=40, tau=0.62, steps=60).materialise()
    shorts = small_specs(10, 3, lo=30, hi=44)  # ~400-1300 tiles each
    say("churn: one long domain, ten short ones")
    ref = {}
    for k, s in enumerate([long_spec] + shorts):
        d = build(capi, s, "fp16s")
        d.step(s.steps)
        ref[k] = d.populations()
        d.destroy()
    b = capi.Batch(1 << 34, "fp16s")
    if cache:
        b.set_cache_block(*cache)
    long_d = build(capi, long_spec, "fp16s")
    long_slot = b.admit(long_d, long_spec.steps)
    active = {}
    queue = list(enumerate(shorts, start=1))
    finished = {}
    while queue or active or long_slot is not None:
        while queue and len(active) < 3:
            k, s = queue.pop(0)
            d = build(capi, s, "fp16s")
            active[b.admit(d, s.steps)] = (k, d)
        b.step(2)
        for slot in b.poll():
            if slot == long_slot:
                b.release(slot)
                finished[0] = long_d.populations()
                long_d.destroy()
                long_slot = None
            else:
                k, d = active.pop(slot)
                b.release(slot)
                finished[k] = d.populations()
                d.destroy()
    b.destroy()
    for k in ref:
        assert np.array_equal(finished[k], ref[k]), f"domain {k} differs"


def test_serving_alone_equals_mix(capi):
    from paper_2204_10566_amd import serve

    tr = I.serving_trace(count=6, rate=200.0, seed=5, steps_lo=20, steps_hi=80)
    for r in tr:  # shrink the grids for the test
        n = 32 if r.rid % 2 else 40
        r.nozzle = I.Nozzle(n=n, length=4 * n, R=n / 4.0, r_throat=n / 4.0 * 0.4, inlet_len=n / 2.0,
                            throat_len=n)
    say("serving: 6 small requests, continuous vs one-at-a-time")
    mix, s_mix = serve.serve_continuous(tr, storage="fp16s", budget_bytes=1 << 32, steps_per_tick=4,
                                        keep_fields=True, realtime=False)
    alone, s_alone = serve.serve_serial(tr, storage="fp16s", keep_fields=True, realtime=False)
    say(f"  {s_mix}\n  {s_alone}")
    # the requests were resident together: more updated cells at once than
    # the largest request alone
    assert s_mix["peak_resident_cells"] > max(o.updated_cells for o in alone)
    by = {o.rid: o for o in alone}
    for o in mix:
        a = by[o.rid]
        assert o.status == a.status
        assert np.array_equal(o.rho, a.rho) and np.array_equal(o.u, a.u), f"request {o.rid} differs"


def test_admission_failure_leaves_batch_consistent(capi):
    """An allocation or upload that fails during admission (forced from the
    host with lbm_debug_fail_after, at each fallible step in turn, including
    a table growth) returns LBM_ERR_OOM, leaves the domain stand-alone and
    the batch working: the domain is admitted again afterwards, and every
    domain ends bit for bit where it ends alone."""
    specs = small_specs(3, 11)
    ref = []
    for s in specs:
        d = build(capi, s, "fp16s")
        d.step(s.steps)
        ref.append(d.populations())
        d.destroy()
    failures = 0
    for n in range(1, 9):
        doms = [build(capi, s, "fp16s") for s in specs]
        b = capi.Batch(1 << 33, "fp16s")
        s0 = b.admit(doms[0], specs[0].steps)
        b.step(2)
        capi.check(capi.lbm_debug_fail_after(n))
        failed = b.admit(doms[1], specs[1].steps)
        capi.check(capi.lbm_debug_fail_after(0))
        if failed is None:
            failures += 1
            # still stand-alone: a resident domain would refuse this call
            assert doms[1].step_status(0) == capi.OK
            s1 = b.admit(doms[1], specs[1].steps)
        else:
            s1 = failed
        s2 = b.admit(doms[2], specs[2].steps)
        slots = {s0: 0, s1: 1, s2: 2}
        done = set()
        while len(done) < 3:
            b.step(4)
            for s in b.poll():
                assert s in slots, f"unknown slot {s} reported"
                done.add(s)
        for s, k in slots.items():
            b.release(s)
            assert np.array_equal(doms[k].populations(), ref[k]), f"injection {n}: domain {k} differs"
            doms[k].destroy()
        b.destroy()
        say(f"failure injected at fallible step {n}: {'admission failed' if failed is None else 'no failure'}")
    assert failures >= 4


def test_serving_budget_bounds_device_memory(capi):
    """Every byte the service holds on the device counts against its budget
    (resident, released, prepared and waiting, being prepared): with room
    for about two requests, the held bytes never exceed the budget; a
    request that can never fit is answered with LBM_ERR_OOM and the others
    are served; results equal the requests served alone."""
    from paper_2204_10566_amd import serve

    tr = I.serving_trace(count=6, rate=200.0, seed=9, steps_lo=20, steps_hi=60)
    for r in tr:
        n = 32 if r.rid % 2 else 40
        r.nozzle = I.Nozzle(n=n, length=4 * n, R=n / 4.0, r_throat=n / 4.0 * 0.4, inlet_len=n / 2.0,
                            throat_len=n)
    big = max(serve.estimate_device_bytes(r, "fp16s") for r in tr)
    budget = int(2.5 * big)
    giant = tr[3]
    giant.nozzle = I.Nozzle(n=96, length=384, R=24.0, r_throat=9.6, inlet_len=48.0, throat_len=96.0)
    assert serve.estimate_device_bytes(giant, "fp16s") > budget
    say(f"serving under a budget of {budget} bytes, one request too large")
    mix, s_mix = serve.serve_continuous(tr, storage="fp16s", budget_bytes=budget, steps_per_tick=4,
                                        keep_fields=True, realtime=False, work_cap_cells=None)
    say(f"  peak held {s_mix['peak_held_bytes']} of {budget}")
    assert 0 < s_mix["peak_held_bytes"] <= budget
    alone, _ = serve.serve_serial([r for r in tr if r.rid != giant.rid], storage="fp16s", keep_fields=True,
                                  realtime=False)
    by = {o.rid: o for o in alone}
    for o in mix:
        if o.rid == giant.rid:
            assert o.status == capi.ERR_OOM
            continue
        a = by[o.rid]
        assert o.status == a.status == 0
        assert np.array_equal(o.rho, a.rho) and np.array_equal(o.u, a.u), f"request {o.rid} differs"


def test_serving_work_cap(capi):
    """With a cap on resident updated cells, admission holds requests back
    until earlier ones finish (never more than the cap resident, unless a
    single request exceeds it), and every result still equals the request
    served alone."""
    from paper_2204_10566_amd import serve

    tr = I.serving_trace(count=6, rate=200.0, seed=7, steps_lo=20, steps_hi=60)
    for r in tr:
        n = 32 if r.rid % 2 else 40
        r.nozzle = I.Nozzle(n=n, length=4 * n, R=n / 4.0, r_throat=n / 4.0 * 0.4, inlet_len=n / 2.0,
                            throat_len=n)
    say("serving with a cap of two small requests")
    alone, _ = serve.serve_serial(tr, storage="fp16s", keep_fields=True, realtime=False)
    cells = {o.rid: o.updated_cells for o in alone}
    cap = sorted(cells.values())[-1] + sorted(cells.values())[0]
    mix, s_mix = serve.serve_continuous(tr, storage="fp16s", budget_bytes=1 << 32, steps_per_tick=4,
                                        keep_fields=True, realtime=False, work_cap_cells=cap)
    say(f"  cap {cap}, peak resident {s_mix['peak_resident_cells']}")
    assert 0 < s_mix["peak_resident_cells"] <= max(cap, max(cells.values()))
    assert s_mix["peak_resident_cells"] < sum(cells.values())
    by = {o.rid: o for o in alone}
    for o in mix:
        a = by[o.rid]
        assert o.status == a.status
        assert np.array_equal(o.rho, a.rho) and np.array_equal(o.u, a.u), f"request {o.rid} differs"


def test_unstable_domain_is_evicted(capi):
    """A domain that goes unstable inside a batch is reported long before
    its step count, released as unstable, and the other domains finish with
    their stand-alone results.  The instability is forced from the host: the
    domain starts from a negative-density state."""
    specs = small_specs(3, 4)
    for s in specs:
        s.steps = 200
    ref = {}
    for k in (0, 2):
        d = build(capi, specs[k], "fp16s")
        d.step(specs[k].steps)
        ref[k] = d.populations()
        d.destroy()
    doms = [build(capi, s, "fp16s") for s in specs]
    bad = doms[1]
    bad.set_populations(-0.01 * np.ones((27,) + specs[1].flags.shape, np.float32))
    say("eviction of an unstable domain")
    b = capi.Batch(1 << 34, "fp16s")
    slots = [b.admit(d, s.steps) for d, s in zip(doms, specs)]
    # poll after each tick waits for the device, so that a tick is exactly
    # two steps and the report time does not depend on how far the host
    # runs ahead of the device
    reported = {}
    ticks = 0
    while len(reported) < 3:
        b.step(2)
        ticks += 1
        for s in b.poll(wait=True):
            reported[s] = ticks
    assert reported[slots[1]] <= 2  # evicted after its first steps, not after 200
    assert reported[slots[0]] == reported[slots[2]] == 100
    for k, s in enumerate(slots):
        b.release(s)
    assert doms[1].step_status(0) == capi.ERR_UNSTABLE
    for k in (0, 2):
        assert doms[k].step_status(0) == capi.OK
        assert np.array_equal(doms[k].populations(), ref[k])
    for d in doms:
        d.destroy()
    b.destroy()


def test_graph_replays_match_eager_steps(capi):
    """lbm_step(69) replays the 64-step graph once and runs 5 eager steps
    (ending on an odd count); three such calls with host reads in between
    equal 207 single eager steps."""
    spec = I.DomainSpec(kind="channel", nx=36, ny=18, nz=12, tau=0.57, steps=207).materialise()
    say("graph replays vs eager steps")
    g = build(capi, spec, "fp32")
    for _ in range(3):
        g.step(69)
        g.moments()
    e = build(capi, spec, "fp32")
    for _ in range(207):
        e.step(1)
    assert np.array_equal(g.populations(), e.populations())


def test_batch_state_errors(capi):
    """A domain resident in a batch refuses stand-alone calls
    (LBM_ERR_STATE); the batch refuses a second admission of it, a domain of
    another storage, a non-positive step count, releasing a slot before its
    steps have completed or a slot that does not exist, and destruction while
    it holds domains.  After release the domain works stand-alone again."""
    import ctypes

    spec = small_specs(1, 21)[0]
    d = build(capi, spec, "fp16s")
    other = build(capi, spec, "fp32")
    b = capi.Batch(1 << 32, "fp16s")
    slot = b.admit(d, 10)
    say("batch state errors")
    h = d.h
    pops = np.zeros(27 * d.ncells, np.float32).ctypes.data_as(capi._fp)
    n_in = int(d.info().n_inlet)
    uin = np.zeros(max(1, 3 * n_in), np.float32).ctypes.data_as(capi._fp)
    nimg = ctypes.c_size_t()
    assert capi.lbm_state_bytes(h, ctypes.byref(nimg)) == 0
    img = np.zeros(nimg.value, np.uint8)
    state = {
        "lbm_save_state": capi.lbm_save_state(h, img.ctypes.data_as(capi._vp), img.nbytes),
        "lbm_load_state": capi.lbm_load_state(h, img.ctypes.data_as(capi._vp), img.nbytes),
        "lbm_step": capi.lbm_step(h, 1),
        "lbm_step_async": capi.lbm_step_async(h, 1),
        "lbm_step_wait": capi.lbm_step_wait(h),
        "lbm_set_params": capi.lbm_set_params(h, 0.6, 1 / 0.6, 1.0),
        "lbm_set_rates": capi.lbm_set_rates(h, 1.5, 1.5, 1.0),
        "lbm_set_order_rates": capi.lbm_set_order_rates(h, 1.0, 1.0, 1.0, 1.0),
        "lbm_set_outlet": capi.lbm_set_outlet(h, 0, 1.0),
        "lbm_set_wall_distances": capi.lbm_set_wall_distances(h, None),
        "lbm_set_inlet_cells": capi.lbm_set_inlet_cells(h, uin),
        "lbm_init_fields": capi.lbm_init_fields(h, None, None),
        "lbm_get_populations": capi.lbm_get_populations(h, pops),
        "lbm_set_populations": capi.lbm_set_populations(h, pops),
        "lbm_stats_enable": capi.lbm_stats_enable(h, 1),
        "lbm_destroy": capi.lbm_destroy(h),
    }
    assert all(rc == capi.ERR_STATE for rc in state.values()), state
    s = ctypes.c_int()
    dp = ctypes.c_void_p()
    assert capi.lbm_batch_admit(b.h, h, 5, ctypes.byref(s)) == capi.ERR_STATE
    assert capi.lbm_batch_admit(b.h, other.h, 5, ctypes.byref(s)) == capi.ERR_ARG
    assert capi.lbm_batch_admit(b.h, other.h, 0, ctypes.byref(s)) == capi.ERR_ARG
    assert capi.lbm_batch_step(b.h, -1) == capi.ERR_ARG
    for bad_window in (0, 65):
        assert capi.lbm_batch_set_cache_block(b.h, 1 << 20, bad_window) == capi.ERR_ARG
    assert capi.lbm_batch_release(b.h, slot, ctypes.byref(dp)) == capi.ERR_STATE
    assert capi.lbm_batch_release(b.h, 999, ctypes.byref(dp)) == capi.ERR_ARG
    assert capi.lbm_batch_destroy(b.h) == capi.ERR_STATE
    b.step(10)
    assert b.poll(wait=True) == [slot]
    b.release(slot)
    d.step(3)
    d.destroy()
    other.destroy()
    b.destroy()


def test_batched_workload_full_size_packed_equals_alone(capi):
    """The 64-domain packed workload the benchmark times (periodic cubes and
    2:1:1 boxes, edges 16..128, 58 M cells, FP16S), over 40 steps with the
    default cache blocks: every domain ends bit for bit where it ends alone."""
    specs = I.batched_domains(count=64, seed=0, steps=40, materialise=True)
    say(f"full-size packed workload: {sum(s.ncells for s in specs)} cells")
    import hashlib

    def digest(d):  # the populations' bits, without holding 6 GB of them on the host
        return hashlib.sha256(d.populations().tobytes()).hexdigest()

    alone = []
    for s in specs:
        d = build(capi, s, "fp16s")
        d.step(s.steps)
        alone.append(digest(d))
        d.destroy()
    doms = [build(capi, s, "fp16s") for s in specs]
    b = capi.Batch(sum(int(d.info().device_bytes) for d in doms) + (1 << 30), "fp16s")
    slots = [b.admit(d, s.steps) for d, s in zip(doms, specs)]
    b.step(40)
    assert sorted(b.poll(wait=True)) == sorted(slots)
    for k, sl in enumerate(slots):
        b.release(sl)
        assert digest(doms[k]) == alone[k], f"domain {k} differs"
        doms[k].destroy()
    b.destroy()
