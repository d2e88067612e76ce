"""Independence of the launch shape (race check).

In a step no two lanes touch one slot: the streaming step reads and writes
slot a_k(x) only from the lane of x, the local step only its own slots.  The
result therefore cannot depend on which wave takes which tile or in what
order the waves run.  Launching every step on 8 or 24 blocks, so that each
wave walks many tiles in turn (and the eight XCDs split the list
differently), must give the same bits as one wave per tile: on random
configurations of every boundary option, in FP32, FP16S and BF16S, with
statistics, through graph replays and an odd step count."""
import numpy as np
import pytest

from test_gpu_random_configs import build_domain, make_case

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def capi():
    from paper_2204_10566_amd import capi

    return capi


def run(capi, c, storage, blocks, steps, stats):
    d = build_domain(capi, c, storage)
    if blocks:
        d.debug_step_grid(blocks)
    if stats:
        d.stats_enable(True)
    d.step(steps)
    out = [d.populations(), *d.moments()]
    if stats:
        out += list(d.stats()[:3])
    d.destroy()
    return out


@pytest.mark.parametrize("k", range(12))
def test_launch_shape_does_not_change_the_result(capi, k):
    c = make_case(500 + k)
    storage = ("fp32", "fp16s", "bf16s")[k % 3]
    steps = 2 * c["steps"] + 5
    stats = k % 2 == 0
    say(f"case {k}: shape {c['fl'].shape} periodic {c['periodic']} {storage} steps {steps} outlet {c['outlet']} "
        f"curved {c['q'] is not None} stats {stats}")
    ref = run(capi, c, storage, 0, steps, stats)
    for blocks in (8, 24):
        got = run(capi, c, storage, blocks, steps, stats)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), f"{blocks} blocks"


def test_bad_grid_rejected(capi):
    c = make_case(3, "fp32")
    d = build_domain(capi, c, "fp32")
    for bad in (-8, 12, 7):
        with pytest.raises(capi.LbmError) as e:
            d.debug_step_grid(bad)
        assert e.value.code == capi.ERR_ARG
    d.destroy()
