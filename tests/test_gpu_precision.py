"""Precision of the stored-population formats against the FP64 oracle on the
under-resolved nozzle: the 128 x 128 x 1536 Re 6500 configuration (inlet
noise 1 %) at its full size over its first 200 steps (16384 sampled cells
of the slab around the end of the throat and the sudden expansion, where
the jet forms), and at a quarter of its linear size, from the plug-flow
start (tau - 1/2 = 7e-5), over two windows: its first 200 steps and the
2000-step window.  The reference fields are written by
tests/golden/make_precision_reference.py (oracle only).

Errors: e_u = |u - u_ref|_2 / |u_ref|_2 and e_p = |rho - rho_ref|_2 /
|rho_ref - mean(rho_ref)|_2 over the updated cells (pressure p = rho / 3).

FP32 storage rounds each stored population to 2^-24 relative, FP16-shifted
storage to 2^-11 of (f - w) 2^14, i.e. about 3e-5 absolute on f, BF16 to
2^-8 of (f - w).  Over the first 200 steps the difference is that rounding,
accumulated step by step (measured: FP32 5.5e-5, FP16 5.3e-4, BF16 4.9e-3):
FP32 is held to 1e-4, FP16 to the 1e-3 velocity error the method is held
to, BF16 to 1e-2.  The pressure error is held to ten times the velocity
bound: a storage rounding moves rho and j by sums of the same roundings,
but e_p divides by the density fluctuation |rho - mean|, about 3 U^2 = 1e-2
of rho at these speeds, against U = 6e-2 for e_u, a factor of about 6
(measured e_p / e_u: 1.3 to 7.4).  Between steps 200 and 2000 the jet behind the throat is
unstable at this Reynolds number: two FP64 oracle runs from starts 1e-7
apart drift 200-fold further apart (a CPU test pins this on the stored
fields), and the rounding of every step is amplified alike (measured: FP32
2.8e-3, FP16 3.4e-2, BF16 0.48, where BF16 has lost the flow's detail).
There no format below FP64 can be held to a fixed bound; the test checks
instead what the argument predicts for FP32: its distance from FP64 is no
more than twice the distance between two FP32 runs whose starts differ by
1e-7 (relative, about FP32 rounding), measured in the same run (0.66 times
measured).  An FP32 error of the method itself would exceed that by orders
of magnitude.  The FP16 and BF16 departures in that window are reported by
the benchmark, not bounded here."""
import os

import numpy as np
import pytest

from paper_2204_10566_amd import inputs as I

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
BOUND_U = {"fp32": 1e-4, "fp16s": 1e-3, "bf16s": 1e-2}
BOUND_P = {k: 10.0 * v for k, v in BOUND_U.items()}
FULL_REF = os.path.join(GOLDEN, "precision_re6500_full_200_sampled.npz")


def ref_path(steps):
    return os.path.join(GOLDEN, f"precision_re6500_quarter_{steps}.npz")


@pytest.fixture(scope="module")
def capi():
    from paper_2204_10566_amd import capi

    return capi


def say(msg):
    print(f"[gpu] {msg}", flush=True)


def run_nozzle(capi, which, storage, steps, u0=None):
    cfg = I.nozzle_config(which)
    fl = cfg["flags"]
    d = capi.Domain(fl, periodic=0, storage=storage)
    d.set_params(cfg["tau"])
    d.set_inlet(cfg["uin"].astype(np.float32))
    d.init_fields(None, cfg["u0"].astype(np.float32) if u0 is None else u0)
    st = d.step_status(steps)
    rho, u = d.moments()
    d.destroy()
    return st, fl, rho, u


def errors(ug, dr, ur, rr):
    e_u = float(np.linalg.norm(ug - ur) / np.linalg.norm(ur))
    e_p = float(np.linalg.norm(dr - rr) / np.linalg.norm(rr - rr.mean()))
    return e_u, e_p


def precision_errors(capi, storage, steps):
    ref = np.load(ref_path(steps))
    st, fl, rho, u = run_nozzle(capi, "re6500_quarter", storage, int(ref["steps"]))
    upd = ((fl == I.FLUID) | (fl == I.OUTLET)).ravel()
    ug = u.reshape(3, -1)[:, upd].astype(np.float64)
    dr = rho.ravel()[upd].astype(np.float64) - 1.0
    e_u, e_p = errors(ug, dr, ref["u"].astype(np.float64), ref["drho"].astype(np.float64))
    return st, e_u, e_p


@pytest.mark.parametrize("storage", ["fp32", "fp16s", "bf16s"])
def test_precision_against_fp64_200_steps(capi, storage):
    if not os.path.exists(ref_path(200)):
        pytest.skip("reference not generated")
    st, e_u, e_p = precision_errors(capi, storage, 200)
    say(f"re6500 quarter, 200 steps, {storage}: e_u={e_u:.3e} e_p={e_p:.3e}")
    assert st == 0
    assert e_u <= BOUND_U[storage]
    assert e_p <= BOUND_P[storage]


@pytest.mark.parametrize("storage", ["fp32", "fp16s", "bf16s"])
def test_full_size_precision_against_fp64(capi, storage):
    """The full 128 x 128 x 1536 configuration, 200 steps, at the sampled
    cells of the FP64 reference: the same velocity bounds as at quarter
    scale."""
    ref = np.load(FULL_REF)
    st, _, rho, u = run_nozzle(capi, "re6500", storage, int(ref["steps"]))
    cells = ref["cells"]
    ug = u.reshape(3, -1)[:, cells].astype(np.float64)
    dr = rho.ravel()[cells].astype(np.float64) - 1.0
    e_u, e_p = errors(ug, dr, ref["u"], ref["drho"])
    say(f"re6500 128x128x1536, 200 steps, {storage}: e_u={e_u:.3e} e_p={e_p:.3e} at {cells.size} cells")
    assert st == 0
    assert e_u <= BOUND_U[storage]
    assert e_p <= BOUND_P[storage]


def test_fp32_2000_steps_within_flow_amplification(capi):
    if not os.path.exists(ref_path(2000)):
        pytest.skip("reference not generated")
    ref = np.load(ref_path(2000))
    cfg = I.nozzle_config("re6500_quarter")
    st, fl, _, u = run_nozzle(capi, "re6500_quarter", "fp32", 2000)
    u0 = cfg["u0"].astype(np.float32).astype(np.float64)
    u0p = (u0 * (1.0 + 1e-7 * np.random.default_rng(1).standard_normal(u0.shape))).astype(np.float32)
    stp, _, _, up = run_nozzle(capi, "re6500_quarter", "fp32", 2000, u0p)
    upd = ((fl == I.FLUID) | (fl == I.OUTLET)).ravel()
    ug = u.reshape(3, -1)[:, upd].astype(np.float64)
    ugp = up.reshape(3, -1)[:, upd].astype(np.float64)
    ur = ref["u"].astype(np.float64)
    e_ref = float(np.linalg.norm(ug - ur) / np.linalg.norm(ur))
    e_pert = float(np.linalg.norm(ugp - ug) / np.linalg.norm(ug))
    say(f"re6500 quarter, 2000 steps, fp32: e_u vs FP64 {e_ref:.3e}, FP32 from a 1e-7 perturbed start {e_pert:.3e}")
    assert st == 0 and stp == 0
    assert e_ref <= 2.0 * e_pert
