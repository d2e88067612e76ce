"""Writes the FP64 oracle references of the precision comparison:
the 128 x 128 x 1536 Re 6500 nozzle at a quarter of its linear size
(32 x 32 x 384, inlet noise 1 %, seed 0) advanced from the plug-flow start
with the paper's rates (omega_bulk = 1/tau, omega_high = 1), over the
2000-step window and over its first 200 steps (before the flow's own
instability amplifies round-off).  Stores rho - 1 and u at the updated
cells, in ascending cell order, one file per window.

Run from the repository root:
    python tests/golden/make_precision_reference.py [steps ...]   (default: 200 2000)
Only the oracle and the seeded input generators are used.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2204_10566_amd import inputs as I  # noqa: E402

WINDOWS = (200, 2000)


def out_path(steps):
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), f"precision_re6500_quarter_{steps}.npz")


def write(steps):
    out = out_path(steps)
    cfg = I.nozzle_config("re6500_quarter")
    fl = cfg["flags"]
    uin = cfg["uin"].astype(np.float32)
    u0 = cfg["u0"].astype(np.float32)
    t0 = time.time()
    f = oracle.init_fields(fl, None, u0)
    st, f = oracle.step(fl, f, oracle.rates_vector(1.0 / cfg["tau"]), steps, periodic=0, uin=uin)
    if st != 0:
        raise SystemExit(f"oracle status {st}")
    rho, u = oracle.moments(fl, f)
    upd = ((fl == I.FLUID) | (fl == I.OUTLET)).ravel()
    np.savez_compressed(out, steps=steps, tau=cfg["tau"], drho=(rho.ravel()[upd] - 1.0).astype(np.float32),
                        u=u.reshape(3, -1)[:, upd].astype(np.float32), threads=oracle.max_threads(),
                        seconds=time.time() - t0)
    print(f"wrote {out} in {time.time() - t0:.0f} s")


def main():
    for steps in ([int(a) for a in sys.argv[1:]] or WINDOWS):
        write(steps)


if __name__ == "__main__":
    main()
