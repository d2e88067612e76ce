"""Writes the FP64 oracle reference of the precision comparison:
the 128 x 128 x 1536 Re 6500 nozzle at a quarter of its linear size
(32 x 32 x 384, inlet noise 1 %, seed 0) advanced 2000 steps from the
plug-flow start with the paper's rates (omega_bulk = 1/tau, omega_high = 1).
Stores rho - 1 and u at the updated cells, in ascending cell order.

Run from the repository root:  python tests/golden/make_precision_reference.py
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

STEPS = 2000
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "precision_re6500_quarter.npz")


def main():
    cfg = I.nozzle_config("re6500_quarter")
    fl = cfg["flags"]
    uin = cfg["uin"].astype(np.float32)
    u0 = cfg["u0"].astype(np.float32)
    t0 = time.time()
    f = oracle.init_fields(fl, None, u0)
    st, f = oracle.step(fl, f, oracle.rates_vector(1.0 / cfg["tau"]), STEPS, periodic=0, uin=uin)
    if st != 0:
        raise SystemExit(f"oracle status {st}")
    rho, u = oracle.moments(fl, f)
    upd = ((fl == I.FLUID) | (fl == I.OUTLET)).ravel()
    np.savez_compressed(OUT, steps=STEPS, tau=cfg["tau"], drho=(rho.ravel()[upd] - 1.0).astype(np.float32),
                        u=u.reshape(3, -1)[:, upd].astype(np.float32), threads=oracle.max_threads(),
                        seconds=time.time() - t0)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
