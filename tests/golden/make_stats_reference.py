"""Writes the FP64 oracle reference of the long-window statistics test
(Sec. 2.2, Eqs. (15)-(19)): a periodic 8 x 16 x 2 box holding a uniform
stream U = 0.05 along x with decaying shear waves on it,
  u_x = U + A sin(2 pi y / 16), u_y = B sin(2 pi x / 8), u_z = C cos(2 pi y / 16),
A = 0.01, B = 0.004, C = 0.006, rho = 1, tau = 0.5015 (the paper's rates),
advanced 20000 steps.  The library samples every second step (its
local-phase steps 2, 4, ..., 20000) the pre-collision state of that step;
here the same states are formed by streaming the oracle's post-collision
state of the step before.  Stores the means of u, u_a u_b (products and sums
in FP64) and sigma over those 10000 samples, [component][z][y][x], and the
velocity field after the last step.

Run from the repository root:
    python tests/golden/make_stats_reference.py
Only the oracle and the seeded input generators are used."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402

SHAPE = (2, 16, 8)  # nz, ny, nx
U, A, B, C = 0.05, 0.01, 0.004, 0.006
TAU = 0.5015
STEPS = 20000
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "stats_stream_waves_20000.npz")


def initial_velocity():
    nz, ny, nx = SHAPE
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u = np.zeros((3,) + SHAPE)
    u[0] = U + A * np.sin(2 * np.pi * y / ny)
    u[1] = B * np.sin(2 * np.pi * x / nx)
    u[2] = C * np.cos(2 * np.pi * y / ny)
    return u.astype(np.float32)


def main():
    fl = np.zeros(SHAPE, np.uint8)
    rates = oracle.rates_vector(1.0 / TAU)
    f = oracle.init_fields(fl, None, initial_velocity())
    su = np.zeros((3,) + SHAPE)
    suu = np.zeros((6,) + SHAPE)
    ss = np.zeros((6,) + SHAPE)
    pa, pb = [0, 1, 2, 0, 0, 1], [0, 1, 2, 1, 2, 2]
    n = 0
    t0 = time.time()
    oracle.set_threads(1)
    for k in range(1, STEPS + 1):
        if k % 2 == 0:
            pre = oracle.stream(fl, f, periodic=7)
            _, u = oracle.moments(fl, pre)
            su += u
            for c in range(6):
                suu[c] += u[pa[c]] * u[pb[c]]
            ss += oracle.stress(fl, pre, 1.0 / TAU)
            n += 1
        st, f = oracle.step(fl, f, rates, 1, periodic=7)
        if st != 0:
            raise SystemExit(f"oracle status {st} at step {k}")
    _, u_end = oracle.moments(fl, f)
    np.savez_compressed(OUT, steps=STEPS, samples=n, tau=TAU, mean_u=su / n, mean_uu=suu / n, mean_sigma=ss / n,
                        u_end=u_end)
    print(f"wrote {OUT} ({n} samples) in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
