"""Writes the FP64 oracle reference of the benchmark nozzle (96 x 96 x 768,
x axial, Re 500, Poiseuille velocity inlet, zero-gradient outlet; the
paper's rates: omega_bulk = 1/tau, orders >= 3 at one) over its first 200
steps from the plug-flow start, the window the oracle can run in full.

Stores, at updated cells drawn with numpy PCG64 (seed 5) in ascending cell
order:
  * the 27 populations f_i (phase-0 form, i = (cx+1) + 3(cy+1) + 9(cz+1))
    at 2048 cells: 256 next to the inlet plane (x = 1), 256 on the outlet
    plane, 512 next to a wall (a solid cell at y +- 1), 512 in the
    throat and the sudden expansion (256 <= x < 448) and 512 anywhere;
  * rho - 1 and u at 16384 updated cells anywhere.

Run from the repository root (about 45 minutes on 8 host threads):
    python tests/golden/make_nozzle_reference.py
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

STEPS = 200
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"nozzle_re500_{STEPS}_sampled.npz")


def sample_cells(fl):
    """(population cells, moment cells), both ascending."""
    nz, ny, nx = fl.shape
    upd = np.flatnonzero(((fl == I.FLUID) | (fl == I.OUTLET)).ravel())
    x = upd % nx
    solid = fl.ravel() == I.SOLID
    near = upd[solid[np.clip(upd + nx, 0, fl.size - 1)] | solid[np.clip(upd - nx, 0, fl.size - 1)]]
    rng = np.random.Generator(np.random.PCG64(5))
    pick = lambda pool, n: rng.choice(pool, size=n, replace=False)  # noqa: E731
    pops = np.concatenate([pick(upd[x == 1], 256), pick(upd[x == nx - 1], 256), pick(near, 512),
                           pick(upd[(x >= 256) & (x < 448)], 512), pick(upd, 512)])
    pops = np.unique(pops)
    moms = np.sort(pick(upd, 16384))
    return pops, moms


def main():
    cfg = I.nozzle_config("re500")
    fl = cfg["flags"]
    uin = cfg["uin"].astype(np.float32)
    u0 = cfg["u0"].astype(np.float32)
    pops, moms = sample_cells(fl)
    t0 = time.time()
    f = oracle.init_fields(fl, None, u0)
    st, f = oracle.step(fl, f, oracle.rates_vector(1.0 / cfg["tau"]), STEPS, periodic=0, uin=uin)
    if st != 0:
        raise SystemExit(f"oracle status {st}")
    rho, u = oracle.moments(fl, f)
    f = f.reshape(27, -1)
    np.savez_compressed(OUT, steps=STEPS, tau=cfg["tau"], pop_cells=pops.astype(np.int64), f=f[:, pops],
                        moment_cells=moms.astype(np.int64), drho=rho.ravel()[moms] - 1.0,
                        u=u.reshape(3, -1)[:, moms], threads=oracle.max_threads(), seconds=time.time() - t0)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
