"""Writes the FP64 oracle references of the precision comparison:
the 128 x 128 x 1536 Re 6500 nozzle at a quarter of its linear size
(32 x 32 x 384, inlet noise 1 %, seed 0) advanced from the plug-flow start
with the paper's rates (omega_bulk = 1/tau, omega_high = 1), over the
2000-step window and over its first 200 steps (before the flow's own
instability amplifies round-off).  Stores rho - 1 and u at the updated
cells, in ascending cell order, one file per window.

With --full-size it writes the reference of the full 128 x 128 x 1536
configuration over its first 200 steps at 16384 sampled updated cells
(numpy PCG64, seed 2) of the slab 490 <= x < 570 around the end of the
throat and the sudden expansion, where the jet forms: the oracle's sampled
run computes only the dependency cone of those cells, which keeps the FP64
run to about half an hour on 8 host threads.  Stores the sampled cell
indices, rho - 1 and u there.

With --perturb EPS it writes the same windows from an initial velocity
multiplied by (1 + EPS xi), xi standard normal per cell and component
(numpy PCG64, seed 1), in one run (the 200-step state on the way to 2000):
the divergence of two FP64 runs that differ by about FP32 rounding, which
shows how much the flow itself amplifies a perturbation of that size.

Run from the repository root:
    python tests/golden/make_precision_reference.py [steps ...]   (default: 200 2000)
    python tests/golden/make_precision_reference.py --perturb 1e-7
    python tests/golden/make_precision_reference.py --full-size
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


def out_path(steps, perturbed=False):
    tag = "_perturbed" if perturbed else ""
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), f"precision_re6500_quarter_{steps}{tag}.npz")


def save(out, fl, f, steps, tau, t0, **extra):
    rho, u = oracle.moments(fl, f)
    upd = ((fl == I.FLUID) | (fl == I.OUTLET)).ravel()
    np.savez_compressed(out, steps=steps, tau=tau, drho=(rho.ravel()[upd] - 1.0).astype(np.float32),
                        u=u.reshape(3, -1)[:, upd].astype(np.float32), threads=oracle.max_threads(),
                        seconds=time.time() - t0, **extra)
    print(f"wrote {out} in {time.time() - t0:.0f} s", flush=True)


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
    save(out, fl, f, steps, cfg["tau"], t0)


def write_perturbed(eps):
    cfg = I.nozzle_config("re6500_quarter")
    fl = cfg["flags"]
    uin = cfg["uin"].astype(np.float32)
    u0 = cfg["u0"].astype(np.float32).astype(np.float64)
    u0 = u0 * (1.0 + eps * np.random.default_rng(1).standard_normal(u0.shape))
    rates = oracle.rates_vector(1.0 / cfg["tau"])
    t0 = time.time()
    f = oracle.init_fields(fl, None, u0)
    done = 0
    for steps in WINDOWS:
        st, f = oracle.step(fl, f, rates, steps - done, periodic=0, uin=uin)
        if st != 0:
            raise SystemExit(f"oracle status {st}")
        done = steps
        save(out_path(steps, True), fl, f, steps, cfg["tau"], t0, perturbation=eps)


FULL_SLAB = (490, 570)
FULL_SAMPLES = 16384
FULL_STEPS = 200


def full_size_path():
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), f"precision_re6500_full_{FULL_STEPS}_sampled.npz")


def full_size_cells(fl):
    """The sampled cells of the full-size reference: FULL_SAMPLES distinct
    updated cells of the slab FULL_SLAB, ascending."""
    nx = fl.shape[2]
    upd = np.flatnonzero(((fl == I.FLUID) | (fl == I.OUTLET)).ravel())
    x = upd % nx
    pool = upd[(x >= FULL_SLAB[0]) & (x < FULL_SLAB[1])]
    rng = np.random.Generator(np.random.PCG64(2))
    return np.sort(rng.choice(pool, size=FULL_SAMPLES, replace=False))


def write_full_size():
    cfg = I.nozzle_config("re6500")
    fl = cfg["flags"]
    cells = full_size_cells(fl)
    uin = cfg["uin"].astype(np.float32)
    u0 = cfg["u0"].astype(np.float32)
    t0 = time.time()
    st, f = oracle.run_cells(fl, cells, oracle.rates_vector(1.0 / cfg["tau"]), FULL_STEPS, periodic=0, uin=uin,
                             u0=u0)
    if st != 0:
        raise SystemExit(f"oracle status {st}")
    rho = np.zeros(cells.size)
    u = np.zeros((3, cells.size))
    for k in range(cells.size):
        rho[k], u[:, k] = oracle.cell_moments(f[:, k])
    np.savez_compressed(full_size_path(), steps=FULL_STEPS, tau=cfg["tau"], cells=cells.astype(np.int64),
                        slab=np.array(FULL_SLAB), drho=(rho - 1.0).astype(np.float64), u=u.astype(np.float64),
                        threads=oracle.max_threads(), seconds=time.time() - t0)
    print(f"wrote {full_size_path()} in {time.time() - t0:.0f} s", flush=True)


def main():
    args = sys.argv[1:]
    if args[:1] == ["--full-size"]:
        write_full_size()
        return
    if args[:1] == ["--perturb"]:
        write_perturbed(float(args[1]))
        return
    for steps in ([int(a) for a in args] or WINDOWS):
        write(steps)


if __name__ == "__main__":
    main()
