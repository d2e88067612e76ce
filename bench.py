"""Benchmark of the fused D3Q27 CHM-MRT stream-collide step on one MI355X.

Workload: the synthetic sudden-expansion nozzle on a 96 x 96 x 768 voxel grid
(x axial; inlet pipe radius 24, 20-degree cone to a throat of radius 8, throat
8 R long, sudden expansion back to R), Re 500 on the throat diameter,
Ma <= 0.1, halfway bounce-back walls, Poiseuille velocity inlet,
zero-gradient outlet, FP32 populations.  A step is the whole fused update
of every fluid cell (gather with boundary resolution, moments, forward
central-Hermite transform, relaxation, inverse transform, store), one kernel
launch.  The library runs steps in place on one population array and
alternates two kernels: the streaming step (neighbour slots) and the local
step (own slots); both move the same algorithmic bytes.  The timed steps are
replayed from HIP graphs of 64, 32, ..., 2 steps (the longest that fit),
built before the timed region.

Prints one JSON line.  value = fluid-cell MLUPS over the timed steps, with
all state resident in HBM.  roofline.achieved = algorithmic bytes per launch
(216 B per updated cell for FP32: 27 loads + 27 stores) / average launch
duration over the timed launches (both kernels), timed with HIP events on
the library's stream: the start event, the steps enqueued without waiting
(lbm_step_async), the end event, then the wait for them and the check of
their status word (lbm_step_wait), which so stays outside the window.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "MLUPS + % peak HBM BW (D3Q27 CHM); batched p50/p99 latency vs serial"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    import hashlib

    path = os.path.join(ROOT, "paper_2204_10566_amd", "csrc", "lbm_device.hpp")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def read_kernel_profile(storage: str, workload: str):
    """Per-kernel average durations of the step kernels from the committed
    rocprofv3 kernel-trace summary, with the fraction of 8 TB/s each
    reaches on the algorithmic bytes; None when absent or when the kernel
    source has changed since the trace was taken."""
    import re

    path = os.path.join(ROOT, "profiles", f"step_{storage}_{workload}.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"sha256\[:16\]: (\w+)", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    out = {"source": os.path.relpath(path, ROOT)}
    for k in ("k_stream_collide", "k_local_collide"):
        m = re.search(rf"  {k}: avg ([\d.]+) us -> (\d+) GB/s \(([\d.]+)% of 8 TB/s\)", text)
        if m:
            out[k] = {"avg_us": float(m.group(1)), "achieved_gbs": float(m.group(2)),
                      "frac": round(float(m.group(3)) / 100, 4)}
    return out


def read_traffic(kernel: str, storage: str, workload: str):
    """HBM traffic per launch measured with rocprofv3 counters, from the
    committed summary; None when absent or when the kernel source has
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{storage}_{workload}.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return float(fields["traffic_bytes_per_launch"]) if "traffic_bytes_per_launch" in fields else None


def time_steps(capi, torch, cfg, storage, steps, warmup, stream, feq_order=6):
    d = capi.Domain(cfg["flags"], periodic=cfg["periodic"], storage=storage, stream=stream.cuda_stream)
    d.set_params(cfg["tau"], 1.0 / cfg["tau"], 1.0)
    d.set_equilibrium_order(feq_order)
    d.set_inlet(cfg["uin"])
    d.init_fields(None, cfg["u0"])
    info = d.info()
    if warmup:
        d.step(warmup)
    d.prepare_steps()  # the step graphs are built before the timed region
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    d.step_async(steps)
    e1.record(stream)
    rc = d.wait_status()
    e1.synchronize()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    rho, u = d.moments()
    d.destroy()
    return info, ms, rc, rho, u


def copy_ceiling(torch, stream, nbytes, reps=20):
    """A plain device-to-device copy moving the same number of bytes as one
    step (half read, half written): the practical HBM ceiling on this machine,
    and the reference kernel for scaling the rocprofv3 byte counters."""
    n = int(nbytes // 2 // 4)
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    with torch.cuda.stream(stream):
        # an elementwise kernel reading n floats and writing n floats
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            torch.mul(src, 1.0, out=dst)
        e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return {"gbs": round(2 * n * 4 / (ms * 1e-3) / 1e9, 1), "bytes_per_copy": 2 * n * 4, "us_per_copy": round(ms * 1e3, 2)}


def batched_leg(storage="fp16s"):
    """64 independent periodic / channel domains (edges 16..128, cubes and
    2:1:1 boxes, tau in [0.51, 0.8]), 500 steps each: packed launches
    (cache-blocked windows of steps) versus one domain after another."""
    from paper_2204_10566_amd import inputs as I
    from paper_2204_10566_amd import serve

    specs = I.batched_domains(count=64, seed=0, steps=500, materialise=True)
    out = serve.run_packed(specs, storage=storage)
    out["storage"] = storage
    return out


def serving_leg(full: bool, storage="fp16s"):
    """Poisson arrivals (20 requests/s, seed 0) of nozzle-like solves (64..128
    cross section, length 4n..8n, throat/pipe ratio 0.25..0.5, Re
    500..6500): continuous batching (with the default cap on resident cells,
    and without a cap) versus one at a time on the same trace.  The full
    trace is 200 requests of 1000-5000 steps; it offers several times what
    the GPU can serve, so its latencies are mostly queueing.  A labelled
    extra serves the same trace at 8.4 requests/s, about 70 % of what the
    GPU sustains, where queues stay short."""
    from paper_2204_10566_amd import inputs as I
    from paper_2204_10566_amd import serve

    def policies(tr, uncapped=True):
        out = {}
        _, out["continuous"] = serve.serve_continuous(tr, storage=storage)
        log(f"serving continuous: {out['continuous']}")
        if uncapped:
            _, out["continuous_uncapped"] = serve.serve_continuous(tr, storage=storage, work_cap_cells=None)
            log(f"serving continuous, no cap on resident cells: {out['continuous_uncapped']}")
        _, out["serial"] = serve.serve_serial(tr, storage=storage)
        log(f"serving serial: {out['serial']}")
        out["p50_ratio_serial_over_continuous"] = round(out["serial"]["p50_s"] / out["continuous"]["p50_s"], 3)
        out["p99_ratio_serial_over_continuous"] = round(out["serial"]["p99_s"] / out["continuous"]["p99_s"], 3)
        return out

    if full:
        tr = I.serving_trace(count=200, rate=20.0, seed=0)
        res = {"trace": "200 requests at 20/s (Poisson, seed 0), 1000-5000 steps each", "storage": storage}
        res.update(policies(tr))
        log("serving: the same trace at 8.4 requests/s")
        slow = I.serving_trace(count=200, rate=8.4, seed=0)
        res["at_8.4_per_s"] = {"trace": "the same 200 requests at 8.4/s (about 70 % of what the GPU sustains)",
                               **policies(slow, uncapped=False)}
        return res
    tr = I.serving_trace(count=60, rate=20.0, seed=0, steps_lo=250, steps_hi=1250)
    res = {"trace": "first 60 requests of the trace with step counts scaled by 1/4 (250-1250)", "storage": storage}
    res.update(policies(tr))
    return res


def precision_leg(capi, torch, stream):
    """Error of each storage format against the FP64 oracle references
    (tests/golden/precision_re6500_quarter_{200,2000}.npz, written by the
    oracle): the Re 6500 nozzle at a quarter of the 128 x 128 x 1536 size
    after 200 and after 2000 steps; then the full 128 x 128 x 1536 Re 6500
    nozzle timed in each format."""
    import numpy as np

    from paper_2204_10566_amd import inputs as I

    out = {}
    cfg = I.nozzle_config("re6500_quarter")
    fl = cfg["flags"]
    upd = ((fl == 0) | (fl == 3)).ravel()
    for steps in (200, 2000):
        ref_path = os.path.join(ROOT, "tests", "golden", f"precision_re6500_quarter_{steps}.npz")
        if not os.path.exists(ref_path):
            continue
        ref = np.load(ref_path)
        ur = ref["u"].astype(np.float64)
        rr = ref["drho"].astype(np.float64)
        res = {"workload": "128x128x1536 Re 6500 nozzle at quarter scale (32x32x384), inlet noise 1 %, "
                           f"{int(ref['steps'])} steps from plug flow, tau={float(ref['tau']):.7f}",
               "reference": f"tests/golden/precision_re6500_quarter_{steps}.npz (FP64 oracle)"}
        def run(st, u0):
            d = capi.Domain(fl, periodic=0, storage=st, stream=stream.cuda_stream)
            d.set_params(cfg["tau"])
            d.set_inlet(cfg["uin"].astype(np.float32))
            d.init_fields(None, u0)
            rc = d.step_status(int(ref["steps"]))
            rho, u = d.moments()
            d.destroy()
            return rc, rho.ravel()[upd].astype(np.float64) - 1.0, u.reshape(3, -1)[:, upd].astype(np.float64)

        u32 = {}
        for st in ("fp32", "fp16s", "bf16s"):
            rc, dr, ug = run(st, cfg["u0"].astype(np.float32))
            u32[st] = ug
            res[st] = {"e_u": float(np.linalg.norm(ug - ur) / np.linalg.norm(ur)),
                       "e_p": float(np.linalg.norm(dr - rr) / np.linalg.norm(rr - rr.mean())), "status": int(rc)}
            log(f"precision {steps} steps {st}: {res[st]}")
        # sensitivity of the flow itself: FP32 from an initial velocity
        # perturbed by 1e-7 relative (about FP32 rounding) against FP32
        u0 = cfg["u0"].astype(np.float32).astype(np.float64)
        u0p = (u0 * (1.0 + 1e-7 * np.random.default_rng(1).standard_normal(u0.shape))).astype(np.float32)
        rc, _, up = run("fp32", u0p)
        res["fp32_perturbed_1e-7_vs_fp32"] = {"e_u": float(np.linalg.norm(up - u32["fp32"]) /
                                                          np.linalg.norm(u32["fp32"])), "status": int(rc)}
        log(f"precision {steps} steps fp32 perturbed 1e-7 vs fp32: {res['fp32_perturbed_1e-7_vs_fp32']}")
        out[f"quarter_scale_vs_fp64_{steps}_steps"] = res
    cfg = I.nozzle_config("re6500")
    for k in ("uin", "u0"):
        cfg[k] = cfg[k].astype(np.float32)
    ref_path = os.path.join(ROOT, "tests", "golden", "precision_re6500_full_200_sampled.npz")
    if os.path.exists(ref_path):
        ref = np.load(ref_path)
        cells = ref["cells"]
        res = {"workload": "synthetic nozzle 128x128x1536, Re 6500, inlet noise 1 %, "
                           f"{int(ref['steps'])} steps from plug flow, tau={float(ref['tau']):.7f}",
               "reference": f"tests/golden/precision_re6500_full_200_sampled.npz (FP64 oracle at {cells.size} "
                            f"sampled cells of the slab {int(ref['slab'][0])} <= x < {int(ref['slab'][1])})"}
        for st in ("fp32", "fp16s", "bf16s"):
            d = capi.Domain(cfg["flags"], periodic=0, storage=st, stream=stream.cuda_stream)
            d.set_params(cfg["tau"])
            d.set_inlet(cfg["uin"])
            d.init_fields(None, cfg["u0"])
            rc = d.step_status(int(ref["steps"]))
            rho, u = d.moments()
            d.destroy()
            ug = u.reshape(3, -1)[:, cells].astype(np.float64)
            dr = rho.ravel()[cells].astype(np.float64) - 1.0
            res[st] = {"e_u": float(np.linalg.norm(ug - ref["u"]) / np.linalg.norm(ref["u"])),
                       "e_p": float(np.linalg.norm(dr - ref["drho"]) /
                                    np.linalg.norm(ref["drho"] - ref["drho"].mean())), "status": int(rc)}
            log(f"precision full size {st}: {res[st]}")
            del rho, u
        out["full_size_vs_fp64_200_steps"] = res
    speed = {"workload": "synthetic nozzle 128x128x1536, Re 6500, inlet noise 1 %, 400 steps from plug flow"}
    for st in ("fp32", "fp16s", "bf16s"):
        info, ms, rc, _, _ = time_steps(capi, torch, cfg, st, 400, 64, stream)
        speed[st] = {"mlups": round(info.n_updated * 400 / (ms * 1e-3) / 1e6, 1), "status": int(rc)}
        log(f"re6500 full size {st}: {speed[st]}")
    speed["ratio_fp16s_vs_fp32"] = round(speed["fp16s"]["mlups"] / speed["fp32"]["mlups"], 3)
    out["re6500_full_size"] = speed
    return out


def roofline_probe_leg(capi, torch, stream, n=320, steps=192):
    """Periodic Taylor-Green vortex on n^3 cells: no walls, every cell
    updated, n a multiple of 64 so that rows align with tiles.  At n = 320
    one FP32 step moves 7.1 GB, far beyond the 256 MB Infinity Cache, so this
    is a bandwidth point that the cache does not flatter; FP32 and FP16S,
    beside a plain copy of the same byte count."""
    import numpy as np

    from paper_2204_10566_amd import inputs as I

    fl = I.periodic_box(n)
    u0 = I.taylor_green_velocity(n, n, n, 0.05).astype(np.float32)
    out = {"workload": f"periodic Taylor-Green vortex {n}^3, u0 = 0.05, tau = 0.6, {steps} timed steps"}
    for st in ("fp32", "fp16s"):
        d = capi.Domain(fl, periodic=7, storage=st, stream=stream.cuda_stream)
        d.set_params(0.6)
        d.init_fields(None, u0)
        info = d.info()
        d.step(64)
        d.prepare_steps()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        d.step_async(steps)
        e1.record(stream)
        rc = d.wait_status()
        e1.synchronize()
        d.destroy()
        us = e0.elapsed_time(e1) / steps * 1e3
        gbs = info.n_updated * info.bytes_per_cell_update / (us * 1e-6) / 1e9
        out[st] = {"us_per_step": round(us, 2), "mlups": round(info.n_updated / us, 1),
                   "achieved_gbs": round(gbs, 1), "frac_of_peak": round(gbs / PEAK_HBM_GBS, 4), "status": int(rc)}
        log(f"tgv {n}^3 {st}: {out[st]}")
    del u0
    copy = copy_ceiling(torch, stream, fl.size * 216, reps=10)
    out["copy_ceiling_gbs"] = copy["gbs"]
    out["fp32_frac_of_copy"] = round(out["fp32"]["achieved_gbs"] / copy["gbs"], 4)
    out["ratio_fp16s_vs_fp32"] = round(out["fp16s"]["mlups"] / out["fp32"]["mlups"], 3)
    log(f"tgv {n}^3 plain copy of {copy['bytes_per_copy'] / 1e9:.1f} GB: {copy['gbs']:.0f} GB/s")
    return out


def finest_grid_leg(capi, torch, stream, steps=64):
    """The synthetic nozzle on the paper's finest grid in that run's own
    lattice parameters (Table 2, R4 at Re 6500: cells of 0.0776 mm over the
    12 x 12 x 240 mm domain, 155 x 155 x 3093 = 74.3 M cells, the pipe filling
    the cross-section; tau = 0.50281 and a mean throat velocity of 0.118 cells
    per step, CFL 0.236), constant-pressure outlet, halfway walls.  In FP32 its
    population array (8.0 GB) is past the 4 GiB that buffer instructions
    address, so it steps with the 64-bit addressing kernels; in FP16S (4.0 GB)
    with the 32-bit ones.  nx = 3093 is not a multiple of 64: general
    addressing.  From the plug-flow start, 64 untimed and `steps` timed
    steps."""
    import numpy as np

    from paper_2204_10566_amd import inputs as I

    cfg = I.paper_nozzle("R4", 6500)
    fl = cfg["flags"]
    nz_, ny_, nx_ = fl.shape
    uin = cfg["uin_cells"].astype(np.float32)
    u0 = cfg["u0"].astype(np.float32)
    tau = cfg["tau"]
    out = {"workload": f"synthetic nozzle {ny_}x{nz_}x{nx_} (x axial) in the paper's R4 parameters (Table 2, Re 6500): "
                       f"tau = {tau:.6f}, mean throat velocity {cfg['u_thr']:.4f}, pressure outlet, {steps} timed steps",
           "cells": int(fl.size)}
    for st in ("fp32", "fp16s"):
        d = capi.Domain(fl, periodic=0, storage=st, stream=stream.cuda_stream)
        d.set_params(tau, 1.0 / tau, 1.0)
        d.set_inlet_cells(uin)
        d.set_outlet("pressure", 1.0)
        d.init_fields(None, u0)
        info = d.info()
        wide = d.is_wide()
        d.step(64)
        d.prepare_steps()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        d.step_async(steps)
        e1.record(stream)
        rc = d.wait_status()
        e1.synchronize()
        d.destroy()
        us = e0.elapsed_time(e1) / steps * 1e3
        gbs = info.n_updated * info.bytes_per_cell_update / (us * 1e-6) / 1e9
        out[st] = {"array_gb": round(capi.lbm_array_bytes(nx_, ny_, nz_, 0 if st == "fp32" else 1) / 1e9, 2),
                   "addressing": "64-bit" if wide else "32-bit", "fluid_cells": int(info.n_updated),
                   "us_per_step": round(us, 1), "mlups": round(info.n_updated / us, 1), "achieved_gbs": round(gbs, 1),
                   "frac_of_peak": round(gbs / PEAK_HBM_GBS, 4), "status": int(rc)}
        log(f"R4 nozzle {st}: {out[st]}")
    out["ratio_fp16s_vs_fp32"] = round(out["fp16s"]["mlups"] / out["fp32"]["mlups"], 3)
    return out


def paper_regime_leg(capi, steps=20000):
    """The paper's own parameter sets on its coarsest grid (Table 2, R1:
    52 x 52 x 1043): Re 500 (tau = 0.50922, CFL 0.177) and Re 6500 (tau =
    0.50100, CFL 0.249, a peak lattice velocity near 0.25), the synthetic
    nozzle with a constant-pressure outlet, FP32, from the plug-flow start,
    with halfway walls and with the curved walls the paper uses.  Reports
    how many steps each runs before the status word reports an unstable
    cell (all `steps` when it does not)."""
    import numpy as np

    from paper_2204_10566_amd import inputs as I

    out = {"workload": f"synthetic nozzle on the R1 grid in the paper's parameters, up to {steps} steps, FP32"}
    for re in (500, 6500):
        cfg = I.paper_nozzle("R1", re)
        fl = cfg["flags"]
        q = cfg["nozzle"].wall_distances(fl)
        for walls in ("halfway", "curved"):
            d = capi.Domain(fl, periodic=0, storage="fp32")
            d.set_params(cfg["tau"], 1.0 / cfg["tau"], 1.0)
            if walls == "curved":
                d.set_wall_distances(q)
            d.set_inlet_cells(cfg["uin_cells"].astype(np.float32))
            d.set_outlet("pressure", 1.0)
            d.init_fields(None, cfg["u0"].astype(np.float32))
            done, rc = 0, 0
            while done < steps:
                rc = d.step_status(1000)
                if rc != 0:
                    break
                done += 1000
            _, u = d.moments()
            d.destroy()
            key = f"re{re}_{walls}_walls"
            out[key] = {"tau": round(cfg["tau"], 6), "mean_throat_velocity": round(cfg["u_thr"], 4),
                        "stable_steps": done, "status": int(rc),
                        "max_abs_u": None if rc else round(float(np.abs(u).max()), 4)}
            log(f"paper regime R1 Re {re}, {walls} walls: {out[key]}")
    return out


def stability_leg(capi, stream):
    """Stability envelope at tau -> 1/2: a 64^3 periodic double shear layer
    (u0 = 0.1, FP32) run 2000 steps at decreasing tau - 1/2 for several
    settings of the higher-order rates; reports the smallest tau - 1/2 that
    stays stable for each setting."""
    import numpy as np

    from paper_2204_10566_amd import inputs as I

    n = 64
    fl = I.periodic_box(n)
    u0 = I.double_shear_layer_velocity(n, 0.1).astype(np.float32)
    eps = [1e-2, 3e-3, 1e-3, 3e-4, 1e-4, 3e-5, 1e-5]
    # (rates of orders 3..6, equilibrium order): the paper's full equilibrium
    # with several higher-order rates, then the explicit truncated ones
    settings = {"omega_3..6 = 1 (paper)": ((1.0, 1.0, 1.0, 1.0), 6),
                "omega_3..6 = 1.2": ((1.2, 1.2, 1.2, 1.2), 6),
                "omega_3..6 = 1.6": ((1.6, 1.6, 1.6, 1.6), 6),
                "omega_3 = omega (shear), rest 1": (None, 6),
                "second-order equilibrium, omega_3..6 = 1": ((1.0, 1.0, 1.0, 1.0), 2),
                "third-order equilibrium, omega_3..6 = 1": ((1.0, 1.0, 1.0, 1.0), 3),
                "fourth-order equilibrium, omega_3..6 = 1": ((1.0, 1.0, 1.0, 1.0), 4)}
    out = {"workload": "64^3 periodic double shear layer, u0 = 0.1, kappa 80, FP32, 2000 steps per point",
           "tau_minus_half_tried": eps}
    for name, (rates, order) in settings.items():
        smallest = None
        for e in eps:
            tau = 0.5 + e
            d = capi.Domain(fl, periodic=7, storage="fp32", stream=stream.cuda_stream)
            d.set_rates(1.0 / tau, 1.0 / tau, 1.0)
            d.set_order_rates(*(rates if rates is not None else (1.0 / tau, 1.0, 1.0, 1.0)))
            d.set_equilibrium_order(order)
            d.init_fields(None, u0)
            rc = d.step_status(2000)
            d.destroy()
            if rc != capi.OK:
                break
            smallest = e
        out[name] = smallest
        log(f"stability {name}: smallest stable tau - 1/2 = {smallest}")
    return out


def cpu_baseline(cfg, nsteps=4):
    import numpy as np

    import oracle

    fl = cfg["flags"]
    t0 = time.perf_counter()
    f = oracle.init_fields(fl, None, cfg["u0"])
    t1 = time.perf_counter()
    st, f = oracle.step(fl, f, oracle.rates_vector(1.0 / cfg["tau"]), nsteps, periodic=cfg["periodic"],
                        uin=cfg["uin"])
    t2 = time.perf_counter()
    n_upd = int(((fl == 0) | (fl == 3)).sum())
    threads = oracle.max_threads()
    # one thread, on a small sample: the periodic TGV 32^3, 3 steps
    from paper_2204_10566_amd import inputs as I

    n1, s1 = 32, 3
    fl1 = I.periodic_box(n1)
    f1 = oracle.init_fields(fl1, None, I.taylor_green_velocity(n1, n1, n1, 0.05))
    oracle.set_threads(1)
    try:
        t3 = time.perf_counter()
        st1, _ = oracle.step(fl1, f1, oracle.rates_vector(1.0 / 0.6), s1, periodic=7)
        t4 = time.perf_counter()
    finally:
        oracle.set_threads(threads)
    return {
        "value": round(n_upd * nsteps / (t2 - t1) / 1e6, 4),
        "unit": "MLUPS",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{nsteps} FP64 oracle steps (dense 27x27 transform + Gaussian elimination per cell) of the "
                  f"full 96x96x768 nozzle ({n_upd} updated cells) from the plug-flow start; "
                  f"{t2 - t1:.1f} s stepping, {t1 - t0:.1f} s equilibrium init not counted",
        "status": int(st),
        "single_thread": {"value": round(n1 ** 3 * s1 / (t4 - t3) / 1e6, 4), "unit": "MLUPS", "cores": 1,
                          "sample": f"{s1} FP64 oracle steps of the periodic TGV {n1}^3, {t4 - t3:.1f} s",
                          "status": int(st1)},
        "host": {"cpu": _cpu_model(), "logical_cpus": os.cpu_count()},
    }


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16s", "bf16s"])
    ap.add_argument("--serving", default="full", choices=["off", "reduced", "full"])
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-stability", action="store_true")
    ap.add_argument("--no-probe", action="store_true")
    ap.add_argument("--no-finest", action="store_true")
    ap.add_argument("--no-regime", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU path: "
              "the single-domain update runs on one MI355X and independent requests would be sharded per GPU.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2204_10566_amd import capi
    from paper_2204_10566_amd import inputs as I

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    cfg = I.nozzle_config("re500")
    for k in ("uin", "u0"):
        cfg[k] = cfg[k].astype(np.float32)
    log(f"nozzle 96x96x768 re500 tau={cfg['tau']:.6f} storage={args.storage} steps={args.steps} "
        f"warmup={args.warmup}")
    info, ms, rc, rho, u = time_steps(capi, torch, cfg, args.storage, args.steps, args.warmup, stream)
    n_upd = int(info.n_updated)
    ms_step = ms / args.steps
    mlups = n_upd * args.steps / (ms * 1e-3) / 1e6
    all_mlups = info.ncells * args.steps / (ms * 1e-3) / 1e6
    bpc = int(info.bytes_per_cell_update)
    achieved = n_upd * bpc / (ms_step * 1e-3) / 1e9
    log(f"{args.storage}: {ms_step * 1e3:.2f} us/step, {mlups:.0f} fluid MLUPS, {achieved:.0f} GB/s algorithmic, "
        f"status {rc}")
    traffic_bytes = read_traffic("step", args.storage, "nozzle96x96x768")
    traffic = None if traffic_bytes is None else round(traffic_bytes / (ms_step * 1e-3) / 1e9, 2)
    copy = copy_ceiling(torch, stream, n_upd * bpc)
    log(f"plain copy of {copy['bytes_per_copy'] / 1e6:.0f} MB: {copy['gbs']:.0f} GB/s")

    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "fp32" else f"f32 compute, {args.storage} storage",
        "data": "synthetic",
        "config": {
            "workload": "synthetic sudden-expansion nozzle 96x96x768 (x axial), Re 500, FP32 populations, "
                        "halfway bounce-back, Poiseuille velocity inlet, zero-gradient outlet",
            "cells": int(info.ncells),
            "fluid_cells": n_upd,
            "tiles": int(info.n_tiles),
            "wall_tiles": int(info.n_wall_tiles),
            "tau": round(cfg["tau"], 8),
            "storage": args.storage,
            "all_cell_mlups": round(all_mlups, 2),
            "status": int(rc),
            "max_abs_u": float(np.abs(u).max()),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_stream_collide + k_local_collide (alternating; average launch)",
            "achieved": round(achieved, 2),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "traffic_bytes_per_launch": traffic_bytes,
            "algorithmic_bytes_per_launch": n_upd * bpc,
            "bytes_per_fluid_cell": bpc,
            "copy_ceiling_gbs": copy["gbs"],
            "frac_of_copy": round(achieved / copy["gbs"], 4),
            "per_kernel_rocprof": read_kernel_profile(args.storage, "nozzle96x96x768"),
        },
    }
    if not args.no_variants and args.storage == "fp32":
        var = {}
        for st in ("fp16s", "bf16s"):
            vsteps = max(200, args.steps // 4)
            vinfo, vms, vrc, _, _ = time_steps(capi, torch, cfg, st, vsteps, args.warmup, stream)
            v = n_upd * vsteps / (vms * 1e-3) / 1e6
            var[st] = {"mlups": round(v, 2), "ratio_vs_fp32": round(v / mlups, 3),
                       "achieved_gbs": round(n_upd * vinfo.bytes_per_cell_update / (vms / vsteps * 1e-3) / 1e9, 1),
                       "steps": vsteps, "status": int(vrc)}
            log(f"{st}: {v:.0f} fluid MLUPS ({v / mlups:.2f}x fp32)")
        for order in (2, 3):
            vsteps = max(200, args.steps // 4)
            vinfo, vms, vrc, _, _ = time_steps(capi, torch, cfg, "fp32", vsteps, args.warmup, stream, order)
            v = n_upd * vsteps / (vms * 1e-3) / 1e6
            var[f"fp32_equilibrium_order_{order}"] = {"mlups": round(v, 2), "ratio_vs_fp32": round(v / mlups, 3),
                                                       "steps": vsteps, "status": int(vrc)}
            log(f"fp32, explicit equilibrium of order {order}: {v:.0f} fluid MLUPS ({v / mlups:.2f}x)")
        out["variants"] = var
    if not args.no_precision:
        log("precision: storage formats against the FP64 reference; re6500 full-size speed")
        out["precision"] = precision_leg(capi, torch, stream)
    if not args.no_probe:
        log("roofline probe: periodic TGV 320^3")
        out["roofline_probe"] = roofline_probe_leg(capi, torch, stream)
    if not args.no_finest:
        log("finest grid: the nozzle at 155x155x3093")
        out["finest_grid"] = finest_grid_leg(capi, torch, stream)
    if not args.no_regime:
        log("the paper's own parameters on the R1 grid")
        out["paper_regime"] = paper_regime_leg(capi)
    if not args.no_stability:
        log("stability envelope (double shear layer)")
        out["stability"] = stability_leg(capi, stream)
    if not args.no_batched:
        log("batched: 64 domains, packed vs serial")
        out["batched"] = batched_leg()
        log(f"batched: {out['batched']}")
    if args.serving != "off":
        log(f"serving ({args.serving} trace)")
        out["serving"] = serving_leg(args.serving == "full")
    if not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle)")
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
