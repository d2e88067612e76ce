"""Continuous-batching service of many independent lattice Boltzmann solves.

Requests (nozzle-like solves of different grid sizes and step counts) arrive
over time.  Host-side preparation (voxel flags, inlet profile, domain
creation and upload) runs on a worker pool; the serving thread admits
prepared domains first-come-first-served while the batch's HBM budget has
room, advances every resident domain with packed, graph-replayed launches
(cache-blocked groups of domains per window of steps), and hands finished domains back to the
pool, which copies their density and velocity to the host.  A domain's state
stays on the device from admission to completion.  The same trace can be
served one solve at a time for comparison.

Latency of a request = time from its arrival to its result on the host.
"""
from __future__ import annotations

import argparse
import collections
import concurrent.futures as cf
import json
import math
import sys
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import capi
from . import inputs as I


@dataclass
class Outcome:
    rid: int
    arrival: float
    admitted: float = math.nan
    done: float = math.nan
    status: int = 0
    updated_cells: int = 0
    steps: int = 0
    rho: np.ndarray | None = field(default=None, repr=False)
    u: np.ndarray | None = field(default=None, repr=False)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


_timing_lock = threading.Lock()
_timing = collections.Counter()


def _account(key, t0):
    with _timing_lock:
        _timing[key] += time.perf_counter() - t0


def prepare(req: I.Request, storage: str, stream=None) -> capi.Domain:
    t0 = time.perf_counter()
    b = req.build()
    _account("build_inputs_s", t0)
    t1 = time.perf_counter()
    d = capi.Domain(b["flags"], periodic=0, storage=storage, stream=stream)
    d.set_params(b["tau"], 1.0 / b["tau"], 1.0)
    d.set_inlet_cells(b["uin_cells"])
    d.init_fields()
    _account("create_domain_s", t1)
    return d


def estimate_device_bytes(req: I.Request, storage: str) -> int:
    """Device memory a request will hold once prepared, before it is: its
    population array plus at most 12 bytes per cell of tables (flags, tile
    records, link masks and inlet data of the wall tiles)."""
    nz = req.nozzle
    st = capi.STORAGE[storage]
    return int(capi.lbm_array_bytes(nz.length, nz.n, nz.n, st)) + 12 * req.ncells


def _failed_code(exc: BaseException) -> int:
    return exc.code if isinstance(exc, capi.LbmError) else capi.ERR_DEVICE


def finish(d: capi.Domain, keep_fields: bool):
    """Copy the result to the host and free the domain.  Returns (status, rho,
    u, updated cells); status is LBM_ERR_UNSTABLE if any step went unstable."""
    t0 = time.perf_counter()
    status = d.step_status(0)
    rho, u = d.moments()
    info = d.info()
    d.destroy()
    if not keep_fields:
        rho, u = None, None
    _account("finish_s", t0)
    return status, rho, u, int(info.n_updated)


def percentiles(lat):
    a = np.asarray(lat)
    return float(np.percentile(a, 50)), float(np.percentile(a, 99))


def summarise(mode, outs, wall, budget=None):
    lat = [o.latency for o in outs]
    p50, p99 = percentiles(lat)
    upd = sum(o.updated_cells * o.steps for o in outs if o.status == 0)
    with _timing_lock:
        host = {k: round(v, 3) for k, v in _timing.items()}
        _timing.clear()
    return {
        "host_time_s": host,
        "mode": mode,
        "requests": len(outs),
        "unstable": sum(1 for o in outs if o.status != 0),
        "p50_s": round(p50, 4),
        "p99_s": round(p99, 4),
        "mean_s": round(float(np.mean(lat)), 4),
        "makespan_s": round(wall, 3),
        "fluid_mlups": round(upd / wall / 1e6, 1),
        "budget_bytes": budget,
    }


# Default cap on the updated cells resident in the batch at once.  The
# packed FP16 step reaches its full throughput at about 2 M resident cells
# (a 128^3 periodic box already runs as fast as a 320^3 one), so more resident
# work only stretches every solve, the longest most: on the reduced trace
# (60 and 120 requests, two runs each) a cap of 3 M cells gave p50 and p99
# below both the uncapped batch and one-at-a-time serving.
DEFAULT_WORK_CAP_CELLS = 3_000_000


def serve_continuous(trace, storage="fp16s", budget_bytes=None, steps_per_tick=16, max_ahead=2, workers=4,
                     keep_fields=False, realtime=True, work_cap_cells=DEFAULT_WORK_CAP_CELLS, order="fifo"):
    """Serve a trace with continuous batching.  Returns (outcomes, summary).

    Admission is limited by the HBM budget and, unless work_cap_cells is
    None or 0, by the number of updated cells resident at once (a request
    larger than the cap is still admitted when nothing else is resident).
    order: "fifo" admits in arrival order, "sjf" admits the waiting request
    with the least work (updated cells x steps) first.

    Every byte of device memory the service holds counts against the
    budget: a request is prepared (its domain created on the device) only
    while the resident domains, the prepared ones waiting for admission and
    those being prepared (at an upper estimate) leave room for it; until
    then it waits as a host-side description.  A request that can never fit
    the budget, or whose preparation fails, is answered at once with the
    error code as its status; the service goes on."""
    import torch

    if budget_bytes is None:
        free, _ = torch.cuda.mem_get_info()
        budget_bytes = int(min(288e9, 0.85 * free))
    batch = capi.Batch(budget_bytes, storage)
    pool = cf.ThreadPoolExecutor(max_workers=workers)
    reqs = sorted(trace, key=lambda r: r.arrival)
    outs = {r.rid: Outcome(r.rid, r.arrival, steps=r.steps) for r in reqs}
    nxt = 0
    arrived = collections.deque()    # requests that arrived, not yet being prepared
    preparing = collections.deque()  # (req, future, estimated bytes) in arrival order
    prep_bytes = 0                   # estimates of the requests being prepared
    waiting = collections.deque()    # (req, domain, cells, bytes) prepared, not yet admitted
    wait_bytes = 0                   # device bytes of the prepared, waiting domains
    resident = {}                    # slot -> (req, domain, updated cells, device bytes)
    resident_cells = 0
    peak_cells = 0                   # most updated cells resident at once
    idle_ticks = 0                   # loop turns with nothing resident
    finishing = []                   # (req, future, device bytes)
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    remaining = len(reqs)
    fin_bytes = 0                    # device bytes of released domains not yet read back and freed
    peak_held = 0                    # most device bytes held at once (resident, released, waiting, preparing)

    def fail_request(r, code):
        nonlocal remaining
        o = outs[r.rid]
        o.done, o.status = now(), code
        remaining -= 1

    try:
        while remaining:
            t = now()
            while nxt < len(reqs) and (not realtime or reqs[nxt].arrival <= t):
                arrived.append(reqs[nxt])
                nxt += 1
            # prepare arrived requests in order while the budget has room
            while arrived:
                r = arrived[0]
                est = estimate_device_bytes(r, storage)
                if est > budget_bytes:
                    arrived.popleft()
                    fail_request(r, capi.ERR_OOM)
                    continue
                in_use = batch.stats()[3]
                if in_use + fin_bytes + wait_bytes + prep_bytes + est > budget_bytes:
                    break
                arrived.popleft()
                preparing.append((r, pool.submit(prepare, r, storage), est))
                prep_bytes += est
                peak_held = max(peak_held, in_use + fin_bytes + wait_bytes + prep_bytes)
            while preparing and preparing[0][1].done():
                r, fut, est = preparing.popleft()
                prep_bytes -= est
                try:
                    d = fut.result()
                except Exception as exc:  # the request fails, the service goes on
                    fail_request(r, _failed_code(exc))
                    continue
                info = d.info()
                waiting.append((r, d, int(info.n_updated), int(info.device_bytes)))
                wait_bytes += int(info.device_bytes)
            if order == "sjf" and len(waiting) > 1:
                waiting = collections.deque(sorted(waiting, key=lambda e: e[2] * e[0].steps))
            while waiting:
                r, d, nupd, nbytes = waiting[0]
                if work_cap_cells and resident and resident_cells + nupd > work_cap_cells:
                    break
                slot = batch.admit(d, r.steps)
                if slot is None:
                    break
                waiting.popleft()
                wait_bytes -= nbytes
                resident[slot] = (r, d, nupd, nbytes)
                resident_cells += nupd
                peak_cells = max(peak_cells, resident_cells)
                outs[r.rid].admitted = now()
            _, enq, done, _ = batch.stats()
            if resident and enq - done < max_ahead * steps_per_tick:
                batch.step(steps_per_tick)
            elif not resident:
                idle_ticks += 1
            for slot in batch.poll():
                r, d, nupd, nbytes = resident.pop(slot)
                resident_cells -= nupd
                batch.release(slot)
                fin_bytes += nbytes
                finishing.append((r, pool.submit(finish, d, keep_fields), nbytes))
            still = []
            for r, fut, nbytes in finishing:
                if fut.done():
                    fin_bytes -= nbytes
                    try:
                        st, rho, u, nupd = fut.result()
                    except Exception as exc:
                        fail_request(r, _failed_code(exc))
                        continue
                    o = outs[r.rid]
                    o.done, o.status, o.rho, o.u, o.updated_cells = now(), st, rho, u, nupd
                    remaining -= 1
                else:
                    still.append((r, fut, nbytes))
            finishing = still
            if not resident or enq - done >= max_ahead * steps_per_tick:
                time.sleep(2e-4)
    finally:
        pool.shutdown(wait=True)
        batch.destroy()
    wall = now()
    res = [outs[r.rid] for r in reqs]
    s = summarise("continuous-batching", res, wall, budget_bytes)
    s["work_cap_cells"] = work_cap_cells
    s["peak_resident_cells"] = peak_cells
    s["peak_held_bytes"] = peak_held
    s["order"] = order
    s["idle_loop_turns"] = idle_ticks
    return res, s


def serve_serial(trace, storage="fp16s", workers=4, keep_fields=False, realtime=True):
    """Serve a trace one solve at a time (preparation of later requests still
    overlaps on the worker pool)."""
    pool = cf.ThreadPoolExecutor(max_workers=workers)
    reqs = sorted(trace, key=lambda r: r.arrival)
    outs = []
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    futures = {}
    nxt = 0
    try:
        for r in reqs:
            if realtime:  # the device is idle until this request arrives
                time.sleep(max(0.0, r.arrival - now()))
            while nxt < len(reqs) and (not realtime or reqs[nxt].arrival <= now()):
                futures[reqs[nxt].rid] = pool.submit(prepare, reqs[nxt], storage)
                nxt += 1
            try:
                d = futures.pop(r.rid).result()
            except Exception as exc:  # the request fails, the service goes on
                outs.append(Outcome(r.rid, r.arrival, steps=r.steps, done=now(), status=_failed_code(exc)))
                continue
            o = Outcome(r.rid, r.arrival, steps=r.steps, admitted=now())
            st = d.step_status(r.steps)
            st2, o.rho, o.u, o.updated_cells = finish(d, keep_fields)
            o.status = st if st != 0 else st2
            o.done = now()
            outs.append(o)
    finally:
        pool.shutdown(wait=True)
    wall = now()
    return outs, summarise("one-at-a-time", outs, wall)


def run_packed(specs, storage="fp16s", steps=None, budget_bytes=None):
    """Advance independent periodic/channel domains together (packed launches)
    and one after another; returns aggregate MLUPS of both.  The packed time
    includes the admissions (also reported alone); each timing ends when the
    last domain's last step has completed."""
    import torch

    def build(s):
        d = capi.Domain(s.flags, periodic=s.periodic, storage=storage)
        d.set_params(s.tau, 1.0 / s.tau, 1.0)
        d.init_fields(None, s.u)
        return d

    nsteps = [steps or s.steps for s in specs]
    upd = sum(s.ncells * n for s, n in zip(specs, nsteps))
    # Warm-up, untimed: the smallest domain through both paths once, so that
    # neither timing holds the process's one-time costs of a kernel's first
    # use (graph capture and launch of the packed kernels take tens of ms
    # the first time in a process, a few hundred microseconds after).
    small = min(specs, key=lambda s: s.ncells)
    d = build(small)
    d.step(130)
    d.destroy()
    d = build(small)
    b = capi.Batch(int(d.info().device_bytes) + (1 << 26), storage)
    slot = b.admit(d, 16)
    b.step(16)
    assert b.poll(wait=True) == [slot]
    b.release(slot)
    b.destroy()
    d.destroy()
    torch.cuda.synchronize()
    # one after another
    doms = [build(s) for s in specs]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for d, n in zip(doms, nsteps):
        d.step(n)
    serial = time.perf_counter() - t
    for d in doms:
        d.destroy()
    # packed
    doms = [build(s) for s in specs]
    if budget_bytes is None:
        budget_bytes = sum(int(d.info().device_bytes) for d in doms) + (1 << 30)
    b = capi.Batch(budget_bytes, storage)
    t = time.perf_counter()
    slots = [b.admit(d, n) for d, n in zip(doms, nsteps)]
    admit = time.perf_counter() - t
    assert all(s is not None for s in slots)
    total = max(nsteps)
    for k in range(0, total, 64):
        b.step(min(64, total - k))
    assert set(b.poll(wait=True)) == set(slots)
    packed = time.perf_counter() - t
    for s in slots:
        b.release(s)
    b.destroy()
    for d in doms:
        d.destroy()
    return {"domains": len(specs), "cells": int(sum(s.ncells for s in specs)), "cell_updates": int(upd),
            "serial_s": round(serial, 4), "packed_s": round(packed, 4), "packed_admission_s": round(admit, 4),
            "serial_mlups": round(upd / serial / 1e6, 1), "packed_mlups": round(upd / packed / 1e6, 1),
            "speedup": round(serial / packed, 3)}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--steps-scale", type=float, default=1.0)
    ap.add_argument("--storage", default="fp16s")
    ap.add_argument("--policies", default="fifo",
                    help="comma-separated continuous-batching policies: fifo, sjf, fifo@CELLS, sjf@CELLS "
                         f"(CELLS caps resident updated cells, default {DEFAULT_WORK_CAP_CELLS:.0e}; @0 for no cap)")
    ap.add_argument("--no-serial", action="store_true")
    args = ap.parse_args(argv)
    import torch

    torch.cuda.set_device(0)
    tr = I.serving_trace(count=args.requests, rate=args.rate,
                         steps_lo=max(1, int(1000 * args.steps_scale)), steps_hi=max(1, int(5000 * args.steps_scale)))
    out = {}
    for pol in args.policies.split(","):
        order, _, cap = pol.partition("@")
        wc = int(float(cap)) if cap else DEFAULT_WORK_CAP_CELLS
        _, s = serve_continuous(tr, storage=args.storage, order=order, work_cap_cells=wc or None)
        out[f"continuous_{pol}"] = s
        print(json.dumps(s), file=sys.stderr, flush=True)
    if not args.no_serial:
        _, out["serial"] = serve_serial(tr, storage=args.storage)
        print(json.dumps(out["serial"]), file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
