"""ctypes binding of liblbm.so (declared in include/lbm.h).

Argument marshalling only: every step of the update runs in the library's HIP
kernels.  The functions keep the C names; ``Domain`` and ``Batch`` are small
conveniences over them that check status codes.  Importing this module fails
loudly when the built library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBM_LIBRARY") or os.path.join(HERE, "liblbm.so")

FLUID, SOLID, INLET, OUTLET = 0, 1, 2, 3
FP32, FP16S, BF16S = 0, 1, 2
STORAGE = {"fp32": FP32, "fp16s": FP16S, "bf16s": BF16S}
OUTLETS = {"zero_gradient": 0, "pressure": 1}
OK, ERR_ARG, ERR_OOM, ERR_DEVICE, ERR_UNSTABLE, ERR_STATE = 0, -1, -2, -3, -4, -5
Q = 27


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


class DomainInfo(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("storage", ctypes.c_int), ("periodic", ctypes.c_uint),
        ("ncells", ctypes.c_uint64), ("plane_stride", ctypes.c_uint64),
        ("n_updated", ctypes.c_uint64), ("n_tiles", ctypes.c_uint64),
        ("n_wall_tiles", ctypes.c_uint64), ("n_inlet", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64),
        ("bytes_per_cell_update", ctypes.c_uint64),
    ]


_vp = ctypes.c_void_p
_ip = ctypes.POINTER(ctypes.c_int)
_fp = ctypes.POINTER(ctypes.c_float)
_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)

# name -> (restype, argtypes); the exported C ABI
SIGNATURES = {
    "lbm_create_domain": (ctypes.c_int, [_u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint, ctypes.c_int,
                                         _vp, ctypes.POINTER(_vp)]),
    "lbm_create_domain_ext": (ctypes.c_int, [_u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint,
                                             ctypes.c_int, _vp, _vp, ctypes.POINTER(_vp)]),
    "lbm_set_params": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "lbm_set_rates": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "lbm_set_order_rates": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "lbm_set_outlet": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double]),
    "lbm_set_wall_distances": (ctypes.c_int, [_vp, _fp]),
    "lbm_set_inlet": (ctypes.c_int, [_vp, _fp]),
    "lbm_set_inlet_cells": (ctypes.c_int, [_vp, _fp]),
    "lbm_init_fields": (ctypes.c_int, [_vp, _fp, _fp]),
    "lbm_step": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lbm_step_async": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lbm_step_wait": (ctypes.c_int, [_vp]),
    "lbm_prepare_steps": (ctypes.c_int, [_vp]),
    "lbm_get_moments": (ctypes.c_int, [_vp, _fp, _fp]),
    "lbm_get_moments_device": (ctypes.c_int, [_vp, _vp, _vp]),
    "lbm_get_moments_noalloc": (ctypes.c_int, [_vp, _fp, _fp]),
    "lbm_set_equilibrium_order": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lbm_debug_fail_after": (ctypes.c_int, [ctypes.c_int]),
    "lbm_debug_wide_addressing": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lbm_debug_step_grid": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lbm_is_wide": (ctypes.c_int, [_vp, _ip]),
    "lbm_get_populations": (ctypes.c_int, [_vp, _fp]),
    "lbm_set_populations": (ctypes.c_int, [_vp, _fp]),
    "lbm_state_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_save_state": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "lbm_load_state": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "lbm_domain_get_info": (ctypes.c_int, [_vp, ctypes.POINTER(DomainInfo)]),
    "lbm_stats_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lbm_stats_get": (ctypes.c_int, [_vp, _dp, _dp, _dp, ctypes.POINTER(ctypes.c_uint64)]),
    "lbm_destroy": (ctypes.c_int, [_vp]),
    "lbm_last_error": (ctypes.c_char_p, []),
    "lbm_batch_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    "lbm_batch_admit": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _ip]),
    "lbm_batch_set_cache_block": (ctypes.c_int, [_vp, ctypes.c_size_t, ctypes.c_int]),
    "lbm_batch_step": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lbm_batch_poll": (ctypes.c_int, [_vp, ctypes.c_int, _ip, ctypes.c_int, _ip]),
    "lbm_batch_release": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(_vp)]),
    "lbm_batch_stats": (ctypes.c_int, [_vp, _ip, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                       ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_batch_destroy": (ctypes.c_int, [_vp]),
    "lbm_array_bytes": (ctypes.c_uint64, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "lbm_selftest_host": (ctypes.c_int, []),
    "lbm_version": (ctypes.c_char_p, []),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                          "python -m paper_2204_10566_amd.build (there is no CPU fallback)")
    # torch ships its own HIP runtime under the same soname as the system
    # one; loading torch first makes the library and torch share a single
    # runtime (and so share devices, streams and allocations).
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
globals().update({name: getattr(_lib, name) for name in SIGNATURES})


def library():
    return _lib


def check(code: int):
    if code != OK:
        raise LbmError(code, lbm_last_error().decode())
    return code


def _f32(a, n=None):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(a, dtype=np.float32)
    if n is not None and arr.size != n:
        raise ValueError(f"expected {n} values, got {arr.size}")
    return arr, arr.ctypes.data_as(_fp)


class Domain:
    """One simulation domain on the current HIP device."""

    def __init__(self, flags, periodic=0, storage="fp32", stream=None, array=None):
        fl = np.ascontiguousarray(flags, dtype=np.uint8)
        if fl.ndim != 3:
            raise ValueError("flags must be [nz, ny, nx]")
        self.shape = fl.shape
        nz, ny, nx = fl.shape
        st = STORAGE[storage] if isinstance(storage, str) else int(storage)
        h = _vp()
        stream_p = _vp(stream) if stream else None
        if array is None:
            check(lbm_create_domain(fl.ctypes.data_as(_u8p), nx, ny, nz, periodic, st, stream_p, ctypes.byref(h)))
        else:
            check(lbm_create_domain_ext(fl.ctypes.data_as(_u8p), nx, ny, nz, periodic, st, stream_p, _vp(array),
                                        ctypes.byref(h)))
        self.h = h
        self.ncells = nx * ny * nz

    def info(self) -> DomainInfo:
        i = DomainInfo()
        check(lbm_domain_get_info(self.h, ctypes.byref(i)))
        return i

    def set_params(self, tau, omega_bulk=None, omega_high=1.0):
        check(lbm_set_params(self.h, tau, 1.0 / tau if omega_bulk is None else omega_bulk, omega_high))

    def set_rates(self, omega, omega_bulk, omega_high):
        check(lbm_set_rates(self.h, omega, omega_bulk, omega_high))

    def set_order_rates(self, omega3, omega4, omega5, omega6):
        check(lbm_set_order_rates(self.h, omega3, omega4, omega5, omega6))

    def set_equilibrium_order(self, order=6):
        """Order of the equilibrium the collision relaxes to: 6 (full, the
        paper's) or 2..5 (explicit truncated equilibrium)."""
        check(lbm_set_equilibrium_order(self.h, int(order)))

    def is_wide(self):
        """True if the step kernels address the array with 64-bit global
        instructions (arrays past 4 GiB)."""
        w = ctypes.c_int(0)
        check(lbm_is_wide(self.h, ctypes.byref(w)))
        return bool(w.value)

    def debug_wide_addressing(self, on=True):
        """Test hook: step with the 64-bit addressing kernels whatever the
        size (on=False returns to the choice by size)."""
        check(lbm_debug_wide_addressing(self.h, 1 if on else 0))

    def debug_step_grid(self, blocks=0):
        """Test hook: launch each step on `blocks` blocks (a multiple of 8;
        0 returns to one wave per tile)."""
        check(lbm_debug_step_grid(self.h, int(blocks)))

    def set_outlet(self, kind="zero_gradient", rho_out=1.0):
        """Outlet condition: "zero_gradient" or "pressure" (rho_out)."""
        check(lbm_set_outlet(self.h, OUTLETS[kind], float(rho_out)))

    def set_wall_distances(self, q=None):
        """Wall fraction of every link, [27, nz, ny, nx] (None: halfway)."""
        a, p = _f32(q, 27 * self.ncells)
        check(lbm_set_wall_distances(self.h, p))

    def set_inlet(self, uin):
        a, p = _f32(uin, 3 * self.ncells)
        check(lbm_set_inlet(self.h, p))

    def set_inlet_cells(self, u_inlet):
        """u_inlet: [3, n_inlet], inlet cells in ascending cell order."""
        a, p = _f32(u_inlet, 3 * int(self.info().n_inlet))
        check(lbm_set_inlet_cells(self.h, p))

    def init_fields(self, rho=None, u=None):
        ra, rp = _f32(rho, self.ncells)
        ua, up = _f32(u, 3 * self.ncells)
        check(lbm_init_fields(self.h, rp, up))

    def step(self, n=1):
        return check(lbm_step(self.h, int(n)))

    def step_status(self, n=1) -> int:
        return lbm_step(self.h, int(n))

    def step_async(self, n=1):
        """Enqueue n steps on the domain's stream without waiting."""
        check(lbm_step_async(self.h, int(n)))

    def wait_status(self) -> int:
        """Wait for the enqueued steps; their status code (OK or ERR_UNSTABLE)."""
        return lbm_step_wait(self.h)

    def prepare_steps(self):
        """Build the step graphs now (outside a timed run)."""
        check(lbm_prepare_steps(self.h))

    def moments(self):
        rho = np.empty(self.shape, np.float32)
        u = np.empty((3,) + self.shape, np.float32)
        check(lbm_get_moments(self.h, rho.ctypes.data_as(_fp), u.ctypes.data_as(_fp)))
        return rho, u

    def moments_device(self, rho_ptr, u_ptr):
        check(lbm_get_moments_device(self.h, _vp(rho_ptr), _vp(u_ptr)))

    def populations(self):
        f = np.empty((Q,) + self.shape, np.float32)
        check(lbm_get_populations(self.h, f.ctypes.data_as(_fp)))
        return f

    def set_populations(self, f):
        a, p = _f32(f, Q * self.ncells)
        check(lbm_set_populations(self.h, p))

    def save_state(self):
        """The domain's exact state (lbm_save_state) as a uint8 array."""
        n = ctypes.c_size_t()
        check(lbm_state_bytes(self.h, ctypes.byref(n)))
        buf = np.empty(n.value, np.uint8)
        check(lbm_save_state(self.h, buf.ctypes.data_as(_vp), buf.nbytes))
        return buf

    def load_state(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        check(lbm_load_state(self.h, buf.ctypes.data_as(_vp), buf.nbytes))

    def stats_enable(self, on=True):
        check(lbm_stats_enable(self.h, 1 if on else 0))

    def stats(self):
        """(mean u [3,...], mean u_a u_b [6,...], mean sigma [6,...], samples)."""
        mu = np.empty((3,) + self.shape, np.float64)
        muu = np.empty((6,) + self.shape, np.float64)
        ms = np.empty((6,) + self.shape, np.float64)
        n = ctypes.c_uint64()
        check(lbm_stats_get(self.h, mu.ctypes.data_as(_dp), muu.ctypes.data_as(_dp), ms.ctypes.data_as(_dp),
                            ctypes.byref(n)))
        return mu, muu, ms, int(n.value)

    def destroy(self):
        if self.h:
            check(lbm_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lbm_destroy(self.h)
        except Exception:
            pass


class Batch:
    """Packed multi-domain execution (graph-replayed launches, cache-blocked groups)."""

    def __init__(self, budget_bytes, storage="fp16s", stream=None):
        st = STORAGE[storage] if isinstance(storage, str) else int(storage)
        h = _vp()
        check(lbm_batch_create(int(budget_bytes), st, _vp(stream) if stream else None, ctypes.byref(h)))
        self.h = h

    def set_cache_block(self, group_bytes, window_steps=16):
        check(lbm_batch_set_cache_block(self.h, int(group_bytes), int(window_steps)))

    def admit(self, dom: Domain, n_steps: int):
        """Returns the slot id, or None when the budget is exhausted."""
        slot = ctypes.c_int()
        rc = lbm_batch_admit(self.h, dom.h, int(n_steps), ctypes.byref(slot))
        if rc == ERR_OOM:
            return None
        check(rc)
        return slot.value

    def step(self, n=1):
        check(lbm_batch_step(self.h, int(n)))

    def poll(self, wait=False, max_n=4096):
        buf = (ctypes.c_int * max_n)()
        n = ctypes.c_int()
        check(lbm_batch_poll(self.h, 1 if wait else 0, buf, max_n, ctypes.byref(n)))
        return [buf[k] for k in range(n.value)]

    def release(self, slot):
        d = _vp()
        check(lbm_batch_release(self.h, int(slot), ctypes.byref(d)))

    def stats(self):
        """(resident slots, steps enqueued, steps done, bytes in use)."""
        r = ctypes.c_int()
        s = ctypes.c_uint64()
        dn = ctypes.c_uint64()
        b = ctypes.c_size_t()
        check(lbm_batch_stats(self.h, ctypes.byref(r), ctypes.byref(s), ctypes.byref(dn), ctypes.byref(b)))
        return r.value, s.value, dn.value, b.value

    def destroy(self):
        if self.h:
            check(lbm_batch_destroy(self.h))
            self.h = None
