"""The C-ABI library loads without a GPU, exports every function the header
declares, passes its host-only self checks, and rejects bad arguments before
touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def capi():
    from paper_2204_10566_amd import capi

    return capi


def test_header_symbols_exported(capi):
    names = declared_functions()
    assert len(names) >= 20
    lib = capi.library()
    for n in names:
        assert hasattr(lib, n), n
    # the binding covers the same set
    assert set(names) == set(capi.SIGNATURES)


def test_host_selftest(capi):
    assert capi.lbm_selftest_host() == 0, capi.lbm_last_error()


def _create(capi, flags, periodic=0, storage=0):
    h = ctypes.c_void_p()
    fl = np.ascontiguousarray(flags, dtype=np.uint8)
    nz, ny, nx = fl.shape
    rc = capi.lbm_create_domain(fl.ctypes.data_as(capi._u8p), nx, ny, nz, periodic, storage, None, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("case", ["outlet_not_last_plane", "outlet_periodic_x", "bad_flag", "bad_storage",
                                  "bad_periodic"])
def test_create_rejects_bad_arguments(capi, case):
    fl = np.zeros((3, 4, 5), np.uint8)
    per, st = 0, 0
    if case == "outlet_not_last_plane":
        fl[1, 1, 2] = capi.OUTLET
    elif case == "outlet_periodic_x":
        fl[1, 1, 4] = capi.OUTLET
        per = 1
    elif case == "bad_flag":
        fl[0, 0, 0] = 9
    elif case == "bad_storage":
        st = 5
    elif case == "bad_periodic":
        per = 9
    rc, h = _create(capi, fl, per, st)
    assert rc == capi.ERR_ARG and not h.value
    assert capi.lbm_last_error()


def test_create_rejects_bad_sizes(capi):
    h = ctypes.c_void_p()
    fl = np.zeros(8, np.uint8)
    for dims in [(0, 2, 2), (2, -1, 2), (70000, 1, 1)]:
        rc = capi.lbm_create_domain(fl.ctypes.data_as(capi._u8p), *dims, 0, 0, None, ctypes.byref(h))
        assert rc == capi.ERR_ARG
    assert capi.lbm_create_domain(None, 2, 2, 2, 0, 0, None, ctypes.byref(h)) == capi.ERR_ARG


def test_too_many_cells_rejected(capi):
    """Cell indices are 32-bit: a grid of more than 2^32 - 64 cells is
    refused from its sizes, before the flags are read (so a one-byte flag
    buffer suffices here).  Arrays past 4 GiB are accepted; they step with
    the 64-bit addressing kernels (tests/test_gpu_wide.py)."""
    fl = np.zeros(1, np.uint8)
    h = ctypes.c_void_p()
    rc = capi.lbm_create_domain(fl.ctypes.data_as(capi._u8p), 65535, 65535, 2, 0, 0, None, ctypes.byref(h))
    assert rc == capi.ERR_ARG and "2^32 - 64 cells" in capi.lbm_last_error().decode()
    assert not h.value


def test_null_handles(capi):
    assert capi.lbm_step(None, 1) == capi.ERR_ARG
    assert capi.lbm_set_params(None, 0.6, 1.0, 1.0) == capi.ERR_ARG
    assert capi.lbm_destroy(None) == capi.ERR_ARG
    assert capi.lbm_batch_step(None, 1) == capi.ERR_ARG
    assert capi.lbm_batch_destroy(None) == capi.ERR_ARG
    n = ctypes.c_size_t()
    assert capi.lbm_state_bytes(None, ctypes.byref(n)) == capi.ERR_ARG
    assert capi.lbm_save_state(None, None, 0) == capi.ERR_ARG
    assert capi.lbm_load_state(None, None, 0) == capi.ERR_ARG
    assert capi.lbm_batch_set_cache_block(None, 0, 8) == capi.ERR_ARG
    assert capi.lbm_step_async(None, 1) == capi.ERR_ARG
    assert capi.lbm_step_wait(None) == capi.ERR_ARG


def test_missing_library_fails_loudly(tmp_path):
    """Without the built library the binding refuses to import (there is no
    CPU fallback for any step of the update)."""
    import subprocess
    import sys

    env = dict(os.environ, LBM_LIBRARY=str(tmp_path / "missing" / "liblbm.so"))
    r = subprocess.run([sys.executable, "-c", "import paper_2204_10566_amd.capi"], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "no CPU fallback" in r.stderr


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU; asked for more it exits with status 2 and
    says why, before touching a device."""
    import subprocess
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
