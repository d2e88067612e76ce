"""Build the gfx950 shared library liblbm.so in-tree with hipcc.

The kernels of each storage format are compiled in their own translation
units (csrc/lbm_kern.hip with LBM_KERN_ST = 0, 1, 2; LBM_KERN_WIDE = 1 for
the step kernels of arrays past 4 GiB), in parallel with the host
translation unit (csrc/lbm.hip), and linked into one library.

Usage: python -m paper_2204_10566_amd.build  (or build() from Python).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
OBJ_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-result",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]

# (source, extra flags, object)
UNITS = [
    ("lbm.hip", [], "lbm_host.o"),
    ("lbm_kern.hip", ["-DLBM_KERN_ST=0"], "lbm_kern_fp32.o"),
    ("lbm_kern.hip", ["-DLBM_KERN_ST=1"], "lbm_kern_fp16s.o"),
    ("lbm_kern.hip", ["-DLBM_KERN_ST=2"], "lbm_kern_bf16s.o"),
    ("lbm_kern.hip", ["-DLBM_KERN_ST=0", "-DLBM_KERN_WIDE=1"], "lbm_kern_fp32_wide.o"),
    ("lbm_kern.hip", ["-DLBM_KERN_ST=1", "-DLBM_KERN_WIDE=1"], "lbm_kern_fp16s_wide.o"),
    ("lbm_kern.hip", ["-DLBM_KERN_ST=2", "-DLBM_KERN_WIDE=1"], "lbm_kern_bf16s_wide.o"),
]


def _filtered(text: str) -> str:
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip())


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    procs = []
    for src, extra, obj in UNITS:
        cmd = ["hipcc", *HIPCC_FLAGS, *extra, "-c", "-o", os.path.join(OBJ_DIR, obj), os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    failed = False
    for cmd, p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out + err)
            failed = True
        elif verbose and _filtered(err):
            print(_filtered(err), file=sys.stderr)
    if failed:
        raise RuntimeError("hipcc failed building liblbm.so")
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-o", tmp,
           *[os.path.join(OBJ_DIR, obj) for _, _, obj in UNITS], "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking liblbm.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
