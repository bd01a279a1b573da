"""Build the HIP library libtwoscale.so for gfx950 (in-tree, no JIT cache).

Every source is compiled by hipcc as HIP for gfx950 only.  Packed FP32
instructions are disabled in the device code generation.
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libtwoscale.so")
SOURCES = ["ts_topology.cpp", "ts_api.cpp", "k_stencil.hip", "k_misc.hip"]
# the surrogate volume kernel, one unit per (degree q, staging width kpt);
# q = 0 is the constant stencil
INST = [(q, k) for q in (0, 1, 2, 3, 4) for k in (2, 4, 8)]
# the IFEM volume kernel, one unit per staging width (levels up to 8)
IFEM_KPT = (2, 4)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wno-unused-command-line-argument",
]


def build(jobs=8, verbose=True, lib_path=LIB, defines=(), build_dir=None):
    """Compile all sources (always) and link the shared library.

    defines: extra preprocessor definitions (tuning constants such as
    TS_VOL_R, TS_VOL_WAVES) for experiments."""
    bdir = build_dir or os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    units = [(s, os.path.join(bdir, os.path.splitext(s)[0] + ".o"), []) for s in SOURCES]
    units += [("k_surr_inst.hip", os.path.join(bdir, "k_surr_q%d_k%d.o" % (q, k)),
               ["TS_Q=%d" % q, "TS_KPT=%d" % k]) for q, k in INST]
    units += [("k_ifem.hip", os.path.join(bdir, "k_ifem_k%d.o" % k), ["TS_KPT=%d" % k])
              for k in IFEM_KPT]
    objs = [u[1] for u in units]
    procs = []
    for src, obj, extra in units:
        cmd = ([HIPCC] + FLAGS + ["-D" + d for d in list(defines) + extra] +
               ["-c", os.path.join(CSRC, src), "-o", obj])
        if verbose:
            print("[build]", os.path.basename(obj), flush=True)
        procs.append(subprocess.Popen(cmd))
        while len([p for p in procs if p.poll() is None]) >= jobs:
            time.sleep(0.2)
    rc = [p.wait() for p in procs]
    if any(rc):
        raise RuntimeError("hipcc failed for " + ", ".join(u[1] for u, r in zip(units, rc) if r))
    tmp = lib_path + ".tmp"
    subprocess.check_call([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, lib_path)
    return lib_path


if __name__ == "__main__":
    build()
    print(LIB)
    sys.exit(0)
