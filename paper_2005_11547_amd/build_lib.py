"""Build the HIP library libdms.so in-tree (gfx950 only)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libdms.so")
SOURCES = ["dms_api.cpp", "dms_constants.cpp", "dms_plain.hip", "dms_sketch.hip", "dms_estimate.hip",
           "dms_calib.hip", "dms_search.hip", "dms_bbit.hip", "dms_index.hip", "dms_order.hip", "dms_validate.hip", "dms_noalloc.hip",
           "dms_server.cpp", "dms_db.cpp"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-fno-fast-math", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    procs = []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(bdir, s + ".o")
        # kernels are HIP; the host-side runtime files are plain C++ against the HIP runtime API
        lang = ["-x", "hip"] if s.endswith(".hip") else ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
        cmd = ["hipcc"] + FLAGS + lang + ["-c", src, "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = False
    for cmd, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if verbose or p.returncode:
            sys.stderr.write(text)
        if p.returncode:
            failed = True
            sys.stderr.write("FAILED: %s\n" % " ".join(cmd))
    if failed:
        raise RuntimeError("HIP build failed")
    tmp = OUT + ".tmp%d" % os.getpid()
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
