"""Build step of the HIP library ``libfch.so`` (gfx950).

Compiles ``csrc/*.hip`` with hipcc into an in-tree shared object next to this
file.  Packed FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfch.so")
# host code with AddressSanitizer and UndefinedBehaviorSanitizer (device code
# unchanged); load it with FCH_LIB and the clang ASan runtime preloaded
LIB_SAN = os.path.join(HERE, "libfch_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-shared-libsan"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["fch_capi.hip", "fch_ensemble.hip", "fch_registry.hip", "fch_kern_small.hip", "fch_nn.hip"] + [
    "fch_kern_n%d.hip" % n for n in (4096, 2048, 1024, 512, 256, 128, 64, 32, 16)]


def build(verbose: bool = True, sanitize: bool = False) -> str:
    t0 = time.time()
    objdir = os.path.join(HERE, "_build_san" if sanitize else "_build")
    extra = SAN_FLAGS if sanitize else []
    lib = LIB_SAN if sanitize else LIB
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    jobs = int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))
    for src in SOURCES:
        while sum(pr.poll() is None for _, pr in procs) >= jobs:
            time.sleep(0.2)
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-c", *extra,
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-command-line-argument",
               "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               "-o", obj, os.path.join(CSRC, src)]
        procs.append((src, subprocess.Popen(cmd, stderr=None if verbose else subprocess.DEVNULL)))
    for src, pr in procs:
        if pr.wait() != 0:
            raise RuntimeError("hipcc failed on %s" % src)
    tmp = lib + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *extra, "-o", tmp,
                           *objs])
    os.replace(tmp, lib)
    if verbose:
        print("built %s in %.1fs" % (lib, time.time() - t0), file=sys.stderr)
    return lib


if __name__ == "__main__":
    build(sanitize="--sanitize" in sys.argv)
