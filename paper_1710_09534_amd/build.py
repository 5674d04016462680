"""Builds the HIP library ``libtlb.so`` in-tree for gfx950 with hipcc.

    python -m paper_1710_09534_amd.build            # build
    python -m paper_1710_09534_amd.build --resources  # also print VGPR/LDS use
    python -m paper_1710_09534_amd.build --sanitize   # libtlb_hostsan.so: host code
                                                      # with AddressSanitizer and UBSan

The sanitized library instruments host code only (each -fsanitize flag is
scoped to the host compilation by -Xarch_host; device code is built as
usual).  It is for the CPU tests of the C ABI, run with the sanitizer runtime
preloaded and TLB_LIBRARY pointing at it (tests/test_host_sanitizers.py).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtlb.so")
SAN_LIB = os.path.join(HERE, "libtlb_hostsan.so")
SOURCES = ["tlb_kernels.hip", "tlb_host.cpp", "tlb_server.cpp", "tlb3d_kernels.hip", "tlb3d_host.cpp",
           "tlb_probe.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 arithmetic is disabled: some of its forms have given wrong results
# on gfx950 without any error, in ways tests do not reliably show.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument", "-munsafe-fp-atomics"]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def build(resources: bool = False, verbose: bool = False, sanitize: bool = False) -> str:
    objs = []
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    extra = SAN_FLAGS if sanitize else []
    tag = ".san" if sanitize else ""
    for src in sources():
        obj = os.path.join(CSRC, os.path.basename(src) + tag + ".o")
        cmd = [HIPCC] + HIP_FLAGS + extra + inc + ["-c", src, "-o", obj]
        if src.endswith(".hip"):
            cmd = [HIPCC, "-x", "hip"] + HIP_FLAGS + extra + inc + ["-c", src, "-o", obj]
            if resources:
                cmd.insert(1, "-Rpass-analysis=kernel-resource-usage")
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        objs.append(obj)
    out = SAN_LIB if sanitize else LIB
    tmp = out + ".tmp%d" % os.getpid()
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp]
    if sanitize:
        link += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-shared-libsan"]
    subprocess.run(link + objs, check=True)
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    return out


if __name__ == "__main__":
    print(build(resources="--resources" in sys.argv, verbose="-v" in sys.argv,
                sanitize="--sanitize" in sys.argv))
