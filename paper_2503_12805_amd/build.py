"""Build the HIP library libwke (gfx950) in-tree.

    python -m paper_2503_12805_amd.build

compiles csrc/*.hip with hipcc for --offload-arch=gfx950 and links
paper_2503_12805_amd/_wke.so.  Packed-FP32 instruction selection is switched
off (-packed-fp32-ops); hipcc's host pass warns that it does not know that
target feature, which is harmless.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "_wke.so")
BUILD_DIR = os.path.join(ROOT, "_build")
SOURCES = ["wke_kernels.hip", "wke_api.hip", "wke_exact.hip", "wke_layout.cpp"]
ARCH = os.environ.get("WKE_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the wke library needs ROCm's hipcc")


def flags():
    return ["-O3", "--offload-arch=" + ARCH, "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + INCLUDE, "-I" + CSRC]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    cc = hipcc()
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [cc] + flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), cmd))
        objs.append(obj)
    for p, cmd in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # drop the host pass's note about the device-only target feature
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            sys.stderr.write("\n".join(lines) + "\n")
            raise RuntimeError("hipcc failed: " + " ".join(cmd))
        if verbose and lines:
            print("\n".join(lines))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([cc, "-shared", "--offload-arch=" + ARCH] + objs + ["-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
