"""Build libbblock.so for gfx950 with hipcc (in-tree, next to this file)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("bb_fast_bf16.hip", "bb_fast_fp32.hip", "bb_w3.hip", "bb_pord.hip", "bb_zgemm.hip", "bb_f64.hip", "bb_f64p.hip", "bb_f32p.hip", "bb_kernels.hip",
                                             "bb_api.hip")]
HEADERS = [os.path.join(CSRC, "bb_internal.h"), os.path.join(CSRC, "bb_fast.h"),
           os.path.join(os.path.dirname(HERE), "include", "bblock.h")]
BUILD_DIR = os.path.join(HERE, "_build")
OUT = os.path.join(HERE, "libbblock.so")

# Packed FP32 instructions are disabled for all device code.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]
NOISE = "is not a recognized feature for this target"


def _clean(stderr: str) -> str:
    return "\n".join(l for l in (stderr or "").splitlines() if NOISE not in l)


def build(verbose: bool = False) -> str:
    """Compile every translation unit (in parallel) and link libbblock.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(BUILD_DIR, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
        objs.append(obj)
        procs.append((src, subprocess.Popen([hipcc] + FLAGS + ["-c", "-o", obj, src], stdout=subprocess.PIPE,
                                            stderr=subprocess.PIPE, text=True)))
    errors = []
    for src, p in procs:
        _, err = p.communicate()
        if p.returncode != 0:
            errors.append("%s:\n%s" % (os.path.basename(src), _clean(err)))
        elif verbose and _clean(err).strip():
            print(_clean(err), file=sys.stderr)
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    tmp = OUT + ".tmp%d" % os.getpid()
    res = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs,
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + _clean(res.stderr))
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
