"""Register budget of the contraction kernels, read from the code objects of
the built library (no GPU needed).

The contraction kernels keep their accumulators and the operands in flight in
registers; a change that makes the compiler spill them to scratch memory
(private segment) slows a kernel by 10-20 % without changing any result, so
no parity test would notice.  This test reads each kernel's private segment
size from the AMDGPU metadata notes and holds the hot kernels to their
budgets."""
from __future__ import annotations

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2211_16278_amd", "libbblock.so")
LLVM = "/opt/rocm/llvm/bin"

# Private segment bytes per lane allowed for each kernel family (mangled-name
# prefix): none for the FP64 kernel and the BF16X3 contraction kernels, a few
# spilled values outside the main loop for the others.
BUDGET = {
    "_ZN2bb3f648contract": 0,       # FP64 kernel 5
    "_ZN2bb2w39contract8": 0,       # BF16X3 kernel 4
    "_ZN2bb2w38contract": 64,       # BF16X3 kernel 2
    "_ZN2bb4fast7bb_fastILi1": 160,  # FP32 kernel 1
    "_ZN2bb4pord8contract": 160,    # BF16X3 kernel 3 (its zero-momentum form: 132)
    "_ZN2bb4f64p8contract": 0,      # FP64 kernel 6
    "_ZN2bb4f32p8contract": 32,     # FP32 kernel 7 (two fragments in 128 VGPRs: 12-28)
}


# Kernels the planner runs two workgroups of 512 threads per CU: at most 128
# VGPRs each (four waves per SIMD), or the second workgroup does not fit and
# the planner's wave-filling split counts leave a second, mostly empty wave.
TWO_PER_CU = ("_ZN2bb4f32p8contractILi1ELi16E", "_ZN2bb4f32p8contractILi2ELi16E")


def kernel_scratch(tmp_path):
    lib = tmp_path / "libbblock.so"
    shutil.copy(LIB, lib)
    # Unbundles next to the copy: one host and one gfx950 object per source.
    subprocess.run([os.path.join(LLVM, "llvm-objdump"), "--offloading", str(lib)], check=True,
                   capture_output=True, cwd=tmp_path)
    sizes = {}
    objs = [p for p in os.listdir(tmp_path) if p.endswith("gfx950")]
    assert objs, "no gfx950 code object in the library"
    for obj in objs:
        notes = subprocess.run([os.path.join(LLVM, "llvm-readelf"), "--notes", str(tmp_path / obj)], check=True,
                               capture_output=True, text=True).stdout
        name = None
        for line in notes.splitlines():
            m = re.match(r"\s+\.name:\s+(\S+)", line)
            if m:
                name = m.group(1)
                continue
            m = re.match(r"\s+\.private_segment_fixed_size:\s+(\d+)", line)
            if m and name:
                sizes[name] = [int(m.group(1)), None]
                continue
            m = re.match(r"\s+\.vgpr_count:\s+(\d+)", line)
            if m and name in sizes:
                sizes[name][1] = int(m.group(1))
                name = None
    return sizes


@pytest.mark.skipif(not os.path.exists(LIB) or not os.path.exists(os.path.join(LLVM, "llvm-readelf")),
                    reason="library not built or LLVM tools missing")
def test_contraction_kernels_within_register_budget(tmp_path):
    sizes = kernel_scratch(tmp_path)
    over = []
    for prefix, budget in BUDGET.items():
        found = {k: v[0] for k, v in sizes.items() if k.startswith(prefix)}
        assert found, "no kernel %s in the library" % prefix
        over += ["%s: %d bytes (budget %d)" % (k, v, budget) for k, v in found.items() if v > budget]
    for prefix in TWO_PER_CU:
        found = {k: v[1] for k, v in sizes.items() if k.startswith(prefix)}
        assert found, "no kernel %s in the library" % prefix
        over += ["%s: %s VGPRs (two workgroups per CU need at most 128)" % (k, v) for k, v in found.items()
                 if v is None or v > 128]
    assert not over, "kernels over their register budget:\n" + "\n".join(sorted(over))
