"""Host-side accounting of bench.py (no GPU): the flop counts behind the
roofline objects and the kernel names the profile summaries are matched by.

The counts follow the per-block figures of the method: F_gemm = 24 N_mom V
n^3 for the fused contraction (8 real flops per complex multiply-add over
K = 3 V), F_alg = 42 V n^2 + (22 + 8 N_mom) V n^3 for the paper's order
(diquark, singlet, projection)."""
from __future__ import annotations

import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402
from paper_2211_16278_amd import synth  # noqa: E402


def test_flop_counts_at_the_headline():
    V, n, n_mom = 32 ** 3, 32, 7
    f_gemm, f_alg = bench.flops(V, n, n, n, n_mom)
    assert f_gemm == 24 * 7 * V * n ** 3
    assert f_alg == 42 * V * n * n + (22 + 8 * 7) * V * n ** 3
    assert abs(f_gemm - 1.804e11) / 1.804e11 < 1e-3
    assert abs(f_alg - 8.52e10) / 8.52e10 < 1e-3


def test_executed_flops_per_kernel():
    V, n = 32 ** 3, 32
    vn3 = V * n ** 3
    f_gemm = 24.0 * 7 * vn3
    # Fused kernels: three BF16 passes, one FP32 pass, kernel 5's three real products.
    assert bench.executed_flops("bf16x3", {"kernel": 4, "nb": 7}, V, n, 7) == 3 * f_gemm
    assert bench.executed_flops("fp32", {"kernel": 1, "nb": 7}, V, n, 7) == f_gemm
    assert bench.executed_flops("fp64", {"kernel": 5, "nb": 7}, V, n, 7) == 0.75 * f_gemm
    # Kernel 8: 7 momenta pad to 8 in fragments of 4; kernel 6 to 16.
    vec = 23.0 * vn3 + 42.0 * V * n * n
    assert bench.executed_flops("fp64", {"kernel": 8, "nb": 2}, V, n, 7) == 6.0 * 8 * vn3 + vec
    assert bench.executed_flops("fp64", {"kernel": 6, "nb": 1}, V, n, 7) == 6.0 * 16 * vn3 + vec
    # 33 momenta with the zero one on the vector unit: 32 columns in 2 fragments of 16.
    assert bench.executed_flops("fp64", {"kernel": 6, "nb": 2}, V, n, 33, zero_off=True) == 6.0 * 32 * vn3 + vec
    assert bench.executed_flops("fp32", {"kernel": 7, "nb": 2}, V, n, 33, zero_off=True) == 6.0 * 32 * vn3
    assert bench.executed_flops("fp32", {"kernel": 7, "nb": 3}, V, n, 33) == 8.0 * 48 * vn3
    # Kernel 7 up to two fragments: three real products.
    assert bench.executed_flops("fp32", {"kernel": 7, "nb": 1}, V, n, 7) == 6.0 * 16 * vn3
    # Kernel 9: 7 momenta pad to 8 in fragments of 4; four real products above two fragments.
    assert bench.executed_flops("fp32", {"kernel": 9, "nb": 2}, V, n, 7) == 6.0 * 8 * vn3
    assert bench.executed_flops("fp32", {"kernel": 9, "nb": 3}, V, n, 10) == 8.0 * 12 * vn3


def test_zero_momentum_rule():
    L = 64
    shell = synth.momenta("shell4")   # 33, zero first
    cube = synth.momenta("cube")      # 27
    assert bench.zero_on_vector_unit({"kernel": 6, "nb": 2}, shell, L)
    assert bench.zero_on_vector_unit({"kernel": 7, "nb": 2}, shell, L)
    assert bench.zero_on_vector_unit({"kernel": 3, "nb": 1}, shell, L)
    assert not bench.zero_on_vector_unit({"kernel": 3, "nb": 2}, shell, L)    # two fragments: no saving
    assert not bench.zero_on_vector_unit({"kernel": 8, "nb": 4}, shell, L)    # fragments of 4 keep it a column
    assert not bench.zero_on_vector_unit({"kernel": 6, "nb": 2}, cube, L)     # 27 is not 16 k + 1
    no_zero = np.delete(shell, 0, axis=0)
    no_zero = np.vstack([no_zero, [[3, 0, 0]]])
    assert not bench.zero_on_vector_unit({"kernel": 6, "nb": 2}, no_zero, L)
    wrapped = shell.copy()
    wrapped[0] = [L, 0, -L]                                                   # zero mod L
    assert bench.zero_on_vector_unit({"kernel": 6, "nb": 2}, wrapped, L)


def test_kernel_names_match_the_profiled_instantiations():
    assert bench.kernel_name("fp64", {"kernel": 8, "nb": 2}, 32, 32) == "bb::f64p::contract<2, 16, false, false, 4, 2>"
    assert bench.kernel_name("fp64", {"kernel": 6, "nb": 2}, 64, 64, True) == \
        "bb::f64p::contract<2, 16, false, true, 16, 2>"
    assert bench.kernel_name("fp64", {"kernel": 6, "nb": 3}, 64, 64) == "bb::f64p::contract<3, 16, false, false, 16, 1>"
    assert bench.kernel_name("bf16x3", {"kernel": 3, "nb": 1}, 64, 64, True) == "bb::pord::contract<1, 32, false, true>"
    assert bench.kernel_name("bf16x3", {"kernel": 4, "nb": 7}, 32, 32) == "bb::w3::contract8<7, 32, false>"
    assert bench.kernel_name("fp32", {"kernel": 1, "nb": 7}, 32, 32) == "bb::fast::bb_fast<1, 7, 32, 32, false>"
    assert bench.kernel_name("fp32", {"kernel": 7, "nb": 1}, 32, 32) == "bb::f32p::contract<1, 16, false, false, 16>"
    assert bench.kernel_name("fp32", {"kernel": 7, "nb": 3}, 64, 64, True) == "bb::f32p::contract<3, 32, false, true, 16>"
    assert bench.kernel_name("fp32", {"kernel": 9, "nb": 2}, 32, 32) == "bb::f32p::contract<2, 16, false, false, 4>"
    for name in ("bb::f64p::contract<2, 16, false, false, 4, 2>", "bb::w3::contract8<7, 32, false>",
                 "bb::fast::bb_fast<1, 7, 32, 32, false>"):
        assert bench.sources_of(name)
