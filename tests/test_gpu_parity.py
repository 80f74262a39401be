"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Error metric (per block): err_max = max|B - R| / max|R|, R the oracle.
Individual entries of B are sums of random-sign terms and may be arbitrarily
small (exactly zero for identical fields), so an entrywise relative error has
no bound; the max-normalised error is the one the tolerances refer to.
Tolerances: FP64 path 1e-10; FP32 and BF16x3 split paths 1e-5.
"""
from __future__ import annotations

import ctypes
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2211_16278_amd import binding, synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-5}
PRECS = ("fp64", "fp32", "bf16x3")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not os.path.exists(binding.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return torch, torch.device("cuda:0")


def err_max(got, ref):
    return float(np.abs(got - ref).max() / np.abs(ref).max())


def gpu_block(torch_dev, prec, L, qs, mom, dtype="c128", plan=None, graph=True, max_ndil=64, workspace_cap=0):
    torch, dev = torch_dev
    tq = [torch.from_numpy(np.ascontiguousarray(q)).to(dev) for q in qs]
    with binding.BaryonBlocks(L, prec=prec, in_dtype=dtype, max_ndil=max_ndil, workspace_cap=workspace_cap) as bb:
        bb.set_graph(graph)
        if plan is not None:
            bb.set_plan(qs[0].shape[-1], qs[1].shape[-1], qs[2].shape[-1], len(mom), plan)
        out = bb.compute(*tq, mom)
        bb.sync()
    return out[0].cpu().numpy()


def fields(L, ns, workload=100, dtype=np.complex128, t=0):
    return [synth.gaussian_field(L, n, workload=workload, role=i, t=t, dtype=dtype) for i, n in enumerate(ns)]


# ------------------------------------------------------------ full blocks
@pytest.mark.parametrize("prec", PRECS)
def test_tiny_workload_full_block(torch_dev, prec):
    """12^3 sites, N_dil = 32, zero momentum: every entry against the oracle."""
    L, n = 12, 32
    qs = synth.gaussian_fields(L, (n, n, n), workload=1)
    mom = synth.momenta("zero")
    say("case tiny-12", prec)
    ref = oracle.bblock(L, *qs, mom)
    got = gpu_block(torch_dev, prec, L, qs, mom)
    e = err_max(got, ref)
    say("  err_max %.3e" % e)
    assert e < TOL[prec]


SHAPES = [(3, (5, 3, 7), "axis"), (5, (33, 17, 40), "cube"), (2, (1, 1, 1), "axis"), (4, (64, 2, 9), "zero"),
          (7, (9, 31, 13), "shell4")]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L,ns,mset", SHAPES)
def test_ragged_shapes_full_block(torch_dev, prec, L, ns, mset):
    """Shapes that leave ragged row, column and site tiles, and several tiles."""
    qs = fields(L, ns, workload=101)
    mom = synth.momenta(mset)
    say("case ragged", prec, L, ns, mset)
    ref = oracle.bblock(L, *qs, mom)
    got = gpu_block(torch_dev, prec, L, qs, mom)
    e = err_max(got, ref)
    say("  err_max %.3e" % e)
    assert e < TOL[prec]


def _random_momenta(n, seed):
    g = synth.rng(120, seed)
    return g.integers(-9, 10, size=(n, 3)).astype(np.int32)  # components past +-L reduce mod L


EDGES = [(1, (3, 4, 5), 3), (3, (5, 6, 7), 128), (2, (70, 3, 40), 2), (5, (8, 16, 17), 19)]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L,ns,n_mom", EDGES)
def test_edge_sizes(torch_dev, prec, L, ns, n_mom):
    """A single site (L = 1), the largest momentum set (128), dilution sizes far
    apart and past the tiled kernels' minimum, momentum components beyond
    +-L: every entry against the oracle."""
    qs = fields(L, ns, workload=121)
    mom = _random_momenta(n_mom, L)
    say("case edge", prec, L, ns, n_mom)
    ref = oracle.bblock(L, *qs, mom)
    got = gpu_block(torch_dev, prec, L, qs, mom, max_ndil=128)
    e = err_max(got, ref)
    say("  err_max %.3e" % e)
    assert e < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_complex64_inputs(torch_dev, prec):
    L, ns = 6, (20, 24, 28)
    qs = fields(L, ns, workload=102, dtype=np.complex64)
    mom = synth.momenta("axis")
    say("case c64", prec)
    ref = oracle.bblock(L, *qs, mom)  # the oracle upcasts the same complex64 values exactly
    got = gpu_block(torch_dev, prec, L, qs, mom, dtype="c64")
    e = err_max(got, ref)
    say("  err_max %.3e" % e)
    assert e < TOL[prec]


def test_identical_fields_antisymmetric_fp64(torch_dev):
    L, n = 4, 6
    q = synth.gaussian_field(L, n, workload=103)
    mom = synth.momenta("axis")
    say("case identical fields")
    got = gpu_block(torch_dev, "fp64", L, [q, q, q], mom)
    scale = np.abs(got).max()
    assert np.abs(got + np.transpose(got, (0, 2, 1, 3))).max() < 1e-12 * scale
    assert np.abs(got + np.transpose(got, (0, 1, 3, 2))).max() < 1e-12 * scale
    assert err_max(got, oracle.bblock(L, q, q, q, mom)) < 1e-10


# --------------------------------------------------------- plan variants
def _plans(prec):
    """Every (kernel, nb, splits, persistent) the planner or autotuner may pick."""
    out = []
    kernels = [(0, nb) for nb in ((1, 2, 4, 7, 14) if prec == "fp64" else (1, 2, 4, 7))]
    if prec == "fp64":
        kernels += [(5, 2), (5, 4), (5, 7), (6, 1), (6, 2), (6, 3), (8, 1), (8, 2), (8, 3), (8, 4)]
    if prec != "fp64":
        kernels += [(1, 4), (1, 7)]
    if prec == "fp32":
        kernels += [(7, 1), (7, 2), (7, 3), (7, 4), (9, 1), (9, 2), (9, 3), (9, 4)]
    if prec == "bf16x3":
        kernels += [(2, 4), (2, 5), (2, 6), (2, 7), (3, 1), (3, 2), (4, 4), (4, 5), (4, 6), (4, 7)]
    for kernel, nb in kernels:
        for splits in (1, 3, 16):
            for persistent in (0, 1):
                out.append(dict(kernel=kernel, nb=nb, splits=splits, persistent=persistent,
                                grid=7 if persistent else 0))
    return out


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L,ns", [(5, (19, 21, 23)), (4, (40, 33, 35))])
def test_every_plan_candidate_passes(torch_dev, prec, L, ns):
    """Each kernel / tile shape / split / persistence the autotuner may pick is
    correct, on shapes with ragged edges for both tile families."""
    qs = fields(L, ns, workload=104)
    mom = synth.momenta("axis")
    ref = oracle.bblock(L, *qs, mom)
    for plan in _plans(prec):
        say("case plan", prec, L, ns, plan)
        e = err_max(gpu_block(torch_dev, prec, L, qs, mom, plan=plan), ref)
        assert e < TOL[prec], (plan, e)


@pytest.mark.parametrize("prec", PRECS)
def test_determinism_graph_persistent(torch_dev, prec):
    """Graph replay, eager launch, persistent and one-tile-per-workgroup
    schedules give bitwise identical blocks (ordered FP64 split reduction)."""
    L, ns = 6, (24, 24, 24)
    qs = fields(L, ns, workload=105)
    mom = synth.momenta("axis")
    say("case determinism", prec)
    a = gpu_block(torch_dev, prec, L, qs, mom, graph=False)
    b = gpu_block(torch_dev, prec, L, qs, mom, graph=True)
    kernel = 5 if prec == "fp64" else 1
    nb = 7
    c = gpu_block(torch_dev, prec, L, qs, mom, plan=dict(kernel=kernel, nb=nb, splits=0, persistent=1))
    d = gpu_block(torch_dev, prec, L, qs, mom, plan=dict(kernel=kernel, nb=nb, splits=0, persistent=0))
    assert np.array_equal(a, b)
    assert np.array_equal(c, d)
    assert err_max(a, oracle.bblock(L, *qs, mom)) < TOL[prec]


@pytest.mark.parametrize("L,ns,dtype", [(6, (24, 24, 24), "c128"), (5, (19, 40, 23), "c128"), (4, (33, 16, 35), "c64"),
                                        (4, (12, 56, 47), "c128")])
def test_precomputed_w_matches_pipelined_bitwise(torch_dev, L, ns, dtype):
    """BF16x3: the kernel with precomputed W images (plan kernel 2) forms the
    same products in the same order as the kernel that builds W in LDS (plan
    kernel 1), whatever its tile shape (4..7 column fragments; d2 blocks of
    8, 16 or 32; d3 blocks of any size in [16, 32]), so the blocks are
    bitwise equal; persistent and one-tile-per-workgroup schedules of kernel
    2 agree too.  Its eight-wave form (plan kernel 4: two waves per SIMD
    splitting the column fragments) gives the same blocks bitwise."""
    qs = fields(L, ns, workload=112, dtype=np.complex64 if dtype == "c64" else np.complex128)
    mom = synth.momenta("cube")
    a = gpu_block(torch_dev, "bf16x3", L, qs, mom, dtype=dtype, plan=dict(kernel=1, nb=7, splits=3, persistent=0))
    for nb in (7, 6, 5, 4):
        say("case w3 vs pipelined", L, ns, dtype, nb)
        b = gpu_block(torch_dev, "bf16x3", L, qs, mom, dtype=dtype, plan=dict(kernel=2, nb=nb, splits=3, persistent=0))
        c = gpu_block(torch_dev, "bf16x3", L, qs, mom, dtype=dtype,
                      plan=dict(kernel=2, nb=nb, splits=3, persistent=1, grid=5))
        assert np.array_equal(a, b)
        assert np.array_equal(b, c)
        say("case w3 eight waves", L, ns, dtype, nb)
        d = gpu_block(torch_dev, "bf16x3", L, qs, mom, dtype=dtype, plan=dict(kernel=4, nb=nb, splits=3, persistent=0))
        e = gpu_block(torch_dev, "bf16x3", L, qs, mom, dtype=dtype,
                      plan=dict(kernel=4, nb=nb, splits=3, persistent=1, grid=5))
        assert np.array_equal(a, d)
        assert np.array_equal(a, e)
    assert err_max(b, oracle.bblock(L, *qs, mom)) < TOL["bf16x3"]


@pytest.mark.parametrize("L,ns,mset,dtype", [(5, (19, 21, 33), "cube", "c128"), (4, (16, 17, 64), "shell4", "c128"),
                                             (5, (24, 9, 40), "shell4", "c64"), (4, (7, 5, 16), "axis", "c128")])
def test_paper_order_kernel(torch_dev, L, ns, mset, dtype):
    """BF16x3 paper-order kernel (singlet on the VALU, momentum GEMM on MFMA)
    for one and two column fragments and both d3 blocks, ragged pair and d3
    edges, against the oracle; persistent and one-tile-per-workgroup
    schedules agree bitwise."""
    qs = fields(L, ns, workload=115, dtype=np.complex64 if dtype == "c64" else np.complex128)
    mom = synth.momenta(mset)
    ref = oracle.bblock(L, *qs, mom)
    for nb in (1, 2):
        say("case paper-order", L, ns, mset, dtype, nb)
        a = gpu_block(torch_dev, "bf16x3", L, qs, mom, dtype=dtype, plan=dict(kernel=3, nb=nb, splits=3, persistent=0))
        b = gpu_block(torch_dev, "bf16x3", L, qs, mom, dtype=dtype,
                      plan=dict(kernel=3, nb=nb, splits=3, persistent=1, grid=6))
        assert np.array_equal(a, b)
        assert err_max(a, ref) < TOL["bf16x3"], err_max(a, ref)


@pytest.mark.parametrize("L,ns,mset,dtype", [(5, (19, 21, 33), "cube", "c128"), (4, (16, 17, 64), "shell4", "c128"),
                                             (5, (24, 9, 40), "shell4", "c64"), (4, (7, 5, 16), "axis", "c128"),
                                             (3, (9, 11, 50), "zero", "c128")])
@pytest.mark.parametrize("prec,kernel,nbs", [("fp64", 6, (1, 2, 3)), ("fp32", 7, (1, 2, 3, 4)),
                                             ("fp64", 8, (1, 2, 3, 4)), ("fp32", 9, (1, 2, 3, 4))])
def test_paper_order_fp64_fp32_kernels(torch_dev, prec, kernel, nbs, L, ns, mset, dtype):
    """FP64 paper-order kernels 6 and 8 (fragments of 16 and of 4 momenta)
    and FP32 kernels 7 and 9 (the same, in single precision; singlet on the
    vector unit in the MFMA operand layout, momentum GEMM on the matrix
    cores) for every momentum-fragment
    count and both d3 blocks, ragged pair, d3 and
    momentum edges and sites that end inside a chunk, against the oracle at
    the precision's tolerance; persistent and one-tile-per-workgroup
    schedules agree bitwise."""
    qs = fields(L, ns, workload=116, dtype=np.complex64 if dtype == "c64" else np.complex128)
    mom = synth.momenta(mset)
    ref = oracle.bblock(L, *qs, mom)
    for nb in nbs:
        say("case paper-order", prec, kernel, L, ns, mset, dtype, nb)
        a = gpu_block(torch_dev, prec, L, qs, mom, dtype=dtype, plan=dict(kernel=kernel, nb=nb, splits=3, persistent=0))
        b = gpu_block(torch_dev, prec, L, qs, mom, dtype=dtype,
                      plan=dict(kernel=kernel, nb=nb, splits=3, persistent=1, grid=6))
        assert np.array_equal(a, b)
        assert err_max(a, ref) < TOL[prec], err_max(a, ref)


def _zero_momentum_sets(L):
    """Momentum sets of 16 k + 1 that hold a momentum zero mod L (the FP64 and
    FP32 paper-order kernels then sum it on the vector unit and project on
    the other 16 k), and a control without one."""
    cube, shell = synth.momenta("cube"), synth.momenta("shell4")
    mid = cube[:17]                                   # (0, 0, 0) at position 13
    wrapped = np.delete(shell, 0, axis=0)
    wrapped = np.insert(wrapped, 20, [L, 0, -L], axis=0)  # zero mod L at position 20
    twice = shell.copy()
    twice[9] = 0                                      # a second zero: a column of its own
    none = np.delete(cube, 13, axis=0)[:17]           # 17 momenta, none zero
    return {"mid-17": mid, "wrapped-33": wrapped, "twice-33": twice, "none-17": none}


@pytest.mark.parametrize("mset", ["mid-17", "wrapped-33", "twice-33", "none-17"])
@pytest.mark.parametrize("prec,kernel,nbs", [("fp64", 6, (1, 2, 3)), ("fp32", 7, (1, 2, 3, 4)),
                                             ("fp64", 8, (1, 2, 3, 4)), ("fp32", 9, (1, 2, 3, 4)),
                                             ("bf16x3", 3, (1, 2))])
def test_zero_momentum_on_vector_unit(torch_dev, prec, kernel, nbs, mset):
    """The zero momentum of a 16 k + 1 set summed on the vector unit (wherever
    it sits in the set, also as a multiple of L, once when repeated): every
    column width, split partials, both schedules bitwise equal, and the
    oracle at the precision's tolerance.  Kernels 8 and 9 (fragments of 4)
    keep the zero momentum a column of its own in the same sets; BF16X3 kernel 3
    takes it off its one fragment of 32 at 33 momenta."""
    L, ns = 5, (19, 21, 40)
    qs = fields(L, ns, workload=117)
    mom = _zero_momentum_sets(L)[mset]
    ref = oracle.bblock(L, *qs, mom)
    for nb in nbs:
        say("case zero momentum", prec, kernel, mset, nb)
        a = gpu_block(torch_dev, prec, L, qs, mom, plan=dict(kernel=kernel, nb=nb, splits=3, persistent=0))
        b = gpu_block(torch_dev, prec, L, qs, mom, plan=dict(kernel=kernel, nb=nb, splits=3, persistent=1, grid=6))
        assert np.array_equal(a, b)
        assert err_max(a, ref) < TOL[prec], err_max(a, ref)
    c = gpu_block(torch_dev, prec, L, qs, mom)  # the default plan
    assert err_max(c, ref) < TOL[prec], err_max(c, ref)


def test_precomputed_w_small_workspace_falls_back(torch_dev):
    """A workspace cap too small for the W images: the planner runs the block
    with the in-LDS W kernel instead, with the same result."""
    L, ns = 6, (24, 24, 24)
    qs = fields(L, ns, workload=113)
    mom = synth.momenta("axis")
    say("case w3 fallback")
    # 1 MiB holds neither the images nor split partials: one split, kernel 1.
    small = gpu_block(torch_dev, "bf16x3", L, qs, mom, workspace_cap=1 << 20)
    k1 = gpu_block(torch_dev, "bf16x3", L, qs, mom, plan=dict(kernel=1, nb=7, splits=1, persistent=0))
    assert np.array_equal(small, k1)
    assert err_max(small, oracle.bblock(L, *qs, mom)) < TOL["bf16x3"]


@pytest.mark.parametrize("kernel", [2, 4])
def test_precomputed_w_in_rounds_matches(torch_dev, kernel):
    """W images larger than the workspace run in rounds of splits (each round:
    images, then the contraction of its splits; the reduction after the last),
    bitwise equal to the single-round run with the same split count."""
    torch, dev = torch_dev
    L, ns = 6, (24, 24, 24)
    qs = fields(L, ns, workload=114)
    mom = synth.momenta("axis")
    say("case w3 rounds, kernel", kernel)
    # Plan kernel 2 (or 4), nb 7, 9 splits of 3 chunks: partials 9 * 2 * 576 * 168 * 4
    # = 6967296 bytes; images (one n-tile: 7 momenta x d3 block 24) 3 * 45056
    # bytes per split; the cap holds 3 splits' images: 3 rounds.
    plan = dict(kernel=kernel, nb=7, splits=9, persistent=0)
    tq = [torch.from_numpy(np.ascontiguousarray(q)).to(dev) for q in qs]
    outs, launches = [], []
    for cap in (0, 6967296 + 3 * 3 * 45056 + 1000):
        with binding.BaryonBlocks(L, prec="bf16x3", in_dtype="c128", max_ndil=64, workspace_cap=cap) as bb:
            bb.set_plan(*ns, len(mom), plan)
            bb.profile(True)
            out = bb.compute(*tq, mom)
            launches.append(bb.profile_read()[3])
            outs.append(out[0].cpu().numpy())
    say("  contraction launches", launches)
    assert launches == [1, 3]
    assert np.array_equal(outs[0], outs[1])
    assert err_max(outs[1], oracle.bblock(L, *qs, mom)) < TOL["bf16x3"]


# ------------------------------------------------------ spin projection
def _projected_case(torch_dev, prec, L, ns_list, groups, coefs, workload, workspace_cap=0, graph=True):
    """Blocks i with fields of shape ns_list[i] summed with coefs[i] into output groups[i]."""
    torch, dev = torch_dev
    fields_i = [fields(L, ns, workload=workload, t=i) for i, ns in enumerate(ns_list)]
    mom = synth.momenta("axis")
    outs = {}
    for g, ns in zip(groups, ns_list):
        if g not in outs:
            outs[g] = torch.empty((len(mom), ns[0], ns[1], ns[2]), dtype=torch.complex128, device=dev)
    tq = [[torch.from_numpy(q).to(dev) for q in f] for f in fields_i]
    descs = [(t[0], t[1], t[2], outs[g]) for t, g in zip(tq, groups)]
    with binding.BaryonBlocks(L, prec=prec, in_dtype="c128", max_ndil=64, workspace_cap=workspace_cap) as bb:
        bb.set_graph(graph)
        bb.compute_projected(descs, coefs, mom)
        bb.compute_projected(descs, coefs, mom)  # a repeat (cached tables, graph replay) overwrites
        bb.sync()
    got = {g: o.cpu().numpy() for g, o in outs.items()}
    refs = {}
    for g in got:
        idx = [i for i, gg in enumerate(groups) if gg == g]
        refs[g] = oracle.bblock_projected(L, [fields_i[i] for i in idx], [coefs[i] for i in idx], mom)
    return got, refs


@pytest.mark.parametrize("prec", PRECS)
def test_projected_groups(torch_dev, prec):
    """Three outputs of 1, 2 and 4 spin-triple terms (eq. (1)), complex
    coefficients, against the oracle's sum of blocks."""
    L = 5
    ns_list = [(19, 21, 23)] * 1 + [(16, 17, 18)] * 2 + [(24, 24, 24)] * 4
    groups = [0, 1, 1, 2, 2, 2, 2]
    coefs = [1.0 + 0.0j, 0.5 - 1.0j, -2.0 + 0.25j, 1.0j, -1.0, 0.75 + 0.75j, 0.125 - 3.0j]
    say("case projected", prec)
    got, refs = _projected_case(torch_dev, prec, L, ns_list, groups, coefs, workload=120)
    for g in got:
        assert err_max(got[g], refs[g]) < TOL[prec], (g, err_max(got[g], refs[g]))


def test_projected_single_term_equals_block(torch_dev):
    """One term with coefficient 1 reproduces the plain block bitwise (same
    partials, same FP64 split sum)."""
    torch, dev = torch_dev
    L, ns = 6, (24, 24, 24)
    qs = fields(L, ns, workload=121)
    mom = synth.momenta("axis")
    say("case projected single term")
    tq = [torch.from_numpy(q).to(dev) for q in qs]
    a = torch.empty((len(mom),) + ns, dtype=torch.complex128, device=dev)
    b = torch.empty_like(a)
    with binding.BaryonBlocks(L, prec="bf16x3", in_dtype="c128", max_ndil=32) as bb:
        bb.compute_batch([(tq[0], tq[1], tq[2], a)], mom)
        bb.compute_projected([(tq[0], tq[1], tq[2], b)], [1.0], mom)
        bb.sync()
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


@pytest.mark.parametrize("prec", ("fp32", "bf16x3"))
def test_projected_group_across_sub_batches(torch_dev, prec):
    """A workspace that holds one block's partials splits a 4-term output over
    four sub-batches (the later ones add to the output): bitwise equal to the
    single-launch result, which sums the terms in the same order."""
    L = 6
    ns_list = [(24, 24, 24)] * 4
    groups = [0, 0, 0, 0]
    coefs = [1.0 - 0.5j, 2.0, -0.25j, 0.5 + 0.5j]
    say("case projected sub-batches", prec)
    full, refs = _projected_case(torch_dev, prec, L, ns_list, groups, coefs, workload=122)
    # One 24^3-dilution block at 7 momenta: 9 splits of 576 x 168 partials
    # (7.0 MB) plus its W images (2.4 MB); 12 MiB holds one block, not two.
    small, _ = _projected_case(torch_dev, prec, L, ns_list, groups, coefs, workload=122, workspace_cap=12 << 20)
    assert np.array_equal(full[0], small[0])
    assert err_max(full[0], refs[0]) < TOL[prec]


def test_plan_validation_and_defaults(torch_dev):
    """Plan control around the precomputed-W kernels: kernel 4 (eight waves)
    and kernel 2 are accepted for BF16X3 with 4-7 column fragments and
    rejected otherwise (other fragment counts, other precisions, unknown
    kernel ids); the default BF16X3 plan is kernel 4 up to 16 momenta and the
    paper-order kernel 3 beyond."""
    say("case plan validation")
    L, n = 6, 24
    with binding.BaryonBlocks(L, prec="bf16x3", in_dtype="c128", max_ndil=64) as bb:
        for kernel in (2, 4):
            for nb in (4, 5, 6, 7):
                bb.set_plan(n, n, n, 7, dict(kernel=kernel, nb=nb, splits=0, persistent=0, grid=0))
                got = bb.get_plan(n, n, n, 7)
                assert (got["kernel"], got["nb"]) == (kernel, nb) and got["splits"] >= 1
            for nb in (1, 2, 3, 8):
                with pytest.raises(binding.BBlockError):
                    bb.set_plan(n, n, n, 7, dict(kernel=kernel, nb=nb, splits=0, persistent=0, grid=0))
        for kernel in (5, -1):
            with pytest.raises(binding.BBlockError):
                bb.set_plan(n, n, n, 7, dict(kernel=kernel, nb=7, splits=0, persistent=0, grid=0))
        bb.set_plan(n, n, n, 7, None)
        assert bb.get_plan(n, n, n, 7)["kernel"] == 4
        assert bb.get_plan(n, n, n, 16)["kernel"] == 4
        assert bb.get_plan(n, n, n, 17)["kernel"] == 3
    for prec in ("fp32", "fp64"):
        with binding.BaryonBlocks(L, prec=prec, in_dtype="c128", max_ndil=64) as bb:
            for kernel in (2, 4):
                with pytest.raises(binding.BBlockError):
                    bb.set_plan(n, n, n, 7, dict(kernel=kernel, nb=7, splits=0, persistent=0, grid=0))
            assert bb.get_plan(n, n, n, 7)["kernel"] == (8 if prec == "fp64" else 9)
            if prec == "fp64":  # kernel 5 up to 4 momenta, kernel 8 from 5 to 12, kernel 6 beyond
                assert bb.get_plan(n, n, n, 4)["kernel"] == 5
                for nm in (5, 8, 9, 12):
                    got = bb.get_plan(n, n, n, nm)
                    assert (got["kernel"], got["nb"]) == (8, -(-nm // 4))
                assert bb.get_plan(n, n, n, 13)["kernel"] == 6
                assert bb.get_plan(n, n, 8, 33)["kernel"] == 5  # n3 below kernel 6's d3 block
                assert bb.get_plan(n, n, 8, 7)["kernel"] == 5  # and kernel 8's
                for nb in (1, 2, 3, 4):
                    bb.set_plan(n, n, n, 7, dict(kernel=8, nb=nb, splits=0, persistent=0, grid=0))
                    assert bb.get_plan(n, n, n, 7)["kernel"] == 8
                with pytest.raises(binding.BBlockError):  # kernel 8 has 1 to 4 fragments of 4
                    bb.set_plan(n, n, n, 7, dict(kernel=8, nb=5, splits=0, persistent=0, grid=0))
                bb.set_plan(n, n, n, 7, None)
                # 33 momenta with the zero one: 32 columns, two fragments.
                assert (bb.get_plan(n, n, n, 33)["kernel"], bb.get_plan(n, n, n, 33)["nb"]) == (6, 2)
            if prec == "fp32":
                for kernel, nb in ((5, 7), (6, 2), (8, 2)):  # kernels 5, 6 and 8 are FP64 only
                    with pytest.raises(binding.BBlockError):
                        bb.set_plan(n, n, n, 7, dict(kernel=kernel, nb=nb, splits=0, persistent=0, grid=0))
                # Kernel 1 up to 4 momenta, kernel 9 (fragments of 4) from 5 to 8, kernel 7 beyond.
                assert bb.get_plan(n, n, n, 4)["kernel"] == 1
                for nm in (5, 7, 8):
                    got = bb.get_plan(n, n, n, nm)
                    assert (got["kernel"], got["nb"]) == (9, -(-nm // 4))
                assert bb.get_plan(n, n, n, 9)["kernel"] == 7
                assert bb.get_plan(n, n, 8, 7)["kernel"] != 9  # n3 below kernel 9's d3 block
                with pytest.raises(binding.BBlockError):  # kernel 9 has 1 to 4 fragments of 4
                    bb.set_plan(n, n, n, 7, dict(kernel=9, nb=5, splits=0, persistent=0, grid=0))
                # 33 momenta with the zero one: 32 columns, two fragments.
                assert (bb.get_plan(n, n, n, 33)["kernel"], bb.get_plan(n, n, n, 33)["nb"]) == (7, 2)
                with pytest.raises(binding.BBlockError):  # kernel 7 has 1 to 4 momentum fragments
                    bb.set_plan(n, n, n, 27, dict(kernel=7, nb=5, splits=0, persistent=0, grid=0))
            else:
                for nb in (1, 2, 3):
                    bb.set_plan(n, n, n, 27, dict(kernel=6, nb=nb, splits=0, persistent=0, grid=0))
                    assert bb.get_plan(n, n, n, 27)["kernel"] == 6
                for nb in (4, 7):
                    with pytest.raises(binding.BBlockError):
                        bb.set_plan(n, n, n, 27, dict(kernel=6, nb=nb, splits=0, persistent=0, grid=0))
                with pytest.raises(binding.BBlockError):  # n3 below the d3 block of 16
                    bb.set_plan(n, n, 8, 27, dict(kernel=6, nb=2, splits=0, persistent=0, grid=0))
                with pytest.raises(binding.BBlockError):  # kernel 7 is FP32 only
                    bb.set_plan(n, n, n, 27, dict(kernel=7, nb=2, splits=0, persistent=0, grid=0))
                bb.set_plan(n, n, n, 27, None)


def test_projected_argument_errors(torch_dev):
    torch, dev = torch_dev
    L = 4
    q = [torch.zeros((L ** 3, 3, n), dtype=torch.complex128, device=dev) for n in (4, 4, 4)]
    q5 = torch.zeros((L ** 3, 3, 5), dtype=torch.complex128, device=dev)
    out = torch.zeros((1, 4, 4, 4), dtype=torch.complex128, device=dev)
    mom = [[0, 0, 0]]
    with binding.BaryonBlocks(L, prec="fp32", in_dtype="c128", max_ndil=8) as bb:
        with pytest.raises(binding.BBlockError):
            bb.compute_projected([(q[0], q[1], q[2], out), (q[0], q[1], q5, out)], [1.0, 1.0], mom)
        with pytest.raises(binding.BBlockError):
            bb.compute_projected([(q[0], q[1], q[2], out)], [float("nan")], mom)
        with pytest.raises(ValueError):
            bb.compute_projected([(q[0], q[1], q[2], out)], [1.0, 2.0], mom)
        bb.sync()


@pytest.mark.parametrize("prec", PRECS)
def test_graph_replays_match_eager(torch_dev, prec):
    """One handle: replay the captured grouped launch several times, with eager
    work and synchronisation in between, each replay equal to the eager result."""
    torch, dev = torch_dev
    L, ns = 5, (16, 12, 20)
    qs = [fields(L, ns, workload=106, t=t) for t in range(3)]
    mom = synth.momenta("cube")
    with binding.BaryonBlocks(L, prec=prec, in_dtype="c128", max_ndil=32) as bb:
        tq = [[torch.from_numpy(q).to(dev) for q in trip] for trip in qs]
        outs = [torch.zeros((len(mom), *ns), dtype=torch.complex128, device=dev) for _ in qs]
        descs = [(a, b_, c, o) for (a, b_, c), o in zip(tq, outs)]
        bb.set_graph(False)
        bb.compute_batch(descs, mom)
        bb.sync()
        eager = [o.cpu().numpy().copy() for o in outs]
        bb.set_graph(True)
        for rep in range(4):
            say("case graph replay", prec, rep)
            for o in outs:
                o.fill_(float("nan"))
            bb.compute_batch(descs, mom)
            bb.sync()
            _ = (torch.ones(1000, device=dev) * rep).sum().item()  # eager work between replays
            for o, e in zip(outs, eager):
                assert np.array_equal(o.cpu().numpy(), e)
        # The default mode replays only long schedules; this one runs eagerly.
        bb.set_graph("auto")
        for o in outs:
            o.fill_(float("nan"))
        bb.compute_batch(descs, mom)
        bb.sync()
        for o, e in zip(outs, eager):
            assert np.array_equal(o.cpu().numpy(), e)
        with pytest.raises(binding.BBlockError):
            bb.set_graph(3)
    for trip, e in zip(qs, eager):
        assert err_max(e, oracle.bblock(L, *trip, mom)) < TOL[prec]


# ----------------------------------------------------------- timeslices
@pytest.mark.parametrize("prec", PRECS)
def test_timeslice_range(torch_dev, prec):
    torch, dev = torch_dev
    L, ns, T = 4, (8, 6, 10), 4
    per_t = [fields(L, ns, workload=107, t=t) for t in range(T)]
    Q = [np.stack([per_t[t][i] for t in range(T)]) for i in range(3)]
    mom = synth.momenta("axis")
    say("case timeslices", prec)
    with binding.BaryonBlocks(L, prec=prec, in_dtype="c128", max_ndil=16) as bb:
        out = bb.compute(*[torch.from_numpy(q).to(dev) for q in Q], mom, t_begin=1, t_end=4)
        bb.sync()
    got = out.cpu().numpy()
    assert got.shape == (3, len(mom), *ns)
    for i, t in enumerate(range(1, 4)):
        assert err_max(got[i], oracle.bblock(L, *per_t[t], mom)) < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_uneven_batch(torch_dev, prec):
    """Blocks with N_dil in {16, 32, 64} (and mixed within a block) in one grouped launch."""
    torch, dev = torch_dev
    L = 4
    shapes = [(16, 16, 16), (64, 64, 64), (32, 32, 32), (16, 64, 32), (32, 16, 64)]
    mom = synth.momenta("axis")
    trips = [fields(L, s, workload=108, t=i, dtype=np.complex64) for i, s in enumerate(shapes)]
    say("case uneven batch", prec)
    with binding.BaryonBlocks(L, prec=prec, in_dtype="c64", max_ndil=64) as bb:
        tq = [[torch.from_numpy(q).to(dev) for q in trip] for trip in trips]
        outs = [torch.empty((len(mom), *s), dtype=torch.complex128, device=dev) for s in shapes]
        bb.compute_batch([(*t, o) for t, o in zip(tq, outs)], mom)
        bb.sync()
    for trip, o in zip(trips, outs):
        assert err_max(o.cpu().numpy(), oracle.bblock(L, *trip, mom)) < TOL[prec]


def test_tune_then_compute(torch_dev):
    L, ns = 6, (24, 24, 24)
    qs = fields(L, ns, workload=109)
    mom = synth.momenta("axis")
    torch, dev = torch_dev
    say("case tune")
    with binding.BaryonBlocks(L, prec="bf16x3", in_dtype="c128", max_ndil=32) as bb:
        bb.tune(*ns, len(mom))
        plan = bb.get_plan(*ns, len(mom))
        assert plan["kernel"] in (0, 1, 2, 3, 4) and plan["nb"] in (1, 2, 4, 5, 6, 7) and plan["splits"] >= 1
        out = bb.compute(*[torch.from_numpy(q).to(dev) for q in qs], mom)
        bb.sync()
    assert err_max(out[0].cpu().numpy(), oracle.bblock(L, *qs, mom)) < TOL["bf16x3"]


def test_tune_times_each_candidate(torch_dev):
    """The autotuner times every candidate plan on its own schedule: at
    32^3, N_dil = 32 the candidates differ by more than 10x (generic tiles
    against the precomputed-W kernels), so a tuned plan slower than the
    default by 30 % means the candidates were not told apart (as when a
    cached schedule of an earlier candidate was replayed for all of them)."""
    torch, dev = torch_dev
    L, n = 32, 32
    mom = synth.momenta("axis")
    say("case tune timing")
    g = torch.Generator(device="cpu").manual_seed(7)
    qs = [torch.randn((L ** 3, 3, n), dtype=torch.complex128, generator=g).to(dev) for _ in range(3)]
    out = torch.empty((1, len(mom), n, n, n), dtype=torch.complex128, device=dev)

    def ms(bb):
        for _ in range(5):
            bb.compute(*qs, mom, out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(bb.stream)
        for _ in range(30):
            bb.compute(*qs, mom, out=out)
        e1.record(bb.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 30

    with binding.BaryonBlocks(L, prec="bf16x3", in_dtype="c128", max_ndil=32) as bb:
        t_default = ms(bb)
        bb.tune(n, n, n, len(mom))
        plan = bb.get_plan(n, n, n, len(mom))
        t_tuned = ms(bb)
    say("  default %.3f ms, tuned %.3f ms with %s" % (t_default, t_tuned, plan))
    assert t_tuned < 1.3 * t_default, (plan, t_default, t_tuned)


# ------------------------------------------- split counts and the accuracy floor
def test_forced_plan_respects_accuracy_floor(torch_dev):
    """At 32^3 a split of the FP32-accumulating paths holds at most 4096 sites,
    so at least 8 splits.  Forcing the paper-order kernel with splits = 0 at
    N_dil 64 (1024 tiles, a wave-filling count of one split) resolves to at
    least 8 splits; an explicit count below 8 is refused; the forced plan's
    block matches the oracle on sampled entries."""
    torch, dev = torch_dev
    L, n = 32, 64
    mom = synth.momenta("shell4")
    say("case forced plan, accuracy floor")
    qs = synth.gaussian_fields(L, (n, n, n), workload=130)
    with binding.BaryonBlocks(L, prec="bf16x3", in_dtype="c128", max_ndil=64) as bb:
        bb.set_plan(n, n, n, len(mom), dict(kernel=3, nb=2, splits=0, persistent=0))
        plan = bb.get_plan(n, n, n, len(mom))
        say("  plan", plan)
        assert plan["kernel"] == 3 and plan["splits"] >= 8
        for bad in (1, 7):
            with pytest.raises(binding.BBlockError) as ei:
                bb.set_plan(n, n, n, len(mom), dict(kernel=3, nb=2, splits=bad, persistent=0))
            assert ei.value.status == 1
        out = bb.compute(*[torch.from_numpy(q).to(dev) for q in qs], mom)
        bb.sync()
    g = np.random.default_rng(5)
    ents = np.stack([g.integers(0, n, 48) for _ in range(3)], axis=1).astype(np.int32)
    ref = oracle.bblock_entries(L, *qs, mom, ents)
    got = out[0].cpu().numpy()[:, ents[:, 0], ents[:, 1], ents[:, 2]]
    assert err_max(got, ref) < TOL["bf16x3"]


def test_single_block_splits_in_whole_waves(torch_dev):
    """32^3, N_dil 48, 7 momenta, BF16X3: the default plan's split count is
    raised to the accuracy floor (8) in whole multiples of the wave-filling
    count (kernel 4 at N_dil 48: d2 blocks of 16, d3 blocks of 24, 6 column
    fragments -> 18 x 2 = 36 tiles per split, floor(256 / 36) = 7 -> 14
    splits); sampled entries against the oracle."""
    torch, dev = torch_dev
    L, n = 32, 48
    mom = synth.momenta("axis")
    say("case single-block split rounding")
    qs = synth.gaussian_fields(L, (n, n, n), workload=131)
    with binding.BaryonBlocks(L, prec="bf16x3", in_dtype="c128", max_ndil=64) as bb:
        plan = bb.get_plan(n, n, n, len(mom))
        say("  plan", plan)
        assert plan["kernel"] == 4 and plan["nb"] == 6
        assert plan["splits"] >= 8 and plan["splits"] % 7 == 0
        out = bb.compute(*[torch.from_numpy(q).to(dev) for q in qs], mom)
        bb.sync()
    g = np.random.default_rng(6)
    ents = np.stack([g.integers(0, n, 64) for _ in range(3)], axis=1).astype(np.int32)
    ref = oracle.bblock_entries(L, *qs, mom, ents)
    got = out[0].cpu().numpy()[:, ents[:, 0], ents[:, 1], ents[:, 2]]
    assert err_max(got, ref) < TOL["bf16x3"]


# --------------------------------------------------------- error paths
def test_error_paths_enqueue_nothing(torch_dev):
    torch, dev = torch_dev
    lib = binding.load()
    L, n = 3, 4
    q = torch.zeros((L ** 3, 3, n), dtype=torch.complex128, device=dev)
    out = torch.full((1, n, n, n), 7.0, dtype=torch.complex128, device=dev)
    m = (ctypes.c_int32 * 3)(0, 0, 0)
    h = binding.bblock_create(L, binding.FP64, binding.C128, 8)
    try:
        p, o = q.data_ptr(), out.data_ptr()
        cases = {
            "null q": (None, p, p, n, n, n, m, 1, 0, 1, o),
            "null out": (p, p, p, n, n, n, m, 1, 0, 1, None),
            "n > max_ndil": (p, p, p, 9, n, n, m, 1, 0, 1, o),
            "n = 0": (p, p, p, 0, n, n, m, 1, 0, 1, o),
            "empty t range": (p, p, p, n, n, n, m, 1, 1, 1, o),
            "negative t": (p, p, p, n, n, n, m, 1, -1, 1, o),
            "n_mom = 0": (p, p, p, n, n, n, m, 0, 0, 1, o),
            "null momenta": (p, p, p, n, n, n, None, 1, 0, 1, o),
            "misaligned": (p + 8, p, p, n, n, n, m, 1, 0, 1, o),
        }
        for name, args in cases.items():
            say("case error path", name)
            assert lib.bblock_compute(h, *args) == 1, name
            assert binding.bblock_last_error(h)
        binding.bblock_sync(h)
        assert torch.all(out == 7.0).item()
    finally:
        binding.bblock_destroy(h)
