"""Grouped launches: walking tiles, one sub-batch per kernel instantiation and
shared W images, through the C ABI.

A walking tile's workgroup runs all site splits of its (block, m-tile,
n-tile) in order and sums each split's FP32 (or FP64) result into the FP64
output; the split-K path stores the same per-split results as partials and
the reduction sums them in the same order.  So for a fixed split count the
two give bitwise equal blocks.  At 20^3 sites the FP32 accumulation bound
(4096 sites per split) asks for 2 splits, so the walks are real.
"""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

import oracle
from paper_2211_16278_amd import binding, synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-5}


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


def _walk_env(value):
    class _Env:
        def __enter__(self):
            self.old = os.environ.get("BBLOCK_SPLIT_WALK")
            os.environ["BBLOCK_SPLIT_WALK"] = value

        def __exit__(self, *exc):
            if self.old is None:
                os.environ.pop("BBLOCK_SPLIT_WALK", None)
            else:
                os.environ["BBLOCK_SPLIT_WALK"] = self.old
    return _Env()


def _run(torch_dev, prec, L, trips, mom, walk, plans=None, dtype="c128", profile=False):
    torch, dev = torch_dev
    tq = [[torch.from_numpy(np.ascontiguousarray(q)).to(dev) for q in t] for t in trips]
    outs = [torch.full((len(mom), *(q.shape[-1] for q in t)), float("nan"), dtype=torch.complex128, device=dev)
            for t in trips]
    with _walk_env(walk):
        with binding.BaryonBlocks(L, prec=prec, in_dtype=dtype, max_ndil=64) as bb:
            for shape, plan in (plans or {}).items():
                bb.set_plan(*shape, len(mom), plan)
            if profile:
                bb.profile(True)
                bb.profile_read()
            bb.compute_batch([(*t, o) for t, o in zip(tq, outs)], mom)
            launches = bb.profile_read()[3] if profile else None
            bb.sync()
    return [o.cpu().numpy() for o in outs], launches


def _fields(L, shapes, workload, dtype=np.complex128):
    return [[synth.gaussian_field(L, n, workload=workload, t=i, role=r, dtype=dtype) for r, n in enumerate(s)]
            for i, s in enumerate(shapes)]


CASES = [("fp32", 1, 7), ("fp32", 1, 4), ("bf16x3", 1, 7), ("bf16x3", 2, 7), ("bf16x3", 4, 5), ("bf16x3", 3, 1),
         ("bf16x3", 3, 2), ("fp32", 0, 4), ("bf16x3", 0, 2), ("fp64", 5, 7), ("fp64", 5, 2), ("fp64", 6, 2),
         ("fp64", 6, 3), ("fp64", 0, 7), ("fp32", 7, 2), ("fp32", 7, 4), ("fp64", 8, 2), ("fp64", 8, 4),
         ("fp32", 9, 2), ("fp32", 9, 4)]


@pytest.mark.parametrize("prec,kernel,nb", CASES)
def test_walking_tiles_bitwise_equal_to_split_reduction(torch_dev, prec, kernel, nb):
    """Every kernel family: a batch run with walking tiles equals the split-K
    partials + reduction run bitwise (2 splits at 20^3), and the oracle."""
    L = 20
    shapes = [(24, 20, 32), (24, 20, 32), (17, 33, 21)]
    trips = _fields(L, shapes, workload=160)
    mom = synth.momenta("cube" if kernel in (3, 6, 7) else "axis")  # the paper-order kernels: many momenta
    plans = {s: dict(kernel=kernel, nb=nb, splits=2, persistent=0) for s in set(shapes)}
    say("case walk vs split reduction", prec, kernel, nb)
    a, _ = _run(torch_dev, prec, L, trips, mom, "0", plans)
    b, _ = _run(torch_dev, prec, L, trips, mom, "1", plans)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    ref = oracle.bblock(L, *trips[2], mom)
    assert err_max(b[2], ref) < TOL[prec]


@pytest.mark.parametrize("prec,kernel,nb", (("fp64", 6, 2), ("fp32", 7, 2), ("bf16x3", 3, 1)))
def test_walking_tiles_zero_momentum_on_vector_unit(torch_dev, prec, kernel, nb):
    """The paper-order FP64/FP32 kernels with the 33-momentum shell (the zero
    momentum summed on the vector unit): walking tiles equal the split-K run
    bitwise, and the oracle."""
    L = 20
    shapes = [(24, 20, 32), (17, 33, 21)]
    trips = _fields(L, shapes, workload=163)
    mom = synth.momenta("shell4")
    plans = {s: dict(kernel=kernel, nb=nb, splits=2, persistent=0) for s in set(shapes)}
    say("case walk vs split reduction, zero momentum on the vector unit", prec, kernel)
    a, _ = _run(torch_dev, prec, L, trips, mom, "0", plans)
    b, _ = _run(torch_dev, prec, L, trips, mom, "1", plans)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    ref = oracle.bblock(L, *trips[1], mom)
    assert err_max(b[1], ref) < TOL[prec]


@pytest.mark.parametrize("prec", ("fp64", "fp32", "bf16x3"))
def test_uneven_batch_one_launch_per_instantiation(torch_dev, prec):
    """Blocks of N_dil 16, 32 and 64 interleaved as the uneven workload orders
    them: sorted into one sub-batch per kernel instantiation (at most 2 here),
    each a single launch with walking tiles; every block against the oracle
    on sampled entries."""
    L = 20
    ndil = [16, 32, 64, 16, 32, 64, 16, 32]
    trips = _fields(L, [(n, n, n) for n in ndil], workload=161, dtype=np.complex64)
    mom = synth.momenta("axis")
    say("case uneven batch launches", prec)
    outs, launches = _run(torch_dev, prec, L, trips, mom, "1", dtype="c64", profile=True)
    say("  contraction launches", launches)
    assert launches <= 2
    g = np.random.default_rng(12)
    for t, o in zip(trips, outs):
        n = t[0].shape[-1]
        ents = np.stack([g.integers(0, n, 16) for _ in range(3)], axis=1).astype(np.int32)
        ref = oracle.bblock_entries(L, *t, mom, ents)
        assert err_max(o[:, ents[:, 0], ents[:, 1], ents[:, 2]], ref) < TOL[prec]


@pytest.mark.parametrize("kernel", (2, 4))
def test_shared_w_images(torch_dev, kernel):
    """BF16x3 precomputed-W kernels: blocks that share their third field
    share one set of W images (produced once); each block equals the block
    computed alone, bitwise."""
    L = 20
    n = 24
    base = _fields(L, [(n, n, n)] * 3, workload=162)
    q3 = base[0][2]
    trips = [(base[0][0], base[0][1], q3), (base[1][0], base[1][1], q3), (base[2][0], base[2][1], q3),
             (base[1][0], base[0][1], base[1][2])]
    mom = synth.momenta("axis")
    plans = {(n, n, n): dict(kernel=kernel, nb=7, splits=2, persistent=0)}
    say("case shared W images, kernel", kernel)
    together, _ = _run(torch_dev, "bf16x3", L, trips, mom, "1", plans)
    for i, t in enumerate(trips):
        alone, _ = _run(torch_dev, "bf16x3", L, [t], mom, "1", plans)
        assert np.array_equal(together[i], alone[0]), i
    assert err_max(together[1], oracle.bblock(L, *trips[1], mom)) < TOL["bf16x3"]
