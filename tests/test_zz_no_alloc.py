"""The allocation-free entry point bblock_compute_noalloc against
bblock_compute, through the C ABI: calls in a row on one handle (each with a
smaller input than the one before, so that the scratch array still holds the
earlier calls' larger contents), in every precision, to the error contract of the
precision (FP64 1e-10, FP32 and BF16X3 1e-5 of the block's largest entry);
and a batch too large for the static scratch array is refused with a clear
error and leaves the output untouched."""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

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


def _fields(torch, dev, L, ns, T, workload):
    per_t = [[synth.gaussian_field(L, n, workload=workload, t=t, role=i) for i, n in enumerate(ns)]
             for t in range(T)]
    return [torch.from_numpy(np.stack([per_t[t][i] for t in range(T)])).to(dev) for i in range(3)]


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("prec", ("fp64", "fp32", "bf16x3"))
def test_noalloc_matches_compute_two_calls(torch_dev, prec):
    torch, dev = torch_dev
    L = 8
    # Each call's input is smaller than the one before; the second runs the
    # many-momenta plans (FP64 kernel 6, BF16X3 kernel 3).
    calls = [((24, 20, 28), 2, "axis"), ((20, 18, 24), 1, "cube"), ((5, 3, 7), 1, "cube")]
    with binding.BaryonBlocks(L, prec=prec, in_dtype="c128", max_ndil=32) as bb:
        for k, (ns, T, mset) in enumerate(calls):
            say("case noalloc", prec, "call", k, ns, T, mset)
            q = _fields(torch, dev, L, ns, T, workload=140 + k)
            mom = synth.momenta(mset)
            ref = bb.compute(*q, mom)
            out = torch.full_like(ref, float("nan"))
            bb.compute_noalloc(*q, mom, out=out)
            bb.sync()
            e = _rel(out.cpu().numpy(), ref.cpu().numpy())
            say("  rel err %.3e" % e)
            assert e < TOL[prec]


def test_noalloc_headline_size_fp64(torch_dev):
    """32^3 sites, N_dil 32, 7 momenta (split partials of tens of MB in the
    scratch array), then N_dil 16 on the same handle."""
    torch, dev = torch_dev
    L = 32
    with binding.BaryonBlocks(L, prec="fp64", in_dtype="c128", max_ndil=32) as bb:
        for k, n in enumerate((32, 16)):
            say("case noalloc headline-size fp64, N_dil", n)
            g = torch.Generator(device=dev).manual_seed(150 + k)
            q = [torch.randn((1, L ** 3, 3, n), dtype=torch.complex128, device=dev, generator=g) for _ in range(3)]
            mom = synth.momenta("axis")
            ref = bb.compute(*q, mom)
            out = torch.full_like(ref, float("nan"))
            bb.compute_noalloc(*q, mom, out=out)
            bb.sync()
            e = _rel(out.cpu().numpy(), ref.cpu().numpy())
            say("  rel err %.3e" % e)
            assert e < TOL["fp64"]


def test_noalloc_refuses_what_does_not_fit(torch_dev):
    """FP32 at 32^3, N_dil 64 with the fused kernel 1 forced: its tiles do not
    fill the device twice, so it keeps split partials, and at least 8 splits
    of 4096 x 448 complex FP32 partials (117 MB) exceed the 64 MiB array:
    BBLOCK_ENOMEM, nothing written.  The default plan (the paper-order kernel
    9, enough tiles to walk) needs no partials and runs in the array, within
    the FP32 contract of the allocating entry point's result."""
    torch, dev = torch_dev
    L, n = 32, 64
    say("case noalloc too large")
    g = torch.Generator(device=dev)
    g.manual_seed(16278 * 1000 + 93)
    q = [torch.view_as_complex(torch.empty((1, L ** 3, 3, n, 2), dtype=torch.float64, device=dev).normal_(generator=g))
         for _ in range(3)]
    mom = synth.momenta("axis")
    out = torch.full((1, len(mom), n, n, n), 7.0, dtype=torch.complex128, device=dev)
    with binding.BaryonBlocks(L, prec="fp32", in_dtype="c128", max_ndil=64) as bb:
        bb.set_plan(n, n, n, len(mom), dict(kernel=1, nb=7, splits=0, persistent=0, grid=0))
        with pytest.raises(binding.BBlockError) as ei:
            bb.compute_noalloc(*q, mom, out=out)
        assert ei.value.status == 2 and "static scratch" in str(ei.value)
        bb.sync()
        assert torch.all(out == 7.0).item()
        bb.set_plan(n, n, n, len(mom), None)
        say("  default plan", bb.get_plan(n, n, n, len(mom)))
        bb.compute_noalloc(*q, mom, out=out)
        ref = bb.compute(*q, mom)
        bb.sync()
    e = _rel(out.cpu().numpy(), ref.cpu().numpy())
    say("  rel err against the allocating entry point %.3e" % e)
    assert e < 1e-5
