"""GPU parity of the LapH-subspace entry points (through the C ABI) against
the oracle in oracle/modes.py: eq. (2) reconstruction, eq. (4) mode triplets
and the contraction of coefficients onto them.

Error metric: max|got - ref| / max|ref|.  The reconstruction and the
contraction are FP64 complex GEMMs on the matrix cores: they differ from the
oracle's numpy products only in summation order, so the bound is 1e-12
(K <= 128 terms of unit size, each rounded at 2^-53).  A complex64 output is
the FP64 sum rounded once: within one FP32 rounding of the oracle's value.
The mode triplets come from the block kernels, with their tolerances.
"""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

import oracle
from oracle import modes
from paper_2211_16278_amd import binding, synth

pytestmark = pytest.mark.gpu

TOL_GEMM = 1e-12
TOL_BLOCK = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-5}


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


def dev(torch_dev, a):
    torch, d = torch_dev
    return torch.from_numpy(np.ascontiguousarray(a)).to(d)


# ------------------------------------------------------------ reconstruction
# (L, n_ev, n_dil, n_q): M = 3 L^3 rows with ragged tails, N = n_q n_dil
# through all three tile shapes, K = n_ev from 1 to past several chunks.
RECON = [(2, 1, 1, 1), (3, 13, 5, 1), (5, 13, 13, 3), (4, 64, 40, 2), (6, 70, 32, 4), (5, 9, 100, 1)]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("L,n_ev,n_dil,n_q", RECON)
def test_reconstruct_matches_oracle(torch_dev, L, n_ev, n_dil, n_q, dtype):
    say("case reconstruct", L, n_ev, n_dil, n_q, dtype)
    phi = synth.laplacian_modes(L, n_ev, workload=300, t=n_ev)
    Q = synth.coefficients(n_q, n_dil, n_ev, workload=300, t=n_dil)
    ref = modes.reconstruct(Q, phi)
    with binding.BaryonBlocks(L, prec="fp64", in_dtype=dtype, max_ndil=8) as bb:
        got = bb.reconstruct(dev(torch_dev, phi), dev(torch_dev, Q))
        bb.sync()
    got = got.cpu().numpy()
    assert got.shape == (n_q, L ** 3, 3, n_dil)
    if dtype == "c128":
        e = err_max(got, ref)
        say("  err_max %.3e" % e)
        assert e < TOL_GEMM
    else:
        # One FP32 rounding (half an ulp, 2^-24 relative) of an FP64 sum that
        # itself is within 1e-12 of the oracle, per component.
        slack = TOL_GEMM * np.abs(ref).max()
        for part in (np.real, np.imag):
            r, g_ = part(ref), part(got).astype(np.float64)
            assert np.all(np.abs(g_ - r) <= 2.0 ** -24 * np.abs(r) + slack)


def test_reconstruct_feeds_the_block_kernel(torch_dev):
    """Reconstructed fields go straight into bblock_compute: the block of the
    reconstructed fields equals the oracle block of the oracle's fields."""
    torch, d = torch_dev
    L, n_ev, ns = 4, 20, (6, 5, 7)
    phi = synth.laplacian_modes(L, n_ev, workload=301)
    Qs = [synth.coefficients(1, n, n_ev, workload=301, role=i) for i, n in enumerate(ns)]
    mom = synth.momenta("axis")
    ref = oracle.bblock(L, *[modes.reconstruct(Q, phi)[0] for Q in Qs], mom)
    with binding.BaryonBlocks(L, prec="fp64", in_dtype="c128", max_ndil=8) as bb:
        qs = [bb.reconstruct(dev(torch_dev, phi), dev(torch_dev, Q))[0] for Q in Qs]
        got = bb.compute(*qs, mom)[0]
        bb.sync()
    e = err_max(got.cpu().numpy(), ref)
    say("case reconstruct->block err_max %.3e" % e)
    assert e < TOL_BLOCK["fp64"]


# ------------------------------------------------------------- mode triplets
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_mode_triplets_match_oracle(torch_dev, prec):
    L, n_ev = 4, 18
    mom = np.array([[0, 0, 0], [1, 0, 0], [0, 2, 1], [-1, 1, 1]], dtype=np.int32)
    phi = synth.laplacian_modes(L, n_ev, workload=302)
    ref = modes.mode_triplets(L, phi, mom)
    with binding.BaryonBlocks(L, prec=prec, in_dtype="c128", max_ndil=32) as bb:
        got = bb.mode_triplets(dev(torch_dev, phi), mom)
        bb.sync()
    got = got.cpu().numpy()
    e = err_max(got, ref)
    say("case mode triplets", prec, "err_max %.3e" % e)
    assert e < TOL_BLOCK[prec]
    # Antisymmetry holds to the same tolerance (the kernels do not impose it).
    assert np.abs(got + got.transpose(0, 2, 1, 3)).max() < 2 * TOL_BLOCK[prec] * np.abs(ref).max()


# --------------------------------------------------------------- contraction
# (n_ev, n1, n2, n3, n_mom): every GEMM shape class, ragged tails, degenerate 1s.
CONTRACT = [(1, 1, 1, 1, 1), (5, 3, 4, 2, 2), (13, 33, 17, 40, 3), (40, 16, 64, 9, 2), (70, 8, 8, 33, 1),
            (24, 64, 64, 64, 2)]


@pytest.mark.parametrize("n_ev,n1,n2,n3,n_mom", CONTRACT)
def test_mode_contract_matches_oracle(torch_dev, n_ev, n1, n2, n3, n_mom):
    say("case mode contract", n_ev, n1, n2, n3, n_mom)
    g = synth.rng(303, n_ev, n1)
    T = g.standard_normal((n_mom, n_ev, n_ev, n_ev)) + 1j * g.standard_normal((n_mom, n_ev, n_ev, n_ev))
    Qs = [synth.coefficients(1, n, n_ev, workload=303, role=i)[0] for i, n in enumerate((n1, n2, n3))]
    ref = modes.mode_contract(*Qs, T)
    with binding.BaryonBlocks(4, prec="fp64", in_dtype="c128", max_ndil=8) as bb:
        got = bb.mode_contract(dev(torch_dev, T), *[dev(torch_dev, Q) for Q in Qs])
        bb.sync()
    e = err_max(got.cpu().numpy(), ref)
    say("  err_max %.3e" % e)
    assert e < TOL_GEMM


@pytest.mark.parametrize("layout", range(6))
def test_every_gemm_layout(torch_dev, monkeypatch, layout):
    """Each wave layout of the complex GEMM (2x2, 1x4, 4x1 output blocks; 1x2 and
    2x1 with two k-groups; 1x1 with four) on ragged reconstruction and
    contraction shapes."""
    monkeypatch.setenv("BBLOCK_ZGEMM_LAYOUT", str(layout))
    say("case gemm layout", layout)
    L, n_ev, n_dil, n_q = 5, 37, 23, 3
    phi = synth.laplacian_modes(L, n_ev, workload=308)
    Q = synth.coefficients(n_q, n_dil, n_ev, workload=308)
    n_e2, ns, n_mom = 19, (21, 9, 35), 2
    g = synth.rng(309)
    T = g.standard_normal((n_mom, n_e2, n_e2, n_e2)) + 1j * g.standard_normal((n_mom, n_e2, n_e2, n_e2))
    Qs = [synth.coefficients(1, n, n_e2, workload=309, role=i)[0] for i, n in enumerate(ns)]
    with binding.BaryonBlocks(L, prec="fp64", in_dtype="c128", max_ndil=8) as bb:
        q = bb.reconstruct(dev(torch_dev, phi), dev(torch_dev, Q))
        B = bb.mode_contract(dev(torch_dev, T), *[dev(torch_dev, x) for x in Qs])
        bb.sync()
    e1 = err_max(q.cpu().numpy(), modes.reconstruct(Q, phi))
    e2 = err_max(B.cpu().numpy(), modes.mode_contract(*Qs, T))
    say("  err_max %.3e %.3e" % (e1, e2))
    assert e1 < TOL_GEMM and e2 < TOL_GEMM


def test_mode_contract_in_momentum_rounds_is_bitwise(torch_dev):
    """A workspace cap that holds one momentum's intermediates gives the same bits."""
    n_ev, ns, n_mom = 20, (6, 7, 5), 5
    g = synth.rng(304)
    T = g.standard_normal((n_mom, n_ev, n_ev, n_ev)) + 1j * g.standard_normal((n_mom, n_ev, n_ev, n_ev))
    Qs = [synth.coefficients(1, n, n_ev, workload=304, role=i)[0] for i, n in enumerate(ns)]
    tT, tQ = dev(torch_dev, T), [dev(torch_dev, Q) for Q in Qs]
    per_mom = (ns[0] * n_ev * n_ev + ns[0] * ns[1] * n_ev) * 16
    outs = []
    for cap in (0, per_mom + 100):
        with binding.BaryonBlocks(4, prec="fp64", in_dtype="c128", max_ndil=8, workspace_cap=cap) as bb:
            outs.append(bb.mode_contract(tT, *tQ).cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    assert err_max(outs[0], modes.mode_contract(*Qs, T)) < TOL_GEMM


@pytest.mark.parametrize("n_ev,n1,n2,n3,n_mom,n_c", [(13, 5, 7, 3, 2, 3), (24, 32, 16, 9, 3, 16), (7, 1, 1, 1, 1, 5)])
def test_mode_contract_batch_matches_oracle(torch_dev, n_ev, n1, n2, n3, n_mom, n_c):
    """n_c coefficient triples in one call (rows of the first GEMM stacked,
    the others batched over the triples): each block against the oracle and
    against the single-triple call."""
    say("case mode contract batch", n_ev, n1, n2, n3, n_mom, n_c)
    g = synth.rng(310, n_ev, n_c)
    T = g.standard_normal((n_mom, n_ev, n_ev, n_ev)) + 1j * g.standard_normal((n_mom, n_ev, n_ev, n_ev))
    Qs = [synth.coefficients(n_c, n, n_ev, workload=310, role=i) for i, n in enumerate((n1, n2, n3))]
    tT, tQ = dev(torch_dev, T), [dev(torch_dev, Q) for Q in Qs]
    with binding.BaryonBlocks(4, prec="fp64", in_dtype="c128", max_ndil=8) as bb:
        got = bb.mode_contract_batch(tT, *tQ).cpu().numpy()
        one = bb.mode_contract(tT, *[Q[n_c - 1] for Q in tQ]).cpu().numpy()
        bb.sync()
    assert got.shape == (n_c, n_mom, n1, n2, n3)
    for c in range(n_c):
        e = err_max(got[c], modes.mode_contract(Qs[0][c], Qs[1][c], Qs[2][c], T))
        assert e < TOL_GEMM, (c, e)
    assert err_max(got[n_c - 1], one) < TOL_GEMM


def test_mode_contract_batch_rounds_and_errors(torch_dev):
    """A cap that holds one momentum's intermediates of all triples runs the
    momenta in rounds with the same result; bad triple counts are rejected."""
    n_ev, ns, n_mom, n_c = 12, (5, 6, 7), 3, 4
    g = synth.rng(311)
    T = g.standard_normal((n_mom, n_ev, n_ev, n_ev)) + 1j * g.standard_normal((n_mom, n_ev, n_ev, n_ev))
    Qs = [synth.coefficients(n_c, n, n_ev, workload=311, role=i) for i, n in enumerate(ns)]
    tT, tQ = dev(torch_dev, T), [dev(torch_dev, Q) for Q in Qs]
    per_mom = n_c * (ns[0] * n_ev * n_ev + ns[0] * ns[1] * n_ev) * 16
    outs = []
    for cap in (0, per_mom + 100):
        with binding.BaryonBlocks(4, prec="fp64", in_dtype="c128", max_ndil=8, workspace_cap=cap) as bb:
            outs.append(bb.mode_contract_batch(tT, *tQ).cpu().numpy())
            with pytest.raises(binding.BBlockError):
                binding.bblock_mode_contract_batch(bb.h, tT, n_ev, n_mom, 0, tQ[0], ns[0], tQ[1], ns[1], tQ[2], ns[2],
                                                   tT)
    assert np.array_equal(outs[0], outs[1])


def test_both_routes_agree_on_the_gpu(torch_dev):
    """Sec. 2: reconstruct + block (eq. (2), (3)) and mode triplets + contraction
    (eq. (4)) give the same block, both computed on the GPU in FP64."""
    torch, d = torch_dev
    L, n_ev, ns = 4, 12, (5, 6, 4)
    mom = synth.momenta("axis")
    phi = synth.laplacian_modes(L, n_ev, workload=305)
    Qs = [synth.coefficients(1, n, n_ev, workload=305, role=i)[0] for i, n in enumerate(ns)]
    tphi, tQ = dev(torch_dev, phi), [dev(torch_dev, Q) for Q in Qs]
    with binding.BaryonBlocks(L, prec="fp64", in_dtype="c128", max_ndil=16) as bb:
        direct = bb.compute(*[bb.reconstruct(tphi, Q) for Q in tQ], mom)[0]
        T = bb.mode_triplets(tphi, mom)
        via_t = bb.mode_contract(T, *tQ)
        bb.sync()
    e = err_max(via_t.cpu().numpy(), direct.cpu().numpy())
    say("case routes err_max %.3e" % e)
    assert e < TOL_BLOCK["fp64"]


# --------------------------------------------------- bench-size parity
def test_bench_sizes_against_oracle(torch_dev):
    """The mode-triplet workload's sizes (32^3 sites, 64 eigenvectors, N_dil 32,
    7 momenta) and the reconstruction workload's (128 eigenvectors, 12
    coefficient sets of 32): full outputs against the oracle."""
    torch, d = torch_dev
    L, mom = 32, synth.momenta("axis")
    phi = synth.laplacian_modes(L, 128, workload=306)
    Q = synth.coefficients(12, 32, 128, workload=306)
    with binding.BaryonBlocks(L, prec="bf16x3", in_dtype="c128", max_ndil=64) as bb:
        q = bb.reconstruct(dev(torch_dev, phi), dev(torch_dev, Q))
        bb.sync()
        e = err_max(q.cpu().numpy(), modes.reconstruct(Q, phi))
        say("case bench reconstruct err_max %.3e" % e)
        assert e < TOL_GEMM
        del q
        n_ev = 64
        g = synth.rng(307)
        T = g.standard_normal((len(mom), n_ev, n_ev, n_ev)) + 1j * g.standard_normal((len(mom), n_ev, n_ev, n_ev))
        Qs = [synth.coefficients(1, 32, n_ev, workload=307, role=i)[0] for i in range(3)]
        got = bb.mode_contract(dev(torch_dev, T), *[dev(torch_dev, x) for x in Qs])
        bb.sync()
        e = err_max(got.cpu().numpy(), modes.mode_contract(*Qs, T))
        say("case bench contract err_max %.3e" % e)
        assert e < TOL_GEMM


# -------------------------------------------------------------- error paths
def test_mode_entry_points_reject_bad_arguments(torch_dev):
    torch, d = torch_dev
    phi = torch.zeros((64, 3, 4), dtype=torch.complex128, device=d)
    Q = torch.zeros((1, 2, 4), dtype=torch.complex128, device=d)
    q = torch.zeros((1, 64, 3, 2), dtype=torch.complex128, device=d)
    T = torch.zeros((1, 4, 4, 4), dtype=torch.complex128, device=d)
    B = torch.zeros((1, 2, 2, 2), dtype=torch.complex128, device=d)
    with binding.BaryonBlocks(4, prec="fp64", in_dtype="c128", max_ndil=8, workspace_cap=512) as bb:
        for call in (lambda: binding.bblock_reconstruct(bb.h, phi, 0, Q, 2, 1, q),
                     lambda: binding.bblock_reconstruct(bb.h, None, 4, Q, 2, 1, q),
                     lambda: binding.bblock_reconstruct(bb.h, phi, 4, Q, 2, 0, q),
                     lambda: binding.bblock_mode_contract(bb.h, T, 4, 0, Q[0], 2, Q[0], 2, Q[0], 2, B),
                     lambda: binding.bblock_mode_contract(bb.h, T, 5000, 1, Q[0], 2, Q[0], 2, Q[0], 2, B),
                     lambda: binding.bblock_mode_triplets(bb.h, phi, 9, [[0, 0, 0]], T)):
            with pytest.raises(binding.BBlockError) as ei:
                call()
            assert "EINVAL" in str(ei.value)
        # Misaligned (8-byte offset) complex128 buffer.
        raw = torch.zeros(2 * 64 * 3 * 4 + 1, dtype=torch.float64, device=d)
        with pytest.raises(binding.BBlockError):
            binding.bblock_reconstruct(bb.h, raw[1:], 4, Q, 2, 1, q)
        # One momentum needs (2 * 4^2 + 2 * 2 * 4) * 16 = 768 bytes of intermediates: over the 512-byte cap.
        with pytest.raises(binding.BBlockError) as ei:
            binding.bblock_mode_contract(bb.h, T, 4, 1, Q[0], 2, Q[0], 2, Q[0], 2, B)
        assert "ENOMEM" in str(ei.value)
        bb.sync()
