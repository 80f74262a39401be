"""Baryon blocks of the stochastic LapH method on AMD Instinct MI355X (gfx950).

The computation lives in libbblock.so (hand-written HIP kernels behind the C
ABI of include/bblock.h); ``binding`` marshals arguments to it, ``synth``
draws seeded synthetic inputs, ``build`` compiles the library with hipcc.

Typical use (torch tensors on the GPU)::

    from paper_2211_16278_amd import BaryonBlocks
    with BaryonBlocks(L=32, prec="bf16x3", in_dtype="c128", max_ndil=64) as bb:
        B = bb.compute(q1, q2, q3, momenta)          # eq. (3): [T, n_mom, n1, n2, n3]
        bb.compute_batch([(q1, q2, q3, out), ...], momenta)   # many blocks, one launch
        bb.compute_projected(descs, coefs, momenta)  # eq. (1): sums of blocks
        q = bb.reconstruct(phi, Q)                    # eq. (2)
        T = bb.mode_triplets(phi, momenta)            # eq. (4)
        B = bb.mode_contract_batch(T, Q1, Q2, Q3)     # blocks from the mode triplets
"""
from .binding import (BaryonBlocks, BBlockError, bblock_compute, bblock_compute_batch,  # noqa: F401
                      bblock_compute_projected, bblock_create, bblock_destroy, bblock_get_plan, bblock_last_error,
                      bblock_mode_contract, bblock_mode_contract_batch, bblock_mode_triplets, bblock_profile,
                      bblock_profile_read, bblock_reconstruct, bblock_set_graph, bblock_set_plan, bblock_sync,
                      bblock_tune, bblock_version)

__all__ = ["BaryonBlocks", "BBlockError", "bblock_create", "bblock_compute", "bblock_compute_batch",
           "bblock_compute_projected", "bblock_reconstruct", "bblock_mode_triplets", "bblock_mode_contract",
           "bblock_mode_contract_batch", "bblock_set_graph", "bblock_tune", "bblock_set_plan", "bblock_get_plan",
           "bblock_profile", "bblock_profile_read", "bblock_sync", "bblock_destroy", "bblock_last_error",
           "bblock_version"]
