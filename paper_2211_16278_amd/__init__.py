"""Baryon blocks of the stochastic LapH method on AMD Instinct MI355X (gfx950).

The computation lives in libbblock.so (hand-written HIP kernels behind the C
ABI of include/bblock.h); ``binding`` marshals arguments to it, ``synth``
draws seeded synthetic inputs, ``build`` compiles the library with hipcc.
"""
from .binding import (BaryonBlocks, BBlockError, bblock_compute, bblock_compute_batch, bblock_create,  # noqa: F401
                      bblock_destroy, bblock_get_plan, bblock_last_error, bblock_profile, bblock_profile_read, bblock_set_graph, bblock_set_plan,
                      bblock_sync, bblock_tune, bblock_version)

__all__ = ["BaryonBlocks", "BBlockError", "bblock_create", "bblock_compute", "bblock_compute_batch",
           "bblock_set_graph", "bblock_tune", "bblock_set_plan", "bblock_get_plan", "bblock_profile",
           "bblock_profile_read", "bblock_sync",
           "bblock_destroy", "bblock_last_error", "bblock_version"]
