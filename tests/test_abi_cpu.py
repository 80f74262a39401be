"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/bblock.h declares, and rejects bad arguments before
touching a device."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

from paper_2211_16278_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bblock.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bblock_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return binding.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 11, names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(binding.EXPORTS)


def test_version(lib):
    assert "gfx950" in binding.bblock_version()


def _create(lib, L=4, prec=0, dtype=0, ndil=8):
    h = ctypes.c_void_p()
    st = lib.bblock_create(ctypes.byref(h), L, prec, dtype, ndil, 0, None)
    return st, h


@pytest.mark.parametrize("L,prec,dtype,ndil,msg", [
    (0, 0, 0, 8, "L=0"), (257, 0, 0, 8, "L=257"), (4, 3, 0, 8, "unknown precision"), (4, -1, 0, 8, "unknown precision"),
    (4, 0, 2, 8, "unknown dtype"), (4, 0, 0, 0, "max_ndil=0"), (4, 0, 0, 5000, "max_ndil=5000")])
def test_create_rejects_bad_arguments(lib, L, prec, dtype, ndil, msg):
    st, h = _create(lib, L, prec, dtype, ndil)
    assert st == 1 and not h.value
    assert msg in binding.bblock_last_error(None)


def test_create_null_out(lib):
    assert lib.bblock_create(None, 4, 0, 0, 8, 0, None) == 1


def test_null_handle_calls(lib):
    assert lib.bblock_destroy(None) == 0
    assert lib.bblock_sync(None) == 1
    assert lib.bblock_set_graph(None, 1) == 1
    assert lib.bblock_tune(None, 4, 4, 4, 1) == 1
    m = (ctypes.c_int32 * 3)(0, 0, 0)
    assert lib.bblock_compute(None, None, None, None, 1, 1, 1, m, 1, 0, 1, None) == 1
    assert lib.bblock_compute_batch(None, None, 0, m, 1) == 1
    assert isinstance(lib.bblock_last_error(None), bytes)


def test_no_gpu_gives_enodev(lib):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except ImportError:
        pass
    st, h = _create(lib)
    assert st == 4 and not h.value
    assert binding.bblock_last_error(None)


def test_python_binding_fails_loudly_without_library(tmp_path):
    saved = binding._lib
    binding._lib = None
    try:
        with pytest.raises(RuntimeError, match="not found"):
            binding.load(str(tmp_path / "missing.so"))
    finally:
        binding._lib = saved
