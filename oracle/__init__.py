"""CPU oracle for the baryon block (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never calls it, and the two share no code: the oracle is
a plain complex128 C loop (``bblock_oracle.c``) that follows eq. (3) of the
paper, Sec. 2, term by term.

Functions
---------
build()              compile ``liboracle.so`` with gcc (OpenMP, no fast-math).
bblock(...)          full block B[p][d1][d2][d3] (eq. (3)).
bblock_rows(...)     B for a list of (d1, d2) pairs, for sampled checks at
                     sizes where the full block would take minutes.
bblock_entries(...)  B for a list of (d1, d2, d3) triples (every momentum),
                     for sampled checks spread over all tiles of a large block.
bblock_projected(...) the spin-projected sum  sum_i c_i B(q1_i, q2_i, q3_i)
                     (eq. (1): a correlator term is a linear combination over
                     spin triples of eq. (3) blocks), and its rows variant.
max_threads()        OpenMP threads the oracle uses.
set_threads(n)       set that count (the CPU baseline runs on 1 and on all).

The LapH-subspace steps around eq. (3) -- eq. (2) reconstruction, eq. (4)
mode triplets and the contraction onto them -- are in ``oracle.modes``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bblock_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle.  -fcx-limited-range selects the textbook complex
    product (no C99 Annex G inf/nan recovery); no reassociation is enabled.
    ``src``/``out`` default to the committed source and the in-tree library."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fcx-limited-range", "-fopenmp", "-fPIC", "-shared",
           "-std=gnu11", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    _lib = load_library(_LIB)
    return _lib


def load_library(path: str):
    """Load a compiled oracle library and declare its entry points."""
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_bblock.argtypes = [ctypes.c_int] * 4 + [dp, dp, dp, ctypes.c_int, ip, dp]
    lib.oracle_bblock.restype = ctypes.c_int
    lib.oracle_bblock_rows.argtypes = ([ctypes.c_int] * 4 + [dp, dp, dp, ctypes.c_int, ip,
                                       ctypes.c_int, ip, dp])
    lib.oracle_bblock_rows.restype = ctypes.c_int
    lib.oracle_bblock_entries.argtypes = ([ctypes.c_int] * 4 + [dp, dp, dp, ctypes.c_int, ip,
                                          ctypes.c_int, ip, dp])
    lib.oracle_bblock_entries.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = ctypes.c_int
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = ctypes.c_int
    return lib


def _field(q: np.ndarray, L: int) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.complex128)  # complex64 upcasts exactly
    if q.ndim != 3 or q.shape[0] != L ** 3 or q.shape[1] != 3:
        raise ValueError("quark field must have shape [L^3, 3, n], got %r" % (q.shape,))
    return q


def _ptr(a: np.ndarray, ty):
    return a.ctypes.data_as(ctypes.POINTER(ty))


def bblock(L: int, q1, q2, q3, mom) -> np.ndarray:
    """B[p][d1][d2][d3] as complex128, shape [n_mom, n1, n2, n3]."""
    q1, q2, q3 = _field(q1, L), _field(q2, L), _field(q3, L)
    mom = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
    n1, n2, n3 = q1.shape[2], q2.shape[2], q3.shape[2]
    out = np.zeros((mom.shape[0], n1, n2, n3), dtype=np.complex128)
    rc = _load().oracle_bblock(L, n1, n2, n3, _ptr(q1, ctypes.c_double), _ptr(q2, ctypes.c_double),
                               _ptr(q3, ctypes.c_double), mom.shape[0], _ptr(mom, ctypes.c_int32),
                               _ptr(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return out


def bblock_rows(L: int, q1, q2, q3, mom, rows) -> np.ndarray:
    """B[p][r][d3] for the (d1, d2) pairs in ``rows``; shape [n_mom, n_rows, n3]."""
    q1, q2, q3 = _field(q1, L), _field(q2, L), _field(q3, L)
    mom = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int32).reshape(-1, 2))
    n1, n2, n3 = q1.shape[2], q2.shape[2], q3.shape[2]
    out = np.zeros((mom.shape[0], rows.shape[0], n3), dtype=np.complex128)
    rc = _load().oracle_bblock_rows(L, n1, n2, n3, _ptr(q1, ctypes.c_double),
                                    _ptr(q2, ctypes.c_double), _ptr(q3, ctypes.c_double),
                                    mom.shape[0], _ptr(mom, ctypes.c_int32), rows.shape[0],
                                    _ptr(rows, ctypes.c_int32), _ptr(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return out


def bblock_entries(L: int, q1, q2, q3, mom, entries) -> np.ndarray:
    """B[p][d1][d2][d3] for the (d1, d2, d3) triples in ``entries``; shape [n_mom, n_entries]."""
    q1, q2, q3 = _field(q1, L), _field(q2, L), _field(q3, L)
    mom = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
    entries = np.ascontiguousarray(np.asarray(entries, dtype=np.int32).reshape(-1, 3))
    n1, n2, n3 = q1.shape[2], q2.shape[2], q3.shape[2]
    out = np.zeros((mom.shape[0], entries.shape[0]), dtype=np.complex128)
    rc = _load().oracle_bblock_entries(L, n1, n2, n3, _ptr(q1, ctypes.c_double),
                                       _ptr(q2, ctypes.c_double), _ptr(q3, ctypes.c_double),
                                       mom.shape[0], _ptr(mom, ctypes.c_int32), entries.shape[0],
                                       _ptr(entries, ctypes.c_int32), _ptr(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return out


def bblock_projected(L: int, triples, coef, mom) -> np.ndarray:
    """sum_i coef[i] * B(triples[i]) in complex128, shape [n_mom, n1, n2, n3]
    (eq. (1) with the spin sum written as a linear combination of blocks)."""
    out = None
    for (q1, q2, q3), c in zip(triples, coef):
        b = complex(c) * bblock(L, q1, q2, q3, mom)
        out = b if out is None else out + b
    return out


def bblock_rows_projected(L: int, triples, coef, mom, rows) -> np.ndarray:
    """The rows variant of bblock_projected: shape [n_mom, n_rows, n3]."""
    out = None
    for (q1, q2, q3), c in zip(triples, coef):
        b = complex(c) * bblock_rows(L, q1, q2, q3, mom, rows)
        out = b if out is None else out + b
    return out


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def set_threads(n: int) -> int:
    """OpenMP threads for later oracle calls; returns the count in force."""
    return int(_load().oracle_set_threads(int(n)))
