"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.

This module holds none of the baryon-block arithmetic: it only draws random
quark fields and lists integer momentum sets and workload shapes.  The fields
stand in for reconstructed LapH quark fields q[x][colour][d] of one spin
component on one timeslice (paper, Sec. 2, eq. (2)); production fields from a
gauge ensemble are not available, so entries are iid standard complex normal
(re, im ~ N(0, 1/2)).  Timing is data independent (dense contraction), so only
the error statistics depend on this choice.

Seeds follow numpy's PCG64 with SeedSequence([16278, workload, t, role, spin]).
"""
from __future__ import annotations

import itertools

import numpy as np


def rng(workload: int, t: int = 0, role: int = 0, spin: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([16278, workload, t, role, spin])))


def gaussian_field(L: int, n: int, *, workload: int = 0, t: int = 0, role: int = 0, spin: int = 0,
                   dtype=np.complex128) -> np.ndarray:
    """Quark field [L^3][3][n], iid complex normal with unit variance."""
    g = rng(workload, t, role, spin)
    v = L ** 3
    s = np.sqrt(0.5)
    re = g.standard_normal((v, 3, n)) * s
    im = g.standard_normal((v, 3, n)) * s
    return (re + 1j * im).astype(dtype)


def gaussian_fields(L: int, ns, **kw):
    """Three independent fields (roles 0, 1, 2) with dilution sizes ns."""
    return [gaussian_field(L, n, role=i, **kw) for i, n in enumerate(ns)]


def laplacian_modes(L: int, n_ev: int, *, workload: int = 0, t: int = 0, dtype=np.complex128) -> np.ndarray:
    """Stand-in for the Laplacian eigenvectors phi^{(l)}_{a x} of one timeslice,
    laid out [L^3][3][n_ev]: iid complex normal entries scaled by 1/sqrt(3 L^3),
    so every column has unit norm on average and distinct columns are nearly
    orthogonal, as eigenvectors are (the real ones need a gauge field)."""
    phi = gaussian_field(L, n_ev, workload=workload, t=t, role=7) / np.sqrt(3.0 * L ** 3)
    return phi.astype(dtype)


def coefficients(n_q: int, n_dil: int, n_ev: int, *, workload: int = 0, t: int = 0, role: int = 0) -> np.ndarray:
    """Quark-field coefficients Q^{(d)}_{l} of n_q spin components / quark lines,
    [n_q][n_dil][n_ev], iid complex normal with unit variance (complex128)."""
    g = rng(workload, t, 100 + role)
    s = np.sqrt(0.5)
    return (g.standard_normal((n_q, n_dil, n_ev)) * s + 1j * g.standard_normal((n_q, n_dil, n_ev)) * s)


# ---------------------------------------------------------------- momenta ---
# Integer momentum vectors n; the physical momentum is p = 2 pi n / L.

def momenta_zero():
    return np.array([[0, 0, 0]], dtype=np.int32)


def momenta_axis():
    """0 and the six unit vectors (7 momenta)."""
    return np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                    dtype=np.int32)


def momenta_cube():
    """{-1, 0, 1}^3 (27 momenta)."""
    return np.array(list(itertools.product((-1, 0, 1), repeat=3)), dtype=np.int32)


def momenta_shell4():
    """All n with |n|^2 <= 4: {-1,0,1}^3 plus the six vectors 2*e_i (33 momenta)."""
    pts = [n for n in itertools.product(range(-2, 3), repeat=3) if sum(c * c for c in n) <= 4]
    pts.sort(key=lambda n: (sum(c * c for c in n), n))
    return np.array(pts, dtype=np.int32)


# -------------------------------------------------------------- workloads ---
# Shapes of the benchmark workloads.  Each entry: lattice extent L, timeslices,
# dilution sizes, momentum set, input dtype, blocks per timeslice.
WORKLOADS = {
    "tiny-12": dict(L=12, T=1, ndil=32, momenta="zero", dtype="c128", blocks_per_t=1),
    "headline-32": dict(L=32, T=1, ndil=32, momenta="axis", dtype="c128", blocks_per_t=1),
    "batched-48": dict(L=48, T=48, ndil=32, momenta="cube", dtype="c64", blocks_per_t=4),
    "uneven-32": dict(L=32, T=16, ndil=(16, 32, 64), momenta="axis", dtype="c64", blocks_per_t=160),
    "large-64": dict(L=64, T=4, ndil=64, momenta="shell4", dtype="c128", blocks_per_t=1),
    # Spin projection: per timeslice 8 spin-triple blocks summed into 2 outputs.
    "projected-32": dict(L=32, T=2, ndil=32, momenta="axis", dtype="c128", blocks_per_t=8),
    # LapH subspace: eigenvector count n_ev, coefficient sets n_q per call.
    "reconstruct-32": dict(L=32, T=1, ndil=32, n_ev=128, n_q=12, dtype="c128"),
    "mode-triplet-32": dict(L=32, T=1, ndil=32, n_ev=64, momenta="axis", dtype="c128", n_c=16),
}

# Spin-projection terms of the projected workload: (output, spin triple,
# coefficient); synthetic, of the +-1, +-i/2 kind spin projectors produce.
PROJECTION_TERMS = (
    (0, (0, 1, 0), 1.0), (0, (1, 0, 0), -1.0), (0, (0, 0, 1), 0.5j), (0, (1, 1, 1), -0.5j),
    (1, (2, 3, 2), 1.0), (1, (3, 2, 2), -1.0), (1, (2, 2, 3), 0.5), (1, (3, 3, 3), -0.5),
)

MOMENTUM_SETS = {"zero": momenta_zero, "axis": momenta_axis, "cube": momenta_cube,
                 "shell4": momenta_shell4}


def momenta(name: str) -> np.ndarray:
    return MOMENTUM_SETS[name]()
