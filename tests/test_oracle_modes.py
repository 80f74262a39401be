"""Pins of the LapH-subspace oracle (oracle/modes.py): eq. (2) reconstruction,
eq. (4) mode triplets and the contraction of coefficients onto them.

None of the checks retypes the oracle's formula.  The reconstruction is
checked by projecting back onto orthonormal eigenvectors (which must return
the coefficients) and by unit coefficients selecting single modes; the mode
triplets against numpy determinants and their total antisymmetry; the
contraction against the other route of Sec. 2 (reconstruct, then the eq. (3)
block oracle) and against identity coefficients.  The mutation test at the
end plants plausible mistakes in a copy of the oracle source and requires a
pin to fail for each.
"""
from __future__ import annotations

import importlib.util

import numpy as np
import pytest

import oracle
from oracle import modes
from paper_2211_16278_amd import synth
from tests.test_oracle_pins import MOM_MIXED, _close, brute_force_det


def _orthonormal_modes(L, n_ev, seed):
    g = synth.rng(940, seed)
    a = g.standard_normal((3 * L ** 3, n_ev)) + 1j * g.standard_normal((3 * L ** 3, n_ev))
    q, _ = np.linalg.qr(a)
    return q.reshape(L ** 3, 3, n_ev)


# --------------------------------------------------------- reconstruction
def test_reconstruct_projection_recovers_coefficients():
    """With orthonormal eigenvectors, projecting q^{(d)} on phi^{(l)} gives Q_{dl} back."""
    L, n_ev = 3, 7
    phi = _orthonormal_modes(L, n_ev, 1)
    Q = synth.coefficients(2, 5, n_ev, workload=941)
    q = modes.reconstruct(Q, phi)
    assert q.shape == (2, L ** 3, 3, 5)
    back = np.einsum("xal,ixad->idl", phi.conj(), q)
    _close(back, Q)


def test_reconstruct_unit_coefficients_select_modes():
    """Q_{dl} = delta_{l, s(d)} gives q^{(d)} = phi^{(s(d))} exactly."""
    L, n_ev = 2, 6
    phi = synth.laplacian_modes(L, n_ev, workload=942)
    sel = [4, 0, 5, 2]
    Q = np.zeros((len(sel), n_ev), dtype=np.complex128)
    Q[np.arange(len(sel)), sel] = 1.0
    q = modes.reconstruct(Q, phi)
    assert np.array_equal(q, phi[:, :, sel])


# ------------------------------------------------------------ mode triplets
def test_mode_triplets_against_determinants():
    L, n_ev = 3, 4
    phi = synth.laplacian_modes(L, n_ev, workload=943)
    _close(modes.mode_triplets(L, phi, MOM_MIXED), brute_force_det(L, phi, phi, phi, MOM_MIXED))


def test_mode_triplets_totally_antisymmetric():
    """eps makes T odd under every exchange of eigenvector indices (so only
    n_ev choose 3 entries are independent, the paper's footnote to eq. (4))."""
    L, n_ev = 3, 5
    T = modes.mode_triplets(L, synth.laplacian_modes(L, n_ev, workload=944), MOM_MIXED)
    scale = np.abs(T).max()
    assert np.abs(T + T.transpose(0, 2, 1, 3)).max() < 1e-13 * scale
    assert np.abs(T + T.transpose(0, 1, 3, 2)).max() < 1e-13 * scale
    for i in range(n_ev):
        assert np.abs(T[:, i, i, :]).max() < 1e-13 * scale


# -------------------------------------------------------------- contraction
def test_mode_contract_equals_reconstruct_route():
    """eq. (4) route == eq. (2) + eq. (3) route (Sec. 2): the block oracle on
    the reconstructed fields."""
    L, n_ev, ns = 3, 6, (2, 3, 4)
    phi = synth.laplacian_modes(L, n_ev, workload=945)
    Qs = [synth.coefficients(1, n, n_ev, workload=945, role=i)[0] for i, n in enumerate(ns)]
    T = modes.mode_triplets(L, phi, MOM_MIXED)
    B = modes.mode_contract(*Qs, T)
    assert B.shape == (len(MOM_MIXED),) + ns
    qs = [modes.reconstruct(Q, phi) for Q in Qs]
    _close(B, oracle.bblock(L, *qs, MOM_MIXED))


def test_mode_contract_identity_coefficients():
    """Q1 = Q2 = Q3 = 1 (n_dil = n_ev) returns T itself; a permutation matrix permutes its axes."""
    g = synth.rng(946)
    n_ev = 4
    T = g.standard_normal((2, n_ev, n_ev, n_ev)) + 1j * g.standard_normal((2, n_ev, n_ev, n_ev))
    eye = np.eye(n_ev)
    assert np.array_equal(modes.mode_contract(eye, eye, eye, T), T)
    P = eye[[2, 0, 3, 1]]
    _close(modes.mode_contract(P, eye, eye, T), T[:, [2, 0, 3, 1]])
    _close(modes.mode_contract(eye, eye, P, T), T[:, :, :, [2, 0, 3, 1]])


def test_mode_oracle_rejects_bad_shapes():
    with pytest.raises(ValueError):
        modes.reconstruct(np.zeros((2, 3)), np.zeros((8, 3, 4)))
    with pytest.raises(ValueError):
        modes.mode_contract(np.zeros((2, 3)), np.zeros((2, 3)), np.zeros((2, 4)), np.zeros((1, 3, 3, 3)))


# ------------------------------------------------------- planted mistakes
PINS = [
    test_reconstruct_projection_recovers_coefficients,
    test_reconstruct_unit_coefficients_select_modes,
    test_mode_triplets_against_determinants,
    test_mode_contract_equals_reconstruct_route,
    test_mode_contract_identity_coefficients,
]

MUTATIONS = {
    "conjugated coefficients": ("flat @ Qi.T", "flat @ Qi.conj().T"),
    "coefficient axes swapped": ("(flat @ Qi.T).reshape(V, 3, Qi.shape[0])",
                                 "(flat @ Qi.T).reshape(Qi.shape[0], V, 3).transpose(1, 2, 0)"),
    "first two triplet indices swapped": ('"ai,bj,ck,pijk->pabc"', '"ai,bj,ck,pjik->pabc"'),
    "output axes swapped": ('"ai,bj,ck,pijk->pabc"', '"ai,bj,ck,pijk->pbac"'),
    "coefficient transposed": ('"ai,bj,ck,pijk->pabc"', '"ia,bj,ck,pijk->pabc"'),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mode_pins_catch_planted_mistake(name, tmp_path, monkeypatch):
    old, new = MUTATIONS[name]
    text = open(modes.__file__).read()
    assert text.count(old) == 1, name
    path = tmp_path / "modes_mutant.py"
    path.write_text(text.replace(old, new))
    spec = importlib.util.spec_from_file_location("modes_mutant", str(path))
    mutant = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mutant)
    for fn in ("reconstruct", "mode_triplets", "mode_contract"):
        monkeypatch.setattr(modes, fn, getattr(mutant, fn))
    failed = []
    for pin in PINS:
        try:
            pin()
        except (AssertionError, ValueError):
            failed.append(pin)
    assert failed, "no pin detects the mutation %r" % name
