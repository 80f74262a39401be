"""The pins in test_oracle_pins.py are sensitive: each plausible mistake
planted in a copy of the oracle source (on the CPU) makes at least one pin
fail.  This guards against pins that would pass for a wrong oracle.  A
mistake in an expression the rows and entries variants share is planted in
both; one in the entries variant alone is caught by its determinant pin."""
from __future__ import annotations

import os

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "bblock_oracle.c")

MUTATIONS = {
    "phase sign": ("return cos(ang) - I * sin(ang);", "return cos(ang) + I * sin(ang);"),
    "epsilon sign": ("return ((a - b) * (b - c) * (c - a)) / 2;", "return -((a - b) * (b - c) * (c - a)) / 2;"),
    "dropped epsilon term": ("if (e == 0) continue;", "if (e == 0 || (a == 2 && b == 1)) continue;"),
    "axis order": ("const int64_t ix = x % L, iy = (x / L) % L,", "const int64_t iy = x % L, ix = (x / L) % L,"),
    "momentum component": ("mod_nonneg(nx * ix + ny * iy + nz * iz, L)", "mod_nonneg(ny * ix + nx * iy + nz * iz, L)"),
    "reversed d3 column": ("* Q3[(x * 3 + c) * n3 + d3];", "* Q3[(x * 3 + c) * n3 + (n3 - 1 - d3)];"),
    "colour/dilution transposed": ("* Q2[(x * 3 + b) * n2 + d2]", "* Q2[(x * n2 + d2) * 3 + b]"),
    "colour of q2 rotated": ("* Q2[(x * 3 + b) * n2 + d2]", "* Q2[(x * 3 + (b + 1) % 3) * n2 + d2]"),
    "phase off by one site": ("ph[p] = phase_of_index(mod_nonneg(nx * ix", "ph[p] = phase_of_index(mod_nonneg(nx * (ix + 1)"),
    "entries: phase index shifted": ("acc[p] += root[mod_nonneg(nx * ix + ny * iy + nz * iz, L)]",
                                     "acc[p] += root[(mod_nonneg(nx * ix + ny * iy + nz * iz, L) + 1) % L]"),
    "entries: epsilon term dropped": ("if (eps == 0) continue;", "if (eps == 0 || (a == 0 && b == 2)) continue;"),
    "entries: d2 read as d1": ("const int d1 = entries[3 * e], d2 = entries[3 * e + 1],",
                               "const int d1 = entries[3 * e], d2 = entries[3 * e] % n2,"),
}

PINS = [
    pins.test_golden_hand_examples,
    lambda: pins.test_bruteforce_determinant(3, (2, 3, 5)),
    lambda: pins.test_translation_phase((1, 2, 3)),
    pins.test_single_site_field,
    pins.test_plane_waves_momentum_conservation,
    pins.test_field_swap_antisymmetry,
    pins.test_dilution_permutation_and_trilinearity,
    pins.test_mode_triplet_route,
    pins.test_entries_against_determinants,
]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path, monkeypatch):
    old, new = MUTATIONS[name]
    text = open(SRC).read()
    assert text.count(old) >= 1, name
    src = tmp_path / "mutant.c"
    src.write_text(text.replace(old, new))  # every occurrence: the variants stay consistent
    lib = oracle.load_library(oracle.build(str(src), str(tmp_path / "mutant.so")))
    monkeypatch.setattr(oracle, "_lib", lib)
    failed = []
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failed.append(pin)
    assert failed, "no pin detects the mutation %r" % name
