"""Mutation tests of the oracle pins (CPU only).

Each mutant is the oracle built with one plausible mistake planted
(-DBBXO_MUTANT=k in bbx_oracle.c).  The pin battery must pass on the
faithful build and fail on every mutant, which shows that the pins can see
a dropped term, a wrong sign, a wrong index or a wrong tie-break anywhere in
the oracle.
"""
from __future__ import annotations

import pytest

import pins
from oracle import Oracle
from oracle.build import build_oracle

MUTANTS = {
    1: "median joins the left child",
    2: "ties broken by descending index",
    3: "split axis fixed to x instead of round-robin",
    4: "reference is the first member, not the nearest to the AABB centre",
    5: "reference ties go to the last member",
    6: "Eq. 2 without the +1 (m = bitlen(D))",
    7: "largest offset taken as the AABB extent instead of the reference's reach",
    8: "axes written in reverse order in the payload",
    9: "bins of width eb instead of 2*eb",
    11: "reconstruction at the bin edge instead of its centre",
    12: "a node of exactly r particles is split",
    13: "members written in reverse order",
    14: "reference code field one bit too narrow",
    15: "relative bound scaled by the smallest range instead of the largest",
    16: "lossless reference field holds the leaf's first member, not its reference",
    17: "lossless reference decoded to its bin centre instead of its stored value",
    18: "rounding guard of a whole FP32 ulp instead of half of one",
    19: "R-index axes in descending instead of ascending entropy",
    20: "R-index with the first axis least significant",
    21: "reduction key: sum of box lengths where the sum of widths is asked, and the reverse",
    22: "reduction ties go to the last box",
    23: "boxes that lose particles keep their old bit box",
    24: "no common particles are absorbed",
    25: "common particles gathered in reverse leaf order",
    26: "lossless fallback stores a particle's axes in reverse order",
    27: "split rule 1 takes the narrowest axis",
    28: "split rule 2 gives the left child the larger half of the leaves",
    29: "split rule 3 sends codes on the midpoint to the left",
    30: "split rule 1 breaks extent ties towards the last axis",
    31: "split rule 3 stops at a one-code-wide axis instead of trying the next",
    32: "split rule 2 makes floor(n/r) leaves",
    33: "Huffman merges prefer the later node on equal weights",
    34: "canonical codes assigned in descending symbol order within a length",
    35: "Huffman merges the heaviest nodes",
    36: "chunk bit offsets one past the chunk's first code",
    37: "codes written least significant bit first",
}


def test_faithful_build_passes_battery(oracle):
    assert pins.run_battery(oracle) == []


@pytest.mark.parametrize("k", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, k):
    lib = build_oracle(str(tmp_path / f"libbbx_oracle_m{k}.so"), mutant=k)
    failed = pins.run_battery(Oracle(lib))
    assert failed, f"mutant {k} ({MUTANTS[k]}) passed every pin"
