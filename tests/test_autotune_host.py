"""The leaf-size and tile choices of the batch autotuner (no GPU): per set the
candidate leaf size with the smallest stream wins, ties go to the larger leaf
size, failed candidates never win unless all failed; the fastest tile wins."""
from __future__ import annotations

import pytest

from paper_2404_02826_amd.autotune import pick_leaf_sizes, pick_tile


def test_pick_leaf_sizes_smallest_stream():
    sizes = {8: [100, 50, 70], 16: [90, 60, 70], 32: [95, 40, 71]}
    assert pick_leaf_sizes(sizes) == [16, 32, 16]


def test_pick_leaf_sizes_failures():
    sizes = {8: [-1, -1], 16: [10, -1], 32: [12, -1]}
    assert pick_leaf_sizes(sizes) == [16, 32]  # all failed -> the largest candidate


def test_pick_leaf_sizes_ties_to_larger():
    assert pick_leaf_sizes({8: [5], 64: [5], 16: [5]}) == [64]


def test_pick_tile():
    assert pick_tile({256: 10.0, 512: 12.0}) == 256
    assert pick_tile({256: 10.0, 512: 10.0}) == 512
    with pytest.raises(ValueError):
        pick_tile({})
