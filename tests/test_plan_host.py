"""The launch planner against what the partition kernels assume of it (CPU
only, no GPU): bbx_plan_check plans a batch exactly as a compress call would
and checks level kinds, chunk shapes, buffer capacities, fused pairs and the
leaf stage.  Swept over set sizes from 10^3 to 2^27 and every block target a
set can get (alone: 1024, or less with the level_blocks cap; in a batch: its
share of 16384 by particle count, 1..4096, reproduced with the cap and, above
1024, with a second set sized to give the first that share)."""
from __future__ import annotations

import numpy as np
import pytest

bbx = pytest.importorskip("paper_2404_02826_amd")

TARGETS = [1, 2, 3, 5, 7, 16, 31, 64, 100, 255, 256, 257, 1000, 1024, 2047, 2048, 3000, 4095, 4096]


def _sizes():
    out = set()
    for e in range(10, 28):
        for d in (-3, -1, 0, 1, 5):
            out.add((1 << e) + d)
    rng = np.random.default_rng(9)
    out.update(int(v) for v in np.exp(rng.uniform(np.log(1e3), np.log(1 << 27), 40)))
    return sorted(v for v in out if 1000 <= v <= (1 << 27))


@pytest.mark.parametrize("tile", [256, 512])
def test_plan_single_sets(tile):
    for n in _sizes():
        for r in (1, 8, 32, 255, 256, 257, 1000, 5000):
            for lb in TARGETS:
                bbx.plan_check([dict(n=n, leaf_size=r, tile=tile, level_blocks=lb)])
            bbx.plan_check([dict(n=n, leaf_size=r, tile=tile, want_perm=True)])
            bbx.plan_check([dict(n=n, leaf_size=r, tile=tile, dims=2, dtype=1, ref_mode=1)])
            for lb in (1, 100, 4096):  # paired global levels
                bbx.plan_check([dict(n=n, leaf_size=r, tile=tile, level_blocks=lb, level_pairs=1)])


def test_plan_batch_shares_above_solo_target():
    # a set of n beside one of m particles gets round(16384 n / (n + m)) blocks
    # per global level, capped at 4096: the shapes above a set alone's 1024
    for n in _sizes()[::3]:
        for share in (1025, 1500, 2048, 3000, 4095, 4096):
            m = max(1, round(n * (16384 / share - 1)))
            bbx.plan_check([dict(n=n, leaf_size=32), dict(n=m, leaf_size=32)])
            bbx.plan_check([dict(n=n, leaf_size=8, want_perm=True), dict(n=m, leaf_size=300)])


def test_plan_batches():
    from synth import batch_plan
    sizes, kinds, ebs = batch_plan(4096, 5)
    sets = [dict(n=int(n), eb=float(e)) for n, e in zip(sizes, ebs)]
    bbx.plan_check(sets)
    rng = np.random.default_rng(4)
    for _ in range(30):
        k = int(rng.integers(2, 40))
        ns = np.exp(rng.uniform(np.log(1e3), np.log(1 << 26), k)).astype(np.int64)
        bbx.plan_check([dict(n=int(n), leaf_size=int(rng.choice([8, 16, 32, 64, 300])),
                             want_perm=bool(rng.random() < 0.3),
                             level_pairs=int(rng.random() < 0.5)) for n in ns])


def test_plan_check_rejects_bad_arguments():
    with pytest.raises(bbx.BitboxError, match="level_blocks"):
        bbx.plan_check([dict(n=5000, level_blocks=5000)])
    with pytest.raises(bbx.BitboxError, match="level_pairs"):
        bbx.plan_check([dict(n=5000, level_pairs=2)])
