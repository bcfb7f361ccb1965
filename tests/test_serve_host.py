"""Host logic of the serving runtime, no GPU: the arena sub-allocator keeps
disjoint 256-byte-aligned blocks inside its budget, places each block in the
smallest free range that holds it, coalesces neighbours on free, and agrees
with a brute-force byte-map model under a long random alloc/free sequence."""
from __future__ import annotations

import numpy as np
import pytest


@pytest.fixture(scope="module")
def bbx():
    import os

    import paper_2404_02826_amd as b
    if not os.path.exists(b.lib_path()):
        from paper_2404_02826_amd import build
        build.build()
    b.load()
    return b


def test_arena_basic(bbx):
    a = bbx.Arena(4096, 256)
    assert a.stats() == dict(used=0, free_total=4096, largest_free=4096, free_ranges=1)
    o1 = a.alloc(1)
    o2 = a.alloc(300)
    o3 = a.alloc(256)
    assert (o1, o2, o3) == (0, 256, 768)
    assert a.stats()["used"] == 1024
    a.free(o2)
    st = a.stats()
    assert st["free_ranges"] == 2 and st["free_total"] == 3584
    # best fit: a 256-byte request goes into the 512-byte hole, not the tail
    assert a.alloc(256) == 256
    a.free(256)
    a.free(o1)
    a.free(o3)
    assert a.stats() == dict(used=0, free_total=4096, largest_free=4096, free_ranges=1)


def test_arena_errors(bbx):
    a = bbx.Arena(1024, 256)
    with pytest.raises(bbx.BitboxError) as e:
        a.alloc(2048)
    assert e.value.name == "ENOMEM"
    o = a.alloc(512)
    with pytest.raises(bbx.BitboxError) as e:
        a.free(o + 256)  # not the start of a block
    assert e.value.name == "EINVAL"
    a.free(o)
    with pytest.raises(bbx.BitboxError):
        a.free(o)  # double free


def test_arena_matches_byte_model(bbx):
    rng = np.random.default_rng(3)
    size, al = 1 << 16, 256
    a = bbx.Arena(size, al)
    owner = np.full(size // al, -1, dtype=np.int64)  # unit -> block start
    live = {}
    for step in range(3000):
        if live and (rng.random() < 0.45 or len(live) > 40):
            off = list(live)[int(rng.integers(len(live)))]
            a.free(off)
            owner[off // al: (off + live.pop(off)) // al] = -1
        else:
            want = int(rng.integers(1, 4 * al))
            need = -(-want // al) * al
            # the model's best fit: smallest free run that holds it, lowest offset on ties
            free = owner < 0
            runs, i = [], 0
            while i < len(free):
                if free[i]:
                    j = i
                    while j < len(free) and free[j]:
                        j += 1
                    runs.append((i * al, (j - i) * al))
                    i = j
                else:
                    i += 1
            fits = [r for r in runs if r[1] >= need]
            if not fits:
                with pytest.raises(bbx.BitboxError):
                    a.alloc(want)
                continue
            exp = min(fits, key=lambda r: (r[1], r[0]))[0]
            off = a.alloc(want)
            assert off == exp, step
            assert (owner[off // al: (off + need) // al] == -1).all()
            owner[off // al: (off + need) // al] = off
            live[off] = need
        st = a.stats()
        assert st["used"] == sum(live.values())
        assert st["used"] + st["free_total"] == size
