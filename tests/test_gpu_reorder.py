"""GPU parity of the two reorderings of Sec. 4.2 (sequences by sum of widths,
members by R-index with the axes in ascending entropy of their widths): the
library's reordered sequence layout and axis order against the oracle's,
byte for byte, over 2-D and 3-D sets, FP32 and FP64, leaves of one member,
of 32, and of more members than the on-chip ranking holds; then the whole
entropy stage (reordered layout, then Huffman coding) against the oracle."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import Oracle
from synth import cosmology, fluid, fluid_lattice_dims, poincare, uniform_cube

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bbx():
    import paper_2404_02826_amd as b
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    b.load()
    return b


@pytest.fixture(scope="module")
def orc():
    return Oracle()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(b: bytes):
    t = torch.zeros(max(len(b), 1) + 16, dtype=torch.uint8, device="cuda")[: len(b)]
    if b:
        t.copy_(torch.from_numpy(np.frombuffer(b, dtype=np.uint8).copy()))
    return t


# (generator, n, dims, dtype, eb, r)
CASES = [
    ("uniform", 1, 3, np.float32, 1e-3, 32),
    ("uniform", 2000, 3, np.float32, 1e-2, 1),
    ("uniform", 65536, 3, np.float32, 1e-3, 32),
    ("cosmology", 40000, 3, np.float32, 1e-4, 32),
    ("cosmology", 30011, 3, np.float64, 1e-5, 16),
    ("fluid", 32768, 3, np.float32, 1e-4, 32),
    ("poincare", 20000, 2, np.float32, 1e-4, 32),
    ("cosmology", 9000, 3, np.float32, 1e-3, 600),   # members ranked from the layout
]


def _gen(kind, n, dims, dt, seed):
    if kind == "uniform":
        return uniform_cube(n, seed=seed, dims=dims, dtype=dt)
    if kind == "cosmology":
        return cosmology(n, seed=seed, dims=dims, dtype=dt)
    if kind == "fluid":
        return fluid(*fluid_lattice_dims(n), seed=seed, dtype=dt)
    return poincare(n, seed=seed, dtype=dt)


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-n{c[1]}-d{c[2]}-{np.dtype(c[3]).name}-r{c[5]}"
                                             for c in CASES])
def test_reordered_layout_parity(orc, bbx, case):
    kind, n, dims, dt, eb, r = case
    _say(f"reordered layout parity: {case}")
    pts = _gen(kind, n, dims, dt, seed=n % 89 + r)
    s = orc.compress(pts, eb, "rel", r, ref_mode=1)
    ref, ref_order = orc.export_sequences_reordered(s)
    got, order = bbx.export_sequences_reordered(_dev(s))
    torch.cuda.synchronize()
    assert order == [int(v) for v in ref_order[:dims]], (order, ref_order)
    gb = got.cpu().numpy().tobytes()
    assert len(gb) == len(ref) and gb == ref, "reordered layout differs from the oracle's"


def test_entropy_stage_end_to_end(orc, bbx):
    pts = cosmology(120000, seed=40)
    x = torch.from_numpy(pts).cuda()
    s = bbx.compress(x, 1e-4, "rel", 32, ref_mode=1)
    ref_s = orc.compress(pts, 1e-4, "rel", 32, ref_mode=1)
    assert s.cpu().numpy().tobytes() == ref_s
    lay, _ = bbx.export_sequences_reordered(s)
    h = bbx.huffman_encode(lay)
    ref_h = orc.huffman_encode(orc.export_sequences_reordered(ref_s)[0])
    assert h.cpu().numpy().tobytes() == ref_h
    assert torch.equal(bbx.huffman_decode(h), lay)


def test_reorder_refuses_code_references(bbx):
    x = torch.from_numpy(uniform_cube(1000, seed=41)).cuda()
    s = bbx.compress(x, 1e-3, "rel", 32)  # ref_mode 0
    with pytest.raises(bbx.BitboxError):
        bbx.export_sequences_reordered(s)
