"""The benchmark-sized workloads against the oracle, byte for byte.

tests/golden/fullsize_digests.json holds SHA-256 digests of the oracle's
stream, perm and decode for the fluid-shaped 2^27 FP32 set (relative bound
1e-4, leaf size 32: the benchmark's own workload and launch configuration),
the fluid-shaped 2^26 FP64 set and the cosmology-shaped 2^24 FP32 set at
1e-4 and 1e-3 (written by tests/golden/make_fullsize_digests.py from the
oracle alone).  The library's outputs must have the same digests.  On the
2^27 set the whole tree and every leaf's bit box are also checked by
properties (every split a median split on the round-robin axis with index
ties, leaves in ascending index, each reference the member nearest its
AABB centre, each width Eq. 2's minimal width), which localise a mismatch;
and every reconstructed coordinate is within eb_abs.  With the reference
stored as its original coordinates (ref_mode 1): every leaf's first decoded
slot is its reference's input coordinate bit for bit, every other slot
decodes exactly as in the code-reference stream, and the meta section grows
by exactly n_leaves * sum_d (32 - G_d) bits.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys

import numpy as np
import pytest

import props
from synth import cosmology, fluid, fluid_lattice_dims

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]

N = 1 << 27
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_digests.json")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sha(t) -> str:
    if isinstance(t, torch.Tensor):
        t = t.cpu().numpy()
    return hashlib.sha256(np.ascontiguousarray(t).tobytes()).hexdigest()


def _points(name, g):
    dt = np.dtype(g["dtype"]).type
    if name.startswith("fluid"):
        return fluid(*fluid_lattice_dims(g["n"]), seed=4, dtype=dt)
    return cosmology(g["n"], seed=2, dtype=dt)


with open(GOLDEN) as _f:
    DIGESTS = json.load(_f)


@pytest.mark.parametrize("name", sorted(DIGESTS))
def test_full_size_digests(name):
    import paper_2404_02826_amd as bbx
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    g = DIGESTS[name]
    _say(f"{name}: generating {g['n']} particles")
    pts = _points(name, g)
    assert _sha(pts) == g["input_sha256"], "generator output drifted"
    x = torch.from_numpy(pts).cuda()
    s, perm = bbx.compress(x, g["eb_rel"], "rel", g["leaf_size"], want_perm=True)
    dec = bbx.decompress(s)
    torch.cuda.synchronize()
    _say(f"{name}: {s.numel()} bytes (oracle {g['stream_bytes']})")
    got = {"stream": _sha(s), "perm": _sha(perm.to(torch.int32)), "decode": _sha(dec)}
    if name == "fluid-2^27-f32":
        _check_fluid_tree(pts, x, s, perm, dec)
    assert s.numel() == g["stream_bytes"], "stream size differs from the oracle's"
    assert got["stream"] == g["stream_sha256"], "stream bytes differ from the oracle's"
    assert got["perm"] == g["perm_sha256"], "perm differs from the oracle's"
    assert got["decode"] == g["decode_sha256"], "decoded positions differ from the oracle's"


def _check_fluid_tree(pts, x, s, perm, dec):
    """Properties of the whole 2^27 stream: permutation and bound on the
    device; tree and bit boxes of every leaf on the host."""
    cnt = torch.bincount(perm.long(), minlength=N)
    assert cnt.numel() == N and bool((cnt == 1).all()), "perm is not a permutation"
    del cnt
    stream = s.cpu().numpy().tobytes()
    h = props.parse_header(stream)
    err = (dec.double() - x[perm.long()].double()).abs().max().item()
    assert err <= h["eb_abs"], f"bound violated: {err} > {h['eb_abs']}"
    sizes = props.leaf_sizes_fast(N, 32)
    assert h["n"] == N and h["n_leaves"] == len(sizes)
    assert len(stream) == props.stream_size(h["meta_bits"], h["payload_bits"])
    _say("tree and bit boxes of every leaf")
    codes = np.empty((3, N), dtype=np.uint32)
    for d in range(3):
        codes[d] = np.floor((pts[:, d].astype(np.float64) - h["origin"][d]) * h["inv_w"] + 0.5)
    order = props.tree_order_from_perm(perm.cpu().numpy().astype(np.int64), sizes)
    props.check_tree(codes, order, N, 32, 3)
    # stored widths and references from the meta records
    G, mbits = h["G"], 5
    S = 3 * mbits + sum(G)
    meta = np.frombuffer(stream, dtype=np.uint8, count=8 * ((h["meta_bits"] + 63) // 64), offset=128)
    bits = np.unpackbits(meta, bitorder="little")
    rec = bits[: len(sizes) * S].reshape(len(sizes), S)[:, : 3 * mbits].astype(np.int64)
    del bits
    m = np.stack([(rec[:, mbits * d: mbits * (d + 1)] << np.arange(mbits)).sum(axis=1)
                  for d in range(3)], axis=1)
    del rec
    # the reference is each leaf's first output slot: its position in tree order
    starts = np.cumsum(sizes) - sizes
    ref_src = perm.cpu().numpy().astype(np.int64)[starts]
    leaf_id = np.repeat(np.arange(len(sizes)), sizes)
    ref_pos = np.zeros(len(sizes), dtype=np.int64)
    hit = order == ref_src[leaf_id]
    ref_pos[leaf_id[hit]] = (np.arange(N) - starts[leaf_id])[hit]
    props.check_bitboxes(codes, order, sizes, ref_pos, m, 3)
    _say("full-size properties hold")


def test_fluid_2p27_lossless_reference():
    import paper_2404_02826_amd as bbx
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    _say("generating the fluid 2^27 workload (lossless references)")
    pts = fluid(*fluid_lattice_dims(N), seed=4)
    x = torch.from_numpy(pts).cuda()
    del pts
    s1, p1 = bbx.compress(x, 1e-4, "rel", 32, want_perm=True, ref_mode=1)
    s0, p0 = bbx.compress(x, 1e-4, "rel", 32, want_perm=True)
    assert torch.equal(p0, p1), "the tree depends on the reference storage"
    del p0
    d1, d0 = bbx.decompress(s1), bbx.decompress(s0)
    torch.cuda.synchronize()
    h1 = props.parse_header(s1[:128].cpu().numpy().tobytes())
    h0 = props.parse_header(s0[:128].cpu().numpy().tobytes())
    assert h1["ref_mode"] == 1 and h0["ref_mode"] == 0
    assert h1["payload_bits"] == h0["payload_bits"]
    assert h1["meta_bits"] - h0["meta_bits"] == h0["n_leaves"] * sum(32 - g for g in h0["G"])
    assert s1.numel() == props.stream_size(h1["meta_bits"], h1["payload_bits"])
    sizes = props.leaf_sizes_fast(N, 32)
    first = torch.zeros(N, dtype=torch.bool, device="cuda")
    first[torch.from_numpy((np.cumsum(sizes) - sizes).astype(np.int64)).cuda()] = True
    src = x[p1.long()]
    assert torch.equal(d1[first].view(torch.int32), src[first].view(torch.int32)), \
        "a reference does not decode to its input coordinate"
    assert torch.equal(d1[~first].view(torch.int32), d0[~first].view(torch.int32)), \
        "members decode differently from the code-reference stream"
    err = (d1.double() - src.double()).abs().max().item()
    assert err <= h1["eb_abs"], f"bound violated: {err} > {h1['eb_abs']}"
    _say("lossless-reference full-size checks passed")
