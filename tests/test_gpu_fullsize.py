"""The full-size workload the benchmark times (fluid-shaped set, 2^27 FP32
particles, relative bound 1e-4, leaf size 32, default tile), checked by
properties that hold at any size and on outputs the oracle computes:

* the perm output is a permutation of the input;
* every reconstructed coordinate is within eb_abs of its source (all 2^27 x 3);
* the stream size and leaf count follow from the header and the size recursion;
* the oracle's decoder, run on the GPU stream, reproduces the GPU decode bit
  for bit;
* on 4096 sampled leaves, recomputed from the source points with the header's
  quantization: the stored reference code is the member nearest the AABB
  centre (first in index order on ties), members follow in ascending index,
  and every stored width is Eq. 2's minimal width;
* with the reference stored as its original coordinates (ref_mode 1): every
  leaf's first decoded slot is its reference's input coordinate bit for bit,
  every other slot decodes exactly as in the code-reference stream, and the
  meta section grows by exactly n_leaves * sum_d (32 - G_d) bits.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import props
from oracle import Oracle
from synth import fluid, fluid_lattice_dims

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 1 << 27


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _bits(stream: bytes, at: int, length: int) -> int:
    lo, hi = at // 8, (at + length + 7) // 8
    return (int.from_bytes(stream[lo:hi], "little") >> (at % 8)) & ((1 << length) - 1)


def _width(D: int) -> int:
    return 0 if D == 0 else D.bit_length() + 1


def test_fluid_2p27_full_size():
    import paper_2404_02826_amd as bbx
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    _say("generating the fluid 2^27 workload")
    pts = fluid(*fluid_lattice_dims(N), seed=4)
    x = torch.from_numpy(pts).cuda()
    s, perm = bbx.compress(x, 1e-4, "rel", 32, want_perm=True)
    dec = bbx.decompress(s)
    torch.cuda.synchronize()
    _say("compressed", s.numel(), "bytes")
    # permutation and bound, on the device
    cnt = torch.bincount(perm.long(), minlength=N)
    assert cnt.numel() == N and bool((cnt == 1).all()), "perm is not a permutation"
    del cnt
    stream = s.cpu().numpy().tobytes()
    h = props.parse_header(stream)
    err = (dec.double() - x[perm.long()].double()).abs().max().item()
    assert err <= h["eb_abs"], f"bound violated: {err} > {h['eb_abs']}"
    # sizes
    sizes = props.leaf_sizes_fast(N, 32)
    assert h["n"] == N and h["n_leaves"] == len(sizes) == Oracle().leaf_count(N, 32)
    assert len(stream) == props.stream_size(h["meta_bits"], h["payload_bits"])
    # the oracle's decoder on the GPU stream
    _say("oracle decode")
    ref_dec = Oracle().decompress(stream)
    assert np.array_equal(ref_dec, dec.cpu().numpy()), "GPU decode differs from the oracle's"
    del ref_dec
    # sampled leaves against the source points
    perm_h = perm.cpu().numpy().astype(np.int64)
    starts = np.cumsum(sizes) - sizes
    G = h["G"]
    dims, mbits = 3, 5
    S = dims * mbits + sum(G)
    rng = np.random.default_rng(11)
    for i in rng.choice(len(sizes), size=4096, replace=False):
        st, sz = int(starts[i]), int(sizes[i])
        src = perm_h[st:st + sz]
        assert (np.diff(src[1:]) > 0).all(), "members after the reference not in index order"
        q = np.floor((pts[src].astype(np.float64) - np.array(h["origin"])) * h["inv_w"] + 0.5).astype(np.int64)
        rec = _bits(stream, 128 * 8 + int(i) * S, S)
        m = [(rec >> (mbits * d)) & ((1 << mbits) - 1) for d in range(dims)]
        qref, at = [], dims * mbits
        for d in range(dims):
            qref.append((rec >> at) & ((1 << G[d]) - 1))
            at += G[d]
        assert list(q[0]) == qref, f"leaf {i}: stored reference code differs"
        qmin, qmax = q.min(axis=0), q.max(axis=0)
        dist = ((2 * q - (qmin + qmax)) ** 2).sum(axis=1)
        best = dist.min()
        cand = src[dist == best]
        assert src[0] == cand.min(), f"leaf {i}: reference is not the nearest (first) member"
        for d in range(dims):
            D = int(max(qref[d] - qmin[d], qmax[d] - qref[d]))
            assert m[d] == _width(D), f"leaf {i} axis {d}: width {m[d]} != {_width(D)}"
    _say("full-size checks passed")


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
