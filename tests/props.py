"""Property checks that hold for any correct compressed stream (any size).

Shared by the oracle pins and the GPU parity tests.  These are definitions
from the paper, checked with vectorised numpy, not a re-implementation of
the compressor:
  P1 bound         every reconstructed coordinate within eb_abs (Sec. 3)
  P2 preservation  the output slots are a permutation of the input (Sec. 2.2)
  P3 tree          each split is a median split along the round-robin axis,
                   ties by index, median on the larger side (Sec. 4.1)
  P4 minimal bits  each leaf's widths hold every offset, one bit fewer fails
                   (Eq. 1 / Eq. 2)
  P5 reference     the stored reference is the member nearest the AABB centre
  P6 size          stream length matches the section sizes (Sec. 4.2 cost model)
"""
from __future__ import annotations

import struct

import numpy as np

HDR = "<4sHBBQIBBBBddddd3d3B5xQQQQ"


def parse_header(stream: bytes) -> dict:
    f = struct.unpack(HDR, bytes(stream[:128]))
    return dict(magic=f[0], version=f[1], dtype=f[2], dims=f[3], n=f[4], r=f[5], eb_mode=f[6],
                split_rule=f[7], ref_mode=f[8], mbits=f[9], eb_user=f[10], eb_abs=f[11],
                eb_eff=f[12], w=f[13], inv_w=f[14], origin=list(f[15:18]), G=list(f[18:21]),
                n_leaves=f[21], meta_bits=f[22], payload_bits=f[23], reserved=f[24])


def leaf_sizes(n: int, r: int) -> np.ndarray:
    """Leaf sizes of the size-only recursion (children floor(s/2), ceil(s/2)),
    computed level by level: at depth k every node has floor(n/2^k) or
    ceil(n/2^k) particles."""
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    sizes = np.array([n], dtype=np.int64)
    done = np.array([n <= r])
    while not done.all():
        out = []
        for s, d in zip(sizes.tolist(), done.tolist()):
            if d:
                out.append((s, True))
            else:
                out.append((s // 2, s // 2 <= r))
                out.append((s - s // 2, s - s // 2 <= r))
        sizes = np.array([o[0] for o in out], dtype=np.int64)
        done = np.array([o[1] for o in out])
    return sizes


def leaf_sizes_fast(n: int, r: int) -> np.ndarray:
    """Same as leaf_sizes, vectorised per level (for large n)."""
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    sizes = np.array([n], dtype=np.int64)
    leaf = sizes <= r
    while not leaf.all():
        lo = sizes // 2
        hi = sizes - lo
        split = ~leaf
        # each split node becomes two entries, leaves stay
        rep = np.where(split, 2, 1)
        new = np.repeat(sizes, rep)
        idx = np.cumsum(rep) - rep
        new[idx[split]] = lo[split]
        new[idx[split] + 1] = hi[split]
        sizes = new
        leaf = sizes <= r
    return sizes


def tree_order_from_perm(perm: np.ndarray, sizes: np.ndarray) -> np.ndarray:
    """Output slots hold [reference, other members ascending]; the tree order
    holds every leaf's members ascending.  Sort each leaf's slots."""
    n = len(perm)
    leaf_id = np.repeat(np.arange(len(sizes)), sizes)
    key = leaf_id.astype(np.uint64) << np.uint64(32) | perm.astype(np.uint64)
    return (np.sort(key) & np.uint64(0xFFFFFFFF)).astype(np.int64)[:n]


def check_bound(points: np.ndarray, decoded: np.ndarray, perm: np.ndarray, eb_abs: float):
    """P1: |x - x_hat| <= eb_abs for every coordinate, compared in FP64."""
    if len(perm) == 0:
        return 0.0
    err = np.abs(decoded.astype(np.float64) - points[perm].astype(np.float64))
    worst = float(err.max())
    assert worst <= eb_abs, f"bound violated: {worst} > {eb_abs}"
    return worst


def check_permutation(perm: np.ndarray, n: int):
    """P2: every particle appears exactly once."""
    assert len(perm) == n
    if n:
        seen = np.zeros(n, dtype=np.int64)
        np.add.at(seen, perm.astype(np.int64), 1)
        assert (seen == 1).all(), "output slots are not a permutation of the input"


def check_tree(codes: np.ndarray, order: np.ndarray, n: int, r: int, dims: int):
    """P3 on the whole tree: for every internal node (depth k, axis k mod
    dims) all of the left child precedes all of the right child in
    (code, index) order, the left child has floor(s/2) particles, every
    leaf holds <= r particles in ascending index order."""
    if n == 0:
        return
    order = order.astype(np.int64)
    sizes = np.array([n], dtype=np.int64)
    depth = 0
    while True:
        inner = sizes > r
        if not inner.any():
            break
        d = depth % dims
        key = (codes[d].astype(np.uint64)[order] << np.uint64(32)) | order.astype(np.uint64)
        starts = np.cumsum(sizes) - sizes
        half = sizes // 2
        bounds = np.empty(2 * len(sizes), dtype=np.int64)
        bounds[0::2] = starts
        bounds[1::2] = starts + half
        lmax = np.maximum.reduceat(key, bounds)[0::2]
        rmin = np.minimum.reduceat(key, bounds)[1::2]
        assert (lmax[inner] < rmin[inner]).all(), f"median split violated at depth {depth}"
        rep = np.where(inner, 2, 1)
        new = np.repeat(sizes, rep)
        at = (np.cumsum(rep) - rep)[inner]
        new[at] = half[inner]
        new[at + 1] = sizes[inner] - half[inner]
        sizes = new
        depth += 1
    assert (sizes <= r).all()
    # ascending index inside every leaf
    leaf_id = np.repeat(np.arange(len(sizes)), sizes)
    same = leaf_id[1:] == leaf_id[:-1]
    assert (order[1:][same] > order[:-1][same]).all(), "leaf members not in ascending index"


def check_bitboxes(codes: np.ndarray, order: np.ndarray, sizes: np.ndarray, ref_pos: np.ndarray,
                   m: np.ndarray, dims: int):
    """P4 + P5 per leaf, vectorised.  order: tree order; ref_pos: position of
    the reference within its leaf; m: [n_leaves, dims] widths."""
    nl = len(sizes)
    if nl == 0:
        return
    starts = np.cumsum(sizes) - sizes
    q = np.stack([codes[d].astype(np.int64)[order] for d in range(dims)], axis=1)  # tree order
    qmin = np.stack([np.minimum.reduceat(q[:, d], starts) for d in range(dims)], axis=1)
    qmax = np.stack([np.maximum.reduceat(q[:, d], starts) for d in range(dims)], axis=1)
    leaf_id = np.repeat(np.arange(nl), sizes)
    C = qmin + qmax
    t = (2 * q - C[leaf_id]).astype(np.uint64)  # |t| <= 2^31; squares wrap exactly mod 2^64
    dist = (t * t).sum(axis=1, dtype=np.uint64)
    best = np.minimum.reduceat(dist, starts)
    # first member attaining the minimum
    hit = dist == best[leaf_id]
    local = np.arange(len(order)) - starts[leaf_id]
    first = np.full(nl, np.iinfo(np.int64).max, dtype=np.int64)
    np.minimum.at(first, leaf_id[hit], local[hit])
    assert np.array_equal(first, ref_pos.astype(np.int64)), "reference is not the member nearest the AABB centre"
    qref = q[starts + ref_pos.astype(np.int64)]
    off = np.abs(q - qref[leaf_id])
    D = np.stack([np.maximum.reduceat(off[:, d], starts) for d in range(dims)], axis=1)
    mm = m.astype(np.int64)
    reach = np.where(mm > 0, (np.int64(1) << np.maximum(mm - 1, 0)) - 1, 0)
    assert (D <= reach).all(), "a member falls outside its bit box"
    smaller = np.maximum(mm - 1, 0)
    reach_less = np.where(smaller > 0, (np.int64(1) << np.maximum(smaller - 1, 0)) - 1, 0)
    assert ((mm == 0) | (D > reach_less)).all(), "bit width is not minimal"


def stream_size(meta_bits: int, payload_bits: int) -> int:
    return 128 + 8 * ((meta_bits + 63) // 64) + 8 * ((payload_bits + 63) // 64)


def psnr(points: np.ndarray, decoded: np.ndarray, perm: np.ndarray) -> float:
    """Sec. 5.1 NRMSE normalised by the largest coordinate range, PSNR = -20 log10 NRMSE."""
    x = points[perm].astype(np.float64)
    y = decoded.astype(np.float64)
    rng = (points.max(axis=0).astype(np.float64) - points.min(axis=0).astype(np.float64)).max()
    nrmse = np.sqrt(np.mean(((x - y) / rng) ** 2))
    return float(-20.0 * np.log10(nrmse))


def reduced_sequences(stream: bytes) -> list:
    """Meta records of a reduced (version 2) stream: per sequence its widths,
    centre codes and particle count (besides the centre)."""
    h = parse_header(stream)
    dims, mbits, G = h["dims"], h["mbits"], h["G"][: h["dims"]]
    mb = 8 * ((h["meta_bits"] + 63) // 64)
    meta = int.from_bytes(bytes(stream[128:128 + mb]), "little")
    out, at = [], 0
    for _ in range(h["reserved"]):
        m = []
        for d in range(dims):
            m.append((meta >> at) & ((1 << mbits) - 1))
            at += mbits
        c = []
        for d in range(dims):
            c.append((meta >> at) & ((1 << G[d]) - 1))
            at += G[d]
        cnt = (meta >> at) & 0xFFFFFFFF
        at += 32
        out.append(dict(m=m, centre=c, count=cnt))
    return out


def check_reduced(points: np.ndarray, stream: bytes, perm: np.ndarray, decoded: np.ndarray,
                  codes: np.ndarray, n_leaves: int):
    """A reduced stream by definitions: every particle once, within the bound,
    every particle of a sequence inside its bit box (its offsets from the
    centre fit the sequence's widths, Eq. 1), at most one sequence per leaf,
    none empty."""
    h = parse_header(stream)
    n, dims = points.shape
    check_permutation(perm, n)
    check_bound(points, decoded, perm, h["eb_abs"])
    seqs = reduced_sequences(stream)
    assert 1 <= len(seqs) <= n_leaves if n else len(seqs) == 0
    slot = 0
    for sq in seqs:
        ctr = perm[slot]
        assert [int(codes[d][ctr]) for d in range(dims)] == sq["centre"], "centre code"
        reach = [(1 << (m - 1)) - 1 if m else 0 for m in sq["m"]]
        for i in perm[slot + 1: slot + 1 + sq["count"]]:
            for d in range(dims):
                assert abs(int(codes[d][i]) - sq["centre"][d]) <= reach[d], "particle outside its box"
        slot += 1 + sq["count"]
    assert slot == n

