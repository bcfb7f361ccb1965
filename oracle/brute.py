"""Pure-Python brute-force re-derivation of the compressor for tiny inputs.

TEST INFRASTRUCTURE ONLY.  A third, independently formulated implementation
used to pin the C oracle: where the C oracle uses closed forms this module
searches exhaustively, and it builds the stream with Python big integers
instead of a bit-at-a-time byte writer.

  * bin widths: smallest m whose Eq. 1 predictable range holds every member
    (searched m = 0, 1, 2, ...), instead of the bitlen(D) + 1 closed form;
  * reference: exact rational distance to the AABB centre (Sec. 4.1), or
    (reference rule 1) every member tried as the reference, keeping the one
    whose searched widths have the smallest sum;
  * tree: the median definition applied with ``sorted`` at every node.
"""
from __future__ import annotations

import math
import struct
from fractions import Fraction

import numpy as np


def _coords(points: np.ndarray):
    return [[float(v) for v in row] for row in points]


def bound_params(points: np.ndarray, eb: float, eb_mode: str):
    """Range, error bound, guard and bin width (Sec. 3 + the rounding guard)."""
    pts = _coords(points)
    n = len(pts)
    dims = points.shape[1]
    f32 = points.dtype == np.float32
    if n == 0:
        return dict(lo=[0.0] * dims, hi=[0.0] * dims, eb_abs=(eb if eb_mode == "abs" else 0.0),
                    eb_eff=0.0, w=0.0, inv_w=0.0, G=[0] * dims)
    lo = [min(p[d] for p in pts) + 0.0 for d in range(dims)]
    hi = [max(p[d] for p in pts) + 0.0 for d in range(dims)]
    delta = max(hi[d] - lo[d] for d in range(dims))
    eb_abs = eb * delta if eb_mode == "rel" else eb
    if delta == 0.0:
        return dict(lo=lo, hi=hi, eb_abs=eb_abs, eb_eff=0.0, w=0.0, inv_w=0.0, G=[0] * dims)
    amax = max(max(abs(lo[d]), abs(hi[d])) for d in range(dims)) + eb_abs
    guard = math.ldexp(amax, -48)
    if f32:
        _, e = math.frexp(amax)
        guard += max(math.ldexp(1.0, e - 25), math.ldexp(1.0, -150))
    eb_eff = eb_abs - guard
    if not eb_eff > 0:
        raise ValueError("EBOUND")
    w = 2.0 * eb_eff
    inv_w = 1.0 / w
    codes = [[math.floor((p[d] - lo[d]) * inv_w + 0.5) for d in range(dims)] for p in pts]
    qmax = [max(c[d] for c in codes) for d in range(dims)]
    if max(qmax) >= (1 << 30):
        raise ValueError("EBOUND")
    G = [int(v).bit_length() for v in qmax]
    return dict(lo=lo, hi=hi, eb_abs=eb_abs, eb_eff=eb_eff, w=w, inv_w=inv_w, G=G, codes=codes)


def quantize(points: np.ndarray, prm: dict):
    if "codes" in prm:
        return prm["codes"]
    return [[0] * points.shape[1] for _ in range(points.shape[0])]


def kd_leaves(codes, r: int, dims: int, rule: int = 0, G=None):
    """Leaves (lists of original indices, ascending) in depth-first order.

    rule 0: halve (floor(s/2) smallest (code, index) pairs go left) until at
    most r, axes in turn; rule 1: the same along the axis whose codes spread
    widest (lowest axis on ties); rule 2: ceil(n/r) leaves, leaf i holding
    the ranks floor(i*n/b) .. floor((i+1)*n/b) - 1, every node giving its
    left child the first half (rounded down) of its leaves; rule 3: cells of
    the code grid [0, 2^G_d) halved at their midpoints, axes in turn with
    one-code-wide axes skipped, empty halves dropped."""
    leaves = []
    n = len(codes)
    b = -(-n // r) if n else 0

    def by_rank(members, d, k):
        ranked = sorted(members, key=lambda i: (codes[i][d], i))
        left = set(ranked[:k])
        return [i for i in members if i in left], [i for i in members if i not in left]

    def split(members, depth, i0, i1, cell):
        d = depth % dims
        if rule == 2:
            if i1 - i0 == 1:
                leaves.append(members)
                return
            im = (i0 + i1) // 2
            lo, hi = by_rank(members, d, im * n // b - i0 * n // b)
            split(lo, depth + 1, i0, im, cell)
            split(hi, depth + 1, im, i1, cell)
            return
        if len(members) <= r:
            leaves.append(members)
            return
        if rule == 3:
            axes = [(d + k) % dims for k in range(dims) if cell[(d + k) % dims][1] > 1]
            if not axes:
                leaves.append(members)
                return
            d = axes[0]
            start, width = cell[d]
            mid = start + width // 2
            lo = [i for i in members if codes[i][d] < mid]
            hi = [i for i in members if codes[i][d] >= mid]
            for part, c in ((lo, (start, width // 2)), (hi, (mid, width // 2))):
                if part:
                    split(part, depth + 1, i0, i1, [c if a == d else cell[a] for a in range(dims)])
            return
        if rule == 1:
            spread = [max(codes[i][a] for i in members) - min(codes[i][a] for i in members)
                      for a in range(dims)]
            d = max(range(dims), key=lambda a: (spread[a], -a))
        lo, hi = by_rank(members, d, len(members) // 2)
        split(lo, depth + 1, i0, i1, cell)
        split(hi, depth + 1, i0, i1, cell)

    if n:
        cell = [(0, 1 << (G[a] if G else 0)) for a in range(dims)]
        split(list(range(n)), 0, 0, b, cell)
    return leaves


def minimal_bits(offsets) -> int:
    """Smallest m whose 2^m - 1 intervals centred on the reference hold every
    offset (Eq. 1 in code units: |o| <= 2^(m-1) - 1; m = 0 holds only 0)."""
    m = 0
    while True:
        reach = 0 if m == 0 else (1 << (m - 1)) - 1
        if all(abs(o) <= reach for o in offsets):
            return m
        m += 1


def bit_box(codes, members, dims, ref_rule=0):
    def widths(ref):
        return [minimal_bits([codes[i][d] - codes[ref][d] for i in members]) for d in range(dims)]
    if ref_rule == 1:
        best = min(range(len(members)), key=lambda j: (sum(widths(members[j])), j))
    else:
        lo = [min(codes[i][d] for i in members) for d in range(dims)]
        hi = [max(codes[i][d] for i in members) for d in range(dims)]
        centre = [Fraction(lo[d] + hi[d], 2) for d in range(dims)]
        best = min(range(len(members)),
                   key=lambda j: (sum((codes[members[j]][d] - centre[d]) ** 2 for d in range(dims)), j))
    return best, widths(members[best])


def _raw_bits(points: np.ndarray, i: int, d: int) -> int:
    """IEEE bits of one input coordinate (32 or 64 of them)."""
    v = points[i, d:d + 1]
    return int(v.view(np.uint32 if points.dtype == np.float32 else np.uint64)[0])


def _from_bits(raw: int, f32: bool):
    if f32:
        return np.array([raw], dtype=np.uint32).view(np.float32)[0]
    return np.array([raw], dtype=np.uint64).view(np.float64)[0]


def lossless_stream(points: np.ndarray, eb: float, eb_mode: str, r: int):
    """Sec. 4.1's lossless escape for a whole set whose bound the grid cannot
    meet: version-3 header, then every coordinate's bits in input order."""
    n, dims = points.shape
    f32 = points.dtype == np.float32
    pts = _coords(points)
    if eb_mode == "rel":
        lo = [min(p[d] for p in pts) + 0.0 for d in range(dims)]
        hi = [max(p[d] for p in pts) + 0.0 for d in range(dims)]
        eb_abs = eb * max(hi[d] - lo[d] for d in range(dims))
    else:
        eb_abs = eb
    M = 32 if f32 else 64
    pay = 0
    at = 0
    for i in range(n):
        for d in range(dims):
            pay |= _raw_bits(points, i, d) << at
            at += M
    header = struct.pack("<4sHBBQIBBBBddddd3d3B5xQQQQ", b"BBX1", 3, 0 if f32 else 1, dims, n, r,
                         0 if eb_mode == "rel" else 1, 0, 0, 5 if f32 else 6, eb, eb_abs, 0.0,
                         0.0, 0.0, 0.0, 0.0, 0.0, 0, 0, 0, 0, 0, at, 0)
    return header + pay.to_bytes(8 * ((at + 63) // 64), "little"), np.arange(n, dtype=np.uint32)


def compress(points: np.ndarray, eb: float, eb_mode: str = "rel", r: int = 32, ref_rule: int = 0,
             ref_mode: int = 0):
    """Returns (stream bytes, perm, details) for an (n, dims) float array.
    ref_mode 1 stores each reference's original coordinates (32 or 64 bits
    per axis) in place of its codes."""
    n, dims = points.shape
    f32 = points.dtype == np.float32
    mbits = 5 if f32 else 6
    M = 32 if f32 else 64
    try:
        prm = bound_params(points, eb, eb_mode)
    except ValueError:
        s, perm = lossless_stream(points, eb, eb_mode, r)
        return s, perm, None
    codes = quantize(points, prm)
    leaves = kd_leaves(codes, r, dims)
    G = prm["G"]
    meta = 0
    mpos = 0
    pay = 0
    ppos = 0
    perm = []
    boxes = []
    for members in leaves:
        j, m = bit_box(codes, members, dims, ref_rule)
        ref = members[j]
        boxes.append((j, m))
        for d in range(dims):
            meta |= m[d] << mpos
            mpos += mbits
        for d in range(dims):
            if ref_mode:
                meta |= _raw_bits(points, ref, d) << mpos
                mpos += M
            else:
                meta |= codes[ref][d] << mpos
                mpos += G[d]
        perm.append(ref)
        for i in members:
            if i == ref:
                continue
            perm.append(i)
            for d in range(dims):
                if m[d]:
                    pay |= (codes[i][d] - codes[ref][d] + (1 << (m[d] - 1))) << ppos
                    ppos += m[d]
    mbytes = 8 * ((mpos + 63) // 64)
    pbytes = 8 * ((ppos + 63) // 64)
    lo3 = list(prm["lo"]) + [0.0] * (3 - dims)
    G3 = list(G) + [0] * (3 - dims)
    header = struct.pack(
        "<4sHBBQIBBBBddddd3d3B5xQQQQ", b"BBX1", 1, 0 if f32 else 1, dims, n, r,
        0 if eb_mode == "rel" else 1, 0, ref_mode, mbits, eb, prm["eb_abs"], prm["eb_eff"], prm["w"],
        prm["inv_w"], *lo3, *G3, len(leaves), mpos, ppos, 0)
    assert len(header) == 128
    stream = header + meta.to_bytes(mbytes, "little") + pay.to_bytes(pbytes, "little")
    details = dict(prm=prm, codes=codes, leaves=leaves, boxes=boxes)
    return stream, np.array(perm, dtype=np.uint32), details


def decompress(stream: bytes) -> np.ndarray:
    """Independent decoder for tiny streams (big-integer bit extraction)."""
    (magic, ver, dt, dims, n, r, mode, _s, ref_mode, mbits, _eu, _ea, _ee, w, inv_w, o0, o1, o2, g0,
     g1, g2, nl, meta_bits, pay_bits, _res) = struct.unpack("<4sHBBQIBBBBddddd3d3B5xQQQQ",
                                                            stream[:128])
    if ver == 2:
        return decompress_reduced(stream)
    if ver == 3:  # every coordinate stored as its bits
        M = 32 if dt == 0 else 64
        pay = int.from_bytes(stream[128:], "little")
        raw = [(pay >> (M * k)) & ((1 << M) - 1) for k in range(n * dims)]
        return np.array(raw, dtype=np.uint32 if dt == 0 else np.uint64).view(
            np.float32 if dt == 0 else np.float64).reshape(n, dims)
    assert magic == b"BBX1" and ver == 1
    origin = [o0, o1, o2][:dims]
    G = [g0, g1, g2][:dims]
    mbytes = 8 * ((meta_bits + 63) // 64)
    meta = int.from_bytes(stream[128:128 + mbytes], "little")
    pay = int.from_bytes(stream[128 + mbytes:], "little")
    sizes = []

    def rec(s):
        if s <= r:
            sizes.append(s)
        else:
            rec(s // 2)
            rec(s - s // 2)

    if n:
        rec(n)
    assert len(sizes) == nl
    T = np.float32 if dt == 0 else np.float64
    M = 32 if dt == 0 else 64
    out = np.zeros((n, dims), dtype=T)
    mpos = ppos = slot = 0
    for s in sizes:
        m = []
        for d in range(dims):
            m.append((meta >> mpos) & ((1 << mbits) - 1))
            mpos += mbits
        ref = []
        exact = None
        for d in range(dims):
            if ref_mode:
                # the stored coordinate, and the code the encoder gave it
                x = _from_bits((meta >> mpos) & ((1 << M) - 1), dt == 0)
                mpos += M
                exact = (exact or []) + [x]
                ref.append(math.floor((float(x) - origin[d]) * inv_w + 0.5))
            else:
                ref.append((meta >> mpos) & ((1 << G[d]) - 1))
                mpos += G[d]
        rows = [ref]
        for _ in range(s - 1):
            q = []
            for d in range(dims):
                if m[d]:
                    u = (pay >> ppos) & ((1 << m[d]) - 1)
                    ppos += m[d]
                    q.append(ref[d] + u - (1 << (m[d] - 1)))
                else:
                    q.append(ref[d])
            rows.append(q)
        for k, q in enumerate(rows):
            if k == 0 and exact is not None:
                out[slot] = exact
            else:
                out[slot] = [T(origin[d] + float(q[d]) * w) for d in range(dims)]
            slot += 1
    assert ppos == pay_bits
    return out


def compress_split(points: np.ndarray, eb: float, eb_mode: str = "rel", r: int = 32,
                   split_rule: int = 0, ref_rule: int = 0, reduce: int = 0):
    """The partition under a split rule (see kd_leaves), bit boxes, then
    either one sequence per leaf (reduce 0) or the reduction below (reduce 1:
    key sum of widths, 2: sum of box lengths).  Version-2 stream unless rule
    0 without the reduction (then the version-1 stream of compress).
    Returns (stream, perm)."""
    if split_rule == 0 and reduce == 0:
        s, perm, _ = compress(points, eb, eb_mode, r, ref_rule)
        return s, perm
    return _sequences(points, eb, eb_mode, r, split_rule, ref_rule, reduce)


def compress_reduced(points: np.ndarray, eb: float, eb_mode: str = "rel", r: int = 32,
                     key_rule: int = 0):
    return _sequences(points, eb, eb_mode, r, 0, 0, key_rule + 1)


def _sequences(points, eb, eb_mode, r, split_rule, ref_rule, reduce):
    """The bit box reduction of Sec. 4.1 restated with Python sets: a box is
    its reference and widths; the key is the sum of widths (reduce 1) or
    the sum of the Eq. 3 box lengths (reduce 2); two boxes meet when their
    Eq. 1 predictable ranges overlap (closed intervals, in bins of 2*eps); a
    particle is inside a box when the box's widths can encode its offsets
    (searched, as for the widths themselves).  Returns (stream, perm)."""
    n, dims = points.shape
    f32 = points.dtype == np.float32
    mbits = 5 if f32 else 6
    try:
        prm = bound_params(points, eb, eb_mode)
    except ValueError:
        return lossless_stream(points, eb, eb_mode, r)
    codes = quantize(points, prm)
    G = prm["G"]
    leaves = kd_leaves(codes, r, dims, split_rule, G)
    boxes = []
    for members in leaves:
        j, m = bit_box(codes, members, dims, ref_rule)
        boxes.append({"left": set(members), "ref": members[j], "m": m, "order": list(members)})
    key_rule = reduce - 1

    def key(b):
        if key_rule == 0:
            return sum(b["m"])
        return sum(Fraction(4) * (Fraction(2) ** (md - 1) - Fraction(1, 2)) for md in b["m"])

    def half(md):  # Eq. 1 half-range in bins: 2^(m-1) - 1/2 (zero for m = 0)
        return Fraction(2) ** (md - 1) - Fraction(1, 2)

    def meet(a, b):
        return all(abs(codes[a["ref"]][d] - codes[b["ref"]][d]) <= half(a["m"][d]) + half(b["m"][d])
                   for d in range(dims))

    def inside(b, i):
        return all(minimal_bits([codes[i][d] - codes[b["ref"]][d]]) <= b["m"][d] for d in range(dims))

    seqs = []
    live = [k for k in range(len(boxes))] if reduce else []
    if not reduce:
        seqs = [(B["ref"], list(B["m"]), [i for i in B["order"] if i != B["ref"]]) for B in boxes]
    while live:
        cur = min(live, key=lambda k: (key(boxes[k]), k))
        B = boxes[cur]
        parts = [i for i in B["order"] if i in B["left"] and i != B["ref"]]
        for k in sorted(live):
            if k == cur or not meet(B, boxes[k]):
                continue
            other = boxes[k]
            common = [i for i in other["order"] if i in other["left"] and inside(B, i)]
            if not common:
                continue
            parts += common
            other["left"] -= set(common)
            if other["left"]:
                rest = [i for i in other["order"] if i in other["left"]]
                j, m = bit_box(codes, rest, dims)
                other["ref"], other["m"] = rest[j], m
        seqs.append((B["ref"], list(B["m"]), parts))
        live = [k for k in live if k != cur and boxes[k]["left"]]
    meta = mpos = pay = ppos = 0
    perm = []
    for ref, m, parts in seqs:
        for d in range(dims):
            meta |= m[d] << mpos
            mpos += mbits
        for d in range(dims):
            meta |= codes[ref][d] << mpos
            mpos += G[d]
        meta |= len(parts) << mpos
        mpos += 32
        perm.append(ref)
        for i in parts:
            perm.append(i)
            for d in range(dims):
                if m[d]:
                    pay |= (codes[i][d] - codes[ref][d] + (1 << (m[d] - 1))) << ppos
                    ppos += m[d]
    lo3 = list(prm["lo"]) + [0.0] * (3 - dims)
    G3 = list(G) + [0] * (3 - dims)
    header = struct.pack(
        "<4sHBBQIBBBBddddd3d3B5xQQQQ", b"BBX1", 2, 0 if f32 else 1, dims, n, r,
        0 if eb_mode == "rel" else 1, split_rule, 0, mbits, eb, prm["eb_abs"], prm["eb_eff"], prm["w"],
        prm["inv_w"], *lo3, *G3, len(leaves), mpos, ppos, len(seqs))
    stream = (header + meta.to_bytes(8 * ((mpos + 63) // 64), "little")
              + pay.to_bytes(8 * ((ppos + 63) // 64), "little"))
    return stream, np.array(perm, dtype=np.uint32)


def decompress_reduced(stream: bytes) -> np.ndarray:
    """Decoder of the reduced stream (version 2) with big integers."""
    (magic, ver, dt, dims, n, _r, _mode, _s, _rm, mbits, _eu, _ea, _ee, w, _iw, o0, o1, o2, g0,
     g1, g2, _nl, meta_bits, pay_bits, nseq) = struct.unpack("<4sHBBQIBBBBddddd3d3B5xQQQQ",
                                                             stream[:128])
    assert magic == b"BBX1" and ver == 2
    origin = [o0, o1, o2][:dims]
    G = [g0, g1, g2][:dims]
    mbytes = 8 * ((meta_bits + 63) // 64)
    meta = int.from_bytes(stream[128:128 + mbytes], "little")
    pay = int.from_bytes(stream[128 + mbytes:], "little")
    T = np.float32 if dt == 0 else np.float64
    out = np.zeros((n, dims), dtype=T)
    mpos = ppos = slot = 0
    for _ in range(nseq):
        m, ref = [], []
        for d in range(dims):
            m.append((meta >> mpos) & ((1 << mbits) - 1))
            mpos += mbits
        for d in range(dims):
            ref.append((meta >> mpos) & ((1 << G[d]) - 1))
            mpos += G[d]
        cnt = (meta >> mpos) & 0xFFFFFFFF
        mpos += 32
        rows = [ref]
        for _ in range(cnt):
            q = []
            for d in range(dims):
                if m[d]:
                    q.append(ref[d] + ((pay >> ppos) & ((1 << m[d]) - 1)) - (1 << (m[d] - 1)))
                    ppos += m[d]
                else:
                    q.append(ref[d])
            rows.append(q)
        for q in rows:
            out[slot] = [T(origin[d] + float(q[d]) * w) for d in range(dims)]
            slot += 1
    assert slot == n and ppos == pay_bits
    return out


def export_sequences(stream: bytes) -> bytes:
    """Sec. 4.2 sequence layout of a ref_mode 1 stream, rebuilt with big
    integers: per leaf the centre's coordinate bits, the widths, the member
    codes and a 32-bit end mark of all ones."""
    (magic, ver, dt, dims, n, r, _mode, _s, ref_mode, mbits, _eu, _ea, _ee, _w, _iw, _o0, _o1, _o2,
     _g0, _g1, _g2, nl, meta_bits, pay_bits, _res) = struct.unpack("<4sHBBQIBBBBddddd3d3B5xQQQQ",
                                                                    stream[:128])
    assert magic == b"BBX1" and ver == 1 and ref_mode == 1
    M = 32 if dt == 0 else 64
    mbytes = 8 * ((meta_bits + 63) // 64)
    meta = int.from_bytes(stream[128:128 + mbytes], "little")
    pay = int.from_bytes(stream[128 + mbytes:], "little")
    sizes = []

    def rec(s):
        if s <= r:
            sizes.append(s)
        else:
            rec(s // 2)
            rec(s - s // 2)

    if n:
        rec(n)
    out, opos, mpos, ppos = 0, 0, 0, 0
    for s in sizes:
        m = [(meta >> (mpos + mbits * d)) & ((1 << mbits) - 1) for d in range(dims)]
        centre = [(meta >> (mpos + mbits * dims + M * d)) & ((1 << M) - 1) for d in range(dims)]
        mpos += dims * (mbits + M)
        for c in centre:
            out |= c << opos
            opos += M
        for w in m:
            out |= w << opos
            opos += mbits
        length = (s - 1) * sum(m)
        out |= ((pay >> ppos) & ((1 << length) - 1)) << opos
        ppos += length
        opos += length
        out |= 0xFFFFFFFF << opos
        opos += 32
    assert ppos == pay_bits
    return out.to_bytes(8 * ((opos + 63) // 64), "little")


def export_sequences_reordered(stream: bytes):
    """The two reorderings of Sec. 4.2 on the sequence layout, restated with
    Python sorts: sequences by ascending sum of widths (stable), members by
    ascending R-index (codes concatenated with the axes in ascending entropy
    of their widths, the lower axis first on equal entropy; stable).
    Returns (layout, axis order)."""
    plain = export_sequences(stream)
    (_m, _v, dt, dims, n, r, _e, _s, _rm, mbits) = struct.unpack("<4sHBBQIBBBB", stream[:24])
    M = 32 if dt == 0 else 64
    bits = int.from_bytes(plain, "little")
    sizes = []

    def rec(s):
        if s <= r:
            sizes.append(s)
        else:
            rec(s // 2)
            rec(s - s // 2)

    if n:
        rec(n)
    seqs, pos = [], 0
    for s in sizes:
        hdr = bits >> pos & ((1 << (dims * (M + mbits))) - 1)
        m = [(bits >> (pos + dims * M + mbits * d)) & ((1 << mbits) - 1) for d in range(dims)]
        at = pos + dims * (M + mbits)
        mem = []
        for _ in range(s - 1):
            u = []
            for d in range(dims):
                u.append((bits >> at) & ((1 << m[d]) - 1))
                at += m[d]
            mem.append(u)
        seqs.append((hdr, m, mem))
        pos = at + 32
    ent = []
    for d in range(dims):
        counts = {}
        for _, m, _ in seqs:
            counts[m[d]] = counts.get(m[d], 0) + 1
        ent.append(sum(c * math.log2(c) for c in counts.values()))
    order = sorted(range(dims), key=lambda d: (-ent[d], d))
    out, opos = 0, 0
    for k in sorted(range(len(seqs)), key=lambda i: (sum(seqs[i][1]), i)):
        hdr, m, mem = seqs[k]
        out |= hdr << opos
        opos += dims * (M + mbits)
        for u in sorted(mem, key=lambda u: tuple(u[d] for d in order)):
            for d in range(dims):
                out |= u[d] << opos
                opos += m[d]
        out |= 0xFFFFFFFF << opos
        opos += 32
    return out.to_bytes(8 * ((opos + 63) // 64), "little"), order


# ---------------------------------------------------------------- entropy coding

HUF_MAXLEN, HUF_CHUNK = 12, 4096


def huffman_lengths(counts):
    """Huffman's construction restated with a priority queue: entries
    (weight, creation number); leaves numbered first in symbol order, merged
    nodes after them in creation order; depth of each leaf; rebuilt from the
    halved weights (rounded up) while some depth exceeds HUF_MAXLEN."""
    import heapq
    w = [int(c) for c in counts]
    while True:
        syms = [s for s in range(256) if w[s] > 0]
        if not syms:
            return [0] * 256
        if len(syms) == 1:
            out = [0] * 256
            out[syms[0]] = 1
            return out
        heap = [(w[s], i) for i, s in enumerate(syms)]
        heapq.heapify(heap)
        children = {}
        nid = len(syms)
        while len(heap) > 1:
            a = heapq.heappop(heap)
            b = heapq.heappop(heap)
            children[nid] = (a[1], b[1])
            heapq.heappush(heap, (a[0] + b[0], nid))
            nid += 1
        depth = {}
        stack = [(heap[0][1], 0)]
        while stack:
            node, dpt = stack.pop()
            if node in children:
                for ch in children[node]:
                    stack.append((ch, dpt + 1))
            else:
                depth[node] = dpt
        lens = [0] * 256
        for i, s in enumerate(syms):
            lens[s] = depth[i]
        if max(lens) <= HUF_MAXLEN:
            return lens
        w = [(x + 1) // 2 if x else 0 for x in w]


def canonical_codes(lens):
    """Codes in (length, symbol) order, consecutive, shifted at each longer length."""
    order = sorted((L, s) for s, L in enumerate(lens) if L)
    codes, c, prev = {}, 0, None
    for L, s in order:
        if prev is not None:
            c = (c + 1) << (L - prev)
        codes[s] = c
        prev = L
    return codes


def huffman_encode(data: bytes) -> bytes:
    n = len(data)
    counts = [0] * 256
    for b in data:
        counts[b] += 1
    lens = huffman_lengths(counts)
    codes = canonical_codes(lens)
    chunks = -(-n // HUF_CHUNK)
    pay, pos, offs = 0, 0, []
    for i, b in enumerate(data):
        if i % HUF_CHUNK == 0:
            offs.append(pos)
        L = lens[b]
        for k in range(L):  # most significant code bit first
            pay |= ((codes[b] >> (L - 1 - k)) & 1) << pos
            pos += 1
    nib = bytearray(128)
    for s in range(256):
        nib[s // 2] |= lens[s] << (4 if s & 1 else 0)
    head = struct.pack("<4sHBBQIIQQQ", b"BBXH", 1, HUF_MAXLEN, 0, n, HUF_CHUNK, 0, chunks, pos, 0)
    return (head + bytes(nib) + b"".join(struct.pack("<Q", o) for o in offs)
            + pay.to_bytes(8 * ((pos + 63) // 64), "little"))


def huffman_optimal_cost(counts):
    """Smallest sum of count x length over every length assignment with
    Kraft sum <= 1 (exhaustive; tiny alphabets only)."""
    import itertools
    syms = [c for c in counts if c > 0]
    if len(syms) <= 1:
        return sum(syms)
    best = None
    for L in itertools.product(range(1, len(syms)), repeat=len(syms)):
        if sum(Fraction(1, 2 ** x) for x in L) <= 1:
            cost = sum(c * x for c, x in zip(syms, L))
            best = cost if best is None else min(best, cost)
    return best
