"""Pins of the CPU oracle against the paper and mathematics (no GPU).

Each test checks the oracle against something other than itself: the
worked example of Sec. 4.1, the brute-force re-derivation on tiny inputs,
closed forms (Eq. 1-3), definitions (error bound, median split, nearest
reference, minimal widths, storage-cost model), and special cases that
reduce to textbook routines.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import pins
import props
from oracle import OracleError, brute
from synth import cosmology, fluid, uniform_cube


def test_worked_example(oracle):
    pins.pin_worked_example(oracle)


def test_worked_example_codes(oracle):
    """Sec. 4.1 example in bins of 2*eps: the x offsets of the AABB corners from
    the reference are 1400 and 1600 bins (FP64), giving m_x = 12."""
    g = pins.w1_case()
    st_ = oracle.stages(np.array(g["points"], dtype=np.float64), g["eps_abs"], "abs", r=3)
    assert st_["q"][:, 2].tolist() == [1400, 1, 110]
    assert st_["q"][:, 1].tolist() == [3000, 2, 200]


def test_eq2_closed_form_exact():
    """Eq. 2 evaluated with exact rationals equals the oracle's integer form for
    every largest offset D < 2^16: m is the least integer with
    2^(m-1) >= D + 1/2 (log2(D + 1/2) + 1 <= m)."""
    from oracle import Oracle
    orc = Oracle()
    for D in range(1 << 16):
        target = Fraction(2 * D + 1, 2)
        m = 0
        while Fraction(2) ** (m - 1) < target:
            m += 1
        assert orc.bits_for_offset(D) == m, D
    # the paper's floating-point form agrees on this range as well
    for D in range(1, 1 << 12):
        assert orc.bits_for_offset(D) == math.ceil(math.log2(D + 0.5) + 1)


def test_eq1_eq3_cover_every_member(oracle):
    """Eq. 1: with m bits the predictable range is pv +- 2eps(2^(m-1) - 1/2);
    every member's bin [x-eps, x+eps] lies inside it, and Eq. 3's box length
    l = 4eps(2^(m-1) - 1/2) spans it."""
    pts = cosmology(4000, seed=21)
    s = oracle.stages(pts, 1e-3, "rel", r=37)
    eps = s["eb_eff"]
    q = s["q"].astype(np.int64)
    order = s["order"].astype(np.int64)
    for i in range(s["n_leaves"]):
        mem = order[s["leaf_start"][i]: s["leaf_start"][i] + s["leaf_size"][i]]
        ref = mem[s["leaf_ref"][i]]
        for d in range(3):
            m = int(s["leaf_m"][i][d])
            off = np.abs(q[d][mem] - q[d][ref])
            if m == 0:
                assert (off == 0).all()
                continue
            half_range = 2 * eps * (2 ** (m - 1) - 0.5)
            assert ((off * 2 * eps + eps) <= half_range * (1 + 1e-12)).all()
            assert math.isclose(4 * eps * (2 ** (m - 1) - 0.5), 2 * half_range)


def test_brute_force_tiny(oracle):
    pins.pin_brute_force(oracle, seed=101, count=150)


def test_brute_force_exhaustive_r(oracle):
    """Every leaf capacity r = 1..n+1 on a few tiny sets, 2-D and 3-D."""
    rng = np.random.default_rng(7)
    for dims in (2, 3):
        for dt in (np.float32, np.float64):
            n = 23
            pts = (np.round(rng.random((n, dims)) * 6) / 6).astype(dt)
            for r in range(1, n + 2):
                s1, p1 = oracle.compress(pts, 0.01, "rel", r, want_perm=True)
                s2, p2, _ = brute.compress(pts, 0.01, "rel", r)
                assert s1 == s2 and np.array_equal(p1, p2), (dims, dt, r)


def test_properties_tiny(oracle):
    pins.pin_properties(oracle, seed=102, count=80)


@pytest.mark.parametrize("gen,eb,r", [
    ("uniform", 1e-3, 32), ("cosmology", 1e-4, 32), ("cosmology", 1e-3, 100),
    ("fluid", 1e-4, 32), ("uniform", 1e-4, 5), ("fluid", 1e-3, 1000)])
def test_tree_bitbox_bound_moderate(oracle, gen, eb, r):
    """P1-P6 on moderate generator sets, the whole tree checked level by level."""
    if gen == "uniform":
        pts = uniform_cube(20000, seed=31)
    elif gen == "cosmology":
        pts = cosmology(20000, seed=32)
    else:
        pts = fluid(32, 32, 16, seed=33)
    n = len(pts)
    s = oracle.stages(pts, eb, "rel", r=r)
    stream, perm = oracle.compress(pts, eb, "rel", r, want_perm=True)
    h = props.parse_header(stream)
    dec = oracle.decompress(stream)
    props.check_permutation(perm, n)
    props.check_bound(pts, dec, perm, h["eb_abs"])
    sizes = props.leaf_sizes_fast(n, r)
    assert np.array_equal(sizes, s["leaf_size"].astype(np.int64))
    order = props.tree_order_from_perm(perm, sizes)
    assert np.array_equal(order, s["order"].astype(np.int64))
    props.check_tree(s["q"], order, n, r, 3)
    props.check_bitboxes(s["q"], order, sizes, s["leaf_ref"], s["leaf_m"], 3)
    # P6: section sizes from the storage-cost model in this layout
    mbits = 5
    assert h["meta_bits"] == len(sizes) * (3 * mbits + sum(h["G"]))
    assert h["payload_bits"] == int(((sizes - 1) * s["leaf_m"].astype(np.int64).sum(axis=1)).sum())
    assert len(stream) == props.stream_size(h["meta_bits"], h["payload_bits"])
    # decoded codes of each slot equal the codes of its source particle
    q_dec = np.floor((dec.astype(np.float64) - np.array(h["origin"]))[:, :3] / h["w"] + 0.5)
    assert np.array_equal(q_dec.astype(np.int64).T, s["q"][:, perm].astype(np.int64))


def test_full_plain_workload(oracle):
    """The plain single-set workload (65,536 uniform points, xi = 1e-3, r = 32):
    2,048 leaves of exactly 32, every point within the bound."""
    pts = uniform_cube(65536, seed=1)
    stream, perm = oracle.compress(pts, 1e-3, "rel", 32, want_perm=True)
    h = props.parse_header(stream)
    assert h["n_leaves"] == 2048
    dec = oracle.decompress(stream)
    props.check_permutation(perm, len(pts))
    props.check_bound(pts, dec, perm, h["eb_abs"])


def test_r1_is_uniform_scalar_quantization(oracle):
    """r = 1: every leaf is one particle, every width is 0, the payload is
    empty and the stream is fixed-width uniform scalar quantization with G_d
    bits per coordinate; each reconstruction is the nearest grid point."""
    pts = cosmology(3000, seed=41)
    stream, perm = oracle.compress(pts, 1e-3, "rel", 1, want_perm=True)
    h = props.parse_header(stream)
    assert h["payload_bits"] == 0 and h["n_leaves"] == 3000
    assert h["meta_bits"] == 3000 * (3 * 5 + sum(h["G"]))
    dec = oracle.decompress(stream).astype(np.float64)
    x = pts[perm].astype(np.float64)
    grid = (dec - np.array(h["origin"])) / h["w"]
    assert np.allclose(grid, np.round(grid), atol=1e-6)
    # the chosen grid point is the nearest one (no neighbour is closer, up to rounding)
    for step in (-1, 1):
        alt = dec + step * h["w"]
        assert (np.abs(x - dec) <= np.abs(x - alt) + 1e-9 * np.abs(x).max()).all()


def test_r_ge_n_single_leaf(oracle):
    """r >= n: one leaf whose reference is the brute-force nearest point to the
    AABB centre."""
    pts = uniform_cube(500, seed=42, dtype=np.float64)
    s = oracle.stages(pts, 1e-2, "rel", r=500)
    assert s["n_leaves"] == 1
    q = s["q"].astype(np.int64)
    centre = (q.min(axis=1) + q.max(axis=1)) / 2.0
    dist = ((q - centre[:, None]) ** 2).sum(axis=0)
    assert int(s["order"][s["leaf_ref"][0]]) == int(np.argmin(dist))


def test_all_identical_points_exact(oracle):
    for dt in (np.float32, np.float64):
        pts = np.full((77, 3), -3.25, dtype=dt)
        stream = oracle.compress(pts, 1e-4, "rel", 8)
        h = props.parse_header(stream)
        assert h["payload_bits"] == 0 and h["G"] == [0, 0, 0]
        assert np.array_equal(oracle.decompress(stream), pts)


def test_collinear_constant_axes(oracle):
    """Points on a line along x: widths are 0 in y and z, which reconstruct exactly."""
    rng = np.random.default_rng(3)
    pts = np.zeros((1000, 3), dtype=np.float32)
    pts[:, 0] = rng.random(1000)
    pts[:, 1] = 0.5
    pts[:, 2] = -2.0
    s = oracle.stages(pts, 1e-3, "rel", r=16)
    assert (s["leaf_m"][:, 1:] == 0).all() and (s["leaf_m"][:, 0] > 0).any()
    dec = oracle.decompress(oracle.compress(pts, 1e-3, "rel", 16))
    assert (dec[:, 1] == 0.5).all() and (dec[:, 2] == -2.0).all()


def test_negative_zero_origin(oracle):
    pts = np.array([[-0.0, 1.0], [0.0, 2.0], [-0.0, 3.0]], dtype=np.float32)
    stream = oracle.compress(pts, 0.01, "rel", 2)
    h = props.parse_header(stream)
    assert math.copysign(1.0, h["origin"][0]) == 1.0
    s2, _, _ = brute.compress(pts, 0.01, "rel", 2)
    assert stream == s2


def test_psnr_bounds(oracle):
    """Sec. 5.1 metrics: |err| <= xi*range gives NRMSE <= xi, PSNR >= -20 log10 xi;
    for bin-uniform errors PSNR is close to -20 log10(xi / sqrt(3))."""
    pts = uniform_cube(65536, seed=1)
    xi = 1e-4
    stream, perm = oracle.compress(pts, xi, "rel", 32, want_perm=True)
    dec = oracle.decompress(stream)
    p = props.psnr(pts, dec, perm)
    assert p >= -20 * math.log10(xi)
    assert abs(p - (-20 * math.log10(xi / math.sqrt(3)))) < 0.6


def test_fp64_input(oracle):
    pts = fluid(16, 16, 16, seed=5, dtype=np.float64)
    stream, perm = oracle.compress(pts, 1e-6, "rel", 32, want_perm=True)
    h = props.parse_header(stream)
    assert h["mbits"] == 6 and h["dtype"] == 1
    dec = oracle.decompress(stream)
    props.check_bound(pts, dec, perm, h["eb_abs"])


def test_soa_layout_same_stream(oracle):
    pts = cosmology(3000, seed=6)
    a = oracle.compress(pts, 1e-3, "rel", 16)
    b = oracle.compress(np.ascontiguousarray(pts.T), 1e-3, "rel", 16, layout="soa")
    assert a == b
    assert np.array_equal(oracle.decompress(a, layout="soa"), oracle.decompress(a).T)


def test_determinism(oracle):
    pts = cosmology(5000, seed=7)
    assert oracle.compress(pts, 1e-4, "rel", 32) == oracle.compress(pts.copy(), 1e-4, "rel", 32)


def test_empty_input(oracle):
    pts = np.zeros((0, 3), dtype=np.float32)
    stream = oracle.compress(pts, 1e-3, "rel", 32)
    assert len(stream) == 128
    h = props.parse_header(stream)
    assert h["n"] == 0 and h["n_leaves"] == 0
    assert oracle.decompress(stream).shape == (0, 3)


# -------------------------------------------------------------- error paths

def _expect(status, fn, *a, **k):
    with pytest.raises(OracleError) as ei:
        fn(*a, **k)
    assert ei.value.name == status


def test_errors(oracle):
    pts = uniform_cube(100, seed=9)
    bad = pts.copy()
    bad[5, 1] = np.nan
    _expect("EINVAL", oracle.compress, bad, 1e-3)
    bad[5, 1] = np.inf
    _expect("EINVAL", oracle.compress, bad, 1e-3)
    _expect("EINVAL", oracle.compress, pts, 1e-3, r=0)
    _expect("EINVAL", oracle.compress, pts, 0.0)
    _expect("EINVAL", oracle.compress, pts, -1.0)
    _expect("EUNSUPPORTED", oracle.compress, np.zeros((4, 4), np.float32), 1e-3)
    # a bound the grid cannot meet (below the f32 resolution, or codes >= 2^30)
    # is not an error: the set is stored losslessly (test_lossless_fallback)
    _expect("ENOSPC", oracle.compress, pts, 1e-3, out_cap=100)


def test_corrupt_streams(oracle):
    pts = cosmology(2000, seed=10)
    good = oracle.compress(pts, 1e-3, "rel", 32)
    oracle.decompress(good)

    def mutate(off, val):
        b = bytearray(good)
        b[off] = val
        return bytes(b)

    _expect("ECORRUPT", oracle.decompress, good[:100])
    _expect("ECORRUPT", oracle.decompress, good[:-8])
    _expect("ECORRUPT", oracle.decompress, mutate(0, ord("Q")))      # magic
    _expect("ECORRUPT", oracle.decompress, mutate(7, 4))             # dims
    _expect("ECORRUPT", oracle.decompress, mutate(23, 6))            # mbits vs dtype
    _expect("ECORRUPT", oracle.decompress, mutate(96, good[96] ^ 1))  # n_leaves
    _expect("ECORRUPT", oracle.decompress, mutate(104, good[104] ^ 8))  # meta bits
    _expect("ECORRUPT", oracle.decompress, mutate(120, 1))           # reserved
    # a zero code in the payload is never emitted (codes lie in [1, 2^m - 1])
    h = props.parse_header(good)
    mb = 8 * ((h["meta_bits"] + 63) // 64)
    b = bytearray(good)
    # first leaf's widths, then clear the first member's x code
    meta = int.from_bytes(b[128:128 + 8], "little")
    mx = meta & 31
    assert mx > 0
    word = int.from_bytes(b[128 + mb:128 + mb + 8], "little")
    word &= ~((1 << mx) - 1)
    b[128 + mb:128 + mb + 8] = word.to_bytes(8, "little")
    _expect("ECORRUPT", oracle.decompress, bytes(b))
    # width field m = 1 can never be produced by Eq. 2
    b = bytearray(good)
    b[128] = (b[128] & ~31) | 1
    _expect("ECORRUPT", oracle.decompress, bytes(b))


def test_decompress_capacity(oracle):
    pts = uniform_cube(100, seed=9)
    s = oracle.compress(pts, 1e-3)
    _expect("ENOSPC", oracle.decompress, s, pos_cap_bytes=100)


# -------------------------------------------------------------- hypothesis

_floats32 = st.floats(min_value=-1e6, max_value=1e6, allow_nan=False, allow_infinity=False, width=32)


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(data=st.data())
def test_hypothesis_properties(oracle, data):
    dims = data.draw(st.sampled_from([2, 3]))
    n = data.draw(st.integers(min_value=1, max_value=60))
    base = data.draw(st.lists(st.tuples(*[_floats32] * dims), min_size=1, max_size=8))
    picks = data.draw(st.lists(st.integers(0, len(base) - 1), min_size=n, max_size=n))
    dt = data.draw(st.sampled_from([np.float32, np.float64]))
    pts = np.array([base[i] for i in picks], dtype=dt)
    jitter = data.draw(st.sampled_from([0.0, 1e-3, 1.0]))
    if jitter:
        pts = (pts + np.random.default_rng(n).random(pts.shape) * jitter).astype(dt)
    r = data.draw(st.integers(min_value=1, max_value=n + 1))
    eb = data.draw(st.sampled_from([1e-1, 1e-3, 1e-5]))
    stream, perm = oracle.compress(pts, eb, "rel", r, want_perm=True)
    h = props.parse_header(stream)
    if h["version"] == 3:  # lossless: the grid cannot meet the bound
        assert stream == brute.compress(pts, eb, "rel", r)[0]
        assert np.array_equal(oracle.decompress(stream).view(np.uint8), pts.view(np.uint8))
        return
    dec = oracle.decompress(stream)
    props.check_permutation(perm, n)
    props.check_bound(pts, dec, perm, h["eb_abs"])
    s2, p2, _ = brute.compress(pts, eb, "rel", r)
    assert stream == s2 and np.array_equal(perm, p2)


def test_reference_rule_fewest_bits_brute_force(oracle):
    """Reference rule 1 (an ablation of the paper's AABB-centre rule): the C
    oracle's closed form (widths from the AABB extremes) equals the exhaustive
    search that tries every member as the reference, byte for byte."""
    for pts, eb, mode, r in pins.tiny_cases(seed=211, count=60):
        s1, p1 = oracle.compress(pts, eb, mode, r, want_perm=True, ref_rule=1)
        s2, p2, _ = brute.compress(pts, eb, mode, r, ref_rule=1)
        assert s1 == s2 and np.array_equal(p1, p2), (pts.shape, eb, mode, r)


def test_reference_rule_fewest_bits_never_costs_more(oracle):
    """Per leaf, rule 1's width sum is at most rule 0's (same tree, same AABB),
    and its stream still reconstructs every particle within the bound."""
    pts = cosmology(20000, seed=23)
    a = oracle.stages(pts, 1e-4, "rel", r=32, ref_rule=0)
    b = oracle.stages(pts, 1e-4, "rel", r=32, ref_rule=1)
    assert np.array_equal(a["order"], b["order"]) and np.array_equal(a["leaf_size"], b["leaf_size"])
    sa = a["leaf_m"].astype(int).sum(axis=1)
    sb = b["leaf_m"].astype(int).sum(axis=1)
    assert (sb <= sa).all() and (sb < sa).any()
    s, perm = oracle.compress(pts, 1e-4, "rel", 32, want_perm=True, ref_rule=1)
    out = oracle.decompress(s).astype(np.float64)
    err = np.abs(out - pts[perm].astype(np.float64)).max()
    assert err <= a["eb_abs"]


def test_lossless_reference_mode(oracle):
    """ref_mode 1 (the paper's lossless centre, Sec. 4.2) at a moderate size:
    references exact, others within the bound and equal to the code-reference
    decode, and the stream longer by exactly (M - G_d) bits per leaf and axis
    (before word padding)."""
    for dt, M in ((np.float32, 32), (np.float64, 64)):
        pts = cosmology(20000, seed=29, dtype=dt)
        s0, p0 = oracle.compress(pts, 1e-4, "rel", 32, want_perm=True)
        s1, p1 = oracle.compress(pts, 1e-4, "rel", 32, want_perm=True, ref_mode=1)
        assert np.array_equal(p0, p1)
        h0, h1 = props.parse_header(s0), props.parse_header(s1)
        assert h1["payload_bits"] == h0["payload_bits"]
        assert h1["meta_bits"] - h0["meta_bits"] == h0["n_leaves"] * sum(M - g for g in h0["G"])
        d0, d1 = oracle.decompress(s0), oracle.decompress(s1)
        sizes = props.leaf_sizes(len(pts), 32)
        first = np.zeros(len(pts), dtype=bool)
        first[np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(int)] = True
        assert np.array_equal(d1[first], pts[p1[first]])
        assert np.array_equal(d1[~first], d0[~first])
        props.check_bound(pts, d1, p1, h1["eb_abs"])
        assert len(s1) <= oracle.compress_bound(len(pts), 3, dt, ref_mode=1)
        # the code-reference bound is too small for single-particle leaves
        assert oracle.compress_bound(1000, 3, dt, ref_mode=1) > oracle.compress_bound(1000, 3, dt)
        s = oracle.compress(pts[:1000], 1e-4, "rel", 1, ref_mode=1)
        assert len(s) <= oracle.compress_bound(1000, 3, dt, ref_mode=1)


def test_lossless_reference_corrupt(oracle):
    """A stored reference that is not finite, or whose code falls outside
    [0, 2^G_d), is a corrupt stream; so is a reference-mode byte above 1."""
    pts = cosmology(2000, seed=31)
    good = oracle.compress(pts, 1e-3, "rel", 32, ref_mode=1)
    oracle.decompress(good)
    h = props.parse_header(good)
    # first record: dims widths of 5 bits, then the x coordinate's 32 bits
    off = 128 * 8 + 3 * 5
    meta = int.from_bytes(good[128:136], "little")

    def with_x(bits):
        m = (meta & ~(((1 << 32) - 1) << 15)) | (bits << 15)
        b = bytearray(good)
        b[128:136] = m.to_bytes(8, "little")
        return bytes(b)

    assert off // 8 == 129
    nan = int(np.array([np.nan], dtype=np.float32).view(np.uint32)[0])
    _expect("ECORRUPT", oracle.decompress, with_x(nan))
    far = float(h["origin"][0]) - 4.0 * float(h["w"])  # code -4
    _expect("ECORRUPT", oracle.decompress,
            with_x(int(np.array([far], dtype=np.float32).view(np.uint32)[0])))
    b = bytearray(good)
    b[22] = 2
    _expect("ECORRUPT", oracle.decompress, bytes(b))


def test_sequence_export_matches_brute_force_and_storage_model(oracle):
    """The Sec. 4.2 sequence layout exported from a ref_mode 1 stream equals an
    independent big-integer rebuild, and its length is the paper's
    storage-cost model with one sequence per leaf: dims * M bits of centre,
    dims * mbits of widths, sum_d m_d * (particles - 1) bits of codes and 32
    bits of end mark per sequence (computed from the oracle's stage dump,
    not from the stream)."""
    for pts, eb, mode, r in pins.tiny_cases(seed=301, count=40):
        n, dims = pts.shape
        s = oracle.compress(pts, eb, mode, r, ref_mode=1)
        e = oracle.export_sequences(s)
        assert e == brute.export_sequences(s), (pts.shape, r)
        st = oracle.stages(pts, eb, mode, r)
        M, mbits = (32, 5) if pts.dtype == np.float32 else (64, 6)
        nseq = st["n_leaves"]
        bits = (dims * M * nseq + dims * mbits * nseq
                + int((st["leaf_m"].astype(np.int64).sum(axis=1) * (st["leaf_size"].astype(np.int64) - 1)).sum())
                + 32 * nseq)
        assert len(e) == 8 * ((bits + 63) // 64)
        tail = int.from_bytes(e, "little") >> bits
        assert tail == 0
    pts = cosmology(20000, seed=37)
    s = oracle.compress(pts, 1e-4, "rel", 32, ref_mode=1)
    assert oracle.export_sequences(s) == brute.export_sequences(s)
    _expect("EINVAL", oracle.export_sequences, oracle.compress(pts, 1e-4, "rel", 32))


def test_sequence_reordering_matches_python_sorts(oracle):
    """The two reorderings of Sec. 4.2 (sequences by sum of widths, members by
    R-index with the axes in ascending entropy of their widths) equal a
    restatement with Python sorts, and keep the layout's length and every
    sequence's members (a permutation within each sequence)."""
    for pts, eb, mode, r in pins.tiny_cases(seed=401, count=40):
        s = oracle.compress(pts, eb, mode, r, ref_mode=1)
        got, order = oracle.export_sequences_reordered(s)
        want, worder = brute.export_sequences_reordered(s)
        assert got == want and order == worder, (pts.shape, r)
        assert len(got) == len(oracle.export_sequences(s))
    pts = cosmology(20000, seed=41)
    s = oracle.compress(pts, 1e-4, "rel", 32, ref_mode=1)
    got, order = oracle.export_sequences_reordered(s)
    assert (got, order) == brute.export_sequences_reordered(s)


def test_reduction_worked_examples(oracle):
    """Sec. 4.1 bit box reduction on hand-worked examples (both keys)."""
    pins.pin_reduction_examples(oracle)


def test_reduction_brute_force(oracle):
    pins.pin_reduction_brute(oracle, seed=102, count=120)


def test_reduction_special_cases(oracle):
    pins.pin_reduction_special(oracle)


@pytest.mark.parametrize("gen,n,r,xi", [(cosmology, 20000, 32, 1e-3), (fluid, 32768, 32, 1e-4),
                                        (uniform_cube, 5000, 8, 1e-2)])
def test_reduction_properties_moderate(oracle, gen, n, r, xi):
    """At moderate sizes: every particle once, within the bound, inside its
    sequence's bit box; at most one sequence per leaf."""
    if gen is fluid:
        from synth import fluid_lattice_dims
        pts = fluid(*fluid_lattice_dims(n), seed=3)
    else:
        pts = gen(n, seed=3)
    s, perm = oracle.compress_reduced(pts, xi, "rel", r, want_perm=True)
    st = oracle.stages(pts, xi, "rel", r)
    props.check_reduced(pts, s, perm, oracle.decompress(s), st["q"], st["n_leaves"])
    h = props.parse_header(s)
    assert h["version"] == 2 and h["reserved"] <= st["n_leaves"]


def test_lossless_fallback(oracle):
    pins.pin_lossless_fallback(oracle)

