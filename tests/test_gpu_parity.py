"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Streams must be byte-identical, the perm outputs equal, and decompressed
positions bit-identical, on seeded inputs that span several tiles and
global levels with ragged tails, both key widths (u16/u32 codes), 2-D and
3-D, FP32 and FP64, both layouts, both bound modes, and leaf capacities
below and above the tile capacity.  Full-size workloads are checked by
properties that hold at any size plus sampled leaves.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import props
from oracle import Oracle, OracleError
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


def gen(kind, n, dims=3, dtype=np.float32, seed=1):
    if kind == "uniform":
        return uniform_cube(n, seed=seed, dims=dims, dtype=dtype)
    if kind == "cosmology":
        return cosmology(n, seed=seed, dims=dims, dtype=dtype)
    if kind == "fluid":
        return fluid(*fluid_lattice_dims(n), seed=seed, dtype=dtype)
    if kind == "poincare":  # 2-D, points on curves
        return poincare(n, seed=seed, dtype=dtype)
    if kind == "ties":  # heavy duplication: many equal codes at every median
        rng = np.random.default_rng(seed)
        return (np.floor(rng.random((n, dims)) * 5) / 5).astype(dtype)
    raise ValueError(kind)


def gpu_roundtrip(bbx, pts, eb, mode, r, layout="aos", tile=0, ref_rule=0, ref_mode=0,
                  want_perm=True, scatter_stage=0, level_blocks=0, level_pairs=0):
    host = pts if layout == "aos" else np.ascontiguousarray(pts.T)
    x = torch.from_numpy(host).cuda()
    out = bbx.compress(x, eb, mode, r, layout, want_perm=want_perm, tile=tile, ref_rule=ref_rule,
                       ref_mode=ref_mode, scatter_stage=scatter_stage, level_blocks=level_blocks,
                       level_pairs=level_pairs)
    s, perm = out if want_perm else (out, None)
    dec = bbx.decompress(s, layout)
    torch.cuda.synchronize()
    return (s.cpu().numpy().tobytes(),
            perm.cpu().numpy().astype(np.uint32) if want_perm else None, dec.cpu().numpy())


def first_diff(a: bytes, b: bytes):
    for i in range(min(len(a), len(b))):
        if a[i] != b[i]:
            return i
    return min(len(a), len(b))


def check_parity(orc, bbx, pts, eb, mode, r, layout="aos", tile=0, ref_rule=0, ref_mode=0,
                 want_perm=True, scatter_stage=0, level_blocks=0, ref=None, level_pairs=0):
    host = pts if layout == "aos" else np.ascontiguousarray(pts.T)
    ref_s, ref_p = ref if ref is not None else orc.compress(
        host, eb, mode, r, layout=layout, want_perm=True, ref_rule=ref_rule, ref_mode=ref_mode)
    got_s, got_p, got_d = gpu_roundtrip(bbx, pts, eb, mode, r, layout, tile, ref_rule, ref_mode,
                                        want_perm, scatter_stage, level_blocks, level_pairs)
    if got_s != ref_s:
        h = props.parse_header(ref_s)
        mb = 8 * ((h["meta_bits"] + 63) // 64)
        i = first_diff(got_s, ref_s)
        where = "header" if i < 128 else ("meta" if i < 128 + mb else "payload")
        raise AssertionError(f"stream differs at byte {i} ({where}); sizes {len(got_s)} vs {len(ref_s)}")
    assert got_p is None or np.array_equal(got_p, ref_p), "perm differs"
    ref_d = orc.decompress(ref_s, layout)
    assert np.array_equal(got_d, ref_d), "decompressed positions differ"
    return ref_s


# (generator, n, dims, dtype, eb, mode, r)
CASES = [
    ("uniform", 1, 3, np.float32, 1e-3, "rel", 32),
    ("uniform", 2, 3, np.float32, 1e-3, "rel", 1),
    ("uniform", 3, 2, np.float32, 1e-3, "rel", 1),
    ("uniform", 33, 3, np.float32, 1e-3, "rel", 32),
    ("ties", 1000, 3, np.float32, 1e-3, "rel", 7),
    ("cosmology", 2047, 3, np.float32, 1e-4, "rel", 32),
    ("cosmology", 2048, 3, np.float32, 1e-4, "rel", 32),
    ("cosmology", 2049, 3, np.float32, 1e-4, "rel", 32),
    ("uniform", 4097, 2, np.float32, 1e-3, "rel", 5),
    ("ties", 20000, 3, np.float32, 1e-2, "rel", 32),
    ("cosmology", 20011, 3, np.float64, 1e-6, "rel", 33),     # u32 codes
    ("uniform", 65536, 3, np.float32, 1e-3, "rel", 32),       # the plain single-set workload
    ("cosmology", 65536, 3, np.float32, 1e-4, "rel", 32),
    ("fluid", 32768, 3, np.float32, 1e-4, "rel", 32),
    ("cosmology", 100003, 3, np.float32, 1e-3, "rel", 1),
    ("cosmology", 100003, 2, np.float32, 1e-4, "rel", 100),
    ("uniform", 100003, 3, np.float64, 1e-5, "abs", 16),
    ("cosmology", 300007, 3, np.float32, 1e-4, "rel", 32),
    ("ties", 300007, 3, np.float32, 1e-3, "rel", 32),
    ("cosmology", 150001, 3, np.float32, 1e-7, "rel", 32),    # G > 16 on float32: u32 codes
    ("cosmology", 5000, 3, np.float32, 1e-3, "rel", 2048),    # leaves >= tile capacity
    ("cosmology", 60000, 3, np.float32, 1e-4, "rel", 3000),
    ("cosmology", 60000, 3, np.float32, 1e-4, "rel", 60000),  # single leaf
    ("uniform", 10000, 3, np.float32, 1e-3, "rel", 4999),     # leaves of r+1 split once more
    ("uniform", 3001, 2, np.float32, 1e-2, "rel", 700),       # wavefront level at depth 0, no tiles
    ("ties", 50000, 2, np.float64, 1e-3, "rel", 2100),
    ("poincare", 100003, 2, np.float32, 1e-4, "rel", 32),     # fusion-shaped 2-D
    ("poincare", 300007, 2, np.float32, 1e-3, "rel", 16),
    ("poincare", 65536, 2, np.float64, 1e-6, "rel", 32),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-n{c[1]}-d{c[2]}-{np.dtype(c[3]).name}-{c[4]}-{c[5]}-r{c[6]}")
def test_parity(orc, bbx, case):
    kind, n, dims, dt, eb, mode, r = case
    _say("case", case)
    pts = gen(kind, n, dims, dt, seed=n % 97 + 1)
    check_parity(orc, bbx, pts, eb, mode, r)


# paired global levels (two levels per data movement): the sets with at
# least two levels that use global histograms, with and without indices,
# 16- and 32-bit codes, 2-D and 3-D, few and many chunks per node, and an
# odd count of such levels (the last one alone)
PAIR_CASES = [
    ("cosmology", 300007, 3, np.float32, 1e-4, "rel", 32, True, 0),
    ("ties", 300007, 3, np.float32, 1e-3, "rel", 32, False, 0),
    ("cosmology", 150001, 3, np.float32, 1e-7, "rel", 32, True, 0),   # u32 codes (mid passes)
    ("poincare", 300007, 2, np.float32, 1e-3, "rel", 16, True, 0),
    ("uniform", 100003, 3, np.float64, 1e-5, "abs", 16, True, 0),
    ("fluid", 1 << 20, 3, np.float32, 1e-4, "rel", 32, False, 0),
    ("cosmology", 1 << 20, 3, np.float32, 1e-4, "rel", 32, True, 7),    # few blocks per level
    ("uniform", (1 << 19) + 333, 3, np.float32, 1e-3, "rel", 8, True, 0),
    ("cosmology", 700001, 3, np.float32, 1e-4, "rel", 1000, False, 0),  # leaves above a tile
]


@pytest.mark.parametrize("case", PAIR_CASES,
                         ids=lambda c: f"{c[0]}-n{c[1]}-d{c[2]}-{np.dtype(c[3]).name}-r{c[6]}-perm{int(c[7])}-lb{c[8]}")
def test_level_pairs_parity(orc, bbx, case):
    kind, n, dims, dt, eb, mode, r, perm, lb = case
    _say("pairs", case)
    pts = gen(kind, n, dims, dt, seed=n % 89 + 3)
    ref = check_parity(orc, bbx, pts, eb, mode, r, want_perm=perm, level_blocks=lb, level_pairs=1)
    # and the same stream as one data movement per level
    got, _, _ = gpu_roundtrip(bbx, pts, eb, mode, r, want_perm=False, level_blocks=lb)
    assert got == ref


@pytest.mark.parametrize("layout", ["aos", "soa"])
@pytest.mark.parametrize("tile", [256, 512])
def test_layout_and_tile_invariance(orc, bbx, layout, tile):
    """Tile capacity never changes the bytes; SoA input gives the same stream."""
    _say("layout", layout, "tile", tile)
    pts = cosmology(70001, seed=5)
    check_parity(orc, bbx, pts, 1e-4, "rel", 32, layout=layout, tile=tile)


# sets with levels that use global histograms: both ways of storing a
# partition group (1 = staged in LDS, 2 = straight from the ranks) give the
# oracle's bytes, with and without the source indices carried along
# (generator, n, dims, dtype, eb, mode, r, want_perm, ref_mode)
STAGE_CASES = [
    ("cosmology", 300007, 3, np.float32, 1e-4, "rel", 32, False, 0),
    ("ties", 300007, 3, np.float32, 1e-3, "rel", 32, True, 0),
    ("cosmology", 150001, 3, np.float32, 1e-7, "rel", 32, False, 0),   # u32 codes
    ("cosmology", 100003, 2, np.float32, 1e-4, "rel", 100, True, 0),
    ("uniform", 100003, 3, np.float64, 1e-5, "abs", 16, False, 1),
    ("fluid", 262144, 3, np.float32, 1e-4, "rel", 32, False, 0),
]


@pytest.mark.parametrize("stage", [1, 2])
@pytest.mark.parametrize("case", STAGE_CASES, ids=lambda c: f"{c[0]}-n{c[1]}-d{c[2]}-perm{int(c[7])}-m{c[8]}")
def test_scatter_stage_invariance(orc, bbx, case, stage):
    kind, n, dims, dt, eb, mode, r, want_perm, ref_mode = case
    _say("scatter stage", stage, case)
    pts = gen(kind, n, dims, dt, seed=n % 83 + 7)
    check_parity(orc, bbx, pts, eb, mode, r, want_perm=want_perm, ref_mode=ref_mode,
                 scatter_stage=stage)


RULE1_CASES = [
    ("cosmology", 100003, 3, np.float32, 1e-4, "rel", 32, 0),
    ("cosmology", 100003, 3, np.float32, 1e-4, "rel", 32, 512),
    ("ties", 20000, 3, np.float32, 1e-2, "rel", 7, 0),
    ("uniform", 4097, 2, np.float32, 1e-3, "rel", 5, 0),
    ("cosmology", 20011, 3, np.float64, 1e-6, "rel", 33, 0),      # u32 codes
    ("cosmology", 150001, 3, np.float32, 1e-7, "rel", 32, 0),     # wide tiles
    ("cosmology", 60000, 3, np.float32, 1e-4, "rel", 3000, 0),    # leaves above the tile
    ("poincare", 100003, 2, np.float32, 1e-4, "rel", 32, 0),
]


@pytest.mark.parametrize("case", RULE1_CASES, ids=lambda c: f"{c[0]}-n{c[1]}-d{c[2]}-r{c[6]}-t{c[7]}")
def test_reference_rule_fewest_bits(orc, bbx, case):
    """Reference rule 1 (fewest code bits) matches the oracle's rule 1 byte for
    byte in every leaf stage (tiles of 256 / 512, the 32-bit tile pass,
    leaves above the tile capacity)."""
    kind, n, dims, dt, eb, mode, r, tile = case
    _say("rule 1", case)
    pts = gen(kind, n, dims, dt, seed=n % 89 + 3)
    check_parity(orc, bbx, pts, eb, mode, r, tile=tile, ref_rule=1)


# (generator, n, dims, dtype, eb, mode, r, tile, layout, want_perm)
REF_MODE1_CASES = [
    ("uniform", 1, 3, np.float32, 1e-3, "rel", 32, 0, "aos", False),
    ("uniform", 3, 2, np.float64, 1e-3, "rel", 1, 0, "aos", True),
    ("ties", 20000, 3, np.float32, 1e-2, "rel", 7, 0, "aos", False),
    ("cosmology", 100003, 3, np.float32, 1e-4, "rel", 32, 0, "aos", False),
    ("cosmology", 100003, 3, np.float32, 1e-4, "rel", 32, 512, "soa", True),
    ("cosmology", 20011, 3, np.float64, 1e-6, "rel", 33, 0, "soa", False),  # u32 codes
    ("cosmology", 150001, 3, np.float32, 1e-7, "rel", 32, 0, "aos", False),  # wide tiles
    ("cosmology", 60000, 3, np.float32, 1e-4, "rel", 3000, 0, "aos", False),  # leaves above the tile
    ("ties", 50000, 2, np.float64, 1e-3, "rel", 2100, 0, "soa", False),
    ("poincare", 100003, 2, np.float32, 1e-4, "rel", 32, 0, "aos", False),
    ("fluid", 32768, 3, np.float32, 1e-4, "abs", 32, 0, "aos", True),
    ("uniform", 100003, 3, np.float64, 1e-5, "abs", 1, 0, "aos", False),  # every particle a reference
]


@pytest.mark.parametrize("case", REF_MODE1_CASES,
                         ids=lambda c: f"{c[0]}-n{c[1]}-d{c[2]}-{np.dtype(c[3]).name}-r{c[6]}-t{c[7]}-{c[8]}-p{int(c[9])}")
def test_lossless_reference(orc, bbx, case):
    """Reference stored as its original coordinates (ref_mode 1): the stream
    equals the oracle's byte for byte and decodes identically (references
    exact), with and without a perm output (source indices are carried
    either way), in every leaf stage and both layouts."""
    kind, n, dims, dt, eb, mode, r, tile, layout, want_perm = case
    _say("ref_mode 1", case)
    pts = gen(kind, n, dims, dt, seed=n % 83 + 5)
    if mode == "abs":
        eb = eb * float(np.ptp(pts, axis=0).max() or 1.0)
    check_parity(orc, bbx, pts, eb, mode, r, layout=layout, tile=tile, ref_mode=1,
                 want_perm=want_perm)


def test_lossless_reference_corrupt_on_device(orc, bbx):
    """A non-finite stored reference is a corrupt stream on the device too."""
    pts = cosmology(20000, seed=12)
    good = orc.compress(pts, 1e-3, "rel", 32, ref_mode=1)
    meta = int.from_bytes(good[128:136], "little")
    nan = int(np.array([np.nan], dtype=np.float32).view(np.uint32)[0])
    meta = (meta & ~(((1 << 32) - 1) << 15)) | (nan << 15)  # first record's x coordinate
    b = bytearray(good)
    b[128:136] = meta.to_bytes(8, "little")
    t = torch.from_numpy(np.frombuffer(bytes(b), dtype=np.uint8).copy()).cuda()
    with pytest.raises(bbx.BitboxError) as e:
        bbx.decompress(t)
    assert e.value.name == "ECORRUPT"
    with pytest.raises(OracleError):
        orc.decompress(bytes(b))


# (generator, n, dims, dtype, eb, mode, r)
EXPORT_CASES = [
    ("uniform", 1, 3, np.float32, 1e-3, "rel", 32),
    ("uniform", 4097, 2, np.float64, 1e-3, "rel", 1),            # sequences without codes
    ("ties", 20000, 3, np.float32, 1e-2, "rel", 7),
    ("cosmology", 100003, 3, np.float32, 1e-4, "rel", 32),       # many blocks, shared words
    ("cosmology", 60000, 3, np.float64, 1e-6, "rel", 3000),      # long code segments, 64-bit centres
    ("poincare", 65536, 2, np.float32, 1e-4, "rel", 16),
]


@pytest.mark.parametrize("case", EXPORT_CASES, ids=lambda c: f"{c[0]}-n{c[1]}-d{c[2]}-{np.dtype(c[3]).name}-r{c[6]}")
def test_sequence_export(orc, bbx, case):
    """The Sec. 4.2 sequence layout exported on the GPU from a ref_mode 1
    stream equals the oracle's export byte for byte."""
    kind, n, dims, dt, eb, mode, r = case
    _say("export", case)
    pts = gen(kind, n, dims, dt, seed=n % 71 + 9)
    ref_s = orc.compress(pts, eb, mode, r, ref_mode=1)
    want = orc.export_sequences(ref_s)
    s = bbx.compress(torch.from_numpy(pts).cuda(), eb, mode, r, ref_mode=1)
    assert s.cpu().numpy().tobytes() == ref_s
    got = bbx.export_sequences(s).cpu().numpy().tobytes()
    if got != want:
        raise AssertionError(f"export differs at byte {first_diff(got, want)}; sizes {len(got)} vs {len(want)}")


def test_sequence_export_errors(orc, bbx):
    """A code-reference stream has no lossless centres to export (EINVAL); a
    width field that Eq. 2 never produces is reported as ECORRUPT."""
    pts = cosmology(20000, seed=14)
    s0 = bbx.compress(torch.from_numpy(pts).cuda(), 1e-3, "rel", 32)
    with pytest.raises(bbx.BitboxError) as e:
        bbx.export_sequences(s0)
    assert e.value.name == "EINVAL"
    good = orc.compress(pts, 1e-3, "rel", 32, ref_mode=1)
    b = bytearray(good)
    b[128] = (b[128] & ~31) | 1  # first record's x width: 1
    with pytest.raises(bbx.BitboxError) as e:
        bbx.export_sequences(torch.from_numpy(np.frombuffer(bytes(b), dtype=np.uint8).copy()).cuda())
    assert e.value.name == "ECORRUPT"


def test_empty(orc, bbx):
    pts = np.zeros((0, 3), dtype=np.float32)
    ref = orc.compress(pts, 1e-3, "rel", 32)
    x = torch.zeros((0, 3), dtype=torch.float32, device="cuda")
    s = bbx.compress(x, 1e-3, "rel", 32)
    assert s.cpu().numpy().tobytes() == ref
    assert bbx.decompress(s).shape == (0, 3)


def test_identical_points(orc, bbx):
    pts = np.full((5000, 3), 7.5, dtype=np.float32)
    check_parity(orc, bbx, pts, 1e-4, "rel", 32)


def test_determinism(bbx):
    pts = cosmology(200003, seed=9)
    x = torch.from_numpy(pts).cuda()
    outs = [bbx.compress(x, 1e-4, "rel", 32).cpu().numpy().tobytes() for _ in range(3)]
    assert outs[0] == outs[1] == outs[2]


def test_errors(bbx):
    pts = uniform_cube(5000, seed=3)
    bad = pts.copy()
    bad[17, 2] = np.nan
    for arr, eb, want in ((bad, 1e-3, "EINVAL"),):
        with pytest.raises(bbx.BitboxError) as e:
            bbx.compress(torch.from_numpy(arr).cuda(), eb)
        assert e.value.name == want
    with pytest.raises(bbx.BitboxError) as e:
        bbx.compress(torch.zeros((10, 4), device="cuda"), 1e-3)
    assert e.value.name == "EUNSUPPORTED"
    # out_cap too small: use the raw Compressor with a shrunken capacity
    c = bbx.Compressor(5000)
    c.cap = 256
    with pytest.raises(bbx.BitboxError) as e:
        c(torch.from_numpy(pts).cuda(), 1e-3)
    assert e.value.name == "ENOSPC"


def test_corrupt_payload_detected_on_device(orc, bbx):
    pts = cosmology(20000, seed=10)
    good = orc.compress(pts, 1e-3, "rel", 32)
    h = props.parse_header(good)
    mb = 8 * ((h["meta_bits"] + 63) // 64)
    b = bytearray(good)
    mx = int.from_bytes(b[128:136], "little") & 31
    word = int.from_bytes(b[128 + mb:128 + mb + 8], "little") & ~((1 << mx) - 1)
    b[128 + mb:128 + mb + 8] = word.to_bytes(8, "little")  # first member's x code -> 0
    t = torch.from_numpy(np.frombuffer(bytes(b), dtype=np.uint8).copy()).cuda()
    with pytest.raises(bbx.BitboxError) as e:
        bbx.decompress(t)
    assert e.value.name == "ECORRUPT"
    with pytest.raises(OracleError):
        orc.decompress(bytes(b))


@pytest.mark.parametrize("dt,xi,n,dims,layout", [(np.float32, 1e-12, 5000, 3, "aos"),
                                                  (np.float64, 1e-10, 3001, 3, "soa"),
                                                  (np.float32, 1e-9, 4097, 2, "aos"),
                                                  (np.float32, 1e-12, 2, 3, "aos")])
def test_lossless_fallback(orc, bbx, dt, xi, n, dims, layout):
    """A bound the grid cannot meet (below the input type's resolution, or
    codes of 30 bits or more): the set is stored losslessly (Sec. 4.1's
    escape for coordinates needing more than M bits), byte-identical to the
    oracle, decoded to the input bit for bit, perm the identity; with the
    bit box reduction asked for, the same stream."""
    pts = (uniform_cube(n, seed=n, dims=dims, dtype=np.float64) * 100 - 50).astype(dt)
    ref_s, ref_p = orc.compress(pts if layout == "aos" else np.ascontiguousarray(pts.T), xi, "rel",
                                32, layout=layout, want_perm=True)
    assert props.parse_header(ref_s)["version"] == 3
    for red in (0, 1):
        got_s, got_p, got_d = gpu_roundtrip(bbx, pts, xi, "rel", 32, layout)
        if red:
            host = pts if layout == "aos" else np.ascontiguousarray(pts.T)
            s, p = bbx.compress(torch.from_numpy(host).cuda(), xi, "rel", 32, layout,
                                want_perm=True, reduce=1)
            got_s, got_p = s.cpu().numpy().tobytes(), p.cpu().numpy().astype(np.uint32)
        assert got_s == ref_s, "lossless stream differs from the oracle's"
        assert np.array_equal(got_p, ref_p)
    dec = got_d if layout == "aos" else got_d.T
    assert np.array_equal(np.ascontiguousarray(dec).view(np.uint8), pts.view(np.uint8))


def test_decompress_checks_the_callers_header_copy(bbx):
    """A decode is planned from the caller's host copy of the header; the
    device compares it with the stream's own header and reports a mismatch
    as a corrupt stream (the same stream with its own header decodes)."""
    pts = cosmology(30000, seed=12)
    s = bbx.compress(torch.from_numpy(pts).cuda(), 1e-3)
    good = s[:128].cpu().numpy().tobytes()
    bad = bytearray(good)
    bad[24] ^= 1  # eb_user: still a valid header, not this stream's
    d = bbx.Decompressor(bytes(bad))
    with pytest.raises(bbx.BitboxError) as e:
        d(s)
    assert e.value.name == "ECORRUPT"
    d.d_status.fill_(0)
    d.launch(s)
    torch.cuda.synchronize()
    assert int(d.d_status.item()) == 3  # ECORRUPT in the asynchronous form too
    assert torch.equal(bbx.Decompressor(good)(s), bbx.decompress(s))


def test_decompress_oracle_streams(orc, bbx):
    """The GPU decoder reproduces the oracle's decoder on oracle-written streams."""
    for r in (1, 32, 3000):
        pts = cosmology(30001, seed=r)
        s = orc.compress(pts, 1e-4, "rel", r)
        t = torch.from_numpy(np.frombuffer(s, dtype=np.uint8).copy()).cuda()
        assert np.array_equal(bbx.decompress(t).cpu().numpy(), orc.decompress(s))


def test_full_size_cosmology_1_in_4_oracle(orc, bbx):
    """A quarter of the cosmology workload (2^22 particles, xi = 1e-4), full
    byte parity with the oracle, once with the library's choice of group
    stores and once with every global level staged (the choice of the
    full-size sets, whose chunks hold 16,384 codes or more)."""
    pts = cosmology(1 << 22, seed=2)
    check_parity(orc, bbx, pts, 1e-4, "rel", 32)
    check_parity(orc, bbx, pts, 1e-4, "rel", 32, want_perm=False, scatter_stage=1)


# Sets just above 2^25 particles: depths 12 and 13 (block-local kind) run as
# one 16-wavefront fused pair over nodes of about 8,200 members, half the
# pair's capacity, so every wavefront's lanes past its node's end hold the
# top code of their axis; 16-bit codes with source indices, then 32-bit
# codes (G = 20).  Byte parity with the oracle.
@pytest.mark.timeout(1200)
@pytest.mark.parametrize("kind,xi,seed", [("cosmology", 1e-4, 5), ("uniform", 1e-6, 6)])
def test_fused16_ragged_nodes(orc, bbx, kind, xi, seed):
    n = (1 << 25) + 12345
    _say(f"{kind} n={n} xi={xi}: oracle")
    pts = gen(kind, n, seed=seed)
    check_parity(orc, bbx, pts, xi, "rel", 32)


# Few blocks per global level: every block's chunk spans many 2048-member
# groups (up to the whole node at level_blocks = 1), with a partial last
# group, so the multi-group loop of the global partition (next-group
# prefetch, running below/equal counts, the staged group's reuse) is
# byte-checked at sizes the oracle finishes quickly; the stream must not
# depend on the chunking.
@pytest.mark.parametrize("n,kind,xi", [(262461, "cosmology", 1e-4), (1 << 20, "fluid", 1e-4),
                                       (300007, "ties", 1e-3)])
def test_multi_group_chunks(orc, bbx, n, kind, xi):
    pts = gen(kind, n, seed=31)
    ref = orc.compress(pts, xi, "rel", 32, want_perm=True)
    for lb in (1, 3, 16, 64):
        for stage in (1, 2):
            _say(f"{kind} n={n} level_blocks={lb} scatter_stage={stage}")
            check_parity(orc, bbx, pts, xi, "rel", 32, scatter_stage=stage, level_blocks=lb,
                         want_perm=(lb != 3), ref=ref)

