"""GPU parity of batched compression: every set of one batch launch gives the
oracle's stream and perm for that set alone, byte for byte, whatever the
other sets are (sizes from empty to several global levels, both types, both
layouts, both bound modes, 2-D and 3-D, leaf capacities below and above the
tile), sets that fail report their own status without touching the others,
and a recorded (HIP graph) launch replays to the same bytes on new inputs.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import Oracle, OracleError
from synth import batch_sets, cosmology, uniform_cube

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


# (kind, n, dims, dtype, eb, mode, r, layout, perm)
MIX = [
    ("uniform", 0, 3, np.float32, 1e-3, "rel", 32, "aos", True),
    ("uniform", 1, 3, np.float32, 1e-3, "rel", 32, "aos", True),
    ("uniform", 2, 2, np.float64, 1e-4, "rel", 1, "soa", True),
    ("cosmology", 777, 3, np.float32, 1e-4, "rel", 8, "aos", False),
    ("uniform", 5000, 3, np.float64, 1e-6, "rel", 16, "soa", True),
    ("cosmology", 70001, 3, np.float32, 1e-3, "rel", 32, "aos", True),
    ("uniform", 3001, 2, np.float32, 0.01, "abs", 700, "aos", True),
    ("cosmology", 40000, 3, np.float32, 1e-5, "rel", 1000, "soa", False),
    ("uniform", 513, 3, np.float32, 1e-3, "rel", 512, "aos", True),
    ("cosmology", 250000, 3, np.float32, 1e-4, "rel", 32, "aos", True),
]


def _gen(kind, n, dims, dtype, seed):
    if kind == "uniform":
        return uniform_cube(n, seed=seed, dims=dims, dtype=dtype)
    return cosmology(n, seed=seed, dims=dims, dtype=dtype)


def _specs(cases, seed0=10):
    hosts, specs = [], []
    for i, (kind, n, dims, dt, eb, mode, r, lay, perm) in enumerate(cases):
        pts = _gen(kind, n, dims, dt, seed0 + i)
        host = pts if lay == "aos" else np.ascontiguousarray(pts.T)
        hosts.append(host)
        specs.append(dict(pos=torch.from_numpy(host).cuda(), eb=eb, eb_mode=mode, leaf_size=r,
                          layout=lay, want_perm=perm))
    return hosts, specs


def _check_set(orc, host, spec, got, perm_t, label):
    ref = orc.compress(host, spec["eb"], spec["eb_mode"], spec["leaf_size"],
                       layout=spec["layout"], want_perm=spec["want_perm"])
    ref_s, ref_p = ref if spec["want_perm"] else (ref, None)
    assert not isinstance(got, Exception), f"{label}: {got}"
    assert got.cpu().numpy().tobytes() == ref_s, f"{label}: stream differs from the oracle"
    if ref_p is not None:
        n = len(ref_p)
        assert np.array_equal(perm_t[:n].cpu().numpy().astype(np.uint32), ref_p), f"{label}: perm"


@pytest.mark.parametrize("tile", [0, 256])
def test_batch_mixed_sets_match_oracle(orc, bbx, tile):
    hosts, specs = _specs(MIX)
    _say(f"batch of {len(specs)} mixed sets, tile {tile}")
    bc = bbx.BatchCompressor(specs, tile=tile)
    res = bc()
    for i, (host, spec) in enumerate(zip(hosts, specs)):
        _check_set(orc, host, spec, res[i], bc.perms[i], f"set {i} {MIX[i]}")


@pytest.mark.parametrize("stage", [1, 2])
def test_batch_scatter_stage_invariance(orc, bbx, stage):
    """Forcing either way of storing the global partition's groups for the
    whole batch leaves every set's stream equal to the oracle's."""
    hosts, specs = _specs(MIX, seed0=60)
    _say(f"batch of {len(specs)} mixed sets, scatter_stage {stage}")
    bc = bbx.BatchCompressor(specs, scatter_stage=stage)
    res = bc()
    for i, (host, spec) in enumerate(zip(hosts, specs)):
        _check_set(orc, host, spec, res[i], bc.perms[i], f"set {i} {MIX[i]} stage {stage}")


def test_batch_level_pairs(orc, bbx):
    """Sets with paired global levels (two levels per data movement) batched
    with sets without: each set's key buffers follow its own pairs, and every
    stream equals the oracle's."""
    cases = MIX + [("cosmology", 400000, 3, np.float32, 1e-4, "rel", 32, "aos", False),
                   ("uniform", 300001, 2, np.float32, 1e-3, "rel", 16, "soa", True)]
    hosts, specs = _specs(cases, seed0=90)
    for i, sp in enumerate(specs):
        sp["level_pairs"] = i % 2
    _say(f"batch of {len(specs)} sets, every other one with paired levels")
    bc = bbx.BatchCompressor(specs)
    res = bc()
    for i, (host, spec) in enumerate(zip(hosts, specs)):
        _check_set(orc, host, spec, res[i], bc.perms[i], f"set {i} {cases[i]} pairs {i % 2}")


def test_batch_equals_single_calls(bbx):
    hosts, specs = _specs(MIX[3:8], seed0=40)
    res = bbx.BatchCompressor(specs)()
    for i, spec in enumerate(specs):
        s = bbx.compress(spec["pos"], spec["eb"], spec["eb_mode"], spec["leaf_size"],
                         spec["layout"])
        assert s.cpu().numpy().tobytes() == res[i].cpu().numpy().tobytes(), f"set {i}"


def test_batch_failing_sets_are_isolated(orc, bbx):
    hosts, specs = _specs(MIX[3:7], seed0=70)
    bad_nan = uniform_cube(1000, seed=5).copy()
    bad_nan[417, 1] = np.nan
    bad_eb = uniform_cube(1000, seed=6)
    small = uniform_cube(4000, seed=7)
    extra = [dict(pos=torch.from_numpy(bad_nan).cuda(), eb=1e-3, want_perm=True),
             dict(pos=torch.from_numpy(bad_eb).cuda(), eb=1e-12, want_perm=False),
             dict(pos=torch.from_numpy(small).cuda(), eb=1e-3, out_cap=256)]
    allspecs = specs[:2] + extra + specs[2:]
    allhosts = hosts[:2] + [bad_nan, bad_eb, small] + hosts[2:]
    _say("batch with NaN / too-small eb / too-small output sets")
    bc = bbx.BatchCompressor(allspecs)
    res = bc()
    want = {2: "EINVAL", 4: "ENOSPC"}  # set 3 (bound below the f32 resolution): stored losslessly
    sizes = bc.d_size.cpu().tolist()
    for i, (host, spec) in enumerate(zip(allhosts, allspecs)):
        if i in want:
            assert isinstance(res[i], bbx.BitboxError) and res[i].name == want[i], (i, res[i])
            assert sizes[i] == -1  # UINT64_MAX
            with pytest.raises(OracleError) as e:
                orc.compress(host, spec["eb"], "rel", 32, out_cap=spec.get("out_cap"))
            assert e.value.name == want[i]
        else:
            sp = dict(spec, eb_mode=spec.get("eb_mode", "rel"), leaf_size=spec.get("leaf_size", 32),
                      layout=spec.get("layout", "aos"), want_perm=spec.get("want_perm", False))
            _check_set(orc, host, sp, res[i], bc.perms[i], f"set {i}")


def test_batch_graph_replay(orc, bbx):
    """Record the kernels once; refill the inputs in place and replay."""
    sets = [pos for pos, _, _ in batch_sets(24, seed0=900, hi_exp=5.0)]
    ebs = [eb for _, eb, _ in batch_sets(24, seed0=900, hi_exp=5.0)]
    specs = [dict(pos=torch.from_numpy(p).cuda(), eb=ebs[i], leaf_size=32,
                  want_perm=(i % 3 == 0)) for i, p in enumerate(sets)]
    bc = bbx.BatchCompressor(specs)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        bc.upload(stream)
        bc.launch(stream)  # eager warm-up on the same workspace
    stream.synchronize()
    eager = [r.cpu().numpy().tobytes() for r in bc.results()]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bc.launch()
    for rep in range(3):
        _say(f"graph replay {rep}")
        hosts = []
        for i, p in enumerate(sets):
            # new values of the same shape: each replay compresses a new batch
            rng = np.random.default_rng(7000 + 31 * rep + i)
            host = (p + rng.random(p.shape, dtype=np.float32) * np.float32(0.5)) if rep else p
            hosts.append(host)
            specs[i]["pos"].copy_(torch.from_numpy(host))
        bc.d_status.fill_(99)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        res = bc.results()
        for i, (host, spec) in enumerate(zip(hosts, specs)):
            sp = dict(spec, eb_mode="rel", layout="aos")
            _check_set(orc, host, sp, res[i], bc.perms[i], f"replay {rep} set {i}")
            if rep == 0:
                assert res[i].cpu().numpy().tobytes() == eager[i]


def test_batch_mixed_reference_rules(orc, bbx):
    """Sets of one batch may use different reference rules; each matches the
    oracle under its own rule."""
    cases = [("cosmology", 30011, 3, np.float32, 1e-4, "rel", 32, "aos", False),
             ("uniform", 9001, 2, np.float32, 1e-3, "rel", 16, "aos", True),
             ("cosmology", 60000, 3, np.float32, 1e-4, "rel", 700, "soa", False)]
    hosts, specs = _specs(cases, seed0=40)
    rules = [1, 0, 1]
    for spec, rule in zip(specs, rules):
        spec["ref_rule"] = rule
    _say("batch with reference rules", rules)
    bc = bbx.BatchCompressor(specs)
    res = bc()
    for i, (host, spec) in enumerate(zip(hosts, specs)):
        ref = orc.compress(host, spec["eb"], spec["eb_mode"], spec["leaf_size"],
                           layout=spec["layout"], want_perm=spec["want_perm"],
                           ref_rule=spec["ref_rule"])
        ref_s = ref[0] if spec["want_perm"] else ref
        assert res[i].cpu().numpy().tobytes() == ref_s, f"set {i} rule {rules[i]}"


def test_batch_mixed_reference_modes(orc, bbx):
    """Sets of one batch may store their references differently (codes or
    original coordinates), with or without perm outputs; each matches the
    oracle under its own mode."""
    cases = [("cosmology", 30011, 3, np.float32, 1e-4, "rel", 32, "aos", False),
             ("uniform", 9001, 2, np.float64, 1e-3, "rel", 16, "aos", True),
             ("cosmology", 60000, 3, np.float32, 1e-4, "rel", 700, "soa", False),
             ("uniform", 4000, 3, np.float32, 1e-3, "rel", 8, "soa", False)]
    hosts, specs = _specs(cases, seed0=50)
    modes = [1, 1, 1, 0]
    for spec, m in zip(specs, modes):
        spec["ref_mode"] = m
    _say("batch with reference modes", modes)
    bc = bbx.BatchCompressor(specs)
    res = bc()
    for i, (host, spec) in enumerate(zip(hosts, specs)):
        ref = orc.compress(host, spec["eb"], spec["eb_mode"], spec["leaf_size"],
                           layout=spec["layout"], want_perm=spec["want_perm"],
                           ref_mode=spec["ref_mode"])
        ref_s = ref[0] if spec["want_perm"] else ref
        assert res[i].cpu().numpy().tobytes() == ref_s, f"set {i} mode {modes[i]}"
        if spec["want_perm"]:
            assert np.array_equal(bc.perms[i][:len(ref[1])].cpu().numpy().astype(np.uint32), ref[1])


def test_autotune_picks_smallest_stream(orc, bbx):
    """The autotuner on a small mixed batch: per set, the chosen leaf size
    gives the smallest stream among the candidates (ties to the larger r),
    and the tuned batch equals the oracle at that leaf size at every tile
    capacity (the tile never changes the bytes)."""
    from paper_2404_02826_amd import autotune
    rng = np.random.default_rng(8)
    arrays, specs = [], []
    for i in range(12):
        n = int(10 ** rng.uniform(3, 4.7))
        pts = (uniform_cube if i % 2 else cosmology)(n, seed=300 + i)
        eb = 1e-3 if i % 3 else 1e-4
        arrays.append(pts)
        specs.append(dict(pos=torch.from_numpy(pts).cuda(), eb=eb))
    tuned = autotune.tune(specs, leaf_candidates=(8, 16, 32, 64), reps=1)
    cands = sorted(tuned.per_set_bytes)
    for i in range(len(specs)):
        sizes = {r: tuned.per_set_bytes[r][i] for r in cands}
        best = min(sizes.values())
        assert sizes[tuned.leaf_sizes[i]] == best, (i, sizes, tuned.leaf_sizes[i])
        assert tuned.leaf_sizes[i] == max(r for r in cands if sizes[r] == best)
    assert tuned.tile in (256, 512)
    for tile in (256, 512):
        bc = bbx.BatchCompressor([dict(sp, leaf_size=tuned.leaf_sizes[i]) for i, sp in enumerate(specs)],
                                 tile=tile)
        bc.upload()
        bc.launch()
        torch.cuda.synchronize()
        assert (bc.d_status.cpu().numpy()[: len(specs)] == 0).all()
        sz = bc.d_size.cpu().numpy()
        for i, pts in enumerate(arrays):
            ref = orc.compress(pts, specs[i]["eb"], "rel", tuned.leaf_sizes[i])
            got = bc.out[bc.offsets[i]: bc.offsets[i] + int(sz[i])].cpu().numpy().tobytes()
            assert got == ref, f"tile {tile}, set {i}: stream differs from the oracle's"
            assert len(ref) == tuned.per_set_bytes[tuned.leaf_sizes[i]][i]

