"""Leaf-size and tile autotuner for batched compression.

The leaf capacity r (the largest particle count of an unsplit subregion,
Sec. 4.1) changes the stream: small r stores many bit-box references, large
r mixes dense and sparse space in one box, and the best value depends on the
spatial distribution and on the bound rather than on the set size alone
(parameter analysis, Sec. 5, observations O1-O3).  The tuner therefore
measures instead of guessing: it compresses every set at each candidate r
(one batched launch per candidate) and keeps, per set, the r that gives the
smallest stream (ties go to the larger r, which has fewer leaves to pack).

The tile capacity only changes where the deepest levels of the partition run
(on-chip or through global passes) and never the bytes, so the tuner records
the tuned batch once per tile capacity, replays each recording a few times
and keeps the fastest.

Both choices are plain functions of the measurements (``pick_leaf_sizes``,
``pick_tile``) so that they can be checked without a GPU.
"""
from __future__ import annotations

from dataclasses import dataclass, field

DEFAULT_LEAF_CANDIDATES = (8, 16, 32, 64, 128)
DEFAULT_TILES = (256, 512)


def pick_leaf_sizes(sizes: dict[int, list[int]]) -> list[int]:
    """Per set, the candidate r with the smallest stream; ties to larger r.

    ``sizes[r][i]`` is the stream length of set i at leaf size r, or a
    negative value if that compression failed (such a candidate never wins
    unless every candidate failed, in which case the largest r is kept).
    """
    cands = sorted(sizes)
    if not cands:
        raise ValueError("no candidates")
    nsets = len(sizes[cands[0]])
    out = []
    for i in range(nsets):
        best_r, best = cands[-1], None
        for r in cands:
            v = sizes[r][i]
            if v < 0:
                continue
            if best is None or v < best or (v == best and r > best_r):
                best_r, best = r, v
        out.append(best_r)
    return out


def pick_tile(times_ms: dict[int, float]) -> int:
    """The tile capacity with the smallest measured time (ties to larger)."""
    if not times_ms:
        raise ValueError("no tiles")
    return min(times_ms, key=lambda t: (times_ms[t], -t))


@dataclass
class Tuned:
    leaf_sizes: list[int]
    tile: int
    stream_bytes: dict[int, int] = field(default_factory=dict)  # total per candidate r
    tile_ms: dict[int, float] = field(default_factory=dict)
    tuned_bytes: int = 0
    per_set_bytes: dict[int, list[int]] = field(default_factory=dict)  # [r][set], -1 failed


def tune(specs, leaf_candidates=DEFAULT_LEAF_CANDIDATES, tiles=DEFAULT_TILES, reps: int = 3,
         device="cuda") -> Tuned:
    """Tunes leaf size per set and the tile capacity for a batch.

    ``specs`` are BatchCompressor set dicts (``pos``, ``eb`` and optional
    ``eb_mode``, ``layout``); their ``leaf_size`` and ``want_perm`` are
    ignored here.
    """
    import torch

    from ._binding import BatchCompressor

    base = [dict(pos=s["pos"], eb=s["eb"], eb_mode=s.get("eb_mode", "rel"),
                 layout=s.get("layout", "aos")) for s in specs]
    sizes: dict[int, list[int]] = {}
    for r in leaf_candidates:
        bc = BatchCompressor([dict(b, leaf_size=r) for b in base], device=device)
        bc.upload()
        bc.launch()
        torch.cuda.synchronize()
        st = bc.d_status.cpu().tolist()[: len(base)]
        sz = bc.d_size.cpu().tolist()[: len(base)]
        sizes[r] = [sz[i] if st[i] == 0 else -1 for i in range(len(base))]
        del bc
    leaf = pick_leaf_sizes(sizes)
    tuned_specs = [dict(b, leaf_size=leaf[i]) for i, b in enumerate(base)]
    times: dict[int, float] = {}
    for t in tiles:
        bc = BatchCompressor(tuned_specs, tile=t, device=device)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            bc.upload(stream)
            bc.launch(stream)
        stream.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            bc.launch()
        best = None
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            g.replay()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        times[t] = best
        del g, bc
    tuned_bytes = sum(sizes[leaf[i]][i] for i in range(len(base)) if sizes[leaf[i]][i] >= 0)
    return Tuned(leaf_sizes=leaf, tile=pick_tile(times),
                 stream_bytes={r: sum(v for v in sizes[r] if v >= 0) for r in sizes},
                 tile_ms=times, tuned_bytes=tuned_bytes, per_set_bytes=sizes)
