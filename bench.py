"""Benchmark: compress + decompress throughput of the bit-box particle
compressor on one MI355X, inputs resident in HBM.

One step = one compress of the whole set (range, quantize, k-d partition,
bit boxes, offsets, packing) + one decompress of the resulting stream.
Prints one JSON line (rank 0).  Default workload: the fluid-shaped set,
2^27 FP32 particles on a 512^3 jittered lattice with a 2-cell vortex,
relative bound 1e-4, leaf size 32.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
METRIC = "compress+decompress GB/s (FP32 xyz, rel eb 1e-4), CR, % HBM roofline, p99 latency"

WORKLOADS = {
    # name: (generator, n, dtype, rel eb)
    "fluid-2^27-f32": ("fluid", 1 << 27, "float32", 1e-4),
    "fluid-2^26-f64": ("fluid", 1 << 26, "float64", 1e-4),
    "cosmology-2^24-f32-xi1e-4": ("cosmology", 1 << 24, "float32", 1e-4),
    "cosmology-2^24-f32-xi1e-3": ("cosmology", 1 << 24, "float32", 1e-3),
    "uniform-65536-f32-xi1e-3": ("uniform", 65536, "float32", 1e-3),
    # moderate sets for the bit box reduction (one workgroup runs a set's pops)
    "cosmology-2^18-f32-xi1e-4": ("cosmology", 1 << 18, "float32", 1e-4),
    "fluid-2^18-f32-xi1e-4": ("fluid", 1 << 18, "float32", 1e-4),
    # fusion-shaped 2-D set of the size of the paper's XGC Poincare data
    "poincare-2d-13077313-f32": ("poincare", 13077313, "float32", 1e-4),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_points(kind, n, dtype):
    import numpy as np
    from synth import cosmology, fluid, fluid_lattice_dims, poincare, uniform_cube
    dt = np.float32 if dtype == "float32" else np.float64
    if kind == "fluid":
        return fluid(*fluid_lattice_dims(n), seed=4, dtype=dt)
    if kind == "poincare":
        return poincare(n, seed=8, dtype=dt)
    if kind == "cosmology":
        return cosmology(n, seed=2, dtype=dt)
    return uniform_cube(n, seed=1, dtype=dt)


# Algorithmic bytes per particle of each kernel (no perm): what the kernel
# must read and write, not what it happens to move.
def kernel_bytes_per_particle(name, key_bytes, in_bytes, stream_bytes_pp, dims=3):
    kb = dims * key_bytes
    return {
        "range_minmax": in_bytes,
        "quantize": in_bytes + kb,
        "level_hist_mid": key_bytes,
        "level_hist_last": key_bytes,
        "level_scatter": 2 * kb,
        "level_local": 2 * kb,
        "level_wave": 2 * kb,
        "tile": 2 * kb,
        "pack_payload": kb + stream_bytes_pp,
        "unpack": stream_bytes_pp + in_bytes,
    }.get(name)


def bench_copy(args):
    """A plain device-to-device copy of 1 GiB: the achievable-bandwidth
    reference and the known-size kernel the HBM byte counters are scaled by."""
    import torch
    nbytes = 1 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    for _ in range(args.warmup):
        b.copy_(a)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        b.copy_(a)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    gbps = 2 * nbytes * args.steps / el / 1e9
    print(json.dumps({"metric": "device copy GB/s (read + write)", "value": round(gbps, 1),
                      "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": round(el * 1e3 / args.steps, 4), "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
                      "config": {"workload": "copy-1GiB", "bytes": nbytes},
                      "roofline": {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBS, 4),
                                   "traffic": None},
                      "cpu_baseline": None}), flush=True)


def bench_entropy(args):
    """The entropy stage of Sec. 3 / 4.2 on a workload: the version-1 stream
    with stored-coordinate references, its sequence layout, the layout after
    the two reorderings, and Huffman coding (of the plain stream, the plain
    layout and the reordered layout): sizes, compression ratios and device
    throughput (each call waits; times over K calls after W warm-ups)."""
    import numpy as np  # noqa: F401
    import torch

    import paper_2404_02826_amd as bbx

    kind, n, dtype, xi = WORKLOADS[args.workload]
    log(f"generating {args.workload} ({n} particles)")
    pts = make_points(kind, n, dtype)
    x = torch.from_numpy(pts).cuda()
    B_in = x.numel() * x.element_size()
    s0 = bbx.compress(x, xi, "rel", args.leaf_size)
    s1 = bbx.compress(x, xi, "rel", args.leaf_size, ref_mode=1)
    plain = bbx.export_sequences(s1)
    del x
    torch.cuda.empty_cache()

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t) * 1e3 / args.steps

    (ro, order), t_ro = timed(lambda: bbx.export_sequences_reordered(s1))
    h_ro, t_enc = timed(lambda: bbx.huffman_encode(ro))
    dec, t_dec = timed(lambda: bbx.huffman_decode(h_ro))
    assert torch.equal(dec, ro)
    h_plain = bbx.huffman_encode(plain)
    h_s0 = bbx.huffman_encode(s0)
    L = ro.numel()
    gbps = L / ((t_ro + t_enc) * 1e-3) / 1e9
    print(json.dumps({
        "metric": "entropy stage GB/s (sequence layout bytes through reordering + Huffman coding)",
        "value": round(gbps, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_ro + t_enc, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "leaf_size": args.leaf_size,
                   "input_bytes": B_in, "stream_bytes": s0.numel(),
                   "stream_ref_coords_bytes": s1.numel(), "layout_bytes": L,
                   "huffman_of_stream_bytes": h_s0.numel(),
                   "huffman_of_layout_bytes": h_plain.numel(),
                   "huffman_of_reordered_layout_bytes": h_ro.numel(),
                   "cr_stream": round(B_in / s0.numel(), 4),
                   "cr_layout": round(B_in / L, 4),
                   "cr_huffman_stream": round(B_in / h_s0.numel(), 4),
                   "cr_huffman_layout": round(B_in / h_plain.numel(), 4),
                   "cr_huffman_reordered_layout": round(B_in / h_ro.numel(), 4),
                   "reordering_gain": round(h_plain.numel() / h_ro.numel(), 4),
                   "axis_order": order,
                   "reorder_ms": round(t_ro, 4), "huffman_encode_ms": round(t_enc, 4),
                   "huffman_decode_ms": round(t_dec, 4),
                   "huffman_encode_gbps": round(L / (t_enc * 1e-3) / 1e9, 2),
                   "huffman_decode_gbps": round(L / (t_dec * 1e-3) / 1e9, 2)},
        "roofline": None, "cpu_baseline": None}), flush=True)


def _cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), for the baseline record."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def _sources_digest():
    """SHA-256 over the library's HIP sources (sorted by name): the counter
    summaries record it, and a summary whose digest differs describes other
    kernels."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2404_02826_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per compress + decompress step of `workload`, summed over
    every kernel, from the committed counter summary; None when the library's
    sources have changed since the counters were taken."""
    import re
    path = os.path.join(ROOT, "profiles", f"roundtrip_{workload}_hbm_bytes.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_b = re.search(r"hbm_bytes_per_step:\s*(\d+)", text)
    m_f = re.search(r"sources_sha256:\s*([0-9a-f]{64})", text)
    if not (m_b and m_f) or m_f.group(1) != _sources_digest():
        return None
    return int(m_b.group(1))


def _level_shape_chunks(n, depth):
    """Chunks per node of a global level (mirrors the library's level shape:
    about 4096 blocks per level, chunks of whole 2048-element groups)."""
    nodes = 1 << depth
    maxsz = (n + nodes - 1) >> depth
    cpn = max(1, (4096 + nodes - 1) // nodes)
    elems = (maxsz + cpn - 1) // cpn
    groups = max(1, (elems + 2047) // 2048)
    chunk = groups * 2048
    return max(1, (maxsz + chunk - 1) // chunk)


def _level_kind(n, depth):
    """0: global histograms, 1: one block per node, 2: one wavefront per node."""
    if ((n + (1 << depth) - 1) >> depth) <= 4096:
        return 2
    return 1 if _level_shape_chunks(n, depth) == 1 else 0


def _global_levels(n, r, tile):
    """Levels above the on-chip stage (tile or large-leaf stage)."""
    tile = tile or 256
    if n == 0:
        return 0
    k = 0
    if r < tile:
        while ((n + (1 << k) - 1) >> k) > tile:
            k += 1
        return k
    while (n >> k) > r:
        k += 1
    return k if ((n + (1 << k) - 1) >> k) <= r else k + 1


def _gen_batch_set(job):
    from synth import batch_set
    s, n, kind, seed0 = job
    return batch_set(s, n, kind, seed0)


def _pctl(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, max(0, int(math.ceil(q * len(v))) - 1))]


def bench_batch(args):
    """Batched compress of many independent sets in one recorded launch,
    against one compress call per set on the same GPU."""
    import numpy as np
    import torch
    from concurrent.futures import ProcessPoolExecutor

    import paper_2404_02826_amd as bbx
    from paper_2404_02826_amd import autotune
    from synth import batch_plan

    nsets, seed0 = args.nsets, 5
    sizes, kinds, ebs = batch_plan(nsets, seed0)
    t0 = time.time()
    jobs = [(s, int(sizes[s]), kinds[s], seed0) for s in range(nsets)]
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        arrays = list(ex.map(_gen_batch_set, jobs, chunksize=32))
    log(f"generated {nsets} sets, {int(sizes.sum())} particles in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    xs = [torch.from_numpy(a).to(dev) for a in arrays]
    torch.cuda.synchronize()
    B_in = sum(a.nbytes for a in arrays)
    n_tot = int(sizes.sum())

    base = [dict(pos=xs[i], eb=ebs[i], eb_mode="rel") for i in range(nsets)]
    if args.leaf_size > 0 and args.tile > 0:
        tuned = autotune.Tuned(leaf_sizes=[args.leaf_size] * nsets, tile=args.tile)
    else:
        t1 = time.time()
        tuned = autotune.tune(base)
        log(f"autotuned in {time.time() - t1:.1f}s: tile {tuned.tile}, tile ms {tuned.tile_ms}, "
            f"bytes per r {tuned.stream_bytes}")
    specs = [dict(b, leaf_size=tuned.leaf_sizes[i]) for i, b in enumerate(base)]

    # ---- batched path: upload once, record the kernels once, replay
    bc = bbx.BatchCompressor(specs, tile=tuned.tile)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        bc.upload(side)
        bc.launch(side)
    side.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bc.launch()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    st = bc.d_status.cpu().numpy()[:nsets]
    assert (st == 0).all(), f"batched sets failed: {np.nonzero(st)[0][:8]}"
    b_sizes = bc.d_size.cpu().numpy()[:nsets]
    S_tot = int(b_sizes.sum())

    torch.cuda.synchronize()
    t_start = time.perf_counter()
    evs = []
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        evs.append((e0, e1))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    job_ms = [a.elapsed_time(b) for a, b in evs]
    value = B_in * args.steps / elapsed / 1e9
    log(f"batched: {elapsed * 1e3 / args.steps:.2f} ms/job, {value:.1f} GB/s")

    # ---- per-set path: one bbx_compress per set, same leaf sizes and tile
    comps = [bbx.Compressor(int(sizes[i]), 3, torch.float32, leaf_size=tuned.leaf_sizes[i],
                            tile=tuned.tile) for i in range(nsets)]

    def per_set_job(record):
        marks = []
        for i in range(nsets):
            comps[i].launch(xs[i], ebs[i])
            if record:
                e = torch.cuda.Event(enable_timing=True)
                e.record()
                marks.append(e)
        return marks

    for _ in range(args.warmup):
        per_set_job(False)
    torch.cuda.synchronize()
    ps_job_ms, ps_lat = [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e0.record()
        marks = per_set_job(True)
        torch.cuda.synchronize()
        lat = [e0.elapsed_time(m) for m in marks]
        ps_lat += lat
        ps_job_ms.append(lat[-1])
    ps_elapsed = time.perf_counter() - t_start
    ps_value = B_in * args.steps / ps_elapsed / 1e9
    log(f"per-set: {ps_elapsed * 1e3 / args.steps:.2f} ms/job, {ps_value:.1f} GB/s")

    # every set's stream equals its per-set stream
    same = 0
    for i in range(nsets):
        n_i = int(comps[i].d_size.item())
        if n_i == int(b_sizes[i]) and torch.equal(comps[i].out[:n_i],
                                                  bc.out[bc.offsets[i]: bc.offsets[i] + n_i]):
            same += 1
    log(f"identical streams: {same}/{nsets}")

    # per-kernel times of one batched job (eager launch on the same workspace)
    with bbx.profile() as prof:
        bc.launch()
        torch.cuda.synchronize()
    dname, (dcount, dms) = max(prof.items(), key=lambda kv: kv[1][1])
    # particles a kernel touches per job: level kernels see each set once per
    # global level of their kind (the library's launch plan), the others once
    kinds = {"level_scatter": 0, "level_local": 1, "level_wave": 2}
    if dname in kinds:
        touched = sum(int(sizes[i]) * sum(1 for k in range(_global_levels(int(sizes[i]), tuned.leaf_sizes[i], tuned.tile))
                                          if _level_kind(int(sizes[i]), k) == kinds[dname])
                      for i in range(nsets))
        bpp = 12.0
    else:
        touched = n_tot
        bpp = kernel_bytes_per_particle(dname, 2, 12, S_tot / n_tot)
    roofline = None
    if bpp is not None and touched > 0:
        per_launch = bpp * touched / dcount
        avg_ms = dms / dcount
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "kernel": dname, "avg_ms": round(avg_ms, 4), "launches_per_step": dcount,
                    "alg_bytes_per_launch": int(per_launch)}

    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on all host cores (at most 16, the box's share for one
        # GPU), one set per thread; the C oracle runs outside the GIL
        from concurrent.futures import ThreadPoolExecutor

        from oracle import Oracle
        orc = Oracle()
        threads = min(16, os.cpu_count() or 1)
        order = [int(i) for i in np.random.default_rng(1).permutation(nsets)]
        t, done_b, k, checked = time.perf_counter(), 0, 0, 0
        with ThreadPoolExecutor(max_workers=threads) as ex:
            while time.perf_counter() - t < 15.0 and k < nsets:
                wave = order[k: k + threads]
                outs = list(ex.map(lambda i: orc.compress(arrays[i], ebs[i], "rel",
                                                          tuned.leaf_sizes[i]), wave))
                for i, so in zip(wave, outs):
                    got = bc.out[bc.offsets[i]: bc.offsets[i] + int(b_sizes[i])].cpu().numpy().tobytes()
                    checked += int(got == so)
                    done_b += arrays[i].nbytes
                k += len(wave)
        dt = time.perf_counter() - t
        cpu = {"value": round(done_b / dt / 1e9, 5), "unit": "GB/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{k} randomly chosen sets of the batch ({done_b} bytes), compress only, "
                         f"one set per thread on {threads} threads ({_cpu_model()}); "
                         f"{checked}/{k} oracle streams equal the batched ones"}

    lat_b = [m for m in job_ms for _ in range(nsets)]  # every set completes with its job
    out = {
        "metric": "batched compress GB/s (4,096 FP32 xyz sets, log-uniform 10^3..10^6), p99 set latency",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed * 1e3 / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batch-{nsets}-f32", "nsets": nsets, "particles": n_tot,
                   "input_bytes": B_in, "stream_bytes": S_tot, "cr": round(B_in / S_tot, 4),
                   "tile": tuned.tile, "leaf_sizes": {str(r): tuned.leaf_sizes.count(r)
                                                      for r in sorted(set(tuned.leaf_sizes))},
                   "tuner_stream_bytes_per_r": {str(k): v for k, v in tuned.stream_bytes.items()},
                   "tuner_tile_ms": {str(k): round(v, 3) for k, v in tuned.tile_ms.items()},
                   "batched": {"gbps": round(value, 2), "job_ms_p50": round(_pctl(job_ms, .5), 3),
                               "set_latency_ms_p50": round(_pctl(lat_b, .5), 3),
                               "set_latency_ms_p99": round(_pctl(lat_b, .99), 3)},
                   "per_set_calls": {"gbps": round(ps_value, 2),
                                     "job_ms_p50": round(_pctl(ps_job_ms, .5), 3),
                                     "set_latency_ms_p50": round(_pctl(ps_lat, .5), 3),
                                     "set_latency_ms_p99": round(_pctl(ps_lat, .99), 3)},
                   "identical_to_per_set": f"{same}/{nsets}",
                   "kernels": {k: {"launches": c, "ms": round(ms, 4)} for k, (c, ms) in
                               sorted(prof.items(), key=lambda kv: -kv[1][1])}},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def _serve_session(bbx, torch, reqs, arrivals, inputs, cfg, sample):
    """Runs one served session; returns per-request (latency s, bytes) and
    the results of the sampled requests (device tensors, cloned)."""
    srv = bbx.Server(cfg["budget"], max_jobs=cfg["max_jobs"], max_batch=cfg["max_batch"],
                     nstreams=cfg["nstreams"], tile=cfg.get("tile", 0))
    t0 = srv.now() + 0.05
    arr = [t0 + a for a in arrivals]
    lat, nbytes, kept, jobs_per_launch = {}, {}, {}, []
    ids, k, max_inflight = {}, 0, 0
    while len(lat) < len(reqs):
        now = srv.now()
        while k < len(reqs) and now >= arr[k]:
            n, kind, comp = reqs[k]
            if comp:
                jid = srv.submit_compress(inputs[k]["x"], 1e-4, "rel", 32)
            else:
                jid = srv.submit_decompress(inputs[k]["stream"], inputs[k]["header"])
            ids[jid] = k
            k += 1
        srv.progress()
        max_inflight = max(max_inflight, srv.counts()["inflight"])
        while True:
            jid = srv.pop_done()
            if not jid:
                break
            d = srv.info(jid)
            i = ids[jid]
            if d["status"] != 0:
                raise RuntimeError(f"served request {i} failed: {d}")
            lat[i] = d["t_done"] - arr[i]
            nbytes[i] = 12 * reqs[i][0]
            jobs_per_launch.append(d["batch_jobs"])
            if i in sample:
                kept[i] = srv.result(jid).clone()
            srv.release(jid)
        if srv.now() - t0 > 300:
            raise RuntimeError("served session did not finish in 300 s")
    makespan = max(arr[i] + lat[i] for i in lat) - t0
    launches = srv.counts()["launches"]
    srv.close()
    return lat, nbytes, kept, makespan, launches, max_inflight, jobs_per_launch


def bench_served(args):
    """Poisson arrivals of compress/decompress requests served with
    continuous batching, against one launch per request on the same GPU."""
    import numpy as np
    import torch

    import paper_2404_02826_amd as bbx
    from synth import poisson_arrivals, request_pool, served_requests

    nreq = args.requests
    reqs = served_requests(nreq, seed0=6)
    nmax = max(r[0] for r in reqs)
    t0 = time.time()
    pools = {k: torch.from_numpy(request_pool(k, nmax)).cuda() for k in ("uniform", "cosmology")}
    log(f"pools of {nmax} particles in {time.time() - t0:.1f}s")
    inputs = []
    for n, kind, comp in reqs:
        x = pools[kind][:n]
        d = {"x": x}
        if not comp:
            st = bbx.compress(x, 1e-4, "rel", 32)
            d["stream"] = st
            d["header"] = st[:128].cpu().numpy().tobytes()
        inputs.append(d)
    torch.cuda.synchronize()
    log(f"prepared {nreq} requests ({sum(1 for r in reqs if not r[2])} decompress streams)")
    arrivals = poisson_arrivals(nreq, args.qps, seed=7)
    sample = set(int(i) for i in np.random.default_rng(2).choice(nreq, size=min(64, nreq),
                                                                  replace=False))
    budget = 64 << 30
    cfgs = {"continuous_batching": dict(budget=budget, max_jobs=4096, max_batch=256, nstreams=4),
            "one_launch_per_request": dict(budget=budget, max_jobs=4096, max_batch=1, nstreams=1)}
    res = {}
    for name, cfg in cfgs.items():
        for _ in range(args.warmup):  # a short warm-up session on the first requests
            _serve_session(bbx, torch, reqs[:32], arrivals[:32], inputs[:32], cfg, set())
        lat, nbytes, kept, span, launches, infl, jpl = _serve_session(
            bbx, torch, reqs, arrivals, inputs, cfg, sample)
        ls = [lat[i] * 1e3 for i in range(nreq)]
        res[name] = dict(gbps=round(sum(nbytes.values()) / span / 1e9, 2),
                         makespan_s=round(span, 4), p50_ms=round(_pctl(ls, .5), 3),
                         p99_ms=round(_pctl(ls, .99), 3), launches=launches,
                         max_launches_in_flight=infl,
                         mean_jobs_per_launch=round(float(np.mean(jpl)), 2), kept=kept)
        log(f"{name}: {res[name]['gbps']} GB/s, p50 {res[name]['p50_ms']} ms, "
            f"p99 {res[name]['p99_ms']} ms, {launches} launches")
    # each sampled result is the same alone and in the mix
    same = 0
    for i in sample:
        n, kind, comp = reqs[i]
        alone = (bbx.compress(inputs[i]["x"], 1e-4, "rel", 32) if comp
                 else bbx.decompress(inputs[i]["stream"]).view(torch.uint8).reshape(-1))
        a = res["continuous_batching"]["kept"][i].reshape(-1).view(torch.uint8)
        b = res["one_launch_per_request"]["kept"][i].reshape(-1).view(torch.uint8)
        same += int(torch.equal(a, alone.reshape(-1)) and torch.equal(b, alone.reshape(-1)))
    for r in res.values():
        r.pop("kept")
    cb, pr = res["continuous_batching"], res["one_launch_per_request"]
    out = {
        "metric": "served compress+decompress GB/s and p50/p99 latency (Poisson arrivals, "
                  "10^4..10^7 FP32 xyz particles per request, rel eb 1e-4)",
        "value": cb["gbps"], "unit": "GB/s", "n_gpus": 1, "steps": nreq, "warmup": args.warmup,
        "ms_per_step": round(cb["makespan_s"] * 1e3 / nreq, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"served-poisson-{args.qps:g}qps-{nreq}req", "qps": args.qps,
                   "requests": nreq, "hbm_budget_bytes": budget,
                   "compress_requests": sum(1 for r in reqs if r[2]),
                   "input_bytes": int(sum(12 * r[0] for r in reqs)),
                   "continuous_batching": cb, "one_launch_per_request": pr,
                   "sampled_results_equal_alone": f"{same}/{len(sample)}"},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="fluid-2^27-f32",
                    choices=sorted(WORKLOADS) + ["batch-4096-f32", "served", "copy-1GiB"])
    ap.add_argument("--leaf-size", type=int, default=32,
                    help="leaf size r (batch workload: 0 = autotuned per set)")
    ap.add_argument("--tile", type=int, default=0,
                    help="tile capacity 256 or 512 (0: library default; batch workload: autotuned)")
    ap.add_argument("--ref-rule", type=int, default=0, choices=(0, 1),
                    help="leaf reference: 0 nearest the AABB centre (the paper's), 1 fewest bits")
    ap.add_argument("--ref-mode", type=int, default=0, choices=(0, 1),
                    help="reference stored as 0 its codes, 1 its original coordinates (lossless)")
    ap.add_argument("--reduce", type=int, default=0, choices=(0, 1, 2),
                    help="bit box reduction after the bit boxes: 1 key sum of widths, 2 key sum of "
                         "box lengths (moderate sets: at most 65,536 leaves)")
    ap.add_argument("--level-pairs", type=int, default=0, choices=(0, 1),
                    help="1: two global partition levels per data movement (same stream)")
    ap.add_argument("--split-rule", type=int, default=0, choices=(0, 1, 2, 3),
                    help="partition split rule: 0 median with axes in turn (the library's), "
                         "1 widest axis, 2 ceil(n/r) proportional leaves, 3 midpoint cells "
                         "(ablations, version-2 streams)")
    ap.add_argument("--scatter-stage", type=int, default=0, choices=(0, 1, 2),
                    help="global partition group stores: 0 by chunk size, 1 staged, 2 direct")
    ap.add_argument("--nsets", type=int, default=4096)
    ap.add_argument("--requests", type=int, default=2000, help="served workload: requests")
    ap.add_argument("--qps", type=float, default=400.0, help="served workload: arrival rate")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 23)
    ap.add_argument("--entropy", action="store_true",
                    help="the entropy stage (sequence layout, reorderings, Huffman coding) on the "
                         "workload instead of the compress + decompress step")
    ap.add_argument("--graph", type=int, default=0, choices=(0, 1),
                    help="single set: replay the compress + decompress step as one recorded HIP graph")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    if args.workload.startswith("batch-"):
        bench_batch(args)
        return
    if args.workload == "served":
        bench_served(args)
        return
    if args.workload == "copy-1GiB":
        bench_copy(args)
        return
    if args.entropy:
        bench_entropy(args)
        return

    import numpy as np
    import torch

    import paper_2404_02826_amd as bbx

    kind, n, dtype, xi = WORKLOADS[args.workload]
    t0 = time.time()
    log(f"generating {args.workload} ({n} particles)")
    pts = make_points(kind, n, dtype)
    log(f"generated in {time.time() - t0:.1f}s; copying to the GPU")
    dev = torch.device("cuda:0")
    x = torch.from_numpy(pts).to(dev)
    torch.cuda.synchronize()
    B_in = x.numel() * x.element_size()

    dims = int(x.shape[1])
    if args.reduce and n > 65536 * args.leaf_size:
        print("the bit box reduction runs a set's pops in one workgroup: use a set of at most "
              "65,536 leaves", file=sys.stderr)
        sys.exit(2)
    comp = bbx.Compressor(n, dims, x.dtype, leaf_size=args.leaf_size, tile=args.tile,
                          ref_rule=args.ref_rule, ref_mode=args.ref_mode,
                          scatter_stage=args.scatter_stage, reduce=args.reduce,
                          split_rule=args.split_rule, level_pairs=args.level_pairs)
    s = comp(x, xi)
    S = s.numel()
    S_plain = S
    if args.reduce or args.split_rule:  # the same input with the plain partition: its size only
        alt = bbx.Compressor(n, dims, x.dtype, leaf_size=args.leaf_size, tile=args.tile)
        S_plain = alt(x, xi).numel()
        del alt
    # the other leaf-reference rule, and the other reference storage, on the
    # same input: their stream sizes only
    alt = bbx.Compressor(n, dims, x.dtype, leaf_size=args.leaf_size, tile=args.tile,
                         ref_rule=1 - args.ref_rule, ref_mode=args.ref_mode,
                         split_rule=args.split_rule)
    S_alt = alt(x, xi).numel()
    del alt
    S_alt_mode = None
    if not args.reduce and not args.split_rule:
        alt = bbx.Compressor(n, dims, x.dtype, leaf_size=args.leaf_size, tile=args.tile,
                             ref_rule=args.ref_rule, ref_mode=1 - args.ref_mode)
        S_alt_mode = alt(x, xi).numel()
        del alt
    torch.cuda.empty_cache()
    header = s[:128].cpu().numpy().tobytes()
    info = bbx.stream_info(header)
    dec = bbx.Decompressor(header)
    stream_buf = comp.out
    log(f"stream {S} bytes, CR {B_in / S:.3f}, leaves {info['n_leaves']}")

    def step():
        comp.launch(x, xi)          # async: size stays on the device
        dec.launch(stream_buf[:S])  # async: same input -> same stream geometry

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # correctness guard on the measured configuration: a sampled bound check
    got = dec(stream_buf[:S]).clone()
    eager_stream = stream_buf[:S].clone()
    torch.cuda.synchronize()
    run = step
    if args.graph:
        # the step recorded once (every library call on the capturing stream,
        # no host synchronization inside), then replayed; each replay is
        # checked against the eager result, with eager work in between
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        for _ in range(3):
            dec.pos.zero_()
            stream_buf[:S].zero_()
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            if not (torch.equal(stream_buf[:S], eager_stream) and
                    torch.equal(dec.pos.view(torch.uint8), got.view(torch.uint8))):
                raise RuntimeError("graph replay differs from the eager step")
            step()
            torch.cuda.synchronize()
        run = graph.replay
        for _ in range(args.warmup):
            run()
    log("warmup done")

    # ---- timed region: exactly K steps
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    value = B_in * args.steps / elapsed / 1e9
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {value:.1f} GB/s")

    # ---- per-phase timing and latency distribution (HIP events, same stream)
    st = torch.cuda.current_stream()
    # (a small set is latency-bound: its p50 / p99 come from at least 1,000 runs)
    lat_runs = args.steps if n > (1 << 20) or args.reduce else max(args.steps, 1000)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(lat_runs)]
    for e0, e1, e2 in ev:
        e0.record(st)
        comp.launch(x, xi)
        e1.record(st)
        dec.launch(stream_buf[:S])
        e2.record(st)
    torch.cuda.synchronize()
    tc = [a.elapsed_time(b) for a, b, _ in ev]
    td = [b.elapsed_time(c) for _, b, c in ev]
    tt = sorted(a + b for a, b in zip(tc, td))
    if args.graph:  # round-trip latency of the replayed step
        eg = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(lat_runs)]
        for e0, e1 in eg:
            e0.record(st)
            run()
            e1.record(st)
        torch.cuda.synchronize()
        tt = sorted(a.elapsed_time(b) for a, b in eg)
    p50 = tt[len(tt) // 2]
    p99 = tt[min(len(tt) - 1, int(math.ceil(0.99 * len(tt))) - 1)]
    mc, md = sorted(tc)[len(tc) // 2], sorted(td)[len(td) // 2]

    algo_round_trip = 2 * (B_in + S)

    # ---- per-kernel timing over the same K steps (library HIP events)
    with bbx.profile() as prof:
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
    h = np.frombuffer(header, dtype=np.uint8)
    G = [int(h[88 + d]) for d in range(dims)]
    key_bytes = 2 if max(G) <= 16 else 4
    in_pp = dims * x.element_size()
    S_pp = S / n
    dominant = max(prof.items(), key=lambda kv: kv[1][1])
    dname, (dcount, dms) = dominant
    bpp = kernel_bytes_per_particle(dname, key_bytes, in_pp, S_pp, dims)
    avg_ms = dms / dcount
    dominant_kernel = None
    if bpp is not None:
        per_launch = bpp * n
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        dominant_kernel = {"kernel": dname, "achieved": round(achieved, 1), "unit": "GB/s",
                           "frac": round(achieved / HBM_PEAK_GBS, 4), "avg_ms": round(avg_ms, 4),
                           "launches_per_step": dcount / args.steps,
                           "alg_bytes_per_launch": int(per_launch)}
    # the path's roofline: the round trip's algorithmic bytes (compress reads
    # the input and writes the stream, decompress reads the stream and writes
    # the input) over the HIP-event time of compress + decompress
    rt_ms = sum(a + b for a, b in zip(tc, td)) / len(tc)
    rt_achieved = algo_round_trip / (rt_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload) if args.leaf_size == 32 and args.ref_mode == 0 \
        and args.ref_rule == 0 and args.tile == 0 and not args.reduce and not args.split_rule \
        and not args.level_pairs else None
    roofline = {"bound": "hbm", "achieved": round(rt_achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(rt_achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "alg_bytes_per_step": int(algo_round_trip),
                "avg_ms": round(rt_ms, 4),
                "traffic_over_alg": (round(traffic / algo_round_trip, 3) if traffic else None),
                "dominant_kernel": dominant_kernel}
    kernels = {k: {"launches": c, "ms_per_step": round(ms / args.steps, 4)}
               for k, (c, ms) in sorted(prof.items(), key=lambda kv: -kv[1][1])}

    # ---- the Sec. 4.2 sequence layout of a lossless-reference stream
    export = None
    if args.ref_mode == 1:
        exp = bbx.SequenceExporter(header)
        for _ in range(args.warmup):
            exp.launch(stream_buf[:S])
        ee = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        for e0, e1 in ee:
            e0.record(st)
            exp.launch(stream_buf[:S])
            e1.record(st)
        torch.cuda.synchronize()
        te = sorted(a.elapsed_time(b) for a, b in ee)[len(ee) // 2]
        export = {"bytes": exp.size, "cr": round(B_in / exp.size, 4), "ms": round(te, 4),
                  "gbps_of_input": round(B_in / (te * 1e-3) / 1e9, 2)}
        del exp

    # ---- error bound on the measured output (sampled slots)
    perm_check = None
    try:
        pc = bbx.Compressor(n, dims, x.dtype, leaf_size=args.leaf_size, tile=args.tile,
                            want_perm=True, ref_rule=args.ref_rule, ref_mode=args.ref_mode,
                            reduce=args.reduce, split_rule=args.split_rule)
        s2 = pc(x, xi)
        assert s2.numel() == S
        perm = pc.perm[:n].long()
        idx = torch.randint(0, n, (1 << 20,), device=dev)
        err = (got[idx].double() - x[perm[idx]].double()).abs().max().item()
        perm_check = {"sampled_slots": 1 << 20, "max_abs_err": err, "eb_abs": info["eb_abs"],
                      "within_bound": bool(err <= info["eb_abs"])}
        del pc
    except Exception as e:  # noqa: BLE001
        perm_check = {"error": str(e)}

    # ---- CPU oracle baseline on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import Oracle
        m = min(args.cpu_sample, n)
        sample = np.ascontiguousarray(pts[:m])
        orc = Oracle()
        log(f"cpu oracle on {m} particles")
        t = time.perf_counter()
        if args.reduce or args.split_rule:
            so = orc.compress_split(sample, xi, "rel", args.leaf_size, split_rule=args.split_rule,
                                    ref_rule=args.ref_rule, reduce=args.reduce)
        else:
            so = orc.compress(sample, xi, "rel", args.leaf_size, ref_rule=args.ref_rule,
                              ref_mode=args.ref_mode)
        t1 = time.perf_counter()
        orc.decompress(so)
        t2 = time.perf_counter()
        cpu = {"value": round(sample.nbytes / (t2 - t) / 1e9, 5), "unit": "GB/s", "cores": 1,
               "kind": "oracle",
               "sample": f"first {m} particles of the same shuffled set (a uniform random subset), "
                         f"compress {t1 - t:.2f}s + decompress {t2 - t1:.2f}s, single thread "
                         f"({_cpu_model()})"}

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "dims": dims, "input": dtype, "eb_rel": xi,
                   "leaf_size": args.leaf_size, "ref_rule": args.ref_rule,
                   "ref_mode": args.ref_mode, "scatter_stage": args.scatter_stage,
                   "level_pairs": args.level_pairs,
                   "graph": bool(args.graph),
                   "stream_bytes": S, "cr": round(B_in / S, 4),
                   "cr_other_ref_rule": round(B_in / S_alt, 4),
                   "cr_other_ref_mode": round(B_in / S_alt_mode, 4) if S_alt_mode else None,
                   "reduce": args.reduce, "split_rule": args.split_rule,
                   "n_leaves": info["n_leaves"],
                   "n_seq": int(np.frombuffer(header[120:128], dtype="<u8")[0]),
                   "cr_without_reduce": round(B_in / S_plain, 4),
                   "sequence_export": export,
                   "bpp": round(8 * S / n, 4),
                   "compress_gbps": round(B_in / (mc * 1e-3) / 1e9, 2),
                   "decompress_gbps": round(B_in / (md * 1e-3) / 1e9, 2),
                   "p50_ms": round(p50, 4), "p99_ms": round(p99, 4),
                   "p50_us": round(p50 * 1e3, 1), "p99_us": round(p99 * 1e3, 1),
                   "round_trip_hbm_frac": roofline["frac"],
                   "wall_clock_hbm_frac": round(algo_round_trip / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "latency_runs": len(tt),
                   "bound_check": perm_check, "kernels": kernels},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
