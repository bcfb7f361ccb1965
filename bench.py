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
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_points(kind, n, dtype):
    import numpy as np
    from synth import cosmology, fluid, fluid_lattice_dims, uniform_cube
    dt = np.float32 if dtype == "float32" else np.float64
    if kind == "fluid":
        return fluid(*fluid_lattice_dims(n), seed=4, dtype=dt)
    if kind == "cosmology":
        return cosmology(n, seed=2, dtype=dt)
    return uniform_cube(n, seed=1, dtype=dt)


# Algorithmic bytes per particle of each kernel (u16 codes, 3-D, no perm):
# what the kernel must read and write, not what it happens to move.
def kernel_bytes_per_particle(name, key_bytes, in_bytes, stream_bytes_pp):
    kb = 3 * key_bytes
    return {
        "range_minmax": in_bytes,
        "quantize": in_bytes + kb,
        "level_hist_mid": key_bytes,
        "level_hist_last": key_bytes,
        "level_scatter": 2 * kb,
        "tile": 2 * kb,
        "pack_payload": kb + stream_bytes_pp,
        "unpack": stream_bytes_pp + in_bytes,
    }.get(name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="fluid-2^27-f32", choices=sorted(WORKLOADS))
    ap.add_argument("--leaf-size", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 22)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

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

    comp = bbx.Compressor(n, 3, x.dtype, leaf_size=args.leaf_size)
    s = comp(x, xi)
    S = s.numel()
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
    got = dec(stream_buf[:S])
    torch.cuda.synchronize()
    log("warmup done")

    # ---- timed region: exactly K steps
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    value = B_in * args.steps / elapsed / 1e9
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {value:.1f} GB/s")

    # ---- per-phase timing and latency distribution (HIP events, same stream)
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
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
    p50 = tt[len(tt) // 2]
    p99 = tt[min(len(tt) - 1, int(math.ceil(0.99 * len(tt))) - 1)]
    mc, md = sorted(tc)[len(tc) // 2], sorted(td)[len(td) // 2]

    # ---- per-kernel timing over the same K steps (library HIP events)
    with bbx.profile() as prof:
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
    h = np.frombuffer(header, dtype=np.uint8)
    G = [int(h[88 + d]) for d in range(3)]
    key_bytes = 2 if max(G) <= 16 else 4
    in_pp = 3 * x.element_size()
    S_pp = S / n
    dominant = max(prof.items(), key=lambda kv: kv[1][1])
    dname, (dcount, dms) = dominant
    bpp = kernel_bytes_per_particle(dname, key_bytes, in_pp, S_pp)
    avg_ms = dms / dcount
    roofline = None
    if bpp is not None:
        per_launch = bpp * n
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "kernel": dname, "avg_ms": round(avg_ms, 4),
                    "launches_per_step": dcount / args.steps,
                    "alg_bytes_per_launch": int(per_launch)}
    kernels = {k: {"launches": c, "ms_per_step": round(ms / args.steps, 4)}
               for k, (c, ms) in sorted(prof.items(), key=lambda kv: -kv[1][1])}

    # ---- error bound on the measured output (sampled slots)
    perm_check = None
    try:
        pc = bbx.Compressor(n, 3, x.dtype, leaf_size=args.leaf_size, want_perm=True)
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
        so = orc.compress(sample, xi, "rel", args.leaf_size)
        t1 = time.perf_counter()
        orc.decompress(so)
        t2 = time.perf_counter()
        cpu = {"value": round(sample.nbytes / (t2 - t) / 1e9, 5), "unit": "GB/s", "cores": 1,
               "kind": "oracle",
               "sample": f"first {m} particles of the same shuffled set (a uniform random subset), "
                         f"compress {t1 - t:.2f}s + decompress {t2 - t1:.2f}s, single thread"}

    algo_round_trip = 2 * (B_in + S)
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "input": dtype, "eb_rel": xi,
                   "leaf_size": args.leaf_size, "stream_bytes": S, "cr": round(B_in / S, 4),
                   "bpp": round(8 * S / n, 4),
                   "compress_gbps": round(B_in / (mc * 1e-3) / 1e9, 2),
                   "decompress_gbps": round(B_in / (md * 1e-3) / 1e9, 2),
                   "p50_ms": round(p50, 4), "p99_ms": round(p99, 4),
                   "round_trip_hbm_frac": round(algo_round_trip / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "bound_check": perm_check, "kernels": kernels},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
