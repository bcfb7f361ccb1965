"""Writes fullsize_digests.json: SHA-256 digests of the oracle's stream, its
decode and its perm (source index per output slot) for the benchmark-sized
workloads.  Calls only oracle/ and synth/ (run on a CPU host; the largest set
takes a few minutes and about 10 GB of memory):

    python tests/golden/make_fullsize_digests.py

The GPU tests compare the library's outputs at the same sizes with these.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import Oracle  # noqa: E402
from synth import cosmology, fluid, fluid_lattice_dims  # noqa: E402

# name: (generator, n, dtype, relative bound, leaf size); the generators and
# seeds are those of the benchmark's workloads
CASES = {
    "fluid-2^27-f32": ("fluid", 1 << 27, np.float32, 1e-4, 32),
    "fluid-2^26-f64": ("fluid", 1 << 26, np.float64, 1e-4, 32),
    "cosmology-2^24-f32-xi1e-4": ("cosmology", 1 << 24, np.float32, 1e-4, 32),
    "cosmology-2^24-f32-xi1e-3": ("cosmology", 1 << 24, np.float32, 1e-3, 32),
}


def points(kind, n, dt):
    if kind == "fluid":
        return fluid(*fluid_lattice_dims(n), seed=4, dtype=dt)
    return cosmology(n, seed=2, dtype=dt)


def sha(b) -> str:
    return hashlib.sha256(b).hexdigest()


def main(names):
    path = os.path.join(HERE, "fullsize_digests.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    orc = Oracle()
    for name in names:
        kind, n, dt, xi, r = CASES[name]
        t = time.time()
        pts = points(kind, n, dt)
        s, perm = orc.compress(pts, xi, "rel", r, want_perm=True)
        dec = orc.decompress(s)
        out[name] = {"n": n, "dtype": np.dtype(dt).name, "eb_rel": xi, "leaf_size": r,
                     "input_sha256": sha(pts.tobytes()), "stream_bytes": len(s),
                     "stream_sha256": sha(s), "decode_sha256": sha(dec.tobytes()),
                     "perm_sha256": sha(perm.astype(np.uint32).tobytes())}
        print(f"{name}: {len(s)} bytes in {time.time() - t:.0f} s", flush=True)
        del pts, s, perm, dec
        json.dump(out, open(path, "w"), indent=2, sort_keys=True)
        open(path, "a").write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
