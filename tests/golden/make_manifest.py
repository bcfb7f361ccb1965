"""Writes synth_manifest.json: SHA-256 of small fixed-seed generator outputs.

The manifest guards against drift of numpy's PCG64 streams or of the
generator recipes; it records inputs only (no compressor output).
Run: python tests/golden/make_manifest.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from synth import cosmology, fluid, poincare, sha256_of, uniform_cube  # noqa: E402

CASES = {
    "uniform_65536_seed1_f32": lambda: uniform_cube(65536, seed=1),
    "cosmology_65536_seed2_f32": lambda: cosmology(65536, seed=2),
    "cosmology_4096_seed3_f64": lambda: cosmology(4096, seed=3, dtype=np.float64),
    "fluid_32x32x32_seed4_f32": lambda: fluid(32, 32, 32, seed=4),
    "fluid_16x16x8_seed4_f64": lambda: fluid(16, 16, 8, seed=4, dtype=np.float64),
    "poincare_65536_seed8_f32": lambda: poincare(65536, seed=8),
}


def compute():
    return {k: sha256_of(f()) for k, f in CASES.items()}


if __name__ == "__main__":
    with open(os.path.join(HERE, "synth_manifest.json"), "w") as f:
        json.dump(compute(), f, indent=1, sort_keys=True)
        f.write("\n")
