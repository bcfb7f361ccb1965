"""Fixed-seed generator outputs match the recorded SHA-256 manifest."""
import json
import os
import sys

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))

import make_manifest  # noqa: E402


def test_manifest():
    with open(os.path.join(os.path.dirname(make_manifest.__file__), "synth_manifest.json")) as f:
        want = json.load(f)
    assert make_manifest.compute() == want
