"""The C-ABI library loads and exports every symbol include/bitbox.h declares
(no GPU calls), and the host-only entry points behave."""
from __future__ import annotations

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("bitbox.h", "bitbox_serve.h")]


def _declared():
    names = set()
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(bbx_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    import paper_2404_02826_amd as bbx
    if not os.path.exists(bbx.lib_path()):
        from paper_2404_02826_amd import build
        build.build()
    return bbx.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "bbx_compress" in names and "bbx_decompress" in names
    assert "bbx_compress_batch" in names and "bbx_server_progress" in names
    for nm in names:
        assert hasattr(lib, nm), f"{nm} declared in include/ but not exported"


def test_status_strings(lib):
    assert lib.bbx_status_str(0) == b"OK"
    assert lib.bbx_status_str(3) == b"ECORRUPT"


def test_compress_bound_matches_oracle(lib, oracle):
    import numpy as np
    for n in (0, 1, 7, 1000, 65536, 1 << 27):
        for dims in (2, 3):
            for dt, code in ((np.float32, 0), (np.float64, 1)):
                assert lib.bbx_compress_bound(n, dims, code) == oracle.compress_bound(n, dims, dt)


def test_argument_errors_on_host(lib):
    import paper_2404_02826_amd as bbx
    with pytest.raises(bbx.BitboxError):
        bbx.compress_workspace_size(100, dims=4)
    with pytest.raises(bbx.BitboxError):
        bbx.compress_workspace_size(100, leaf_size=0)
    with pytest.raises(bbx.BitboxError, match="scatter_stage"):
        bbx.compress_workspace_size(100, scatter_stage=3)
    assert bbx.compress_workspace_size(100) > 0
    for stage in (0, 1, 2):  # a tuning choice: the workspace does not depend on it
        assert bbx.compress_workspace_size(100000, scatter_stage=stage) == bbx.compress_workspace_size(100000)


def test_stream_info_parses_oracle_header(lib, oracle):
    import numpy as np
    import paper_2404_02826_amd as bbx
    from synth import cosmology
    pts = cosmology(5000, seed=3)
    s = oracle.compress(pts, 1e-3, "rel", 32)
    info = bbx.stream_info(s[:128])
    assert info["n"] == 5000 and info["dims"] == 3 and info["leaf_size"] == 32
    assert info["n_leaves"] == oracle.leaf_count(5000, 32)
    assert info["stream_bytes"] == len(s)
    bad = bytearray(s[:128])
    bad[0] ^= 1
    with pytest.raises(bbx.BitboxError) as e:
        bbx.stream_info(bytes(bad))
    assert e.value.name == "ECORRUPT"
    bad = bytearray(s[:128])
    bad[96] ^= 1  # leaf count no longer matches (n, r)
    with pytest.raises(bbx.BitboxError):
        bbx.stream_info(bytes(bad))
    assert np.isclose(info["eb_abs"], 1e-3 * (pts.max(0) - pts.min(0)).max())
