"""bitbox: MI355X (gfx950) bit-box particle compressor.

Thin Python binding of the C ABI declared in include/bitbox.h (arXiv
2404.02826: quantize -> k-d median partition -> per-leaf bit box -> offsets
-> bit packing, and unpack -> dequantize).  Every step runs in the HIP
library; this module only marshals arguments.  PyTorch supplies device
memory and the current HIP stream.  There is no CPU fallback: if the built
library is missing, every call raises.
"""
from __future__ import annotations

from ._binding import (  # noqa: F401
    Arena,
    BatchCompressor,
    BitboxError,
    Compressor,
    Decompressor,
    STATUS,
    SequenceExporter,
    Server,
    compress,
    compress_bound,
    compress_static,
    compress_static_limit,
    compress_workspace_size,
    decompress,
    decompress_workspace_size,
    export_sequences,
    export_sequences_reordered,
    huffman_decode,
    huffman_encode,
    lib_path,
    load,
    plan_check,
    profile,
    stream_info,
)
