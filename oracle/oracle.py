"""ctypes wrapper of the C oracle (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
this module.  It never touches the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

STATUS = {0: "OK", 1: "EINVAL", 2: "ENOSPC", 3: "ECORRUPT", 4: "EBOUND", 5: "EUNSUPPORTED",
          6: "EHIP", 7: "ENOMEM"}


class OracleError(RuntimeError):
    def __init__(self, status: int):
        self.status = status
        self.name = STATUS.get(status, f"status {status}")
        super().__init__(self.name)


def _dt(arr: np.ndarray) -> int:
    if arr.dtype == np.float32:
        return 0
    if arr.dtype == np.float64:
        return 1
    raise TypeError("positions must be float32 or float64")


class Oracle:
    """Loads libbbx_oracle.so (building it first if nothing is built)."""

    def __init__(self, path: str | None = None):
        path = path or _build.LIB
        if not os.path.exists(path):
            _build.build_oracle(path)
        self.path = path
        lib = C.CDLL(path)
        u64, u32, i32, dbl, vp = C.c_uint64, C.c_uint32, C.c_int, C.c_double, C.c_void_p
        lib.bbxo_compress_bound.restype = u64
        lib.bbxo_compress_bound.argtypes = [u64, u32, i32]
        lib.bbxo_compress.restype = i32
        lib.bbxo_compress.argtypes = [vp, u64, u32, i32, i32, dbl, i32, u32, vp, u64,
                                      C.POINTER(u64), vp]
        lib.bbxo_decompress.restype = i32
        lib.bbxo_decompress.argtypes = [vp, u64, vp, u64, i32]
        lib.bbxo_stages.restype = i32
        lib.bbxo_stages.argtypes = [vp, u64, u32, i32, i32, dbl, i32, u32, vp, vp, u64, vp, vp,
                                    vp, vp, vp, vp]
        lib.bbxo_compress_ex.restype = i32
        lib.bbxo_compress_ex.argtypes = [vp, u64, u32, i32, i32, dbl, i32, u32, i32, i32, vp,
                                         u64, C.POINTER(u64), vp]
        lib.bbxo_compress_bound_mode.restype = u64
        lib.bbxo_compress_bound_mode.argtypes = [u64, u32, i32, i32]
        lib.bbxo_stages_ex.restype = i32
        lib.bbxo_stages_ex.argtypes = [vp, u64, u32, i32, i32, dbl, i32, u32, i32, vp, vp, u64,
                                       vp, vp, vp, vp, vp, vp]
        lib.bbxo_export_sequences.restype = i32
        lib.bbxo_export_sequences.argtypes = [vp, u64, vp, u64, C.POINTER(u64)]
        lib.bbxo_export_sequences_reordered.restype = i32
        lib.bbxo_export_sequences_reordered.argtypes = [vp, u64, vp, u64, C.POINTER(u64), vp]
        lib.bbxo_leaf_count.restype = u64
        lib.bbxo_leaf_count.argtypes = [u64, u32]
        lib.bbxo_bits_for_offset.restype = u32
        lib.bbxo_bits_for_offset.argtypes = [u64]
        lib.bbxo_compress_reduced.restype = i32
        lib.bbxo_compress_reduced.argtypes = [vp, u64, u32, i32, i32, dbl, i32, u32, i32, vp, u64,
                                              C.POINTER(u64), vp]
        lib.bbxo_compress_split.restype = i32
        lib.bbxo_compress_split.argtypes = [vp, u64, u32, i32, i32, dbl, i32, u32, i32, i32, i32,
                                            vp, u64, C.POINTER(u64), vp]
        lib.bbxo_huffman_lengths.restype = None
        lib.bbxo_huffman_lengths.argtypes = [vp, vp]
        lib.bbxo_huffman_bound.restype = u64
        lib.bbxo_huffman_bound.argtypes = [u64]
        lib.bbxo_huffman_encode.restype = i32
        lib.bbxo_huffman_encode.argtypes = [vp, u64, vp, u64, C.POINTER(u64)]
        lib.bbxo_huffman_decode.restype = i32
        lib.bbxo_huffman_decode.argtypes = [vp, u64, vp, u64, C.POINTER(u64)]
        lib.bbxo_axis_order_by_entropy.restype = None
        lib.bbxo_axis_order_by_entropy.argtypes = [vp, u64, u32, vp]
        lib.bbxo_r_index.restype = u64
        lib.bbxo_r_index.argtypes = [vp, vp, u32, vp, C.POINTER(u64)]
        self.lib = lib

    # -- helpers ---------------------------------------------------------
    @staticmethod
    def _shape(pos: np.ndarray, layout: str):
        if pos.ndim != 2:
            raise ValueError("positions must be 2-D")
        if layout == "aos":
            return pos.shape[0], pos.shape[1], 0
        if layout == "soa":
            return pos.shape[1], pos.shape[0], 1
        raise ValueError(layout)

    def compress_bound(self, n: int, dims: int, dtype, ref_mode: int = 0) -> int:
        dt = 0 if np.dtype(dtype) == np.float32 else 1
        if ref_mode:
            return int(self.lib.bbxo_compress_bound_mode(n, dims, dt, int(ref_mode)))
        return int(self.lib.bbxo_compress_bound(n, dims, dt))

    def leaf_count(self, n: int, r: int) -> int:
        return int(self.lib.bbxo_leaf_count(n, r))

    def bits_for_offset(self, D: int) -> int:
        return int(self.lib.bbxo_bits_for_offset(D))

    def axis_order_by_entropy(self, widths) -> list:
        """Axes in ascending entropy of their width distributions (Sec. 4.2);
        widths is [nseq][dims]."""
        w = np.ascontiguousarray(np.asarray(widths, dtype=np.uint32))
        dims = int(w.shape[1])
        order = np.zeros(3, dtype=np.uint32)
        self.lib.bbxo_axis_order_by_entropy(w.ctypes.data if w.size else None, int(w.shape[0]),
                                            dims, order.ctypes.data)
        return [int(v) for v in order[:dims]]

    def r_index(self, codes, widths, order) -> int:
        """R-index of one member (Sec. 4.2): its codes concatenated in the
        given axis order, first axis most significant."""
        dims = len(codes)
        u = np.zeros(3, dtype=np.uint64)
        m = np.zeros(3, dtype=np.uint32)
        o = np.zeros(3, dtype=np.uint32)
        u[:dims], m[:dims], o[:dims] = codes, widths, order
        hi = C.c_uint64(0)
        lo = self.lib.bbxo_r_index(u.ctypes.data, m.ctypes.data, dims, o.ctypes.data, C.byref(hi))
        return (int(hi.value) << 64) | int(lo)

    # -- API ---------------------------------------------------------------
    def compress(self, pos: np.ndarray, eb: float, eb_mode: str = "rel", r: int = 32,
                 layout: str = "aos", want_perm: bool = False, out_cap: int | None = None,
                 ref_rule: int = 0, ref_mode: int = 0):
        pos = np.ascontiguousarray(pos)
        n, dims, lay = self._shape(pos, layout)
        dt = _dt(pos)
        cap = self.compress_bound(n, dims, pos.dtype, ref_mode) if out_cap is None else out_cap
        out = np.zeros(max(cap, 1), dtype=np.uint8)
        size = C.c_uint64(0)
        perm = np.zeros(max(n, 1), dtype=np.uint32) if want_perm else None
        st = self.lib.bbxo_compress_ex(pos.ctypes.data, n, dims, dt, lay, float(eb),
                                       0 if eb_mode == "rel" else 1, r, int(ref_rule),
                                       int(ref_mode), out.ctypes.data, cap, C.byref(size),
                                       None if perm is None else perm.ctypes.data)
        if st:
            raise OracleError(st)
        stream = out[: size.value].tobytes()
        if want_perm:
            return stream, perm[:n].copy()
        return stream

    def compress_split(self, pos: np.ndarray, eb: float, eb_mode: str = "rel", r: int = 32,
                       layout: str = "aos", split_rule: int = 0, ref_rule: int = 0,
                       reduce: int = 0, want_perm: bool = False):
        """The partition with split rule 0 (median, axes in turn), 1 (widest
        axis), 2 (ceil(n/r) proportional leaves) or 3 (midpoint cells), then
        bit boxes and, with reduce 1 or 2, the reduction of Sec. 4.1.  Rule 0
        without the reduction gives the version-1 stream, anything else
        version 2 (one record per sequence)."""
        pos = np.ascontiguousarray(pos)
        n, dims, lay = self._shape(pos, layout)
        mbits = 5 if pos.dtype == np.float32 else 6
        # version 2 at worst: a record per particle (widths, 30-bit codes,
        # count), or the lossless stream
        v2 = 128 + 8 * ((n * (dims * (mbits + 30 + 31) + 32) + 63) // 64)
        cap = max(self.compress_bound(n, dims, pos.dtype), v2) + 16
        out = np.zeros(max(cap, 1), dtype=np.uint8)
        size = C.c_uint64(0)
        perm = np.zeros(max(n, 1), dtype=np.uint32)
        st = self.lib.bbxo_compress_split(pos.ctypes.data, n, dims, _dt(pos), lay, float(eb),
                                          0 if eb_mode == "rel" else 1, r, int(split_rule),
                                          int(ref_rule), int(reduce), out.ctypes.data, cap,
                                          C.byref(size), perm.ctypes.data)
        if st:
            raise OracleError(st)
        stream = out[: size.value].tobytes()
        return (stream, perm[:n].copy()) if want_perm else stream

    def huffman_lengths(self, counts) -> list:
        c = np.ascontiguousarray(np.asarray(counts, dtype=np.uint64).reshape(256))
        out = np.zeros(256, dtype=np.uint32)
        self.lib.bbxo_huffman_lengths(c.ctypes.data, out.ctypes.data)
        return out.tolist()

    def huffman_encode(self, data: bytes) -> bytes:
        """Huffman coding of bytes (canonical codes, 12-bit limit, chunks of
        16,384 bytes)."""
        a = np.frombuffer(bytes(data), dtype=np.uint8)
        n = len(a)
        cap = int(self.lib.bbxo_huffman_bound(n))
        out = np.zeros(max(cap, 1), dtype=np.uint8)
        size = C.c_uint64(0)
        st = self.lib.bbxo_huffman_encode(a.ctypes.data if n else None, n, out.ctypes.data, cap,
                                          C.byref(size))
        if st:
            raise OracleError(st)
        return out[: size.value].tobytes()

    def huffman_decode(self, stream: bytes) -> bytes:
        b = np.frombuffer(bytes(stream), dtype=np.uint8)
        n = C.c_uint64(0)
        st = self.lib.bbxo_huffman_decode(b.ctypes.data, len(b), None, 0, C.byref(n))
        if st not in (0, 2):
            raise OracleError(st)
        out = np.zeros(max(n.value, 1), dtype=np.uint8)
        st = self.lib.bbxo_huffman_decode(b.ctypes.data, len(b), out.ctypes.data, n.value,
                                          C.byref(n))
        if st:
            raise OracleError(st)
        return out[: n.value].tobytes()

    def compress_reduced(self, pos: np.ndarray, eb: float, eb_mode: str = "rel", r: int = 32,
                         layout: str = "aos", key_rule: int = 0, want_perm: bool = False):
        """Partition, bit boxes, then the bit box reduction of Sec. 4.1
        (version-2 stream: one record per sequence)."""
        pos = np.ascontiguousarray(pos)
        n, dims, lay = self._shape(pos, layout)
        cap = self.compress_bound(n, dims, pos.dtype) + 4 * n + 16
        out = np.zeros(max(cap, 1), dtype=np.uint8)
        size = C.c_uint64(0)
        perm = np.zeros(max(n, 1), dtype=np.uint32)
        st = self.lib.bbxo_compress_reduced(pos.ctypes.data, n, dims, _dt(pos), lay, float(eb),
                                            0 if eb_mode == "rel" else 1, r, int(key_rule),
                                            out.ctypes.data, cap, C.byref(size), perm.ctypes.data)
        if st:
            raise OracleError(st)
        stream = out[: size.value].tobytes()
        return (stream, perm[:n].copy()) if want_perm else stream

    def decompress(self, stream: bytes, layout: str = "aos", pos_cap_bytes: int | None = None):
        buf = np.frombuffer(stream, dtype=np.uint8) if len(stream) else np.zeros(1, np.uint8)
        if len(stream) >= 16:
            n = int.from_bytes(stream[8:16], "little")
            dims = stream[7] if stream[7] in (2, 3) else 3
            dt = np.float64 if stream[6] == 1 else np.float32
        else:
            n, dims, dt = 0, 3, np.float32
        nalloc = max(n, 0) if n < (1 << 31) else 0
        out = np.zeros((nalloc, dims) if layout == "aos" else (dims, nalloc), dtype=dt)
        cap = out.nbytes if pos_cap_bytes is None else pos_cap_bytes
        st = self.lib.bbxo_decompress(buf.ctypes.data, len(stream), out.ctypes.data if out.size else None,
                                      cap, 0 if layout == "aos" else 1)
        if st:
            raise OracleError(st)
        return out

    def export_sequences(self, stream: bytes) -> bytes:
        """The Sec. 4.2 sequence layout of a ref_mode 1 stream."""
        buf = np.frombuffer(stream, dtype=np.uint8) if len(stream) else np.zeros(1, np.uint8)
        size = C.c_uint64(0)
        st = self.lib.bbxo_export_sequences(buf.ctypes.data, len(stream), None, 0, C.byref(size))
        if st not in (0, 2):  # ENOSPC: the size query
            raise OracleError(st)
        out = np.zeros(max(size.value, 8), dtype=np.uint8)
        st = self.lib.bbxo_export_sequences(buf.ctypes.data, len(stream), out.ctypes.data,
                                            out.nbytes, C.byref(size))
        if st:
            raise OracleError(st)
        return out[: size.value].tobytes()

    def export_sequences_reordered(self, stream: bytes):
        """(layout, axis order) after the two reorderings of Sec. 4.2."""
        buf = np.frombuffer(stream, dtype=np.uint8) if len(stream) else np.zeros(1, np.uint8)
        size = C.c_uint64(0)
        order = np.zeros(3, dtype=np.uint32)
        st = self.lib.bbxo_export_sequences_reordered(buf.ctypes.data, len(stream), None, 0,
                                                      C.byref(size), order.ctypes.data)
        if st not in (0, 2):
            raise OracleError(st)
        out = np.zeros(max(size.value, 8), dtype=np.uint8)
        st = self.lib.bbxo_export_sequences_reordered(buf.ctypes.data, len(stream), out.ctypes.data,
                                                      out.nbytes, C.byref(size), order.ctypes.data)
        if st:
            raise OracleError(st)
        return out[: size.value].tobytes(), [int(v) for v in order[: stream[7]]]

    def stages(self, pos: np.ndarray, eb: float, eb_mode: str = "rel", r: int = 32,
               layout: str = "aos", ref_rule: int = 0) -> dict:
        pos = np.ascontiguousarray(pos)
        n, dims, lay = self._shape(pos, layout)
        nl = self.leaf_count(n, r)
        q = np.zeros((dims, max(n, 1)), dtype=np.uint32)
        order = np.zeros(max(n, 1), dtype=np.uint32)
        ls = np.zeros(max(nl, 1), dtype=np.uint32)
        lz = np.zeros(max(nl, 1), dtype=np.uint32)
        lr = np.zeros(max(nl, 1), dtype=np.uint32)
        lm = np.zeros((max(nl, 1), 3), dtype=np.uint8)
        lb = np.zeros(max(nl, 1), dtype=np.uint64)
        sc = np.zeros(16, dtype=np.float64)
        st = self.lib.bbxo_stages_ex(pos.ctypes.data, n, dims, _dt(pos), lay, float(eb),
                                     0 if eb_mode == "rel" else 1, r, int(ref_rule),
                                     q.ctypes.data, order.ctypes.data, nl, ls.ctypes.data,
                                     lz.ctypes.data, lr.ctypes.data, lm.ctypes.data,
                                     lb.ctypes.data, sc.ctypes.data)
        if st:
            raise OracleError(st)
        return {
            "q": q[:, :n], "order": order[:n], "leaf_start": ls[:nl], "leaf_size": lz[:nl],
            "leaf_ref": lr[:nl], "leaf_m": lm[:nl, :dims], "leaf_bits": lb[:nl],
            "eb_abs": sc[0], "eb_eff": sc[1], "w": sc[2], "inv_w": sc[3],
            "lo": sc[4:4 + dims].copy(), "hi": sc[7:7 + dims].copy(),
            "G": sc[10:10 + dims].astype(int), "n_leaves": int(sc[13]),
            "meta_bits": int(sc[14]), "payload_bits": int(sc[15]),
        }


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
