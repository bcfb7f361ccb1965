"""ctypes marshalling for libbitbox.so (include/bitbox.h)."""
from __future__ import annotations

import ctypes as C
import os
from contextlib import contextmanager

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "lib", "libbitbox.so")
_lib = None

STATUS = {0: "OK", 1: "EINVAL", 2: "ENOSPC", 3: "ECORRUPT", 4: "EBOUND", 5: "EUNSUPPORTED",
          6: "EHIP", 7: "ENOMEM"}

F32, F64 = 0, 1
REL, ABS = 0, 1
AOS, SOA = 0, 1


class BitboxError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        self.status = status
        self.name = STATUS.get(status, f"status {status}")
        super().__init__(f"{self.name}: {msg}" if msg else self.name)


class _Params(C.Structure):
    _fields_ = [("leaf_size", C.c_uint32), ("eb_mode", C.c_uint32), ("layout", C.c_uint32),
                ("tile_override", C.c_uint32), ("ref_rule", C.c_uint32), ("ref_mode", C.c_uint32),
                ("scatter_stage", C.c_uint32), ("level_blocks", C.c_uint32),
                ("reduce", C.c_uint32), ("split_rule", C.c_uint32), ("level_pairs", C.c_uint32)]


class _Set(C.Structure):
    _fields_ = [("d_pos", C.c_void_p), ("n", C.c_uint64), ("dims", C.c_uint32),
                ("dtype", C.c_uint32), ("eb", C.c_double), ("params", _Params),
                ("d_out", C.c_void_p), ("out_cap", C.c_size_t), ("d_size", C.c_void_p),
                ("d_status", C.c_void_p), ("d_perm", C.c_void_p)]


class _ServerConfig(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_jobs", C.c_uint32), ("max_batch", C.c_uint32),
                ("nstreams", C.c_uint32), ("tile_override", C.c_uint32)]


class _JobInfo(C.Structure):
    _fields_ = [("state", C.c_uint32), ("status", C.c_uint32), ("bytes", C.c_uint64),
                ("d_result", C.c_void_p), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_launch", C.c_double), ("t_done", C.c_double), ("batch_jobs", C.c_uint32),
                ("kind", C.c_uint32)]


def lib_path() -> str:
    return _LIB_PATH


def load():
    """Loads the built HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built (run __graft_entry__.build())")
    lib = C.CDLL(_LIB_PATH)
    u64, u32, i32, dbl, vp, sz = C.c_uint64, C.c_uint32, C.c_int, C.c_double, C.c_void_p, C.c_size_t
    lib.bbx_compress_bound.restype = sz
    lib.bbx_compress_bound.argtypes = [u64, u32, i32]
    lib.bbx_compress_bound_mode.restype = sz
    lib.bbx_compress_bound_mode.argtypes = [u64, u32, i32, u32]
    lib.bbx_compress_bound_params.restype = sz
    lib.bbx_compress_bound_params.argtypes = [u64, u32, i32, C.POINTER(_Params)]
    lib.bbx_compress_workspace_size.restype = sz
    lib.bbx_compress_workspace_size.argtypes = [u64, u32, i32, C.POINTER(_Params)]
    lib.bbx_compress.restype = i32
    lib.bbx_compress.argtypes = [vp, u64, u32, i32, dbl, C.POINTER(_Params), vp, sz,
                                 C.POINTER(sz), vp, vp, vp, vp, sz, vp]
    lib.bbx_batch_workspace_size.restype = sz
    lib.bbx_batch_workspace_size.argtypes = [C.POINTER(_Set), u32]
    lib.bbx_compress_static_limit.restype = sz
    lib.bbx_compress_static_limit.argtypes = []
    lib.bbx_compress_static.restype = i32
    lib.bbx_compress_static.argtypes = [vp, u64, u32, i32, dbl, C.POINTER(_Params), vp, sz,
                                        C.POINTER(sz), vp, vp, vp, vp]
    lib.bbx_plan_check.restype = i32
    lib.bbx_plan_check.argtypes = [C.POINTER(_Set), u32]
    for nm in ("bbx_batch_upload", "bbx_batch_launch", "bbx_compress_batch"):
        f = getattr(lib, nm)
        f.restype = i32
        f.argtypes = [C.POINTER(_Set), u32, vp, sz, vp]
    vpp = C.POINTER(C.c_void_p)
    lib.bbx_arena_create.restype = i32
    lib.bbx_arena_create.argtypes = [sz, sz, vpp]
    lib.bbx_arena_destroy.restype = None
    lib.bbx_arena_destroy.argtypes = [vp]
    lib.bbx_arena_alloc.restype = i32
    lib.bbx_arena_alloc.argtypes = [vp, sz, C.POINTER(sz)]
    lib.bbx_arena_free.restype = i32
    lib.bbx_arena_free.argtypes = [vp, sz]
    lib.bbx_arena_stats.restype = None
    lib.bbx_arena_stats.argtypes = [vp] + [C.POINTER(sz)] * 4
    lib.bbx_server_create.restype = i32
    lib.bbx_server_create.argtypes = [C.POINTER(_ServerConfig), vp, sz, vpp]
    lib.bbx_server_destroy.restype = i32
    lib.bbx_server_destroy.argtypes = [vp]
    lib.bbx_server_submit_compress.restype = i32
    lib.bbx_server_submit_compress.argtypes = [vp, vp, u64, u32, i32, dbl, C.POINTER(_Params),
                                               C.POINTER(u64)]
    lib.bbx_server_submit_decompress.restype = i32
    lib.bbx_server_submit_decompress.argtypes = [vp, vp, sz, vp, i32, C.POINTER(u64)]
    lib.bbx_server_progress.restype = i32
    lib.bbx_server_progress.argtypes = [vp, C.POINTER(u32)]
    lib.bbx_server_pop_done.restype = u64
    lib.bbx_server_pop_done.argtypes = [vp]
    lib.bbx_server_job_info.restype = i32
    lib.bbx_server_job_info.argtypes = [vp, u64, C.POINTER(_JobInfo)]
    lib.bbx_server_release.restype = i32
    lib.bbx_server_release.argtypes = [vp, u64]
    lib.bbx_server_now.restype = dbl
    lib.bbx_server_now.argtypes = [vp]
    lib.bbx_server_counts.restype = None
    lib.bbx_server_counts.argtypes = [vp] + [C.POINTER(u32)] * 4 + [C.POINTER(u64), C.POINTER(sz)]
    lib.bbx_stream_info.restype = i32
    lib.bbx_stream_info.argtypes = [vp, sz, C.POINTER(u64), C.POINTER(u32), C.POINTER(i32),
                                    C.POINTER(dbl), C.POINTER(u32), C.POINTER(u64), C.POINTER(u64)]
    lib.bbx_decompress_workspace_size.restype = sz
    lib.bbx_decompress_workspace_size.argtypes = [vp, sz]
    lib.bbx_decompress.restype = i32
    lib.bbx_decompress.argtypes = [vp, sz, vp, vp, sz, i32, vp, vp, sz, vp]
    lib.bbx_export_reordered_workspace_size.restype = sz
    lib.bbx_export_reordered_workspace_size.argtypes = [vp, sz]
    lib.bbx_export_sequences_reordered.restype = i32
    lib.bbx_export_sequences_reordered.argtypes = [vp, sz, vp, vp, sz, vp, vp, sz, vp]
    lib.bbx_huffman_bound.restype = sz
    lib.bbx_huffman_bound.argtypes = [u64]
    lib.bbx_huffman_workspace_size.restype = sz
    lib.bbx_huffman_workspace_size.argtypes = [u64]
    lib.bbx_huffman_encode.restype = i32
    lib.bbx_huffman_encode.argtypes = [vp, u64, vp, sz, C.POINTER(sz), vp, sz, vp]
    lib.bbx_huffman_decode.restype = i32
    lib.bbx_huffman_decode.argtypes = [vp, sz, vp, vp, sz, vp, vp, sz, vp]
    lib.bbx_export_sequences_size.restype = sz
    lib.bbx_export_sequences_size.argtypes = [vp, sz]
    lib.bbx_export_sequences.restype = i32
    lib.bbx_export_sequences.argtypes = [vp, sz, vp, vp, sz, vp, vp, sz, vp]
    lib.bbx_status_str.restype = C.c_char_p
    lib.bbx_status_str.argtypes = [i32]
    lib.bbx_last_error.restype = C.c_char_p
    lib.bbx_last_error.argtypes = []
    lib.bbx_profile_enable.restype = None
    lib.bbx_profile_enable.argtypes = [i32]
    lib.bbx_profile_reset.restype = None
    lib.bbx_profile_reset.argtypes = []
    lib.bbx_profile_count.restype = i32
    lib.bbx_profile_count.argtypes = []
    lib.bbx_profile_get.restype = i32
    lib.bbx_profile_get.argtypes = [i32, C.POINTER(C.c_char_p), C.POINTER(u64), C.POINTER(dbl)]
    _lib = lib
    return lib


def _check(st: int):
    if st != 0:
        raise BitboxError(st, load().bbx_last_error().decode())


def _stream_ptr(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError("positions must be float32 or float64")


def _shape(pos: torch.Tensor, layout: str):
    if pos.dim() != 2:
        raise ValueError("positions must be 2-D: (n, dims) for aos or (dims, n) for soa")
    if layout == "aos":
        return pos.shape[0], pos.shape[1], AOS
    if layout == "soa":
        return pos.shape[1], pos.shape[0], SOA
    raise ValueError(layout)


def _params(leaf_size: int, eb_mode: str, layout: int, tile: int, ref_rule: int = 0,
            ref_mode: int = 0, scatter_stage: int = 0, level_blocks: int = 0,
            reduce: int = 0, split_rule: int = 0, level_pairs: int = 0) -> _Params:
    return _Params(leaf_size, REL if eb_mode == "rel" else ABS, layout, tile, ref_rule, ref_mode,
                   scatter_stage, level_blocks, reduce, split_rule, level_pairs)


def compress_bound_params(n: int, dims: int, dtype, params: _Params) -> int:
    code = F32 if dtype == torch.float32 else F64
    return int(load().bbx_compress_bound_params(n, dims, code, C.byref(params)))


def compress_bound(n: int, dims: int = 3, dtype=torch.float32, ref_mode: int = 0) -> int:
    code = F32 if dtype == torch.float32 else F64
    if ref_mode:
        return int(load().bbx_compress_bound_mode(n, dims, code, ref_mode))
    return int(load().bbx_compress_bound(n, dims, code))


def compress_workspace_size(n: int, dims: int = 3, dtype=torch.float32, leaf_size: int = 32,
                            eb_mode: str = "rel", layout: str = "aos", tile: int = 0,
                            ref_rule: int = 0, ref_mode: int = 0, scatter_stage: int = 0,
                            level_blocks: int = 0, reduce: int = 0, split_rule: int = 0,
                            level_pairs: int = 0) -> int:
    p = _params(leaf_size, eb_mode, AOS if layout == "aos" else SOA, tile, ref_rule, ref_mode,
                scatter_stage, level_blocks, reduce, split_rule, level_pairs)
    code = F32 if dtype == torch.float32 else F64
    lib = load()
    v = int(lib.bbx_compress_workspace_size(n, dims, code, C.byref(p)))
    if v == 0:
        # argument errors are reported before any launch: ask bbx_compress for the status
        st = lib.bbx_compress(None, n, dims, code, 1.0, C.byref(p), None, 0, None, None, None,
                              None, None, 0, None)
        raise BitboxError(st if st else 1, lib.bbx_last_error().decode())
    return v


class Compressor:
    """Reusable compress call: owns the workspace and the output buffer.

    ``__call__`` synchronizes once and returns the stream as a uint8 view of
    the output buffer (valid until the next call); ``launch`` enqueues the
    work without waiting and leaves the size in ``d_size`` (device).
    """

    def __init__(self, n: int, dims: int = 3, dtype=torch.float32, leaf_size: int = 32,
                 eb_mode: str = "rel", layout: str = "aos", tile: int = 0, want_perm: bool = False,
                 device="cuda", ref_rule: int = 0, ref_mode: int = 0, scatter_stage: int = 0,
                 level_blocks: int = 0, reduce: int = 0, split_rule: int = 0,
                 level_pairs: int = 0):
        self.n, self.dims, self.dtype = n, dims, dtype
        self.layout = layout
        self.params = _params(leaf_size, eb_mode, AOS if layout == "aos" else SOA, tile, ref_rule,
                              ref_mode, scatter_stage, level_blocks, reduce, split_rule,
                              level_pairs)
        lib = load()
        self.ws_size = compress_workspace_size(n, dims, dtype, leaf_size, eb_mode, layout, tile,
                                               ref_rule, ref_mode, scatter_stage, level_blocks,
                                               reduce, split_rule, level_pairs)
        self.ws = torch.empty(self.ws_size, dtype=torch.uint8, device=device)
        self.cap = compress_bound_params(n, dims, dtype, self.params)
        self.out = torch.empty((self.cap + 7) // 8 * 8, dtype=torch.uint8, device=device)
        self.perm = torch.empty(max(n, 1), dtype=torch.int32, device=device) if want_perm else None
        self.d_size = torch.zeros(1, dtype=torch.int64, device=device)
        self.d_status = torch.zeros(1, dtype=torch.int32, device=device)
        self._lib = lib

    def _call(self, pos: torch.Tensor, eb: float, h_size, stream):
        n, dims, lay = _shape(pos, self.layout)
        if n != self.n or dims != self.dims or pos.dtype != self.dtype:
            raise ValueError("positions do not match this Compressor's shape/type")
        if not pos.is_cuda or not pos.is_contiguous():
            raise ValueError("positions must be a contiguous device tensor")
        return self._lib.bbx_compress(
            pos.data_ptr() if n else None, n, dims, _dtype_code(pos), float(eb), C.byref(self.params),
            self.out.data_ptr(), self.cap, h_size, self.d_size.data_ptr(), self.d_status.data_ptr(),
            self.perm.data_ptr() if self.perm is not None else None, self.ws.data_ptr(),
            self.ws_size, _stream_ptr(stream))

    def launch(self, pos: torch.Tensor, eb: float, stream=None):
        _check(self._call(pos, eb, None, stream))

    def __call__(self, pos: torch.Tensor, eb: float, stream=None):
        size = C.c_size_t(0)
        _check(self._call(pos, eb, C.byref(size), stream))
        return self.out[: size.value]


class Decompressor:
    """Reusable decompress call for streams of one header shape."""

    def __init__(self, header: bytes, layout: str = "aos", device="cuda"):
        lib = load()
        self.header = bytes(header[:128])
        self.info = stream_info(self.header)
        self.layout = layout
        self.ws_size = int(lib.bbx_decompress_workspace_size(self.header, 128))
        if self.ws_size == 0:
            raise BitboxError(3, lib.bbx_last_error().decode())
        self.ws = torch.empty(self.ws_size, dtype=torch.uint8, device=device)
        n, dims = self.info["n"], self.info["dims"]
        dt = torch.float32 if self.info["dtype"] == F32 else torch.float64
        shape = (n, dims) if layout == "aos" else (dims, n)
        self.pos = torch.empty(shape, dtype=dt, device=device)
        self.d_status = torch.zeros(1, dtype=torch.int32, device=device)
        self._lib = lib

    def _call(self, stream_t: torch.Tensor, d_status, stream):
        return self._lib.bbx_decompress(
            stream_t.data_ptr(), stream_t.numel(), self.header, self.pos.data_ptr(),
            self.pos.numel() * self.pos.element_size(), AOS if self.layout == "aos" else SOA,
            d_status, self.ws.data_ptr(), self.ws_size, _stream_ptr(stream))

    def launch(self, stream_t: torch.Tensor, stream=None):
        _check(self._call(stream_t, self.d_status.data_ptr(), stream))

    def __call__(self, stream_t: torch.Tensor, stream=None):
        _check(self._call(stream_t, None, stream))
        return self.pos


class BatchCompressor:
    """Compresses many independent particle sets with one launch sequence.

    ``sets`` is a list of dicts with keys ``pos`` (contiguous device tensor),
    ``eb`` and optionally ``eb_mode``, ``leaf_size``, ``layout``,
    ``want_perm``, ``out_cap``.  The outputs of all sets live in one device buffer
    (set i at byte ``offsets[i]``, capacity ``caps[i]``); ``d_size`` and
    ``d_status`` hold one entry per set.  ``upload`` copies the descriptors
    into the workspace, ``launch`` enqueues the kernels only (so it can be
    recorded in a HIP graph and replayed while the upload stays valid).
    """

    def __init__(self, sets, tile: int = 0, device="cuda", scatter_stage: int = 0):
        lib = load()
        self._lib = lib
        self.nsets = len(sets)
        self.tile = tile
        arr = (_Set * max(self.nsets, 1))()
        caps, offs, perms, total = [], [], [], 0
        for spec in sets:
            pos = spec["pos"]
            layout = spec.get("layout", "aos")
            n, dims, _ = _shape(pos, layout)
            cap = (compress_bound_params(n, dims, pos.dtype, _params(
                spec.get("leaf_size", 32), "rel", AOS, tile, 0, spec.get("ref_mode", 0), 0, 0,
                spec.get("reduce", 0), spec.get("split_rule", 0))) + 7) // 8 * 8
            if "out_cap" in spec:  # a smaller capacity, reported per set as ENOSPC
                cap = int(spec["out_cap"])
            caps.append(cap)
            offs.append(total)
            total += (cap + 7) // 8 * 8
        self.out = torch.empty(max(total, 8), dtype=torch.uint8, device=device)
        self.d_size = torch.zeros(max(self.nsets, 1), dtype=torch.int64, device=device)
        self.d_status = torch.zeros(max(self.nsets, 1), dtype=torch.int32, device=device)
        self.offsets, self.caps, self.perms, self.inputs = offs, caps, [], []
        base = self.out.data_ptr()
        for i, spec in enumerate(sets):
            pos = spec["pos"]
            layout = spec.get("layout", "aos")
            if not pos.is_cuda or not pos.is_contiguous():
                raise ValueError("positions must be contiguous device tensors")
            n, dims, lay = _shape(pos, layout)
            perm = (torch.empty(max(n, 1), dtype=torch.int32, device=device)
                    if spec.get("want_perm") else None)
            self.perms.append(perm)
            self.inputs.append(pos)
            S = arr[i]
            S.d_pos = pos.data_ptr() if n else None
            S.n, S.dims, S.dtype, S.eb = n, dims, _dtype_code(pos), float(spec["eb"])
            S.params = _params(spec.get("leaf_size", 32), spec.get("eb_mode", "rel"), lay, tile,
                               spec.get("ref_rule", 0), spec.get("ref_mode", 0), scatter_stage,
                               spec.get("level_blocks", 0), spec.get("reduce", 0),
                               spec.get("split_rule", 0), spec.get("level_pairs", 0))
            S.d_out = base + offs[i]
            S.out_cap = caps[i]
            S.d_size = self.d_size.data_ptr() + 8 * i
            S.d_status = self.d_status.data_ptr() + 4 * i
            S.d_perm = perm.data_ptr() if perm is not None else None
        self._arr = arr
        self.ws_size = int(lib.bbx_batch_workspace_size(arr, self.nsets))
        if self.ws_size == 0:
            _check(lib.bbx_batch_upload(arr, self.nsets, None, 0, None) or 1)
        self.ws = torch.empty(self.ws_size, dtype=torch.uint8, device=device)

    def upload(self, stream=None):
        _check(self._lib.bbx_batch_upload(self._arr, self.nsets, self.ws.data_ptr(), self.ws_size,
                                          _stream_ptr(stream)))

    def launch(self, stream=None):
        _check(self._lib.bbx_batch_launch(self._arr, self.nsets, self.ws.data_ptr(), self.ws_size,
                                          _stream_ptr(stream)))

    def results(self):
        """Waits for the stream's work and returns, per set, the stream bytes
        (uint8 device view) or a BitboxError."""
        torch.cuda.synchronize()
        sizes = self.d_size.cpu().tolist()
        stats = self.d_status.cpu().tolist()
        res = []
        for i in range(self.nsets):
            if stats[i] != 0:
                res.append(BitboxError(stats[i], f"set {i}"))
            else:
                res.append(self.out[self.offsets[i]: self.offsets[i] + sizes[i]])
        return res

    def __call__(self, stream=None):
        self.upload(stream)
        self.launch(stream)
        return self.results()


class Arena:
    """Host bookkeeping of the serving runtime's device-memory arena
    (offsets only; no device access)."""

    def __init__(self, size: int, align: int = 256):
        self._lib = load()
        h = C.c_void_p()
        _check(self._lib.bbx_arena_create(size, align, C.byref(h)))
        self._h = h

    def alloc(self, nbytes: int) -> int:
        off = C.c_size_t()
        _check(self._lib.bbx_arena_alloc(self._h, nbytes, C.byref(off)))
        return off.value

    def free(self, off: int):
        _check(self._lib.bbx_arena_free(self._h, off))

    def stats(self) -> dict:
        v = [C.c_size_t() for _ in range(4)]
        self._lib.bbx_arena_stats(self._h, *[C.byref(x) for x in v])
        return dict(used=v[0].value, free_total=v[1].value, largest_free=v[2].value,
                    free_ranges=v[3].value)

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.bbx_arena_destroy(self._h)
            self._h = None


JOB_STATES = {0: "queued", 1: "admitted", 2: "running", 3: "done"}


class Server:
    """Continuous-batching server over one device arena of ``hbm_budget``
    bytes (allocated here once; the runtime sub-allocates inside it).

    Jobs reference caller-owned device inputs, which must stay unchanged
    until the job is done.  ``progress()`` never waits for the GPU.
    """

    def __init__(self, hbm_budget: int, max_jobs: int = 1024, max_batch: int = 256,
                 nstreams: int = 4, tile: int = 0, device="cuda"):
        self._lib = load()
        self.arena = torch.empty(hbm_budget, dtype=torch.uint8, device=device)
        cfg = _ServerConfig(hbm_budget, max_jobs, max_batch, nstreams, tile)
        h = C.c_void_p()
        _check(self._lib.bbx_server_create(C.byref(cfg), self.arena.data_ptr(), hbm_budget,
                                           C.byref(h)))
        self._h = h
        self._meta = {}

    def submit_compress(self, pos: torch.Tensor, eb: float, eb_mode: str = "rel",
                        leaf_size: int = 32, layout: str = "aos", ref_rule: int = 0,
                        ref_mode: int = 0) -> int:
        n, dims, lay = _shape(pos, layout)
        if not pos.is_cuda or not pos.is_contiguous():
            raise ValueError("positions must be a contiguous device tensor")
        prm = _params(leaf_size, eb_mode, lay, 0, ref_rule, ref_mode)
        jid = C.c_uint64()
        _check(self._lib.bbx_server_submit_compress(self._h, pos.data_ptr() if n else None, n, dims,
                                                    _dtype_code(pos), float(eb), C.byref(prm),
                                                    C.byref(jid)))
        self._meta[jid.value] = ("c", None)
        return jid.value

    def submit_decompress(self, stream_t: torch.Tensor, header: bytes, layout: str = "aos") -> int:
        hb = bytes(header[:128])
        info = stream_info(hb)
        jid = C.c_uint64()
        _check(self._lib.bbx_server_submit_decompress(self._h, stream_t.data_ptr(),
                                                      stream_t.numel(), hb,
                                                      AOS if layout == "aos" else SOA,
                                                      C.byref(jid)))
        self._meta[jid.value] = ("d", (info, layout))
        return jid.value

    def progress(self) -> int:
        nd = C.c_uint32()
        _check(self._lib.bbx_server_progress(self._h, C.byref(nd)))
        return nd.value

    def pop_done(self) -> int:
        return int(self._lib.bbx_server_pop_done(self._h))

    def info(self, jid: int) -> dict:
        ji = _JobInfo()
        _check(self._lib.bbx_server_job_info(self._h, jid, C.byref(ji)))
        return dict(state=JOB_STATES[ji.state], status=ji.status, bytes=ji.bytes,
                    d_result=ji.d_result, t_submit=ji.t_submit, t_admit=ji.t_admit,
                    t_launch=ji.t_launch, t_done=ji.t_done, batch_jobs=ji.batch_jobs,
                    kind="compress" if ji.kind == 0 else "decompress")

    def result(self, jid: int) -> torch.Tensor:
        """The finished job's result as a view into the arena (valid until
        release): uint8 stream bytes, or positions of the stream's type."""
        d = self.info(jid)
        if d["state"] != "done":
            raise RuntimeError("job not finished")
        if d["status"] != 0:
            raise BitboxError(d["status"], f"job {jid}")
        off = d["d_result"] - self.arena.data_ptr()
        raw = self.arena[off: off + d["bytes"]]
        kind, extra = self._meta[jid]
        if kind == "c":
            return raw
        info, layout = extra
        dt = torch.float32 if info["dtype"] == F32 else torch.float64
        n, dims = info["n"], info["dims"]
        return raw.view(dt).view((n, dims) if layout == "aos" else (dims, n))

    def release(self, jid: int):
        _check(self._lib.bbx_server_release(self._h, jid))
        self._meta.pop(jid, None)

    def now(self) -> float:
        return float(self._lib.bbx_server_now(self._h))

    def counts(self) -> dict:
        v = [C.c_uint32() for _ in range(4)]
        la, au = C.c_uint64(), C.c_size_t()
        self._lib.bbx_server_counts(self._h, *[C.byref(x) for x in v], C.byref(la), C.byref(au))
        return dict(queued=v[0].value, admitted=v[1].value, running=v[2].value,
                    inflight=v[3].value, launches=la.value, arena_used=au.value)

    def close(self):
        if getattr(self, "_h", None):
            _check(self._lib.bbx_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


def stream_info(header: bytes) -> dict:
    lib = load()
    n, dims, dt, eb, r, nl, sb = (C.c_uint64(), C.c_uint32(), C.c_int(), C.c_double(),
                                  C.c_uint32(), C.c_uint64(), C.c_uint64())
    buf = bytes(header[:128])
    _check(lib.bbx_stream_info(buf, len(buf), C.byref(n), C.byref(dims), C.byref(dt),
                               C.byref(eb), C.byref(r), C.byref(nl), C.byref(sb)))
    return dict(n=n.value, dims=dims.value, dtype=dt.value, eb_abs=eb.value, leaf_size=r.value,
                n_leaves=nl.value, stream_bytes=sb.value)


def compress_static(pos: torch.Tensor, eb: float, out: torch.Tensor, eb_mode: str = "rel",
                    leaf_size: int = 32, layout: str = "aos", perm: torch.Tensor | None = None,
                    stream=None) -> int:
    """bbx_compress_static: compress into the caller's ``out`` (uint8 device
    tensor) with the library's static per-device workspace (no device
    allocation by the library or here).  Waits once and returns the stream
    length."""
    n, dims, lay = _shape(pos, layout)
    if not pos.is_cuda or not pos.is_contiguous() or out.dtype != torch.uint8:
        raise ValueError("positions must be a contiguous device tensor, out a uint8 device tensor")
    p = _params(leaf_size, eb_mode, lay, 0)
    size = C.c_size_t(0)
    _check(load().bbx_compress_static(
        pos.data_ptr() if n else None, n, dims, _dtype_code(pos), float(eb), C.byref(p),
        out.data_ptr(), out.numel(), C.byref(size), None, None,
        perm.data_ptr() if perm is not None else None, _stream_ptr(stream)))
    return size.value


def compress_static_limit() -> int:
    return int(load().bbx_compress_static_limit())


def plan_check(sets) -> None:
    """Host-only check of a batch's launch plan (no GPU needed).  ``sets`` is
    a list of dicts with ``n`` and optionally ``dims``, ``dtype`` (0 f32, 1
    f64), ``eb``, ``leaf_size``, ``tile``, ``scatter_stage``,
    ``level_blocks``, ``want_perm``, ``ref_mode``; raises BitboxError naming
    the failing check."""
    arr = (_Set * max(len(sets), 1))()
    for i, spec in enumerate(sets):
        S = arr[i]
        S.d_pos = None
        S.n, S.dims = int(spec["n"]), int(spec.get("dims", 3))
        S.dtype, S.eb = int(spec.get("dtype", F32)), float(spec.get("eb", 1e-4))
        S.params = _params(spec.get("leaf_size", 32), spec.get("eb_mode", "rel"), AOS,
                           spec.get("tile", 0), spec.get("ref_rule", 0), spec.get("ref_mode", 0),
                           spec.get("scatter_stage", 0), spec.get("level_blocks", 0),
                           spec.get("reduce", 0), spec.get("split_rule", 0),
                           spec.get("level_pairs", 0))
        S.d_out, S.out_cap, S.d_size, S.d_status = None, 0, None, None
        S.d_perm = 8 if spec.get("want_perm") else None  # planned, never read
    _check(load().bbx_plan_check(arr, len(sets)))


def decompress_workspace_size(header: bytes) -> int:
    return int(load().bbx_decompress_workspace_size(bytes(header[:128]), 128))


def compress(pos: torch.Tensor, eb: float, eb_mode: str = "rel", leaf_size: int = 32,
             layout: str = "aos", want_perm: bool = False, tile: int = 0, stream=None,
             ref_rule: int = 0, ref_mode: int = 0, scatter_stage: int = 0,
             level_blocks: int = 0, reduce: int = 0, split_rule: int = 0, level_pairs: int = 0):
    """One-shot compress of a device tensor; returns the stream as a uint8
    device tensor (and the int32 source index of every output slot).
    ref_rule: 0 = leaf reference nearest the AABB centre (the paper's rule),
    1 = the member with the fewest code bits.  ref_mode: 0 = the reference
    stored as its codes, 1 = as its original coordinates (decoded exactly).
    scatter_stage: how the global partition levels store their groups (0 =
    by chunk size, 1 = staged, 2 = direct); level_blocks: cap on the blocks
    per global partition level (0 = the library's choice); neither changes
    the stream.  reduce: the bit box reduction of Sec. 4.1 (1: key sum of
    widths, 2: key sum of box lengths), a version-2 stream.  split_rule: how
    the partition splits a node (0: median, axes in turn; 1: median along
    the widest axis; 2: ceil(n/r) proportional leaves; 3: midpoint cells);
    1-3 give a version-2 stream.  level_pairs: 0 = one data movement per
    global partition level, 1 = two levels per movement; it never changes
    the stream."""
    n, dims, _ = _shape(pos, layout)
    c = Compressor(n, dims, pos.dtype, leaf_size, eb_mode, layout, tile, want_perm, pos.device,
                   ref_rule, ref_mode, scatter_stage, level_blocks, reduce, split_rule,
                   level_pairs)
    s = c(pos.contiguous(), eb, stream).clone()
    if want_perm:
        return s, c.perm[:n].clone()
    return s


def decompress(stream_t: torch.Tensor, layout: str = "aos", stream=None) -> torch.Tensor:
    """One-shot decompress of a device uint8 stream."""
    if stream_t.numel() < 128:
        raise BitboxError(3, "stream shorter than its header")
    header = stream_t[:128].cpu().numpy().tobytes()
    d = Decompressor(header, layout, stream_t.device)
    return d(stream_t, stream).clone()


class SequenceExporter:
    """Reusable export of ref_mode 1 streams of one header's geometry to the
    Sec. 4.2 sequence layout: owns the workspace and the output buffer.
    ``__call__`` waits and returns the layout as a uint8 view of the output
    buffer (valid until the next call); ``launch`` only enqueues."""

    def __init__(self, header: bytes, device="cuda"):
        lib = load()
        self._lib = lib
        self.header = bytes(header[:128])
        self.size = int(lib.bbx_export_sequences_size(self.header, 128))
        if self.size == 0 and stream_info(self.header)["n"] > 0:
            raise BitboxError(1, "the sequence layout needs references stored as coordinates (ref_mode 1)")
        self.ws_size = int(lib.bbx_decompress_workspace_size(self.header, 128))
        self.ws = torch.empty(max(self.ws_size, 1), dtype=torch.uint8, device=device)
        self.out = torch.empty(max(self.size, 8), dtype=torch.uint8, device=device)
        self.d_status = torch.zeros(1, dtype=torch.int32, device=device)

    def _call(self, stream_t: torch.Tensor, d_status, stream):
        return self._lib.bbx_export_sequences(
            stream_t.data_ptr(), stream_t.numel(), self.header, self.out.data_ptr(), self.out.numel(),
            d_status, self.ws.data_ptr(), self.ws_size, _stream_ptr(stream))

    def launch(self, stream_t: torch.Tensor, stream=None):
        _check(self._call(stream_t, self.d_status.data_ptr(), stream))

    def __call__(self, stream_t: torch.Tensor, stream=None):
        _check(self._call(stream_t, None, stream))
        return self.out[: self.size]


def export_sequences(stream_t: torch.Tensor, stream=None) -> torch.Tensor:
    """The Sec. 4.2 sequence layout (centre, widths, codes, 32-bit end mark
    per leaf) of a device uint8 stream compressed with ref_mode = 1."""
    if stream_t.numel() < 128:
        raise BitboxError(3, "stream shorter than its header")
    header = stream_t[:128].cpu().numpy().tobytes()
    return SequenceExporter(header, stream_t.device)(stream_t, stream).clone()


def export_sequences_reordered(stream_t: torch.Tensor, stream=None):
    """The Sec. 4.2 sequence layout after its two reorderings (sequences by
    sum of widths, members by R-index with the axes in ascending entropy) of
    a device uint8 stream compressed with ref_mode = 1; returns (layout as a
    uint8 device tensor, axis order)."""
    lib = load()
    if stream_t.numel() < 128:
        raise BitboxError(3, "stream shorter than its header")
    header = stream_t[:128].cpu().numpy().tobytes()
    size = int(lib.bbx_export_sequences_size(header, 128))
    ws_size = int(lib.bbx_export_reordered_workspace_size(header, 128))
    if ws_size == 0:
        raise BitboxError(1, "the sequence layout needs references stored as coordinates (ref_mode 1)")
    ws = torch.empty(ws_size, dtype=torch.uint8, device=stream_t.device)
    out = torch.empty(max(size, 8), dtype=torch.uint8, device=stream_t.device)
    order = (C.c_uint32 * 3)()
    _check(lib.bbx_export_sequences_reordered(stream_t.data_ptr(), stream_t.numel(), header,
                                              out.data_ptr(), out.numel(), order, ws.data_ptr(),
                                              ws_size, _stream_ptr(stream)))
    dims = stream_info(header)["dims"]
    return out[:size].clone(), [int(order[d]) for d in range(dims)]


def huffman_encode(data: torch.Tensor, stream=None) -> torch.Tensor:
    """Huffman coding of a device uint8 tensor (the encoding phase of Sec. 3;
    canonical codes of at most 12 bits, chunks of 4,096 bytes); returns the
    stream as a uint8 device tensor."""
    lib = load()
    if data.dtype != torch.uint8 or not data.is_cuda or not data.is_contiguous():
        raise ValueError("input must be a contiguous uint8 device tensor")
    n = data.numel()
    ws_size = int(lib.bbx_huffman_workspace_size(n))
    ws = torch.empty(ws_size, dtype=torch.uint8, device=data.device)
    cap = int(lib.bbx_huffman_bound(n))
    out = torch.empty((cap + 7) // 8 * 8, dtype=torch.uint8, device=data.device)
    size = C.c_size_t(0)
    _check(lib.bbx_huffman_encode(data.data_ptr() if n else None, n, out.data_ptr(), out.numel(),
                                  C.byref(size), ws.data_ptr(), ws_size, _stream_ptr(stream)))
    return out[: size.value].clone()


def huffman_decode(stream_t: torch.Tensor, stream=None) -> torch.Tensor:
    """Decode a device uint8 Huffman stream (waits for the device's verdict)."""
    lib = load()
    if stream_t.numel() < 176:
        raise BitboxError(3, "Huffman stream shorter than its header")
    header = stream_t[:176].cpu().numpy().tobytes()
    n = int.from_bytes(header[8:16], "little")
    ws_size = int(lib.bbx_huffman_workspace_size(n))
    ws = torch.empty(ws_size, dtype=torch.uint8, device=stream_t.device)
    out = torch.empty(max((n + 7) // 8 * 8, 8), dtype=torch.uint8, device=stream_t.device)
    _check(lib.bbx_huffman_decode(stream_t.data_ptr(), stream_t.numel(), header, out.data_ptr(),
                                  out.numel(), None, ws.data_ptr(), ws_size, _stream_ptr(stream)))
    return out[:n].clone()


@contextmanager
def profile():
    """Collects per-kernel launch counts and summed durations (ms)."""
    lib = load()
    lib.bbx_profile_reset()
    lib.bbx_profile_enable(1)
    result = {}
    try:
        yield result
    finally:
        lib.bbx_profile_enable(0)
        for i in range(lib.bbx_profile_count()):
            name, cnt, ms = C.c_char_p(), C.c_uint64(), C.c_double()
            _check(lib.bbx_profile_get(i, C.byref(name), C.byref(cnt), C.byref(ms)))
            result[name.value.decode()] = (cnt.value, ms.value)
        lib.bbx_profile_reset()
