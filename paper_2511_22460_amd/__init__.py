"""Python binding of libebr (the C ABI declared in include/ebr.h).

Argument marshalling only: every step of the retrieval path runs inside
libebr.so (host runtime + gfx950 kernels). PyTorch supplies device memory
(the index arena, the batch workspace, outputs) and the current HIP stream.
There is no fallback: if the library cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from . import _build

_lib = None

EBR_OK, EBR_EINVAL, EBR_ENOMEM, EBR_EDEVICE, EBR_EAGAIN, EBR_ENOTFOUND, EBR_ESHUTDOWN, \
    EBR_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
F32, BF16, FP8E4M3 = 0, 1, 2
# device scratch of ebr_score_topk_noalloc (EBR_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 256 << 20
_STATUS = {0: "EBR_OK", -1: "EBR_EINVAL", -2: "EBR_ENOMEM", -3: "EBR_EDEVICE", -4: "EBR_EAGAIN",
           -5: "EBR_ENOTFOUND", -6: "EBR_ESHUTDOWN", -7: "EBR_EUNSUPPORTED"}

#: every symbol include/ebr.h declares
EXPORTS = ("ebr_index_size", "ebr_build_index", "ebr_index_stats", "ebr_decode_key", "ebr_decode_keys",
           "ebr_free_index", "ebr_workspace_size", "ebr_score_topk", "ebr_score_dense",
           "ebr_codec_size", "ebr_codec_encode", "ebr_codec_decode", "ebr_last_error",
           "ebr_version", "ebr_set_timing", "ebr_get_timings", "ebr_quantize_bf16",
           "ebr_quantize_fp8", "ebr_dequantize_fp8", "ebr_server_create", "ebr_submit",
           "ebr_poll", "ebr_server_stats", "ebr_server_reset_stats", "ebr_server_destroy",
           "ebr_autotune", "ebr_set_launch_shape", "ebr_get_launch_shape", "ebr_graph_create",
           "ebr_score_topk_graph", "ebr_graph_stats", "ebr_graph_destroy", "ebr_score_topk_noalloc",
           "ebr_device_build_scratch_size", "ebr_device_index_size", "ebr_build_index_device",
           "ebr_server_swap_index")


class EbrError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {_STATUS.get(status, status)}: {msg}")
        self.status = status


class BuildDesc(ctypes.Structure):
    _fields_ = [("n_ads", ctypes.c_int64), ("dim", ctypes.c_int32), ("ad_emb", ctypes.c_void_p),
                ("n_keys", ctypes.c_int64), ("key_offsets", ctypes.c_void_p),
                ("post_ids", ctypes.c_void_p), ("post_w", ctypes.c_void_p),
                ("dtypes", ctypes.c_uint32)]


class IndexInfo(ctypes.Structure):
    _fields_ = [("n_ads", ctypes.c_int64), ("n_keys", ctypes.c_int64),
                ("n_postings", ctypes.c_int64), ("n_chunks", ctypes.c_int64),
                ("n_tiles", ctypes.c_int64), ("dim", ctypes.c_int32), ("tile_ads", ctypes.c_int32),
                ("arena_bytes", ctypes.c_uint64), ("bytes_emb_f32", ctypes.c_uint64),
                ("bytes_emb_bf16", ctypes.c_uint64), ("bytes_emb_fp8", ctypes.c_uint64),
                ("bytes_chunk_headers", ctypes.c_uint64), ("bytes_packed_ids", ctypes.c_uint64),
                ("bytes_weights", ctypes.c_uint64), ("max_err_bf16", ctypes.c_double),
                ("max_err_fp8", ctypes.c_double), ("bits_per_id", ctypes.c_double),
                ("bytes_per_posting", ctypes.c_double), ("encode_ms", ctypes.c_double),
                ("upload_ms", ctypes.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Timings(ctypes.Structure):
    _fields_ = [("decode_ms", ctypes.c_double), ("sample_ms", ctypes.c_double),
                ("score_ms", ctypes.c_double), ("finalize_ms", ctypes.c_double),
                ("host_ms", ctypes.c_double), ("score_first_ms", ctypes.c_double),
                ("rescore_ms", ctypes.c_double), ("rounds", ctypes.c_int32),
                ("uncertified", ctypes.c_int32), ("imprecise", ctypes.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


def set_timing(enable: bool):
    _check(load().ebr_set_timing(1 if enable else 0), "ebr_set_timing")


def last_timings() -> dict:
    t = Timings()
    _check(load().ebr_get_timings(ctypes.byref(t)), "ebr_get_timings")
    return t.as_dict()


class Batch(ctypes.Structure):
    _fields_ = [("n_queries", ctypes.c_int32), ("user_emb", ctypes.c_void_p),
                ("feat_offsets", ctypes.c_void_p), ("feat_keys", ctypes.c_void_p),
                ("feat_mult", ctypes.c_void_p), ("k", ctypes.c_void_p),
                ("scan_dtype", ctypes.c_int), ("rescore_factor", ctypes.c_int32),
                ("wide64", ctypes.c_int32)]


class LaunchShape(ctypes.Structure):
    _fields_ = [("score_ranges", ctypes.c_int32), ("sample_ranges", ctypes.c_int32),
                ("decode_chunks", ctypes.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


TUNE_MAX = 16


class TuneReport(ctypes.Structure):
    _fields_ = [("n_tried", ctypes.c_int32), ("tried", LaunchShape * TUNE_MAX),
                ("tried_ms", ctypes.c_float * TUNE_MAX), ("best", LaunchShape),
                ("best_ms", ctypes.c_float), ("default_ms", ctypes.c_float)]

    def as_dict(self):
        n = self.n_tried
        return {"tried": [(self.tried[i].as_dict(), float(self.tried_ms[i])) for i in range(n)],
                "best": self.best.as_dict(), "best_ms": float(self.best_ms),
                "default_ms": float(self.default_ms)}


class GraphInfo(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_uint64), ("instantiations", ctypes.c_uint64),
                ("updates", ctypes.c_uint64), ("nodes", ctypes.c_uint64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class ServerOpts(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("max_wait_us", ctypes.c_int32),
                ("pipeline", ctypes.c_int32), ("scan_dtype", ctypes.c_int),
                ("rescore_factor", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("f32_below", ctypes.c_int32), ("max_queue", ctypes.c_int32)]


class Query(ctypes.Structure):
    _fields_ = [("user_emb", ctypes.c_void_p), ("n_feats", ctypes.c_int32),
                ("feat_keys", ctypes.c_void_p), ("feat_mult", ctypes.c_void_p),
                ("k", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("queued", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("mean_batch", ctypes.c_double),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("elapsed_ms", ctypes.c_double), ("qps", ctypes.c_double),
                ("busy_ms", ctypes.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


def lib_path() -> str:
    return _build.LIB


def load():
    """Load libebr.so (building it first only if no built library exists)."""
    global _lib
    if _lib is not None:
        return _lib
    try:  # torch first, so its HIP runtime is the one the library binds to
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(_build.LIB):
        _build.build()
    h = ctypes.CDLL(_build.LIB)
    P, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    st = ctypes.c_int
    sig = {
        "ebr_index_size": ([P, ctypes.POINTER(sz)], st),
        "ebr_build_index": ([P, P, sz, P, ctypes.POINTER(P)], st),
        "ebr_index_stats": ([P, P], st),
        "ebr_decode_key": ([P, i64, P, P, i64, ctypes.POINTER(i64), P], st),
        "ebr_decode_keys": ([P, i64, i64, P, P, i64, ctypes.POINTER(i64), P], st),
        "ebr_free_index": ([P], None),
        "ebr_workspace_size": ([P, P, ctypes.POINTER(sz)], st),
        "ebr_score_topk": ([P, P, P, sz, P, P, P], st),
        "ebr_score_topk_noalloc": ([P, P, P, P, P], st),
        "ebr_device_build_scratch_size": ([i64, i64, ctypes.POINTER(sz)], st),
        "ebr_device_index_size": ([P, P, sz, P, ctypes.POINTER(sz)], st),
        "ebr_build_index_device": ([P, P, sz, P, sz, P, ctypes.POINTER(P)], st),
        "ebr_server_swap_index": ([P, P], st),
        "ebr_score_dense": ([P, P, P, sz, P, P, P], st),
        "ebr_codec_size": ([P, i64, ctypes.POINTER(sz)], st),
        "ebr_codec_encode": ([P, i64, P, sz, ctypes.POINTER(sz)], st),
        "ebr_codec_decode": ([P, sz, i64, P], st),
        "ebr_last_error": ([], ctypes.c_char_p),
        "ebr_version": ([], ctypes.c_char_p),
        "ebr_set_timing": ([ctypes.c_int], st),
        "ebr_quantize_bf16": ([P, i64, P], st),
        "ebr_quantize_fp8": ([P, i64, ctypes.c_float, P], st),
        "ebr_dequantize_fp8": ([P, i64, P], st),
        "ebr_get_timings": ([P], st),
        "ebr_server_create": ([P, P, sz, P, ctypes.POINTER(P)], st),
        "ebr_submit": ([P, P, P, P, ctypes.POINTER(ctypes.c_uint64)], st),
        "ebr_poll": ([P, ctypes.c_uint64, i32], st),
        "ebr_server_stats": ([P, P], st),
        "ebr_server_reset_stats": ([P], st),
        "ebr_server_destroy": ([P], st),
        "ebr_autotune": ([P, P, P, sz, P, P, i32, P, P], st),
        "ebr_set_launch_shape": ([P, ctypes.c_int, i32, P], st),
        "ebr_get_launch_shape": ([P, ctypes.c_int, i32, P], st),
        "ebr_graph_create": ([ctypes.POINTER(P)], st),
        "ebr_score_topk_graph": ([P, P, P, P, sz, P, P, P], st),
        "ebr_graph_stats": ([P, P], st),
        "ebr_graph_destroy": ([P], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(h, name)
        f.argtypes = args
        f.restype = res
    _lib = h
    return h


def _check(rc: int, where: str):
    if rc != EBR_OK:
        raise EbrError(rc, where, load().ebr_last_error().decode(errors="replace"))


def version() -> str:
    return load().ebr_version().decode()


def _np(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def _ptr(a):
    return None if a is None else a.ctypes.data


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


# ------------------------------------------------------------------------------ quantisers (host)

def quantize_bf16(x) -> np.ndarray:
    x = _np(x, np.float32)
    out = np.empty(max(1, len(x)), dtype=np.uint16)
    _check(load().ebr_quantize_bf16(_ptr(x), len(x), out.ctypes.data), "ebr_quantize_bf16")
    return out[:len(x)]


def quantize_fp8(x, scale: float = 1.0) -> np.ndarray:
    x = _np(x, np.float32)
    out = np.empty(max(1, len(x)), dtype=np.uint8)
    _check(load().ebr_quantize_fp8(_ptr(x), len(x), float(scale), out.ctypes.data), "ebr_quantize_fp8")
    return out[:len(x)]


def dequantize_fp8(codes) -> np.ndarray:
    c = _np(codes, np.uint8)
    out = np.empty(max(1, len(c)), dtype=np.float32)
    _check(load().ebr_dequantize_fp8(_ptr(c), len(c), out.ctypes.data), "ebr_dequantize_fp8")
    return out[:len(c)]


# ------------------------------------------------------------------------------ codec (host)

def codec_encode(ids) -> bytes:
    ids = _np(ids, np.uint32)
    n = len(ids)
    need = ctypes.c_size_t()
    _check(load().ebr_codec_size(_ptr(ids), n, ctypes.byref(need)), "ebr_codec_size")
    buf = np.zeros(max(1, need.value), dtype=np.uint8)
    used = ctypes.c_size_t()
    _check(load().ebr_codec_encode(_ptr(ids), n, buf.ctypes.data, need.value, ctypes.byref(used)),
           "ebr_codec_encode")
    return buf[:used.value].tobytes()


def codec_decode(blob: bytes, n: int) -> np.ndarray:
    src = np.frombuffer(blob, dtype=np.uint8) if len(blob) else np.zeros(1, np.uint8)
    out = np.empty(max(1, n), dtype=np.uint32)
    _check(load().ebr_codec_decode(src.ctypes.data, len(blob), n, out.ctypes.data),
           "ebr_codec_decode")
    return out[:n]


def index_size(ad_emb, key_offsets, post_ids, post_w=None, dtypes: int = 1) -> int:
    desc, _keep = _desc(ad_emb, key_offsets, post_ids, post_w, dtypes)
    n = ctypes.c_size_t()
    _check(load().ebr_index_size(ctypes.byref(desc), ctypes.byref(n)), "ebr_index_size")
    return n.value


def _desc(ad_emb, key_offsets, post_ids, post_w, dtypes):
    E = _np(ad_emb, np.float32)
    offs = _np(key_offsets, np.int64)
    ids = _np(post_ids, np.uint32)
    w = _np(post_w, np.float32)
    d = BuildDesc(E.shape[0], E.shape[1] if E.ndim == 2 else 0, _ptr(E), len(offs) - 1,
                  _ptr(offs), _ptr(ids) if len(ids) else None, _ptr(w) if w is not None and len(w) else None,
                  dtypes)
    return d, (E, offs, ids, w)


# ------------------------------------------------------------------------------ index

class Index:
    """A resident index: compressed posting lists + embeddings in a torch-owned device arena."""

    def __init__(self, ad_emb, key_offsets, post_ids, post_w=None, dtypes: int = 1, device=None,
                 stream=None):
        import torch
        self.device = torch.device(device if device is not None else "cuda")
        desc, keep = _desc(ad_emb, key_offsets, post_ids, post_w, dtypes)
        n = ctypes.c_size_t()
        _check(load().ebr_index_size(ctypes.byref(desc), ctypes.byref(n)), "ebr_index_size")
        # zeroed: the alignment gaps between sections are then deterministic too
        self.arena = torch.zeros(max(256, n.value), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        _check(load().ebr_build_index(ctypes.byref(desc), self.arena.data_ptr(), self.arena.numel(),
                                      _stream(stream), ctypes.byref(h)), "ebr_build_index")
        self._h = h
        self.n_ads, self.dim = keep[0].shape
        self.n_keys = len(keep[1]) - 1
        self._ws = None

    @classmethod
    def from_workload(cls, wl, **kw):
        return cls(wl.ad_emb, wl.key_offsets, wl.post_ids, wl.post_w, **kw)

    @classmethod
    def build_on_device(cls, ad_emb, key_offsets, post_ids, post_w=None, dtypes: int = 1, stream=None):
        """The same index built on the GPU (ebr_build_index_device) from device tensors:
        ad_emb float32 [N, d], key_offsets int64 [V + 1], post_ids int32/uint32 bits, post_w
        float32 or None. Returns (index, device milliseconds of the size and build calls)."""
        import time
        import torch
        lib = load()
        dev = ad_emb.device
        for t in (ad_emb, key_offsets, post_ids) + ((post_w,) if post_w is not None else ()):
            if t.device != dev or not t.is_contiguous():
                raise ValueError("device build inputs: contiguous tensors on one device")
        V = key_offsets.numel() - 1
        desc = BuildDesc(ad_emb.shape[0], ad_emb.shape[1], ad_emb.data_ptr(), V, key_offsets.data_ptr(),
                         post_ids.data_ptr() if post_ids.numel() else None,
                         post_w.data_ptr() if post_w is not None and post_w.numel() else None, dtypes)
        sb = ctypes.c_size_t()
        _check(lib.ebr_device_build_scratch_size(V, post_ids.numel(), ctypes.byref(sb)),
               "ebr_device_build_scratch_size")
        scratch = torch.empty(max(256, sb.value), dtype=torch.uint8, device=dev)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        n = ctypes.c_size_t()
        _check(lib.ebr_device_index_size(ctypes.byref(desc), scratch.data_ptr(), scratch.numel(), _stream(stream),
                                         ctypes.byref(n)), "ebr_device_index_size")
        self = cls.__new__(cls)
        self.device = dev
        self.arena = torch.zeros(max(256, n.value), dtype=torch.uint8, device=dev)
        h = ctypes.c_void_p()
        _check(lib.ebr_build_index_device(ctypes.byref(desc), scratch.data_ptr(), scratch.numel(),
                                          self.arena.data_ptr(), self.arena.numel(), _stream(stream),
                                          ctypes.byref(h)), "ebr_build_index_device")
        ms = 1000.0 * (time.perf_counter() - t0)
        self._h = h
        self.n_ads, self.dim = int(ad_emb.shape[0]), int(ad_emb.shape[1])
        self.n_keys = V
        self._ws = None
        return self, ms

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().ebr_free_index(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self) -> dict:
        info = IndexInfo()
        _check(load().ebr_index_stats(self._h, ctypes.byref(info)), "ebr_index_stats")
        return info.as_dict()

    def decode_key(self, key: int, stream=None):
        import torch
        n = ctypes.c_int64()
        rc = load().ebr_decode_key(self._h, key, None, None, 0, ctypes.byref(n), _stream(stream))
        if rc not in (EBR_OK, EBR_ENOMEM):
            _check(rc, "ebr_decode_key")
        cap = max(1, n.value)
        ids = torch.empty(cap, dtype=torch.int32, device=self.device)
        w = torch.empty(cap, dtype=torch.float32, device=self.device)
        _check(load().ebr_decode_key(self._h, key, ids.data_ptr(), w.data_ptr(), cap,
                                     ctypes.byref(n), _stream(stream)), "ebr_decode_key")
        return ids[:n.value], w[:n.value]

    def decode_keys(self, key_begin: int, key_end: int, stream=None):
        """GPU decode of the lists of keys [key_begin, key_end), concatenated in key order."""
        import torch
        n = ctypes.c_int64()
        rc = load().ebr_decode_keys(self._h, key_begin, key_end, None, None, 0, ctypes.byref(n),
                                    _stream(stream))
        if rc not in (EBR_OK, EBR_ENOMEM):
            _check(rc, "ebr_decode_keys")
        cap = max(1, n.value)
        ids = torch.empty(cap, dtype=torch.int32, device=self.device)
        w = torch.empty(cap, dtype=torch.float32, device=self.device)
        _check(load().ebr_decode_keys(self._h, key_begin, key_end, ids.data_ptr(), w.data_ptr(), cap,
                                      ctypes.byref(n), _stream(stream)), "ebr_decode_keys")
        return ids[:n.value], w[:n.value]

    # -------------------------------------------------------------------------- batches

    def _batch(self, user_emb, feat_offsets, feat_keys, feat_mult, k, scan_dtype, rescore,
               wide64=False):
        import torch
        if not (isinstance(user_emb, torch.Tensor) and user_emb.is_cuda):
            raise TypeError("user_emb must be a CUDA (HIP) tensor")
        if user_emb.dtype != torch.float32 or user_emb.dim() != 2 or user_emb.shape[1] != self.dim:
            raise ValueError(f"user_emb must be float32 [B, {self.dim}]")
        user_emb = user_emb.contiguous()
        offs = _np(feat_offsets, np.int64)
        keys = _np(feat_keys, np.int32)
        mult = _np(feat_mult, np.float32)
        kq = _np(k, np.int32) if k is not None else None
        B = user_emb.shape[0]
        if len(offs) != B + 1:
            raise ValueError("feat_offsets must have B + 1 entries")
        if kq is not None and len(kq) != B:
            raise ValueError("k must have B entries")
        keep = (user_emb, offs, keys, mult, kq)
        b = Batch(B, user_emb.data_ptr(), _ptr(offs), _ptr(keys) if len(keys) else None,
                  _ptr(mult) if mult is not None and len(mult) else None,
                  _ptr(kq) if kq is not None and len(kq) else None, scan_dtype, rescore,
                  1 if wide64 else 0)
        return b, keep

    def workspace(self, nbytes: int):
        import torch
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(max(256, nbytes), dtype=torch.uint8, device=self.device)
        return self._ws

    def workspace_size(self, user_emb, feat_offsets, feat_keys, k, feat_mult=None,
                       scan_dtype: int = F32, rescore_factor: int = 4, wide64: bool = False) -> int:
        b, keep = self._batch(user_emb, feat_offsets, feat_keys, feat_mult, k, scan_dtype,
                              rescore_factor, wide64)
        n = ctypes.c_size_t()
        _check(load().ebr_workspace_size(self._h, ctypes.byref(b), ctypes.byref(n)),
               "ebr_workspace_size")
        return n.value

    def score_topk(self, user_emb, feat_offsets, feat_keys, k, feat_mult=None,
                   scan_dtype: int = F32, rescore_factor: int = 4, out=None, stream=None,
                   graph: Optional["Graph"] = None, wide64: bool = False):
        """Top-K per query. Returns (ids int32 tensor [sum K], scores float32 tensor [sum K],
        offsets np.int64 [B + 1]); ids are uint32 values stored in int32 (N < 2^31 here).
        With a Graph handle the batch's device work runs as one captured HIP graph; wide64
        asks for 64-bit cross-term cells for every query (FP32 scan)."""
        import torch
        b, keep = self._batch(user_emb, feat_offsets, feat_keys, feat_mult, k, scan_dtype,
                              rescore_factor, wide64)
        kq = keep[4]
        offs = np.zeros(len(kq) + 1, dtype=np.int64)
        np.cumsum(kq, out=offs[1:])
        total = int(offs[-1])
        if out is None:
            ids = torch.empty(max(1, total), dtype=torch.int32, device=self.device)
            scores = torch.empty(max(1, total), dtype=torch.float32, device=self.device)
        else:
            ids, scores = out
        lib = load()
        if graph is None:
            def call(wp, wn):
                return lib.ebr_score_topk(self._h, ctypes.byref(b), wp, wn, ids.data_ptr(),
                                          scores.data_ptr(), _stream(stream))
        else:
            def call(wp, wn):
                return lib.ebr_score_topk_graph(graph._h, self._h, ctypes.byref(b), wp, wn,
                                                ids.data_ptr(), scores.data_ptr(), _stream(stream))
        # the kept workspace is tried first; it grows (one sizing call) only when too small
        ws = self._ws
        rc = call(ws.data_ptr() if ws is not None else None, ws.numel() if ws is not None else 0)
        if rc == EBR_ENOMEM and lib.ebr_last_error().startswith(b"workspace too small"):
            n = ctypes.c_size_t()
            _check(lib.ebr_workspace_size(self._h, ctypes.byref(b), ctypes.byref(n)),
                   "ebr_workspace_size")
            ws = self.workspace(n.value)
            rc = call(ws.data_ptr(), ws.numel())
        _check(rc, "ebr_score_topk" if graph is None else "ebr_score_topk_graph")
        return ids[:total], scores[:total], offs

    def autotune(self, user_emb, feat_offsets, feat_keys, k, feat_mult=None,
                 scan_dtype: int = F32, rescore_factor: int = 4, reps: int = 3, stream=None):
        """Autotune the launch shape on this batch (ebr_autotune) and record it in the index
        for batches of the same dtype and query-group count. Returns the report as a dict and
        the batch's results (ids, scores, offsets)."""
        import torch
        b, keep = self._batch(user_emb, feat_offsets, feat_keys, feat_mult, k, scan_dtype,
                              rescore_factor)
        kq = keep[4]
        offs = np.zeros(len(kq) + 1, dtype=np.int64)
        np.cumsum(kq, out=offs[1:])
        total = int(offs[-1])
        ids = torch.empty(max(1, total), dtype=torch.int32, device=self.device)
        scores = torch.empty(max(1, total), dtype=torch.float32, device=self.device)
        n = ctypes.c_size_t()
        _check(load().ebr_workspace_size(self._h, ctypes.byref(b), ctypes.byref(n)),
               "ebr_workspace_size")
        ws = self.workspace(n.value)
        rep = TuneReport()
        _check(load().ebr_autotune(self._h, ctypes.byref(b), ws.data_ptr(), ws.numel(),
                                   ids.data_ptr(), scores.data_ptr(), int(reps), _stream(stream),
                                   ctypes.byref(rep)), "ebr_autotune")
        return rep.as_dict(), (ids[:total], scores[:total], offs)

    def set_launch_shape(self, scan_dtype: int, n_queries: int, shape: Optional[dict]):
        """Record (dict with score_ranges / sample_ranges / decode_chunks) or clear (None)
        the launch shape of batches of n_queries queries on scan_dtype."""
        sh = None if shape is None else LaunchShape(int(shape.get("score_ranges", 0)),
                                                    int(shape.get("sample_ranges", 0)),
                                                    int(shape.get("decode_chunks", 0)))
        _check(load().ebr_set_launch_shape(self._h, scan_dtype, int(n_queries),
                                           None if sh is None else ctypes.byref(sh)),
               "ebr_set_launch_shape")

    def launch_shape(self, scan_dtype: int, n_queries: int) -> dict:
        sh = LaunchShape()
        _check(load().ebr_get_launch_shape(self._h, scan_dtype, int(n_queries), ctypes.byref(sh)),
               "ebr_get_launch_shape")
        return sh.as_dict()

    def score_dense(self, user_emb, feat_offsets, feat_keys, feat_mult=None, scan_dtype: int = F32,
                    stream=None, wide64: bool = False):
        """Full deep and wide terms [B, N] (FP32 values) as the scan of that dtype computes them
        (wide64: with 64-bit cross-term cells)."""
        import torch
        b, keep = self._batch(user_emb, feat_offsets, feat_keys, feat_mult, None, scan_dtype, 0,
                              wide64)
        n = ctypes.c_size_t()
        # the dense hook needs no selection buffers; size it through the top-K query with K = 0
        kz = np.zeros(max(1, b.n_queries), np.int32)
        b2 = Batch(b.n_queries, b.user_emb, b.feat_offsets, b.feat_keys, b.feat_mult,
                   kz.ctypes.data, scan_dtype, 0, b.wide64)
        _check(load().ebr_workspace_size(self._h, ctypes.byref(b2), ctypes.byref(n)),
               "ebr_workspace_size")
        ws = self.workspace(n.value)
        B = b.n_queries
        deep = torch.empty((B, self.n_ads), dtype=torch.float32, device=self.device)
        wide = torch.empty((B, self.n_ads), dtype=torch.float32, device=self.device)
        _check(load().ebr_score_dense(self._h, ctypes.byref(b), ws.data_ptr(), ws.numel(),
                                      deep.data_ptr(), wide.data_ptr(), _stream(stream)),
               "ebr_score_dense")
        return deep, wide

    def topk_workload(self, wl, qs=None, **kw):
        """Convenience: run a workloads.Workload batch (or a subset of its queries)."""
        import torch
        w = wl if qs is None else wl.subset(qs)
        U = torch.from_numpy(np.ascontiguousarray(w.user_emb)).to(self.device)
        return self.score_topk(U, w.feat_offsets, w.feat_keys, w.k, w.feat_mult, **kw)


class Graph:
    """A captured-batch handle (ebr_graph_*): pass it to Index.score_topk(graph=...) to run a
    batch's device work as one HIP graph. One call at a time per handle."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(load().ebr_graph_create(ctypes.byref(h)), "ebr_graph_create")
        self._h = h

    def stats(self) -> dict:
        info = GraphInfo()
        _check(load().ebr_graph_stats(self._h, ctypes.byref(info)), "ebr_graph_stats")
        return info.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().ebr_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop over a resident Index (ebr_server_*): submit single queries from host
    memory, poll for their results. The scratch arena is a torch-owned device buffer."""

    def __init__(self, index: "Index", scratch_bytes: int, max_batch: int = 256,
                 max_wait_us: int = 200, pipeline: int = 2, scan_dtype: int = F32,
                 rescore_factor: int = 4, graph: bool = False, f32_below: int = 0,
                 max_queue: int = 0):
        import torch
        self.index = index
        self.scratch = torch.empty(max(256, int(scratch_bytes)), dtype=torch.uint8, device=index.device)
        opts = ServerOpts(max_batch, max_wait_us, pipeline, scan_dtype, rescore_factor,
                          1 if graph else 0, int(f32_below), int(max_queue))
        h = ctypes.c_void_p()
        _check(load().ebr_server_create(index._h, self.scratch.data_ptr(), self.scratch.numel(),
                                        ctypes.byref(opts), ctypes.byref(h)), "ebr_server_create")
        self._h = h
        self._pending = {}

    def submit(self, user_emb, feat_keys, k: int, feat_mult=None) -> int:
        """Queue one query (host arrays); returns its ticket."""
        u = _np(user_emb, np.float32)
        keys = _np(feat_keys, np.int32)
        mult = _np(feat_mult, np.float32)
        if u.shape != (self.index.dim,):
            raise ValueError(f"user_emb must have {self.index.dim} entries")
        if mult is not None and len(mult) != len(keys):
            raise ValueError("feat_mult must match feat_keys")
        ids = np.empty(max(1, k), dtype=np.uint32)
        sc = np.empty(max(1, k), dtype=np.float32)
        q = Query(_ptr(u), len(keys), _ptr(keys) if len(keys) else None,
                  _ptr(mult) if mult is not None and len(mult) else None, int(k))
        t = ctypes.c_uint64()
        _check(load().ebr_submit(self._h, ctypes.byref(q), _ptr(ids), _ptr(sc), ctypes.byref(t)),
               "ebr_submit")
        self._pending[t.value] = (ids, sc, int(k))
        return t.value

    def poll(self, ticket: int, timeout_us: int = -1):
        """(ids, scores) once the ticket is done, None if not done within timeout_us."""
        rc = load().ebr_poll(self._h, ticket, int(timeout_us))
        if rc == EBR_EAGAIN:
            return None
        ids, sc, k = self._pending.pop(ticket, (None, None, 0))
        _check(rc, "ebr_poll")
        return ids[:k], sc[:k]

    def swap_index(self, index: "Index"):
        """Online refresh: later submissions run on `index`; returns once every query of the
        previous index has completed (the previous Index may then be freed)."""
        _check(load().ebr_server_swap_index(self._h, index._h), "ebr_server_swap_index")
        self.index = index

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().ebr_server_stats(self._h, ctypes.byref(st)), "ebr_server_stats")
        return st.as_dict()

    def reset_stats(self):
        _check(load().ebr_server_reset_stats(self._h), "ebr_server_reset_stats")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            rc = load().ebr_server_destroy(self._h)
            self._h = None
            self._pending.clear()
            _check(rc, "ebr_server_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
