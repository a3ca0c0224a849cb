"""FP64 CPU oracle for the Wide & Deep ad-retrieval hot path (arXiv 2511.22460).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product library never does.
It shares no code with the GPU library.

Two implementations live here, each written from the paper's definitions:

* ``oracle.cpp`` (C++17 + OpenMP, FP64): per query the dual-tower dot
  (Section 3.1, equation "dual-tower"), plus the HitMatch cross term walked
  over the raw posting lists (Section 3.3, equation "hitmatch"), summed
  (Section 3.1, the three logits are added), then the top-K by
  (score desc, id asc).
* ``dense_scores`` (numpy, FP64, tiny inputs only): the same scores from the
  uncompressed cross-weight table, deep = U E^T and wide = M W with a dense
  W[V x N]; this is the sparse-matrix-times-vector form L * w~ of Section 3.4.
  It is the independent brute force the C++ oracle is pinned against.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_h = None

_P = ctypes.c_void_p


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _lib():
    global _h
    if _h is None:
        if not os.path.exists(_LIB):
            build(force=False)
        h = ctypes.CDLL(_LIB)
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        h.oracle_scores.argtypes = [i64, i32, _P, i64, _P, _P, _P, _P, i32, _P, _P, _P, _P, _P]
        h.oracle_scores.restype = ctypes.c_int
        h.oracle_topk.argtypes = [i64, i32, _P, i64, _P, _P, _P, _P, i32, _P, _P, i64,
                                  _P, _P, _P, _P, _P]
        h.oracle_topk.restype = ctypes.c_int
        h.oracle_topk_batch.argtypes = [i64, i32, _P, i64, _P, _P, _P, i32, _P, _P, _P, _P,
                                        _P, _P, _P, _P, _P]
        h.oracle_topk_batch.restype = ctypes.c_int
        h.oracle_num_threads.argtypes = []
        h.oracle_num_threads.restype = ctypes.c_int
        _h = h
    return _h


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


class Index:
    """The raw (uncompressed) inputs the oracle reads."""

    def __init__(self, ad_emb, key_offsets, post_ids, post_w):
        self.ad_emb = _c(ad_emb, np.float32)
        self.key_offsets = _c(key_offsets, np.int64)
        self.post_ids = _c(post_ids, np.uint32)
        self.post_w = _c(post_w, np.float32)
        self.n_ads, self.dim = self.ad_emb.shape
        self.n_keys = len(self.key_offsets) - 1

    @classmethod
    def of(cls, wl):
        # a binary L (ids only) is the weighted form with every weight 1 (Section 3.3)
        w = wl.post_w if wl.post_w is not None else np.ones(len(wl.post_ids), np.float32)
        return cls(wl.ad_emb, wl.key_offsets, wl.post_ids, w)


def scores(ix: Index, u, keys, mult=None):
    """FP64 (deep, wide, cond) over all ads for one query."""
    u = _c(u, np.float32)
    keys = _c(keys, np.int32)
    mult = _c(mult, np.float32)
    deep = np.empty(ix.n_ads)
    wide = np.empty(ix.n_ads)
    cond = np.empty(ix.n_ads)
    rc = _lib().oracle_scores(ix.n_ads, ix.dim, _ptr(ix.ad_emb), ix.n_keys, _ptr(ix.key_offsets),
                              _ptr(ix.post_ids), _ptr(ix.post_w), _ptr(u), len(keys),
                              _ptr(keys), _ptr(mult), _ptr(deep), _ptr(wide), _ptr(cond))
    if rc:
        raise ValueError("oracle_scores: key or posting id out of range")
    return deep, wide, cond


def topk(ix: Index, u, keys, k, mult=None):
    """Top-k of one query: dict of ids (uint32), score, cond, deep, wide (FP64)."""
    u = _c(u, np.float32)
    keys = _c(keys, np.int32)
    mult = _c(mult, np.float32)
    k = int(k)
    out = {n: np.empty(k) for n in ("score", "cond", "deep", "wide")}
    out["ids"] = np.empty(k, dtype=np.uint32)
    rc = _lib().oracle_topk(ix.n_ads, ix.dim, _ptr(ix.ad_emb), ix.n_keys, _ptr(ix.key_offsets),
                            _ptr(ix.post_ids), _ptr(ix.post_w), _ptr(u), len(keys), _ptr(keys),
                            _ptr(mult), k, _ptr(out["ids"]), _ptr(out["score"]),
                            _ptr(out["cond"]), _ptr(out["deep"]), _ptr(out["wide"]))
    if rc:
        raise ValueError("oracle_topk: bad input")
    return out


def topk_batch(ix: Index, user_emb, feat_offsets, feat_keys, kq, feat_mult=None):
    """Top-K of every query of a batch (OpenMP over queries): dict of ids (uint32), score and
    cond (FP64), each of sum K entries, plus the offsets (query q: [off[q], off[q+1]))."""
    U = _c(user_emb, np.float32).reshape(-1, ix.dim)
    fo = _c(feat_offsets, np.int64)
    fk = _c(feat_keys, np.int32)
    fm = _c(feat_mult, np.float32)
    kq = _c(kq, np.int32)
    B = U.shape[0]
    if len(fo) != B + 1 or len(kq) != B:
        raise ValueError("oracle_topk_batch: batch arrays disagree")
    off = np.zeros(B + 1, np.int64)
    off[1:] = np.cumsum(kq)
    n = int(off[-1])
    out = {"ids": np.empty(n, np.uint32), "score": np.empty(n), "cond": np.empty(n), "offsets": off}
    if fk is None:
        fk = np.zeros(0, np.int32)
    rc = _lib().oracle_topk_batch(ix.n_ads, ix.dim, _ptr(ix.ad_emb), ix.n_keys, _ptr(ix.key_offsets),
                                  _ptr(ix.post_ids), _ptr(ix.post_w), B, _ptr(U), _ptr(fo), _ptr(fk),
                                  _ptr(fm), _ptr(kq), _ptr(off), _ptr(out["ids"]), _ptr(out["score"]),
                                  _ptr(out["cond"]))
    if rc:
        raise ValueError("oracle_topk_batch: bad input")
    return out


def topk_query(wl, q: int, k=None):
    """Top-k of query q of a workload-like object (see workloads.Workload)."""
    ix = getattr(wl, "_oracle_index", None)
    if ix is None:
        ix = Index.of(wl)
        try:
            wl._oracle_index = ix
        except AttributeError:
            pass
    kk = int(wl.k[q]) if k is None else int(k)
    mult = None if wl.feat_mult is None else wl.query_mults(q)
    return topk(ix, wl.user_emb[q], wl.query_keys(q), kk, mult)


def num_threads() -> int:
    return int(_lib().oracle_num_threads())


# ------------------------------------------------------------------------------------------
# Dense brute force (tiny inputs): the sparse product written as a dense one.
# ------------------------------------------------------------------------------------------

def dense_weight_table(key_offsets, post_ids, post_w, n_ads):
    """W[V x N] FP64 with W[k, a] = weight of ad a in key k's list (0 if absent)."""
    V = len(key_offsets) - 1
    W = np.zeros((V, n_ads))
    for k in range(V):
        s, e = int(key_offsets[k]), int(key_offsets[k + 1])
        W[k, post_ids[s:e].astype(np.int64)] = post_w[s:e].astype(np.float64)
    return W


def dense_scores(ad_emb, key_offsets, post_ids, post_w, user_emb, feat_offsets, feat_keys,
                 feat_mult=None):
    """FP64 (deep[B x N], wide[B x N]) by two dense products: U E^T and M W."""
    E = np.asarray(ad_emb, dtype=np.float64)
    U = np.asarray(user_emb, dtype=np.float64)
    N = E.shape[0]
    W = dense_weight_table(key_offsets, post_ids, post_w, N)
    B = U.shape[0]
    M = np.zeros((B, W.shape[0]))
    for q in range(B):
        for j in range(int(feat_offsets[q]), int(feat_offsets[q + 1])):
            M[q, int(feat_keys[j])] += 1.0 if feat_mult is None else float(feat_mult[j])
    return U @ E.T, M @ W
