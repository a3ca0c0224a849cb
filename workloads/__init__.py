"""Seeded synthetic workloads shaped like the paper's ad-retrieval setting.

The paper evaluates on proprietary WeChat ad logs (Section 4.1, "Datasets");
nothing of that data is available, so every input here is synthetic and
seeded. The recipes follow the workload shapes the method is measured on:

* ad embeddings: N(0, 1) per element, each row L2-normalised, stored FP32
  (the towers are 64-d, Section 4.1 "Implementation details");
* posting lists (the columns of the binary feature-to-ad matrix L of the
  HitMatch equation, Section 3.3): per key an exact-length, sorted, uniformly
  random set of distinct ad ids, each with an FP32 cross weight N(0, 0.1);
* queries: a user embedding drawn like an ad row, a set of distinct user
  feature values (keys), and a per-query K.

This module generates inputs only. It holds none of the scoring, ranking or
index arithmetic: the FP64 oracle and the GPU library both consume its output
and share nothing else. Large arrays come from ``gen.c`` (a counter-based
generator, so results do not depend on thread count); small per-query draws
use numpy's ``Generator`` seeded from ``SeedSequence(251122460 + c)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libworkloads.so")
_lib_handle = None

BASE_SEED = 251122460


def build(force: bool = True) -> str:
    """Compile the generator helper with gcc (OpenMP). Returns the .so path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB):
            build(force=False)
        h = ctypes.CDLL(_LIB)
        h.wl_normal_rows.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                     ctypes.c_int32, ctypes.c_void_p]
        h.wl_normal_rows.restype = None
        h.wl_lists.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                               ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
        h.wl_lists.restype = ctypes.c_int
        _lib_handle = h
    return _lib_handle


def normal_rows(seed: int, tag: int, n: int, d: int) -> np.ndarray:
    """n x d FP32 rows of N(0,1) draws, each row L2-normalised."""
    out = np.empty((n, d), dtype=np.float32)
    if n and d:
        _lib().wl_normal_rows(seed, tag, n, d, out.ctypes.data)
    return out


def posting_lists(seed: int, lengths: np.ndarray, n_ads: int, w_sigma: float = 0.1):
    """Exact-length sorted distinct uniform id lists plus N(0, w_sigma) FP32 weights."""
    lengths = np.asarray(lengths, dtype=np.int64)
    if (lengths > n_ads).any() or (lengths < 0).any():
        raise ValueError("list length outside [0, n_ads]")
    offsets = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    total = int(offsets[-1])
    ids = np.empty(total, dtype=np.uint32)
    w = np.empty(total, dtype=np.float32)
    rc = _lib().wl_lists(seed, len(lengths), offsets.ctypes.data, n_ads, float(w_sigma),
                         ids.ctypes.data, w.ctypes.data)
    if rc != 0:
        raise MemoryError("posting list generation failed")
    return offsets, ids, w


@dataclass
class Workload:
    """One seeded index plus one query batch. All arrays live in host memory."""
    name: str
    n_ads: int
    dim: int
    n_keys: int
    ad_emb: np.ndarray          # float32 [n_ads, dim], row-major
    key_offsets: np.ndarray     # int64 [n_keys + 1], CSR over postings
    post_ids: np.ndarray        # uint32, strictly increasing within a key
    post_w: Optional[np.ndarray]  # float32, same length; None for a binary L (ids only)
    user_emb: np.ndarray        # float32 [B, dim]
    feat_offsets: np.ndarray    # int64 [B + 1]
    feat_keys: np.ndarray       # int32, distinct within a query
    feat_mult: Optional[np.ndarray]  # float32 per feature, or None for all-ones
    k: np.ndarray               # int32 [B]
    recipe: dict = field(default_factory=dict)

    @property
    def n_queries(self) -> int:
        return int(self.user_emb.shape[0])

    @property
    def n_postings(self) -> int:
        return int(self.key_offsets[-1])

    def query_keys(self, q: int) -> np.ndarray:
        return self.feat_keys[self.feat_offsets[q]:self.feat_offsets[q + 1]]

    def query_mults(self, q: int) -> np.ndarray:
        n = int(self.feat_offsets[q + 1] - self.feat_offsets[q])
        if self.feat_mult is None:
            return np.ones(n, dtype=np.float32)
        return self.feat_mult[self.feat_offsets[q]:self.feat_offsets[q + 1]]

    def subset(self, qs: Sequence[int]) -> "Workload":
        """Same index, a batch made of the listed queries (in that order)."""
        qs = [int(q) for q in qs]
        lens = [int(self.feat_offsets[q + 1] - self.feat_offsets[q]) for q in qs]
        offs = np.zeros(len(qs) + 1, dtype=np.int64)
        np.cumsum(lens, out=offs[1:])
        keys = (np.concatenate([self.query_keys(q) for q in qs]).astype(np.int32)
                if qs else np.zeros(0, np.int32))
        mult = None
        if self.feat_mult is not None:
            mult = (np.concatenate([self.query_mults(q) for q in qs]).astype(np.float32)
                    if qs else np.zeros(0, np.float32))
        return Workload(self.name + "[sub]", self.n_ads, self.dim, self.n_keys, self.ad_emb,
                        self.key_offsets, self.post_ids, self.post_w,
                        np.ascontiguousarray(self.user_emb[qs]), offs, keys, mult,
                        self.k[qs].astype(np.int32), dict(self.recipe))


# --------------------------------------------------------------------------------------------
# Recipes. Each config seeds numpy from SeedSequence(251122460 + c) and the C generator from
# the same integer seed with separate stream tags.
# --------------------------------------------------------------------------------------------

CONFIGS = {
    # Plain path, CPU-size: 100k ads, 1 query with 8 features, Zipf(1.2) list lengths
    # clipped to 10..20000, top-100.
    "c1": dict(cfg=1, n_ads=100_000, dim=64, n_keys=1000,
               lengths=("zipf_draw", 1.2, 10, 20_000),
               n_queries=1, feats=8, key_draw=("uniform",), k=100),
    # Plain FP32 at scale: 10M ads, 1M keys with rank-power lengths 100..1M (~4e8 postings),
    # 256 queries x 32 keys drawn Zipf(1.0) by rank, top-1000.
    "c2": dict(cfg=2, n_ads=10_000_000, dim=64, n_keys=1_000_000,
               lengths=("rank_power", 1e6, 0.64, 100, 1_000_000),
               n_queries=256, feats=32, key_draw=("zipf_rank", 1.0), k=1000),
    # Uneven batching: the C2 index, 4096 queries, F ~ U{4..128}, K ~ U{100..2000}.
    "c4": dict(cfg=4, n_ads=10_000_000, dim=64, n_keys=1_000_000,
               lengths=("rank_power", 1e6, 0.64, 100, 1_000_000),
               n_queries=4096, feats=(4, 128), key_draw=("zipf_rank", 1.0), k=(100, 2000)),
    # Serving inventory: 50M ads, ~1.5e9 postings, F ~ U{4..128}, K in {100, 500, 2000}.
    "c5": dict(cfg=5, n_ads=50_000_000, dim=64, n_keys=1_000_000,
               lengths=("rank_power", 3.75e6, 0.64, 100, 3_750_000),
               n_queries=2000, feats=(4, 128), key_draw=("zipf_rank", 1.0), k=[100, 500, 2000]),
}


def list_lengths(spec, n_keys: int, n_ads: int, rng: np.random.Generator) -> np.ndarray:
    kind = spec[0]
    if kind == "zipf_draw":
        _, a, lo, hi = spec
        L = np.clip(rng.zipf(a, size=n_keys), lo, hi)
    elif kind == "rank_power":
        _, l0, e, lo, hi = spec
        r = np.arange(1, n_keys + 1, dtype=np.float64)
        L = np.clip(np.round(l0 * r ** (-e)), lo, hi)
    elif kind == "fixed":
        L = np.full(n_keys, spec[1])
    else:
        raise ValueError(kind)
    return np.minimum(L.astype(np.int64), n_ads)


def _draw_count(spec, rng, n):
    if isinstance(spec, tuple):
        return rng.integers(spec[0], spec[1] + 1, size=n)
    if isinstance(spec, list):
        return rng.choice(np.asarray(spec), size=n)
    return np.full(n, int(spec))


def draw_keys(spec, n_keys: int, counts: np.ndarray, rng: np.random.Generator):
    """Per query, counts[q] distinct keys. ("zipf_rank", s): P(key = r - 1) ~ r^-s."""
    kind = spec[0]
    out = []
    cdf = None
    if kind == "zipf_rank":
        w = np.arange(1, n_keys + 1, dtype=np.float64) ** (-spec[1])
        cdf = np.cumsum(w)
        cdf /= cdf[-1]
    for c in counts:
        c = int(min(c, n_keys))
        if kind == "uniform":
            out.append(rng.choice(n_keys, size=c, replace=False).astype(np.int32))
            continue
        got: list = []
        seen = set()
        while len(got) < c:
            draws = np.searchsorted(cdf, rng.random(2 * (c - len(got)) + 4), side="right")
            for x in draws:
                x = int(min(x, n_keys - 1))
                if x not in seen:
                    seen.add(x)
                    got.append(x)
                    if len(got) == c:
                        break
        out.append(np.asarray(got, dtype=np.int32))
    return out


def queries_for(wl: Workload, name: str, **over) -> Workload:
    """A new query batch drawn with recipe `name` (its query fields: n_queries, feats,
    key_draw, k, seed) on the index of an existing workload."""
    spec = dict(CONFIGS[name])
    spec.update(over)
    seed = int(spec.get("seed", BASE_SEED + spec["cfg"]))
    ss = np.random.SeedSequence(seed)
    _, rng_q, rng_k = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3)]
    B = int(spec["n_queries"])
    U = normal_rows(seed, 2, B, wl.dim)
    counts = _draw_count(spec["feats"], rng_q, B)
    keys = draw_keys(spec["key_draw"], wl.n_keys, counts, rng_q)
    offs = np.zeros(B + 1, dtype=np.int64)
    np.cumsum([len(x) for x in keys], out=offs[1:])
    fk = np.concatenate(keys).astype(np.int32) if B else np.zeros(0, np.int32)
    kq = np.minimum(_draw_count(spec["k"], rng_k, B), wl.n_ads).astype(np.int32)
    recipe = dict(wl.recipe)
    recipe.update({"queries": name, "query_seed": seed, **{k: spec[k] for k in ("n_queries", "feats", "k")}})
    return Workload(wl.name + "+" + name, wl.n_ads, wl.dim, wl.n_keys, wl.ad_emb, wl.key_offsets,
                    wl.post_ids, wl.post_w, U, offs, fk, None, kq, recipe)


def binary(wl: Workload, seed_tag: int = 7) -> Workload:
    """The same lists and queries in the paper's binary form (Section 3.3, equation
    "hitmatch"): the lists carry ids only (post_w None, every weight 1) and each query
    feature carries its multiplier w_hat = w x, a learned weight w ~ N(0, 0.1) times a user
    statistic x ~ U(0.5, 2), drawn per (query, feature) from SeedSequence(seed + seed_tag)."""
    seed = int(wl.recipe.get("query_seed", wl.recipe.get("seed", BASE_SEED))) + seed_tag
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    n = len(wl.feat_keys)
    mult = (rng.normal(0.0, 0.1, n) * rng.uniform(0.5, 2.0, n)).astype(np.float32)
    recipe = dict(wl.recipe)
    recipe.update({"binary": True, "mult_seed": seed})
    return Workload(wl.name + "+binary", wl.n_ads, wl.dim, wl.n_keys, wl.ad_emb, wl.key_offsets,
                    wl.post_ids, None, wl.user_emb, wl.feat_offsets, wl.feat_keys, mult, wl.k,
                    recipe)


def widened(wl: Workload, dim: int, seed_tag: int = 11) -> Workload:
    """The same lists and queries with towers of width `dim` (Section 3.2: the IPNN
    concatenation lengthens both vectors): new seeded ad and user rows, N(0, 1) per element
    and L2-normalised, from seed + seed_tag."""
    seed = int(wl.recipe.get("seed", BASE_SEED)) + seed_tag
    A = normal_rows(seed, 1, wl.n_ads, dim)
    U = normal_rows(seed, 2, wl.n_queries, dim)
    recipe = dict(wl.recipe)
    recipe.update({"dim": dim, "tower_seed": seed})
    return Workload(wl.name + f"+d{dim}", wl.n_ads, dim, wl.n_keys, A, wl.key_offsets, wl.post_ids,
                    wl.post_w, U, wl.feat_offsets, wl.feat_keys, wl.feat_mult, wl.k, recipe)


def make(name: str = "c1", **over) -> Workload:
    """Build a workload from a named recipe, with optional overrides of any recipe field.

    Overridable: n_ads, dim, n_keys, lengths, n_queries, feats, key_draw, k, w_sigma, seed.
    """
    spec = dict(CONFIGS[name]) if name in CONFIGS else dict(CONFIGS["c1"])
    spec.update(over)
    seed = int(spec.get("seed", BASE_SEED + spec["cfg"]))
    n_ads, dim, n_keys = int(spec["n_ads"]), int(spec["dim"]), int(spec["n_keys"])
    ss = np.random.SeedSequence(seed)
    rng_len, rng_q, rng_k = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3)]
    lengths = list_lengths(spec["lengths"], n_keys, n_ads, rng_len)
    key_offsets, ids, w = posting_lists(seed, lengths, n_ads, float(spec.get("w_sigma", 0.1)))
    E = normal_rows(seed, 1, n_ads, dim)
    B = int(spec["n_queries"])
    U = normal_rows(seed, 2, B, dim)
    counts = _draw_count(spec["feats"], rng_q, B)
    keys = draw_keys(spec["key_draw"], n_keys, counts, rng_q)
    feat_offsets = np.zeros(B + 1, dtype=np.int64)
    np.cumsum([len(x) for x in keys], out=feat_offsets[1:])
    feat_keys = np.concatenate(keys).astype(np.int32) if B else np.zeros(0, np.int32)
    kq = np.minimum(_draw_count(spec["k"], rng_k, B), n_ads).astype(np.int32)
    recipe = {key: spec[key] for key in spec}
    recipe["seed"] = seed
    return Workload(name, n_ads, dim, n_keys, E, key_offsets, ids, w, U, feat_offsets,
                    feat_keys, None, kq, recipe)
