"""Pins for the FP64 oracle and the workload generator (CPU only).

The oracle is checked against things other than itself:
* a dense brute force, deep = U E^T and wide = M W over the uncompressed
  cross-weight table (the product form L * w~ of Section 3.4);
* paper mode (binary L, per-feature weight w~): the cross term equals the dense
  product L w~ of Section 3.4;
* the hand-executed worked example in tests/golden/paper_mode_example.json
  (its block contents checked by properties of the id set; its scores by hand
  and by L w~);
* the batch entry point against hand-computed results and against the
  single-query entry point;
* closed forms and special cases: F empty gives plain maximum inner product
  search, u = 0 with unit weights gives integer hit counts (massive exact
  ties), one-hot embeddings give 0/1 dots, K = N is a full sort, K = 0 is empty.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W
from parity import ParityError, check_topk

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def small(**kw):
    base = dict(n_ads=3000, dim=16, n_keys=40, lengths=("zipf_draw", 1.3, 5, 2000), n_queries=4,
                feats=(1, 8), key_draw=("uniform",), k=50)
    base.update(kw)
    return W.make("c1", **base)


# ---------------------------------------------------------------------------- generator

def test_generator_is_deterministic_and_well_formed():
    a, b = small(), small()
    for name in ("ad_emb", "key_offsets", "post_ids", "post_w", "user_emb", "feat_offsets",
                 "feat_keys", "k"):
        assert sha(getattr(a, name)) == sha(getattr(b, name)), name
    c = small(seed=7)
    assert sha(c.post_ids) != sha(a.post_ids)
    L = np.diff(a.key_offsets)
    for k in range(a.n_keys):
        ids = a.post_ids[a.key_offsets[k]:a.key_offsets[k + 1]].astype(np.int64)
        assert (np.diff(ids) > 0).all() and (ids < a.n_ads).all()
    assert L.min() >= 5 and L.max() <= 2000
    np.testing.assert_allclose(np.linalg.norm(a.ad_emb.astype(np.float64), axis=1), 1.0, atol=1e-6)
    for q in range(a.n_queries):
        keys = a.query_keys(q)
        assert len(set(keys.tolist())) == len(keys)


def test_generator_exact_lengths_and_uniform_ids():
    lengths = np.array([1, 2, 100, 999, 1000, 0, 500])
    offs, ids, w = W.posting_lists(11, lengths, 1000)
    assert np.array_equal(np.diff(offs), lengths)
    full = ids[offs[4]:offs[5]]
    assert np.array_equal(full, np.arange(1000))
    # ids of many long lists are close to uniform over [0, N)
    offs, ids, w = W.posting_lists(3, np.full(200, 500), 10000)
    hist = np.bincount(ids // 1000, minlength=10)
    assert (np.abs(hist - 10000) < 600).all()
    assert abs(float(w.std()) - 0.1) < 0.002


def test_generator_rank_power_lengths_match_recipe():
    L = W.list_lengths(("rank_power", 1e6, 0.64, 100, 1_000_000), 1_000_000, 10_000_000, None)
    assert L[0] == 1_000_000 and L.min() == 145
    assert abs(L.sum() - 3.993e8) / 3.993e8 < 0.002


# ---------------------------------------------------------------------------- brute force

@pytest.mark.parametrize("dim", [16, 64])
def test_oracle_matches_dense_bruteforce(dim):
    wl = small(dim=dim, n_ads=2048, n_keys=64, n_queries=5)
    rng = np.random.default_rng(5)
    mult = rng.normal(0, 2, size=len(wl.feat_keys)).astype(np.float32)
    deep_d, wide_d = oracle.dense_scores(wl.ad_emb, wl.key_offsets, wl.post_ids, wl.post_w,
                                         wl.user_emb, wl.feat_offsets, wl.feat_keys, mult)
    ix = oracle.Index.of(wl)
    for q in range(wl.n_queries):
        f0, f1 = wl.feat_offsets[q], wl.feat_offsets[q + 1]
        deep, wide, cond = oracle.scores(ix, wl.user_emb[q], wl.feat_keys[f0:f1], mult[f0:f1])
        np.testing.assert_allclose(deep, deep_d[q], rtol=0, atol=1e-12)
        np.testing.assert_allclose(wide, wide_d[q], rtol=0, atol=1e-12)
        assert (cond >= np.abs(deep + wide) - 1e-12).all()
        s = deep_d[q] + wide_d[q]
        k = 77
        r = oracle.topk(ix, wl.user_emb[q], wl.feat_keys[f0:f1], k, mult[f0:f1])
        want = np.lexsort((np.arange(wl.n_ads), -s))[:k]
        assert np.array_equal(r["ids"].astype(np.int64), want)
        np.testing.assert_allclose(r["score"], s[want], rtol=0, atol=1e-12)
        np.testing.assert_allclose(r["deep"] + r["wide"], r["score"], rtol=0, atol=0)


def test_bruteforce_detects_a_dropped_posting():
    # The brute-force comparison is sensitive: removing one posting from the oracle's input
    # changes one ad's wide term by exactly that weight.
    wl = small(n_ads=1024, n_keys=8, n_queries=1, feats=8)
    ix = oracle.Index.of(wl)
    keys = wl.query_keys(0)
    _, wide_full, _ = oracle.scores(ix, wl.user_emb[0], keys)
    k = int(keys[0])
    s, e = int(wl.key_offsets[k]), int(wl.key_offsets[k + 1])
    assert e > s
    ids2 = np.delete(wl.post_ids, s)
    offs2 = wl.key_offsets.copy()
    offs2[k + 1:] -= 1
    _, wide_cut, _ = oracle.scores(oracle.Index(wl.ad_emb, offs2, ids2, np.delete(wl.post_w, s)),
                                   wl.user_emb[0], keys)
    diff = np.nonzero(wide_full != wide_cut)[0]
    assert diff.tolist() == [int(wl.post_ids[s])]
    assert wide_full[diff[0]] - wide_cut[diff[0]] == pytest.approx(float(wl.post_w[s]), abs=1e-12)


# ---------------------------------------------------------------------------- paper mode

def binary_L(lists, n_ads):
    """The feature-to-ad matrix L of the HitMatch equation (Section 3.3): L[a, k] = 1 when ad
    a carries feature value k, else 0."""
    L = np.zeros((n_ads, len(lists)))
    for k, ads in enumerate(lists):
        L[np.asarray(ads, dtype=np.int64), k] = 1.0
    return L


def test_paper_worked_example_golden():
    with open(os.path.join(GOLDEN, "paper_mode_example.json")) as f:
        ex = json.load(f)
    lists = ex["lists"]
    ids = set(lists[0])
    # The hand-built blocks of the fixture, checked by properties of the id set rather than by
    # re-running the indexing steps: a block with header h holds exactly the low bytes of the
    # list's ids whose high part is h; its size n sits in the size class g (n = 1 for g = 0,
    # 2^(g-1) < n <= 2^g otherwise); the blocks together hold every id once.
    seen = []
    for g, want in ex["expected_blocks"].items():
        g = int(g)
        for h, lows in zip(want["header"], want["values"]):
            assert sorted(lows) == sorted(v % 256 for v in ids if v // 256 == h)
            n = len(lows)
            assert (n == 1) if g == 0 else (2 ** (g - 1) < n <= 2 ** g)
            seen += [h * 256 + l for l in lows]
    assert sorted(seen) == sorted(ids)
    N = ex["n_ads"]
    keys, w_hat = ex["query"]["keys"], ex["query"]["w_hat"]
    # oracle in paper mode: W == 1, m_j = w_hat_j
    offs = np.array([0, len(lists[0])], dtype=np.int64)
    ix = oracle.Index(np.zeros((N, 16), np.float32), offs, np.array(lists[0], np.uint32),
                      np.ones(len(lists[0]), np.float32))
    deep, wide, _ = oracle.scores(ix, np.zeros(16, np.float32), keys, w_hat)
    want = np.zeros(N)
    for a, v in ex["expected_nonzero"].items():
        want[int(a)] = v
    assert np.array_equal(wide, want)
    # the same scores as the product L w~ (Section 3.4), w~ placed at the query's keys
    wt = np.zeros(len(lists))
    wt[keys] = w_hat
    assert np.array_equal(binary_L(lists, N) @ wt, want)
    assert wide[ex["padding_victim"]] == 0.0
    assert (deep == 0).all()


def test_oracle_paper_mode_equals_binary_L_product():
    # Paper mode (Section 3.3): a binary L and a per-feature weight w~_k = w_k x_k; the cross
    # term of every ad is the matrix-vector product L w~ (Section 3.4), here a dense numpy
    # product over the whole matrix.
    rng = np.random.default_rng(12)
    N, V = 5000, 30
    lists = [np.sort(rng.choice(N, size=int(rng.integers(1, 600)), replace=False)).tolist()
             for _ in range(V)]
    L = binary_L(lists, N)
    offs = np.zeros(V + 1, np.int64)
    offs[1:] = np.cumsum([len(x) for x in lists])
    ids = np.concatenate([np.array(x, np.uint32) for x in lists])
    ix = oracle.Index(np.zeros((N, 16), np.float32), offs, ids, np.ones(len(ids), np.float32))
    for trial in range(5):
        keys = rng.choice(V, size=int(rng.integers(1, 12)), replace=False)
        w_hat = rng.normal(0, 1, size=len(keys)).astype(np.float32)
        wt = np.zeros(V)
        wt[keys] = w_hat
        _, wide, _ = oracle.scores(ix, np.zeros(16, np.float32), keys.astype(np.int32), w_hat)
        np.testing.assert_allclose(wide, L @ wt, rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------- batch entry

def test_batch_oracle_hand_case():
    # Eight ads with deep(a) = u0 * a (E[a] = a e_0), two posting lists:
    # key 0 -> ads {1, 3} with weights {10, -5}; key 1 -> ads {3, 6} with weights {2, 2}.
    N, d = 8, 16
    E = np.zeros((N, d), np.float32)
    E[:, 0] = np.arange(N)
    offs = np.array([0, 2, 4], np.int64)
    ids = np.array([1, 3, 3, 6], np.uint32)
    w = np.array([10, -5, 2, 2], np.float32)
    ix = oracle.Index(E, offs, ids, w)
    U = np.zeros((4, d), np.float32)
    U[0, 0], U[2, 0] = 1.0, -1.0
    fo = np.array([0, 1, 3, 3, 3], np.int64)
    fk = np.array([0, 0, 1], np.int32)
    fm = np.array([1.0, 1.0, 0.5], np.float32)
    kq = np.array([3, 2, 4, 0], np.int32)
    r = oracle.topk_batch(ix, U, fo, fk, kq, fm)
    # q0: scores a + wide = [0, 11, 2, -2, 4, 5, 6, 7]; q1: wide = [0, 10, 0, -4, 0, 0, 1, 0];
    # q2: -a, no features; q3: K = 0
    assert r["offsets"].tolist() == [0, 3, 5, 9, 9]
    assert r["ids"].tolist() == [1, 7, 6, 1, 6, 0, 1, 2, 3]
    assert r["score"].tolist() == [11.0, 7.0, 6.0, 10.0, 1.0, 0.0, -1.0, -2.0, -3.0]


@pytest.mark.parametrize("n_queries", [3, 40])
def test_batch_oracle_equals_single_queries(n_queries):
    # 3 queries run one after another over all threads, 40 are spread over the threads
    wl = small(n_ads=5000, n_keys=50, n_queries=n_queries, feats=(0, 9), k=(0, 300))
    rng = np.random.default_rng(9)
    mult = rng.normal(0, 3, size=len(wl.feat_keys)).astype(np.float32)
    ix = oracle.Index.of(wl)
    r = oracle.topk_batch(ix, wl.user_emb, wl.feat_offsets, wl.feat_keys, wl.k, mult)
    off = r["offsets"]
    for q in range(wl.n_queries):
        f0, f1 = wl.feat_offsets[q], wl.feat_offsets[q + 1]
        one = oracle.topk(ix, wl.user_emb[q], wl.feat_keys[f0:f1], int(wl.k[q]), mult[f0:f1])
        a, b = off[q], off[q + 1]
        assert b - a == int(wl.k[q])
        assert np.array_equal(r["ids"][a:b], one["ids"])
        assert np.array_equal(r["score"][a:b], one["score"])
        assert np.array_equal(r["cond"][a:b], one["cond"])
    with pytest.raises(ValueError):
        oracle.topk_batch(ix, wl.user_emb, wl.feat_offsets, wl.feat_keys, np.full(n_queries, wl.n_ads + 1))


# ---------------------------------------------------------------------------- special cases

def test_no_features_is_exact_mips():
    wl = small(n_ads=4096, dim=64)
    ix = oracle.Index.of(wl)
    u = wl.user_emb[0]
    r = oracle.topk(ix, u, np.zeros(0, np.int32), 200)
    dots = wl.ad_emb.astype(np.float64) @ u.astype(np.float64)
    want = np.lexsort((np.arange(wl.n_ads), -dots))[:200]
    assert np.array_equal(r["ids"].astype(np.int64), want)
    np.testing.assert_allclose(r["score"], dots[want], rtol=0, atol=1e-13)
    assert (r["wide"] == 0).all()


def test_unit_weights_zero_user_give_integer_counts_and_id_tiebreak():
    wl = small(n_ads=1500, n_keys=20, lengths=("zipf_draw", 1.1, 50, 1500), n_queries=3,
               feats=(5, 12))
    ones = np.ones_like(wl.post_w)
    ix = oracle.Index(wl.ad_emb, wl.key_offsets, wl.post_ids, ones)
    for q in range(wl.n_queries):
        keys = wl.query_keys(q)
        counts = np.zeros(wl.n_ads, np.int64)
        for k in keys:
            for a in wl.post_ids[wl.key_offsets[k]:wl.key_offsets[k + 1]]:
                counts[int(a)] += 1
        k = 300
        r = oracle.topk(ix, np.zeros(wl.dim, np.float32), keys, k)
        want = sorted(range(wl.n_ads), key=lambda a: (-counts[a], a))[:k]
        assert r["ids"].astype(np.int64).tolist() == want
        assert np.array_equal(r["score"], counts[want].astype(np.float64))


def test_one_hot_embeddings_closed_form():
    N, d = 640, 16
    E = np.zeros((N, d), np.float32)
    E[np.arange(N), np.arange(N) % d] = 1.0
    ix = oracle.Index(E, np.zeros(1, np.int64), np.zeros(0, np.uint32), np.zeros(0, np.float32))
    for j in (0, 5, 15):
        u = np.zeros(d, np.float32)
        u[j] = 2.5
        deep, wide, _ = oracle.scores(ix, u, np.zeros(0, np.int32))
        assert np.array_equal(deep, np.where(np.arange(N) % d == j, 2.5, 0.0))
        r = oracle.topk(ix, u, np.zeros(0, np.int32), N // d + 3)
        # the N/d ads with the hot coordinate, ascending ids, then the smallest zero-score ids
        hot = [a for a in range(N) if a % d == j]
        rest = [a for a in range(N) if a % d != j][:3]
        assert r["ids"].tolist() == hot + rest


def test_duplicated_rows_tie_to_lower_id_and_full_sort():
    rng = np.random.default_rng(3)
    base = rng.normal(size=(50, 16)).astype(np.float32)
    E = np.repeat(base, 4, axis=0)           # ads 4i..4i+3 identical
    ix = oracle.Index(E, np.zeros(1, np.int64), np.zeros(0, np.uint32), np.zeros(0, np.float32))
    u = rng.normal(size=16).astype(np.float32)
    N = len(E)
    r = oracle.topk(ix, u, np.zeros(0, np.int32), N)
    dots = E.astype(np.float64) @ u.astype(np.float64)
    assert r["ids"].tolist() == sorted(range(N), key=lambda a: (-dots[a], a))
    for i in range(0, N, 4):
        grp = r["ids"][i:i + 4]
        assert (np.diff(grp.astype(np.int64)) == 1).all()
    assert len(oracle.topk(ix, u, np.zeros(0, np.int32), 0)["ids"]) == 0


def test_additivity_of_deep_and_wide():
    wl = small(n_ads=2500, dim=32)
    ix = oracle.Index.of(wl)
    for q in range(wl.n_queries):
        keys = wl.query_keys(q)
        d1, w1, _ = oracle.scores(ix, wl.user_emb[q], keys)
        d2, w2, _ = oracle.scores(ix, wl.user_emb[q], np.zeros(0, np.int32))
        d3, w3, _ = oracle.scores(ix, np.zeros(wl.dim, np.float32), keys)
        assert np.array_equal(d1, d2) and np.array_equal(w1, w3)
        assert (w2 == 0).all() and (d3 == 0).all()


def test_bad_inputs_are_rejected():
    wl = small(n_ads=500, n_keys=5, lengths=("fixed", 10))
    ix = oracle.Index.of(wl)
    with pytest.raises(ValueError):
        oracle.scores(ix, wl.user_emb[0], np.array([5], np.int32))
    with pytest.raises(ValueError):
        oracle.topk(ix, wl.user_emb[0], np.array([0], np.int32), wl.n_ads + 1)


# ---------------------------------------------------------------------------- criteria helper

def test_parity_criteria_accept_and_reject():
    s = np.array([5.0, 4.0, 4.0, 3.0, 1.0, 0.5])
    ids = np.array([0, 1, 2], np.uint32)
    assert check_topk(ids, s[[0, 1, 2]].astype(np.float32), 3, s) == 1.0
    with pytest.raises(ParityError):          # wrong tie order
        check_topk(np.array([0, 2, 1], np.uint32), s[[0, 2, 1]], 3, s)
    with pytest.raises(ParityError):          # an ad below the band
        check_topk(np.array([0, 1, 3], np.uint32), s[[0, 1, 3]], 3, s)
    with pytest.raises(ParityError):          # a score off by more than the tolerance
        check_topk(ids, np.array([5.0, 4.0, 4.001]), 3, s)
    with pytest.raises(ParityError):          # duplicate id
        check_topk(np.array([0, 1, 1], np.uint32), s[[0, 1, 1]], 3, s)
    # near-ties inside the band may be swapped
    s2 = np.array([1.0, 1.0 + 1e-7, 0.2])
    assert check_topk(np.array([0], np.uint32), np.array([1.0]), 1, s2) == 1.0
    with pytest.raises(ParityError):          # exact mode has no band
        check_topk(np.array([0], np.uint32), np.array([1.0]), 1, s2, exact=True)


def test_parity_against_the_oracles_topk():
    from parity import check_topk_vs_oracle
    s = np.array([5.0, 4.0, 4.0 + 1e-9, 3.0, 1.0, 0.5])
    o_ids = np.array([0, 2, 1], np.int64)          # 4 + 1e-9 ranks before 4
    o_sc = s[o_ids]
    full = lambda: s
    # same set and order: decided without the full scores
    assert check_topk_vs_oracle(np.array([0, 2, 1]), s[[0, 2, 1]], 3, o_ids, o_sc,
                                lambda: pytest.fail("full scores not needed")) == 1.0
    # a swap inside the band: the set differs from nothing, order follows the returned scores
    assert check_topk_vs_oracle(np.array([0, 1, 2]), np.array([5.0, 4.0, 4.0]), 3, o_ids, o_sc, full) == 1.0
    with pytest.raises(ParityError):                # wrong order of the returned scores
        check_topk_vs_oracle(np.array([0, 1, 2]), np.array([5.0, 4.0, 4.00001]), 3, o_ids, o_sc, full)
    with pytest.raises(ParityError):                # an ad below the band: decided by full scores
        check_topk_vs_oracle(np.array([0, 2, 3]), s[[0, 2, 3]], 3, o_ids, o_sc, full)
    with pytest.raises(ParityError):                # a score off by more than the tolerance
        check_topk_vs_oracle(np.array([0, 2, 1]), np.array([5.0, 4.01, 4.0]), 3, o_ids, o_sc, full)
    with pytest.raises(ParityError):                # duplicate ids
        check_topk_vs_oracle(np.array([0, 0, 2]), s[[0, 0, 2]], 3, o_ids, o_sc, full)
