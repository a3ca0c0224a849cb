"""GPU parity of libebr against the FP64 oracle (through the C ABI).

Every case compares the library's top-K (ids, FP32 scores) with the oracle's FP64
scores of all ads under the criteria in parity.py: scores within 1e-5 relative,
the id set exact up to ties inside the tolerance band, ordering by (score desc,
id asc). Tests whose scores are exact in FP32 use a zero band (exact ids and
order). Sizes span many 32-ad tiles, ragged tails and two 256-query groups.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle_check import check_batch_vs_oracle
from parity import check_topk

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2511_22460_amd")

REL = 1e-5


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def run(ix, wl, **kw):
    ids, sc, offs = ix.topk_workload(wl, **kw)
    torch.cuda.synchronize()
    return ids.cpu().numpy().view(np.uint32), sc.cpu().numpy(), offs


def check_all(wl, ids, sc, offs, qs=None, exact=False, cond=False, label=""):
    oix = oracle.Index.of(wl)
    recalls = []
    for q in (range(wl.n_queries) if qs is None else qs):
        mult = None if wl.feat_mult is None else wl.query_mults(q)
        deep, wide, c = oracle.scores(oix, wl.user_emb[q], wl.query_keys(q), mult)
        a, b = offs[q], offs[q + 1]
        recalls.append(check_topk(ids[a:b], sc[a:b], int(wl.k[q]), deep + wide, rel_tol=REL,
                                  cond_all=c if cond else None, exact=exact,
                                  label=f"{label} query {q}"))
    assert min(recalls) == 1.0
    return recalls


def small_wl(**kw):
    base = dict(n_ads=20_017, dim=64, n_keys=600, lengths=("zipf_draw", 1.2, 5, 6000),
                n_queries=300, feats=(0, 24), key_draw=("uniform",), k=(0, 300))
    base.update(kw)
    return W.make("c1", **base)


@pytest.fixture(scope="module")
def small():
    dev()
    wl = small_wl()
    return wl, E.Index.from_workload(wl)


# ----------------------------------------------------------------------------- decode

def test_decode_every_key_bit_exact(small):
    wl, ix = small
    for k in range(wl.n_keys):
        ids, w = ix.decode_key(k)
        s, e = wl.key_offsets[k], wl.key_offsets[k + 1]
        assert np.array_equal(ids.cpu().numpy().view(np.uint32), wl.post_ids[s:e]), k
        assert np.array_equal(w.cpu().numpy().view(np.uint32), wl.post_w[s:e].view(np.uint32)), k
    st = ix.stats()
    assert st["n_postings"] == wl.n_postings and st["bytes_per_posting"] < 6.0
    # the range hook: every list at once, an inner range, an empty range, a bad range
    ids, w = ix.decode_keys(0, wl.n_keys)
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), wl.post_ids)
    assert np.array_equal(w.cpu().numpy().view(np.uint32), wl.post_w.view(np.uint32))
    ids, w = ix.decode_keys(7, 300)
    s, e = wl.key_offsets[7], wl.key_offsets[300]
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), wl.post_ids[s:e])
    assert ix.decode_keys(5, 5)[0].numel() == 0
    with pytest.raises(E.EbrError):
        ix.decode_keys(10, wl.n_keys + 1)


# ----------------------------------------------------------------------------- dense terms

@pytest.mark.parametrize("dim", [16, 48, 64, 128])
def test_dense_terms_match_oracle(dim):
    wl = small_wl(dim=dim, n_ads=3001, n_queries=40, feats=(0, 12))
    rng = np.random.default_rng(dim)
    wl.feat_mult = rng.normal(0, 3, size=len(wl.feat_keys)).astype(np.float32)
    ix = E.Index.from_workload(wl)
    U = torch.from_numpy(wl.user_emb).to(dev())
    deep, wide = ix.score_dense(U, wl.feat_offsets, wl.feat_keys, wl.feat_mult)
    deep, wide = deep.cpu().numpy().astype(np.float64), wide.cpu().numpy().astype(np.float64)
    oix = oracle.Index.of(wl)
    maxw = np.array([np.abs(wl.post_w[wl.key_offsets[k]:wl.key_offsets[k + 1]]).max(initial=0.0)
                     for k in range(wl.n_keys)])
    for q in range(wl.n_queries):
        d, w, c = oracle.scores(oix, wl.user_emb[q], wl.query_keys(q), wl.query_mults(q))
        # FP32 dot: <= d * 2^-24 of the magnitude c. Cross term: each term round(fl(m' w')) at
        # the query's scale 2^S (2^-S <= 2^-29 A, A = sum_j |m_j| max|W[k_j, :]|) errs by
        # 2^-24 |m w| + 2^-(S+1); the exact int32 sum of F terms is converted with one FP32
        # rounding: |error| <= 2^-24 |w| + 2^-24 A + F 2^-30 A.
        A = float(np.sum(np.abs(wl.query_mults(q)) * maxw[wl.query_keys(q)]))
        F = len(wl.query_keys(q))
        assert np.all(np.abs(deep[q] - d) <= 2.0 ** -18 * c)
        assert np.all(np.abs(wide[q] - w) <= 2.0 ** -22 * np.abs(w) + (2.0 ** -23 + F * 2.0 ** -29) * A)
    # additivity: the wide term does not depend on u, the deep term not on the features
    deep0, wide0 = ix.score_dense(torch.zeros_like(U), wl.feat_offsets, wl.feat_keys, wl.feat_mult)
    nof = np.zeros(wl.n_queries + 1, np.int64)
    deep1, wide1 = ix.score_dense(U, nof, np.zeros(0, np.int32))
    assert torch.equal(wide0.cpu(), torch.from_numpy(wide.astype(np.float32)))
    assert torch.equal(deep1.cpu(), torch.from_numpy(deep.astype(np.float32)))
    assert (deep0.cpu() == 0).all() and (wide1.cpu() == 0).all()


# ----------------------------------------------------------------------------- top-K

def test_topk_small_ragged_two_groups(small):
    wl, ix = small
    ids, sc, offs = run(ix, wl)
    assert offs[-1] == int(wl.k.sum())
    check_all(wl, ids, sc, offs, label="small")


def test_topk_is_deterministic_and_same_alone_as_in_a_mix(small):
    wl, ix = small
    ids1, sc1, offs = run(ix, wl)
    ids2, sc2, _ = run(ix, wl)
    assert np.array_equal(ids1, ids2) and np.array_equal(sc1.view(np.uint32), sc2.view(np.uint32))
    for q in (3, 150, 299):
        a_ids, a_sc, _ = run(ix, wl, qs=[q])
        a, b = offs[q], offs[q + 1]
        assert np.array_equal(a_ids, ids1[a:b]), q
        assert np.array_equal(a_sc.view(np.uint32), sc1[a:b].view(np.uint32)), q


@pytest.mark.parametrize("rnd", ["1", "2"])
def test_forced_selection_rounds_give_the_same_result(small, monkeypatch, rnd):
    """The threshold-revision rounds on ordinary inputs: the first threshold follows round 1's
    rule (the sample's K'-th key) or round 2's (no threshold: every ad is a candidate, the
    candidate buffer overflows on 20k ads, and the revised threshold resolves it). The result
    must be the normal path's, bit for bit, and the oracle's."""
    wl, ix = small
    ids, sc, offs = run(ix, wl)
    monkeypatch.setenv("EBR_FORCE_SELECT_ROUND", rnd)
    E.set_timing(True)
    try:
        f_ids, f_sc, _ = run(ix, wl)
        rounds = E.last_timings()["rounds"]
    finally:
        E.set_timing(False)
        monkeypatch.delenv("EBR_FORCE_SELECT_ROUND")
    assert np.array_equal(f_ids, ids) and np.array_equal(f_sc.view(np.uint32), sc.view(np.uint32))
    if rnd == "2":
        assert rounds >= 2
    check_all(wl, f_ids, f_sc, offs, qs=range(0, wl.n_queries, 7), label=f"forced round {rnd}")
    # a small inventory: every ad fits the candidate buffer, so round 2's rule resolves at once
    wl2 = small_wl(n_ads=3_001, n_queries=20, k=(1, 200))
    ix2 = E.Index.from_workload(wl2)
    ids2, sc2, offs2 = run(ix2, wl2)
    monkeypatch.setenv("EBR_FORCE_SELECT_ROUND", rnd)
    try:
        g_ids, g_sc, _ = run(ix2, wl2)
    finally:
        monkeypatch.delenv("EBR_FORCE_SELECT_ROUND")
    assert np.array_equal(g_ids, ids2) and np.array_equal(g_sc.view(np.uint32), sc2.view(np.uint32))
    check_all(wl2, g_ids, g_sc, offs2, label=f"forced round {rnd}, 3k ads")


def test_small_groups_match_the_matrix_core_path_bit_for_bit(small):
    """Groups of at most 16 queries take the per-lane FMA-chain dot product; its scores must
    be the matrix-core path's bit for bit: the same queries inside a group of 40, and the
    dense hook's deep + wide (matrix-core products) for every returned ad."""
    wl, ix = small
    qs = list(range(16))
    few = run(ix, wl, qs=qs)            # one group of 16: the FMA-chain path
    many = run(ix, wl, qs=list(range(40)))  # one group of 40: the matrix-core path
    for i in qs:
        a, b = few[2][i], few[2][i + 1]
        c, d = many[2][i], many[2][i + 1]
        assert np.array_equal(few[0][a:b], many[0][c:d]), i
        assert np.array_equal(few[1][a:b].view(np.uint32), many[1][c:d].view(np.uint32)), i
    for qs1 in ([5], [0, 7, 11]):
        w = wl.subset(qs1)
        U = torch.from_numpy(np.ascontiguousarray(w.user_emb)).to(dev())
        deep, wide = ix.score_dense(U, w.feat_offsets, w.feat_keys, w.feat_mult)
        deep, wide = deep.cpu().numpy(), wide.cpu().numpy()
        ids, sc, offs = run(ix, wl, qs=qs1)
        for i in range(len(qs1)):
            sel = ids[offs[i]:offs[i + 1]].astype(np.int64)
            want = (deep[i, sel] + wide[i, sel]).astype(np.float32)
            want[want == 0] = 0.0  # -0.0 is returned as +0.0
            assert np.array_equal(sc[offs[i]:offs[i + 1]].view(np.uint32), want.view(np.uint32)), qs1


def test_topk_c1_config():
    dev()
    wl = W.make("c1")
    ix = E.Index.from_workload(wl)
    ids, sc, offs = run(ix, wl)
    check_all(wl, ids, sc, offs, label="c1")


@pytest.mark.parametrize("dim", [16, 32, 96])
def test_topk_other_dims(dim):
    wl = small_wl(dim=dim, n_ads=5000, n_queries=20, k=(1, 64))
    ix = E.Index.from_workload(wl)
    ids, sc, offs = run(ix, wl)
    check_all(wl, ids, sc, offs, label=f"d={dim}")


def test_topk_k_edge_cases():
    # K = N returns every ad, including those whose deep and wide terms cancel to near zero;
    # there the score tolerance is relative to the condition magnitude (sum of |terms|).
    wl = small_wl(n_ads=3000, n_queries=5, k=1)
    wl.k = np.array([0, 1, 3000, 2999, 17], np.int32)
    ix = E.Index.from_workload(wl)
    ids, sc, offs = run(ix, wl)
    check_all(wl, ids, sc, offs, cond=True, label="k edge")
    wl.k = np.zeros(5, np.int32)
    ids, sc, offs = ix.topk_workload(wl)
    assert offs[-1] == 0


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_topk_k_beyond_the_lds_sort(dtype):
    # K above 8192 (or rescore_factor x K above it) is answered by a full sort of the query's
    # scores; K = N returns every ad. Scores near zero make the tolerance condition-relative.
    wl = small_wl(n_ads=50_021, n_queries=6, k=1)
    wl.k = np.array([50_021, 8193, 20_000, 100, 0, 12_345], np.int32)
    ix = E.Index.from_workload(wl, dtypes=1 | (1 << E.BF16))
    sd = E.F32 if dtype == "f32" else E.BF16
    ids, sc, offs = run(ix, wl, scan_dtype=sd)
    check_all(wl, ids, sc, offs, cond=True, label=f"large K {dtype}")
    # the full-sort queries give the same result alone and in the batch
    i1, s1, _ = run(ix, wl.subset([2]), scan_dtype=sd)
    assert np.array_equal(i1, ids[offs[2]:offs[3]])
    assert np.array_equal(s1.view(np.uint32), sc[offs[2]:offs[3]].view(np.uint32))


def test_topk_exact_ties_integer_counts():
    # u = 0 and unit weights: every score is an integer hit count, exact in FP32; massive ties
    # are broken by the smaller ad id, so the result must equal the oracle's exactly.
    wl = small_wl(n_ads=40_000, n_keys=50, lengths=("zipf_draw", 1.05, 2000, 30000),
                  n_queries=12, feats=(4, 20), k=(100, 2000))
    wl.post_w = np.ones_like(wl.post_w)
    wl.user_emb = np.zeros_like(wl.user_emb)
    ix = E.Index.from_workload(wl)
    ids, sc, offs = run(ix, wl)
    check_all(wl, ids, sc, offs, exact=True, label="ties")


def test_topk_duplicated_rows_tie_to_lower_id():
    wl = small_wl(n_ads=8192, n_queries=6, feats=0, k=(50, 500))
    base = wl.ad_emb[:1024].copy()
    wl.ad_emb = np.ascontiguousarray(np.repeat(base, 8, axis=0))   # 8 identical rows each
    ix = E.Index.from_workload(wl)
    ids, sc, offs = run(ix, wl)
    check_all(wl, ids, sc, offs, label="dup rows")
    for q in range(wl.n_queries):
        r = ids[offs[q]:offs[q + 1]].astype(np.int64)
        s = sc[offs[q]:offs[q + 1]]
        for i in range(len(r) - 1):
            if s[i] == s[i + 1]:
                assert r[i] < r[i + 1]


def test_topk_cancellation_uses_condition_tolerance():
    # large opposite multipliers make s << cond for many ads
    wl = small_wl(n_ads=6000, n_queries=10, feats=(2, 10), k=(10, 200))
    rng = np.random.default_rng(9)
    wl.feat_mult = (rng.choice([-1, 1], size=len(wl.feat_keys)) * 50).astype(np.float32)
    ix = E.Index.from_workload(wl)
    ids, sc, offs = run(ix, wl)
    check_all(wl, ids, sc, offs, cond=True, label="cancel")


def test_batch_input_errors(small):
    wl, ix = small
    U = torch.from_numpy(wl.user_emb[:2]).to(dev())
    offs = np.array([0, 2, 3], np.int64)
    with pytest.raises(E.EbrError) as ei:
        ix.score_topk(U, offs, np.array([1, 1, 2], np.int32), np.array([5, 5], np.int32))
    assert ei.value.status == E.EBR_EINVAL                      # repeated key
    with pytest.raises(E.EbrError):
        ix.score_topk(U, offs, np.array([1, 2, wl.n_keys], np.int32), np.array([5, 5], np.int32))
    with pytest.raises(E.EbrError):
        ix.score_topk(U, offs, np.array([1, 2, 3], np.int32), np.array([5, wl.n_ads + 1], np.int32))
    Ubad = U.clone()
    Ubad[1, 3] = float("nan")
    with pytest.raises(E.EbrError):
        ix.score_topk(Ubad, offs, np.array([1, 2, 3], np.int32), np.array([5, 5], np.int32))


# ----------------------------------------------------------------------------- full size

@pytest.fixture(scope="module")
def c2():
    dev()
    wl = W.make("c2")
    ix = E.Index.from_workload(wl)
    return wl, ix


@pytest.mark.timeout(900)
def test_c2_full_size_every_query(c2):
    """10M ads, ~4e8 postings, 256 queries x 32 keys, K = 1000, in the benchmark's launch
    (autotuned shape): every query of the batch is checked against the oracle."""
    wl, ix = c2
    ids, sc, offs = run(ix, wl)
    assert offs[-1] == 256 * 1000
    # the benchmark autotunes the launch shape first: the tuned launch gives the same bits
    U = torch.from_numpy(np.ascontiguousarray(wl.user_emb)).to(dev())
    rep, _ = ix.autotune(U, wl.feat_offsets, wl.feat_keys, wl.k, wl.feat_mult, reps=1)
    t_ids, t_sc, _ = run(ix, wl)
    assert np.array_equal(t_ids, ids) and np.array_equal(t_sc.view(np.uint32), sc.view(np.uint32)), rep
    check_batch_vs_oracle(wl, ids, sc, offs, rel_tol=REL, label="c2")


@pytest.mark.timeout(900)
def test_c2_decode_every_key_bit_exact(c2):
    """GPU decode of all 1M lists (~4e8 postings) of the 10M-ad index, in slices of keys,
    against the arrays the index was built from: ids equal, weights equal bit for bit."""
    wl, ix = c2
    V = wl.n_keys
    step = 1 << 17
    for k0 in range(0, V, step):
        k1 = min(V, k0 + step)
        ids, w = ix.decode_keys(k0, k1)
        s, e = int(wl.key_offsets[k0]), int(wl.key_offsets[k1])
        assert ids.numel() == e - s
        assert np.array_equal(ids.cpu().numpy().view(np.uint32), wl.post_ids[s:e]), (k0, k1)
        assert np.array_equal(w.cpu().numpy().view(np.uint32), wl.post_w[s:e].view(np.uint32)), (k0, k1)
        del ids, w
    # the single-key hook agrees on the longest and the last list
    for k in (0, V - 1):
        ids, w = ix.decode_key(k)
        s, e = wl.key_offsets[k], wl.key_offsets[k + 1]
        assert np.array_equal(ids.cpu().numpy().view(np.uint32), wl.post_ids[s:e]), k
