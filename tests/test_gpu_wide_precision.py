"""Cross-term precision with multipliers and weights of very different magnitudes.

The paper's multiplier of a feature is its weight times the user's statistic x (Section 3.3,
equation "hitmatch"), and the statistics it lists are clicks, click-through rates and
conversions (Section 4.1), which differ by orders of magnitude within one user. The cross
term is summed in fixed point with one quantum per query; a query whose quantum is coarse
against its returned scores must still meet the 1e-5 rule relative to each ad's own score,
so such queries are rerun with 64-bit cells (see ebr_batch.wide64). Every check here is
against the FP64 oracle, relative to |s(a)|.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import check_topk

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2511_22460_amd")

REL = 1e-5


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def mixed_wl(n_queries=24, seed=11):
    """20,017 ads, 600 keys. Per-key weight scale log-uniform in [1e-2, 10]; per query one
    multiplier of magnitude ~1e4 on a short list (5..40 ads) and the others log-uniform in
    [1e-3, 1] with random signs, so that most returned ads owe their score to small terms
    while the query's largest possible term is ~1e4 times bigger."""
    wl = W.make("c1", n_ads=20_017, dim=64, n_keys=600, lengths=("zipf_draw", 1.2, 5, 6000),
                n_queries=n_queries, feats=(8, 24), key_draw=("uniform",), k=(50, 300))
    rng = np.random.default_rng(seed)
    lens = np.diff(wl.key_offsets)
    scale = 10.0 ** rng.uniform(-2.0, 1.0, size=wl.n_keys)
    wl.post_w = (wl.post_w.astype(np.float64) * np.repeat(scale, lens)).astype(np.float32)
    short = np.nonzero((lens >= 5) & (lens <= 40))[0]
    assert len(short) > n_queries
    keys, mults = [], []
    for q in range(n_queries):
        kk = wl.query_keys(q).copy()
        cand = np.setdiff1d(short, kk)
        kk[0] = rng.choice(cand)
        m = (10.0 ** rng.uniform(-3.0, 0.0, size=len(kk))) * rng.choice([-1.0, 1.0], size=len(kk))
        m[0] = rng.choice([-1.0, 1.0]) * rng.uniform(0.5, 1.0) * 1e4
        keys.append(kk)
        mults.append(m)
    wl.feat_keys = np.concatenate(keys).astype(np.int32)
    wl.feat_mult = np.concatenate(mults).astype(np.float32)
    return wl


def check_rel(wl, ids, sc, offs, label):
    oix = oracle.Index.of(wl)
    for q in range(wl.n_queries):
        d, w, _ = oracle.scores(oix, wl.user_emb[q], wl.query_keys(q), wl.query_mults(q))
        a, b = offs[q], offs[q + 1]
        assert check_topk(ids[a:b], sc[a:b], int(wl.k[q]), d + w, rel_tol=REL,
                          label=f"{label} query {q}") == 1.0


def run(ix, wl, **kw):
    ids, sc, offs = ix.topk_workload(wl, **kw)
    torch.cuda.synchronize()
    return ids.cpu().numpy().view(np.uint32), sc.cpu().numpy(), offs


@pytest.fixture(scope="module")
def mixed():
    dev()
    wl = mixed_wl()
    return wl, E.Index.from_workload(wl, dtypes=1 | (1 << E.BF16) | (1 << E.FP8E4M3))


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_mixed_magnitudes_meet_the_per_ad_tolerance(mixed, dtype):
    wl, ix = mixed
    sd = {"f32": E.F32, "bf16": E.BF16, "fp8": E.FP8E4M3}[dtype]
    E.set_timing(True)
    try:
        ids, sc, offs = run(ix, wl, scan_dtype=sd)
        t = E.last_timings()
    finally:
        E.set_timing(False)
    # the coarse queries went through the 64-bit rerun (the 32-bit quantum here is ~1e-5 of
    # a typical returned score, above the 2^-18 acceptance bound)
    assert t["imprecise"] > 0
    check_rel(wl, ids, sc, offs, f"mixed {dtype}")


def test_mixed_results_do_not_depend_on_the_batch(mixed):
    wl, ix = mixed
    ids, sc, offs = run(ix, wl)
    for q in (0, 7, 23):
        i1, s1, o1 = run(ix, wl.subset([q]))
        assert np.array_equal(i1, ids[offs[q]:offs[q + 1]])
        assert np.array_equal(s1.view(np.uint32), sc[offs[q]:offs[q + 1]].view(np.uint32))
    # and mixed with ordinary queries of the same index
    plain = W.make("c1", n_ads=20_017, dim=64, n_keys=600, lengths=("zipf_draw", 1.2, 5, 6000),
                   n_queries=8, feats=(8, 24), key_draw=("uniform",), k=(50, 300))
    both = W.Workload("mix", wl.n_ads, wl.dim, wl.n_keys, wl.ad_emb, wl.key_offsets, wl.post_ids,
                      wl.post_w, np.concatenate([plain.user_emb, wl.user_emb[:4]]),
                      np.concatenate([plain.feat_offsets, plain.feat_offsets[-1] + wl.feat_offsets[1:5]]),
                      np.concatenate([plain.feat_keys, wl.feat_keys[:wl.feat_offsets[4]]]).astype(np.int32),
                      np.concatenate([np.ones(len(plain.feat_keys), np.float32),
                                      wl.feat_mult[:wl.feat_offsets[4]]]).astype(np.float32),
                      np.concatenate([plain.k, wl.k[:4]]).astype(np.int32))
    ib, sb, ob = run(ix, both)
    for i in range(4):
        q = 8 + i
        assert np.array_equal(ib[ob[q]:ob[q + 1]], ids[offs[i]:offs[i + 1]])
        assert np.array_equal(sb[ob[q]:ob[q + 1]].view(np.uint32), sc[offs[i]:offs[i + 1]].view(np.uint32))
    check_rel(both, ib, sb, ob, "mixed with plain")


def test_forced_64_bit_cells_match_the_oracle_and_the_rerun(mixed):
    wl, ix = mixed
    ids, sc, offs = run(ix, wl, wide64=True)
    check_rel(wl, ids, sc, offs, "wide64")
    # the automatic rerun runs exactly this path for the queries it reruns
    E.set_timing(True)
    try:
        ia, sa, _ = run(ix, wl)
        n_imp = E.last_timings()["imprecise"]
    finally:
        E.set_timing(False)
    same = sum(np.array_equal(ia[offs[q]:offs[q + 1]], ids[offs[q]:offs[q + 1]]) and
               np.array_equal(sa[offs[q]:offs[q + 1]].view(np.uint32), sc[offs[q]:offs[q + 1]].view(np.uint32))
               for q in range(wl.n_queries))
    assert n_imp > 0 and same >= n_imp
    with pytest.raises(E.EbrError):
        ix.topk_workload(wl, scan_dtype=E.BF16, wide64=True)


@pytest.mark.parametrize("dim", [64, 128])
def test_dense_64_bit_cells_bound(dim):
    # 64-bit cells: each term errs by 2^-24 |m w| (the FP32 product) plus half a quantum of
    # 2^-S <= 2^-61 A; one FP32 rounding of the sum
    wl = mixed_wl(n_queries=6)
    if dim != 64:
        wl = W.make("c1", n_ads=20_017, dim=dim, n_keys=600, lengths=("zipf_draw", 1.2, 5, 6000),
                    n_queries=6, feats=(8, 24), key_draw=("uniform",), k=(50, 300))
        wl.feat_mult = (10.0 ** np.random.default_rng(3).uniform(-3, 4, size=len(wl.feat_keys))).astype(np.float32)
    ix = E.Index.from_workload(wl)
    U = torch.from_numpy(wl.user_emb).to(dev())
    _, wide = ix.score_dense(U, wl.feat_offsets, wl.feat_keys, wl.feat_mult, wide64=True)
    wide = wide.cpu().numpy().astype(np.float64)
    oix = oracle.Index.of(wl)
    maxw = np.array([np.abs(wl.post_w[wl.key_offsets[k]:wl.key_offsets[k + 1]]).max(initial=0.0)
                     for k in range(wl.n_keys)])
    for q in range(wl.n_queries):
        _, w, c = oracle.scores(oix, wl.user_emb[q], wl.query_keys(q), wl.query_mults(q))
        A = float(np.sum(np.abs(wl.query_mults(q)) * maxw[wl.query_keys(q)]))
        F = len(wl.query_keys(q))
        assert np.all(np.abs(wide[q] - w) <= 2.0 ** -23 * np.abs(w) + 2.0 ** -23 * c + F * 2.0 ** -60 * A)
