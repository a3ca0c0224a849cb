"""Batches of several query groups with split buckets: the batch's keys are hot (the longest
lists, users in each work-group's LDS), warm (users found in global memory) or cold (at most
as many users as query groups: each (posting, user) pair is placed in its group's bucket with
its rounded term). The cross term is an exact integer sum, so every route gives the same
bits: a query's results do not depend on its batch, and match the FP64 oracle.

The workload makes all three kinds: 600 queries (three groups) of 40..80 keys drawn Zipf over
3,000 keys, every list 2,500 of 4,099 ads long, so that the popular keys have more users than
the groups' LDS holds (warm), the tail keys have at most three users (cold), and a tile holds
hundreds of one group's cold pairs."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import check_topk

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2511_22460_amd")


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def split_wl(n_queries=600, seed=None):
    over = dict(n_ads=4099, dim=64, n_keys=3000, lengths=("fixed", 2500), n_queries=n_queries,
                feats=(40, 80), key_draw=("zipf_rank", 1.0), k=(10, 300))
    if seed is not None:
        over["seed"] = seed
    return W.make("c1", **over)


def kinds(wl, gq=256):
    """Hot / warm / cold key counts by the planner's rules, taking keys in id order (the
    planner takes equal-length lists in order of first use): a precondition of this test,
    which needs every kind to be present, not the planner's exact split."""
    G = (wl.n_queries + gq - 1) // gq
    grp = np.repeat(np.arange(wl.n_queries) // gq, np.diff(wl.feat_offsets))
    uk, inv = np.unique(wl.feat_keys, return_inverse=True)
    cnt = np.zeros((len(uk), G), np.int64)
    np.add.at(cnt, (inv, grp), 1)
    U = cnt.sum(1)
    cold = U <= G
    hu = np.zeros(G, np.int64)
    hot = np.zeros(len(uk), bool)
    for i in range(len(uk)):
        if cold[i] or hot.sum() == 2048:
            continue
        if np.all(hu + cnt[i] <= 8192):
            hu += cnt[i]
            hot[i] = True
    return int(hot.sum()), int((~hot & ~cold).sum()), int(cold.sum())


@pytest.fixture(scope="module")
def split():
    dev()
    wl = split_wl()
    return wl, E.Index.from_workload(wl, dtypes=1 | (1 << E.BF16))


def test_workload_has_every_kind(split):
    wl, _ = split
    h, w, c = kinds(wl)
    assert h > 0 and w > 0 and c > 0, (h, w, c)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_split_batch_matches_the_oracle(split, dtype):
    wl, ix = split
    sd = E.F32 if dtype == "f32" else E.BF16
    ids, sc, offs = ix.topk_workload(wl, scan_dtype=sd)
    torch.cuda.synchronize()
    ids, sc = ids.cpu().numpy().view(np.uint32), sc.cpu().numpy()
    oix = oracle.Index.of(wl)
    for q in range(wl.n_queries):
        d, w, c = oracle.scores(oix, wl.user_emb[q], wl.query_keys(q))
        a, b = offs[q], offs[q + 1]
        assert check_topk(ids[a:b], sc[a:b], int(wl.k[q]), d + w, cond_all=c,
                          label=f"split {dtype} query {q}") == 1.0


def test_split_results_do_not_depend_on_the_batch(split):
    wl, ix = split
    ids, sc, offs = ix.topk_workload(wl)
    ids, sc = ids.cpu().numpy(), sc.cpu().numpy()
    for qs in ([0], [599], [255, 256], list(range(200, 330))):
        i2, s2, o2 = ix.topk_workload(wl, qs=qs)
        i2, s2 = i2.cpu().numpy(), s2.cpu().numpy()
        for j, q in enumerate(qs):
            assert np.array_equal(i2[o2[j]:o2[j + 1]], ids[offs[q]:offs[q + 1]])
            assert np.array_equal(s2[o2[j]:o2[j + 1]].view(np.uint32), sc[offs[q]:offs[q + 1]].view(np.uint32))


def test_split_dense_terms_equal_single_query_terms(split):
    # the dense hook walks every tile of every sub-range: the batch's wide terms equal each
    # query's own (one group, no split) bit for bit
    wl, ix = split
    U = torch.from_numpy(np.ascontiguousarray(wl.user_emb)).to(dev())
    _, wide = ix.score_dense(U, wl.feat_offsets, wl.feat_keys, wl.feat_mult)
    wide = wide.cpu().numpy()
    for q in (0, 1, 300, 599):
        s = wl.subset([q])
        _, w1 = ix.score_dense(U[q:q + 1], s.feat_offsets, s.feat_keys, s.feat_mult)
        assert np.array_equal(w1.cpu().numpy()[0].view(np.uint32), wide[q].view(np.uint32))


def test_split_with_64_bit_cells(split):
    # 128-query groups (five here), 64-bit cells: the same split, checked against the oracle
    wl, ix = split
    ids, sc, offs = ix.topk_workload(wl, wide64=True)
    torch.cuda.synchronize()
    ids, sc = ids.cpu().numpy().view(np.uint32), sc.cpu().numpy()
    oix = oracle.Index.of(wl)
    for q in range(0, wl.n_queries, 7):
        d, w, c = oracle.scores(oix, wl.user_emb[q], wl.query_keys(q))
        a, b = offs[q], offs[q + 1]
        assert check_topk(ids[a:b], sc[a:b], int(wl.k[q]), d + w, cond_all=c,
                          label=f"split wide64 query {q}") == 1.0
