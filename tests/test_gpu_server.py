"""GPU tests of the serving loop (ebr_server_*): single queries submitted from host memory,
batched on the device under a scratch budget, results polled back.

Every served result is checked against the FP64 oracle (parity.py rules) and must be
bit-identical to the same query run alone through ebr_score_topk: the cross term is an
exact fixed-point sum and the dot product's order does not depend on the batch, so a
query's scores do not depend on which queries share its batch.
"""
import threading

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


@pytest.fixture(scope="module")
def served():
    dev()
    wl = W.make("c1", n_ads=40_009, dim=64, n_keys=800, lengths=("zipf_draw", 1.2, 5, 8000),
                n_queries=96, feats=(0, 40), key_draw=("uniform",), k=(0, 400))
    ix = E.Index.from_workload(wl, dtypes=1 | (1 << E.BF16))
    return wl, ix


def alone(ix, wl, q, **kw):
    ids, sc, _ = ix.topk_workload(wl, qs=[q], **kw)
    torch.cuda.synchronize()
    return ids.cpu().numpy().view(np.uint32), sc.cpu().numpy()


def submit_all(srv, wl, qs):
    return {q: srv.submit(wl.user_emb[q], wl.query_keys(q), int(wl.k[q]),
                          None if wl.feat_mult is None else wl.query_mults(q)) for q in qs}


def check_served(wl, ix, results, kw=None, oracle_qs=None):
    oix = oracle.Index.of(wl)
    for q, (ids, sc) in results.items():
        a_ids, a_sc = alone(ix, wl, q, **(kw or {}))
        assert np.array_equal(ids, a_ids), f"query {q}: served ids differ from the query alone"
        assert np.array_equal(sc.view(np.uint32), a_sc.view(np.uint32)), f"query {q}: scores differ"
        if oracle_qs is None or q in oracle_qs:
            d, w, _ = oracle.scores(oix, wl.user_emb[q], wl.query_keys(q))
            assert check_topk(ids, sc, int(wl.k[q]), d + w, label=f"query {q}") == 1.0


def test_served_results_equal_alone_and_oracle(served):
    wl, ix = served
    with E.Server(ix, scratch_bytes=256 << 20, max_batch=64, max_wait_us=2000) as srv:
        t = submit_all(srv, wl, range(wl.n_queries))
        res = {q: srv.poll(tk) for q, tk in t.items()}
        st = srv.stats()
    assert st["completed"] == wl.n_queries and st["failed"] == 0
    assert st["batches"] >= 2 and st["p99_ms"] >= st["p50_ms"] > 0
    check_served(wl, ix, res)


def test_small_scratch_budget_splits_batches(served):
    wl, ix = served
    qs = list(range(48))
    # a slot that holds the largest single query but not the whole set: admission trims
    U = torch.from_numpy(wl.user_emb).to(ix.device)
    def ws(sub):
        w = wl.subset(sub)
        return ix.workspace_size(U[:len(sub)], w.feat_offsets, w.feat_keys, w.k)
    slot = max(ws([q]) for q in qs) + (2 << 20)
    assert ws(qs) > slot
    with E.Server(ix, scratch_bytes=2 * slot, max_batch=64, max_wait_us=5000, pipeline=2) as srv:
        t = submit_all(srv, wl, qs)
        res = {q: srv.poll(tk) for q, tk in t.items()}
        st = srv.stats()
    assert st["completed"] == len(qs) and st["mean_batch"] < len(qs)
    check_served(wl, ix, res, oracle_qs=set(qs[::6]))


def test_threads_submit_concurrently(served):
    wl, ix = served
    out, errs = {}, []
    with E.Server(ix, scratch_bytes=256 << 20, max_batch=32, max_wait_us=500, pipeline=3) as srv:
        def client(qs):
            try:
                for q in qs:
                    tk = srv.submit(wl.user_emb[q], wl.query_keys(q), int(wl.k[q]))
                    out[q] = srv.poll(tk)
            except Exception as e:  # reported below
                errs.append(e)
        th = [threading.Thread(target=client, args=(range(i, wl.n_queries, 4),)) for i in range(4)]
        for x in th:
            x.start()
        for x in th:
            x.join()
    assert not errs and len(out) == wl.n_queries
    check_served(wl, ix, out, oracle_qs=set(range(0, wl.n_queries, 8)))


def test_bf16_server_with_rescore(served):
    wl, ix = served
    qs = list(range(0, wl.n_queries, 3))
    kw = dict(scan_dtype=E.BF16, rescore_factor=4)
    with E.Server(ix, scratch_bytes=512 << 20, max_batch=64, max_wait_us=2000, **kw) as srv:
        t = submit_all(srv, wl, qs)
        res = {q: srv.poll(tk) for q, tk in t.items()}
    check_served(wl, ix, res, kw=kw)


def test_small_batches_on_the_fp32_scan_give_the_same_bits(served):
    # a BF16 server whose batches of at most 8 queries take the FP32 scan: queries served one
    # at a time (FP32) and in a burst (BF16 + rescore) both equal the query run alone on
    # either scan, bit for bit
    wl, ix = served
    kw = dict(scan_dtype=E.BF16, rescore_factor=4)
    with E.Server(ix, scratch_bytes=512 << 20, max_batch=64, max_wait_us=0, f32_below=8, **kw) as srv:
        res = {}
        for q in range(0, 12):  # one at a time
            res[q] = srv.poll(srv.submit(wl.user_emb[q], wl.query_keys(q), int(wl.k[q])))
        t = submit_all(srv, wl, range(12, wl.n_queries))
        res.update({q: srv.poll(tk) for q, tk in t.items()})
        st = srv.stats()
    assert st["completed"] == wl.n_queries and st["failed"] == 0
    check_served(wl, ix, res, kw=kw, oracle_qs={0, 5, 50})
    for q in (0, 7, 40, 90):
        f_ids, f_sc = alone(ix, wl, q)
        assert np.array_equal(res[q][0], f_ids) and np.array_equal(res[q][1].view(np.uint32), f_sc.view(np.uint32)), q


def test_submission_errors(served):
    wl, ix = served
    u = wl.user_emb[0]
    with E.Server(ix, scratch_bytes=64 << 20, max_batch=8) as srv:
        for keys, k, user, code in [([3, 3], 10, u, E.EBR_EINVAL),
                                    ([wl.n_keys], 10, u, E.EBR_EINVAL),
                                    ([1], 10, np.full(wl.dim, np.nan, np.float32), E.EBR_EINVAL),
                                    ([1], 8193, u, E.EBR_EINVAL),
                                    ([1], -1, u, E.EBR_EINVAL)]:
            with pytest.raises(E.EbrError) as ei:
                srv.submit(user, keys, k)
            assert ei.value.status == code
        with pytest.raises(E.EbrError) as ei:
            srv.poll(987654321, 0)
        assert ei.value.status == E.EBR_ENOTFOUND
        assert srv.stats()["submitted"] == 0
    with pytest.raises(E.EbrError) as ei:        # index has no FP8 copy
        E.Server(ix, scratch_bytes=64 << 20, scan_dtype=E.FP8E4M3)
    assert ei.value.status == E.EBR_EUNSUPPORTED


def test_query_larger_than_a_slot_is_refused(served):
    wl, ix = served
    big = np.argsort(-np.diff(wl.key_offsets))[:40].astype(np.int32)   # the longest lists
    one = ix.workspace_size(torch.zeros(1, wl.dim, device=ix.device), [0, 0], [], [10])
    with E.Server(ix, scratch_bytes=2 * (one + (1 << 20)), max_batch=8) as srv:
        with pytest.raises(E.EbrError) as ei:
            srv.submit(wl.user_emb[0], big, 10)
        assert ei.value.status == E.EBR_ENOMEM
        tk = srv.submit(wl.user_emb[0], big[:1], 10)     # a small query still runs
        ids, sc = srv.poll(tk)
        assert len(ids) == 10


def test_destroy_drains_unpolled_tickets(served):
    wl, ix = served
    srv = E.Server(ix, scratch_bytes=128 << 20, max_batch=16, max_wait_us=100000)
    held = []
    for q in range(20):
        t = srv.submit(wl.user_emb[q], wl.query_keys(q), int(wl.k[q]))
        held.append((q, t, srv._pending[t]))
    srv.close()                      # waits for every queued query
    for q, t, (ids, sc, k) in held:
        a_ids, a_sc = alone(ix, wl, q)
        assert np.array_equal(ids[:k], a_ids)


def test_full_queue_returns_eagain_then_accepts_after_polling(served):
    wl, ix = served
    # one slot, batches of up to 64 and a long batching window: the worker holds off for a
    # full second, so the first two submissions stay queued and the third finds the queue full
    with E.Server(ix, scratch_bytes=256 << 20, max_batch=64, max_wait_us=1_000_000, pipeline=1,
                  max_queue=2) as srv:
        t0 = srv.submit(wl.user_emb[0], wl.query_keys(0), int(wl.k[0]))
        t1 = srv.submit(wl.user_emb[1], wl.query_keys(1), int(wl.k[1]))
        with pytest.raises(E.EbrError) as ei:
            srv.submit(wl.user_emb[2], wl.query_keys(2), int(wl.k[2]))
        assert ei.value.status == E.EBR_EAGAIN
        st = srv.stats()
        assert st["rejected"] == 1 and st["submitted"] == 2
        res = {0: srv.poll(t0), 1: srv.poll(t1)}
        # the queue has drained into a batch: the same query is accepted now
        t2 = srv.submit(wl.user_emb[2], wl.query_keys(2), int(wl.k[2]))
        res[2] = srv.poll(t2)
        assert srv.stats()["completed"] == 3
    check_served(wl, ix, res)


def test_injected_device_fault_reaches_every_ticket_of_its_batch(served, monkeypatch):
    wl, ix = served
    # batch 1 (the second) fails: its four tickets get EBR_EDEVICE, batches 0 and 2 are served
    monkeypatch.setenv("EBR_FAULT_BATCH", "1")
    with E.Server(ix, scratch_bytes=256 << 20, max_batch=4, max_wait_us=5_000_000, pipeline=1) as srv:
        monkeypatch.delenv("EBR_FAULT_BATCH")
        outcome = {}
        for b in range(3):
            qs = list(range(4 * b, 4 * b + 4))
            t = submit_all(srv, wl, qs)   # four queries: a full batch, launched at once
            for q, tk in t.items():
                try:
                    outcome[q] = srv.poll(tk)
                except E.EbrError as e:
                    outcome[q] = e.status
        st = srv.stats()
    failed = sorted(q for q, r in outcome.items() if not isinstance(r, tuple))
    assert failed == [4, 5, 6, 7]
    assert all(outcome[q] == E.EBR_EDEVICE for q in failed)
    assert st["failed"] == 4 and st["completed"] == 8 and st["batches"] == 3
    check_served(wl, ix, {q: r for q, r in outcome.items() if isinstance(r, tuple)})


@pytest.mark.timeout(900)
def test_served_50m_inventory_matches_the_oracle():
    """The serving inventory: 50M ads x 64-d (FP32 master + BF16 scan copy), ~1.5e9 postings,
    resident on one GPU; queries with 4..128 features and K in {100, 500, 2000} submitted as
    the serving benchmark does (BF16 scan with 4 K rescored, batches of at most 16 queries on
    the FP32 scan): a burst of 40 (batched on the BF16 scan) and four singles. Twelve served
    results, from the burst and the singles, are checked against the oracle."""
    from oracle_check import check_batch_vs_oracle
    dev()
    wl = W.make("c5", n_queries=44)
    assert wl.n_ads == 50_000_000 and wl.n_postings > 1_400_000_000
    assert set(int(k) for k in wl.k) <= {100, 500, 2000}
    ix = E.Index.from_workload(wl, dtypes=1 | (1 << E.BF16))
    with E.Server(ix, scratch_bytes=8 << 30, max_batch=256, max_wait_us=20_000, pipeline=2,
                  scan_dtype=E.BF16, rescore_factor=4, f32_below=16) as srv:
        t = submit_all(srv, wl, range(40))
        res = {q: srv.poll(tk) for q, tk in t.items()}
        st_burst = srv.stats()
        for q in range(40, 44):
            res[q] = srv.poll(srv.submit(wl.user_emb[q], wl.query_keys(q), int(wl.k[q])))
        st = srv.stats()
    assert st["completed"] == 44 and st["failed"] == 0
    assert st_burst["mean_batch"] > 16, st_burst   # the burst ran on the BF16 scan
    qs = [0, 7, 13, 21, 29, 35, 38, 39, 40, 41, 42, 43]
    sub = wl.subset(qs)
    ids = np.concatenate([res[q][0] for q in qs])
    sc = np.concatenate([res[q][1] for q in qs])
    offs = np.zeros(len(qs) + 1, np.int64)
    offs[1:] = np.cumsum(sub.k)
    del ix
    check_batch_vs_oracle(sub, ids, sc, offs, label="served 50M")
