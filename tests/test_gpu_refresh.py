"""Online refresh: the index built on the GPU (ebr_build_index_device) from lists and
embeddings in device memory must be the host build's index, arena byte for byte, with the
same statistics and the same search results; invalid inputs are refused, found on the GPU."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as W
from parity import check_topk

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2511_22460_amd")

ALL = 1 | (1 << E.BF16) | (1 << E.FP8E4M3)


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def on_device(wl, d):
    ids = torch.from_numpy(wl.post_ids.view(np.int32)).to(d)
    w = torch.from_numpy(wl.post_w).to(d) if wl.post_w is not None else None
    return (torch.from_numpy(np.ascontiguousarray(wl.ad_emb)).to(d), torch.from_numpy(wl.key_offsets).to(d), ids, w)


def device_build(wl, dtypes):
    e, ko, ids, w = on_device(wl, dev())
    ix, ms = E.Index.build_on_device(e, ko, ids, w, dtypes=dtypes)
    torch.cuda.synchronize()
    return ix


def same_index(a, b):
    sa, sb = a.stats(), b.stats()
    for k in sa:
        if k not in ("encode_ms", "upload_ms"):
            assert sa[k] == sb[k], (k, sa[k], sb[k])
    n = sa["arena_bytes"]
    assert torch.equal(a.arena[:n], b.arena[:n])


@pytest.mark.parametrize("case", ["weighted_d64", "weighted_d96", "binary_d32", "empty_lists"])
def test_device_build_equals_host_build(case):
    d = dev()
    if case == "weighted_d64":
        wl = W.make("c1", n_ads=20_011, dim=64, n_keys=700, lengths=("zipf_draw", 1.2, 1, 12_000), n_queries=4)
    elif case == "weighted_d96":
        wl = W.make("c1", n_ads=5_003, dim=96, n_keys=300, lengths=("zipf_draw", 1.1, 1, 5_003), n_queries=4)
    elif case == "binary_d32":
        wl = W.binary(W.make("c1", n_ads=30_001, dim=32, n_keys=500, lengths=("zipf_draw", 1.2, 1, 20_000),
                             n_queries=4))
    else:
        wl = W.make("c1", n_ads=4_099, dim=64, n_keys=200, lengths=("zipf_draw", 1.3, 1, 300), n_queries=4)
        lens = np.diff(wl.key_offsets)
        keep = np.ones(wl.n_postings, bool)
        for k in range(0, wl.n_keys, 3):  # every third list emptied
            keep[wl.key_offsets[k]:wl.key_offsets[k + 1]] = False
            lens[k] = 0
        wl.post_ids, wl.post_w = wl.post_ids[keep], wl.post_w[keep]
        wl.key_offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    host = E.Index.from_workload(wl, dtypes=ALL)
    devx = device_build(wl, ALL)
    same_index(host, devx)


def test_device_built_index_serves_the_same_results():
    wl = W.make("c1", n_ads=30_011, dim=64, n_keys=500, lengths=("zipf_draw", 1.2, 5, 8000),
                n_queries=40, feats=(0, 24), key_draw=("uniform",), k=(1, 300))
    host = E.Index.from_workload(wl, dtypes=ALL)
    devx = device_build(wl, ALL)
    for sd in (E.F32, E.BF16, E.FP8E4M3):
        i1, s1, o1 = host.topk_workload(wl, scan_dtype=sd)
        i2, s2, o2 = devx.topk_workload(wl, scan_dtype=sd)
        assert np.array_equal(i1.cpu().numpy(), i2.cpu().numpy())
        assert np.array_equal(s1.cpu().numpy().view(np.uint32), s2.cpu().numpy().view(np.uint32))
    ids, sc = i2.cpu().numpy().view(np.uint32), s2.cpu().numpy()
    oix = oracle.Index.of(wl)
    for q in range(wl.n_queries):
        dd, ww, c = oracle.scores(oix, wl.user_emb[q], wl.query_keys(q))
        assert check_topk(ids[o2[q]:o2[q + 1]], sc[o2[q]:o2[q + 1]], int(wl.k[q]), dd + ww, cond_all=c,
                          label=f"device-built query {q}") == 1.0


@pytest.mark.parametrize("fault", ["decreasing_ids", "id_out_of_range", "nan_weight", "nan_embedding"])
def test_device_build_refuses_invalid_input(fault):
    d = dev()
    wl = W.make("c1", n_ads=5_000, dim=32, n_keys=50, lengths=("zipf_draw", 1.2, 5, 400), n_queries=2)
    e, ko, ids, w = on_device(wl, d)
    k = int(np.argmax(np.diff(wl.key_offsets)))  # a long list
    p = int(wl.key_offsets[k]) + 3
    if fault == "decreasing_ids":
        ids[p] = ids[p - 1]
    elif fault == "id_out_of_range":
        ids[int(wl.key_offsets[k + 1]) - 1] = 5_000
    elif fault == "nan_weight":
        w[p] = float("nan")
    else:
        e[17, 5] = float("nan")
    with pytest.raises(E.EbrError) as ei:
        E.Index.build_on_device(e, ko, ids, w, dtypes=1)
    assert ei.value.status == E.EBR_EINVAL
    msg = E.load().ebr_last_error().decode()
    assert ("ad 17" in msg) if fault == "nan_embedding" else (f"key {k}" in msg), msg


def test_server_swap_queries_straddling_a_swap():
    """Queries submitted before a swap run on the old index, later ones on the new one (built
    on the GPU from refreshed lists); the swap returns only when the old index's queries have
    completed; each result matches the FP64 oracle of the index it ran on."""
    d = dev()
    old = W.make("c1", n_ads=20_011, dim=64, n_keys=400, lengths=("zipf_draw", 1.2, 5, 6000),
                 n_queries=48, feats=(1, 20), key_draw=("uniform",), k=(1, 200))
    # the refresh: same ads, new feature-to-ad lists and weights
    new = W.make("c1", n_ads=20_011, dim=64, n_keys=400, lengths=("zipf_draw", 1.2, 5, 6000),
                 n_queries=1, seed=777)
    new.ad_emb = old.ad_emb
    ix_old = E.Index.from_workload(old, dtypes=1 | (1 << E.BF16))
    ix_new = device_build(new, 1 | (1 << E.BF16))
    qs_before, qs_after = list(range(0, 24)), list(range(24, 48))
    with E.Server(ix_old, scratch_bytes=256 << 20, max_batch=8, max_wait_us=20_000, pipeline=2,
                  scan_dtype=E.BF16) as srv:
        tb = [srv.submit(old.user_emb[q], old.query_keys(q), int(old.k[q])) for q in qs_before]
        srv.swap_index(ix_new)
        # every query of the old index has completed: its results are ready without waiting
        before = [srv.poll(t, 0) for t in tb]
        assert all(r is not None for r in before)
        ta = [srv.submit(old.user_emb[q], old.query_keys(q), int(old.k[q])) for q in qs_after]
        after = [srv.poll(t) for t in ta]
        with pytest.raises(E.EbrError):  # another width: refused
            other = E.Index.from_workload(W.make("c1", n_ads=20_011, dim=32, n_keys=400, n_queries=1))
            srv.swap_index(other)
    del ix_old  # the previous index may be freed once the swap has returned
    for idx, (qs, res) in ((oracle.Index.of(old), (qs_before, before)), (oracle.Index.of(new), (qs_after, after))):
        for q, (ids, sc) in zip(qs, res):
            dd, ww, c = oracle.scores(idx, old.user_emb[q], old.query_keys(q))
            assert check_topk(ids, sc, int(old.k[q]), dd + ww, cond_all=c, label=f"swap query {q}") == 1.0
    # and the queries really ran on different lists: for some, the two indexes disagree
    o1, o2 = oracle.Index.of(old), oracle.Index.of(new)
    differ = sum(not np.allclose(sum(oracle.scores(o1, old.user_emb[q], old.query_keys(q))[:2]),
                                 sum(oracle.scores(o2, old.user_emb[q], old.query_keys(q))[:2])) for q in qs_after)
    assert differ > 0
