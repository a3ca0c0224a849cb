"""The paper's binary L (Section 3.3, equation "hitmatch"): postings without weights, each
query feature carrying its multiplier w_hat = w * x (Algorithm 2's query input). The index is
built with post_w = NULL and stores ids only; the oracle is given W = 1 explicitly."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W
from parity import check_topk

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2511_22460_amd")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_golden_worked_example_on_an_ids_only_index():
    d = dev()
    with open(os.path.join(GOLDEN, "paper_mode_example.json")) as f:
        g = json.load(f)
    n = int(g["n_ads"])
    lists = g["lists"]
    offs = np.zeros(len(lists) + 1, np.int64)
    offs[1:] = np.cumsum([len(l) for l in lists])
    ids = np.concatenate([np.array(l, np.uint32) for l in lists])
    emb = np.zeros((n, 16), np.float32)
    ix = E.Index(emb, offs, ids, None)
    st = ix.stats()
    assert st["bytes_weights"] == 0
    # decoded ids exact, weights 1
    dids, dw = ix.decode_key(0)
    assert np.array_equal(dids.cpu().numpy().view(np.uint32), ids)
    assert np.all(dw.cpu().numpy() == 1.0)
    q = g["query"]
    U = torch.zeros((1, 16), dtype=torch.float32, device=d)
    fo = np.array([0, len(q["keys"])], np.int64)
    fk = np.array(q["keys"], np.int32)
    fm = np.array(q["w_hat"], np.float32)
    _, wide = ix.score_dense(U, fo, fk, fm)
    wide = wide.cpu().numpy()[0]
    want = np.zeros(n, np.float32)
    for a, v in g["expected_nonzero"].items():
        want[int(a)] = v
    assert np.array_equal(wide, want)
    assert wide[int(g["padding_victim"])] == 0.0
    # top-7: the six listed ads (0.75 each, by id), then the lowest-id ad of the zero scores
    out_ids, out_sc, _ = ix.score_topk(U, fo, fk, np.array([7], np.int32), fm)
    got = out_ids.cpu().numpy().view(np.uint32)
    assert list(got) == sorted(int(a) for a in g["expected_nonzero"]) + [0]
    assert list(out_sc.cpu().numpy()) == [0.75] * 6 + [0.0]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_binary_L_batch_matches_the_oracle(dtype):
    dev()
    wl = W.make("c1", n_ads=30_011, dim=64, n_keys=500, lengths=("zipf_draw", 1.2, 5, 8000),
                n_queries=60, feats=(1, 24), key_draw=("uniform",), k=(10, 400))
    rng = np.random.default_rng(5)
    # w_hat = w * x: a learned weight times a user statistic, either sign
    wl.feat_mult = (rng.normal(0, 0.5, size=len(wl.feat_keys)) *
                    rng.uniform(0.1, 3.0, size=len(wl.feat_keys))).astype(np.float32)
    ones = np.ones_like(wl.post_w)
    ix = E.Index(wl.ad_emb, wl.key_offsets, wl.post_ids, None, dtypes=1 | (1 << E.BF16))
    full = E.Index(wl.ad_emb, wl.key_offsets, wl.post_ids, ones, dtypes=1 | (1 << E.BF16))
    assert ix.stats()["arena_bytes"] < full.stats()["arena_bytes"]
    sd = E.F32 if dtype == "f32" else E.BF16
    ids, sc, offs = ix.topk_workload(wl, scan_dtype=sd)
    torch.cuda.synchronize()
    ids, sc = ids.cpu().numpy().view(np.uint32), sc.cpu().numpy()
    # the same results as an index that stores the unit weights explicitly
    i2, s2, _ = full.topk_workload(wl, scan_dtype=sd)
    assert np.array_equal(ids, i2.cpu().numpy().view(np.uint32))
    assert np.array_equal(sc.view(np.uint32), s2.cpu().numpy().view(np.uint32))
    oix = oracle.Index(wl.ad_emb, wl.key_offsets, wl.post_ids, ones)
    for q in range(wl.n_queries):
        d_, w_, c_ = oracle.scores(oix, wl.user_emb[q], wl.query_keys(q), wl.query_mults(q))
        a, b = offs[q], offs[q + 1]
        assert check_topk(ids[a:b], sc[a:b], int(wl.k[q]), d_ + w_, rel_tol=1e-5, cond_all=c_,
                          label=f"binary L {dtype} query {q}") == 1.0
