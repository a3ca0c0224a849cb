"""GPU parity for uneven batches: several 256-query groups in one launch, per-query feature
counts U{4..128} and K U{100..2000} (the uneven-batching workload), on FP32 and on the
reduced-precision scans with exact rescoring."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle_check import check_batch_vs_oracle
from parity import check_topk

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2511_22460_amd")

ALL = 1 | (1 << 1) | (1 << 2)


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def check(wl, ids, sc, offs, qs):
    oix = oracle.Index.of(wl)
    for q in qs:
        d, w, _ = oracle.scores(oix, wl.user_emb[q], wl.query_keys(q))
        a, b = offs[q], offs[q + 1]
        assert check_topk(ids[a:b], sc[a:b], int(wl.k[q]), d + w, label=f"query {q}") == 1.0


@pytest.fixture(scope="module")
def uneven():
    dev()
    wl = W.make("c4", n_ads=300_007, n_keys=40_000, lengths=("rank_power", 3e4, 0.64, 10, 30_000),
                n_queries=700)
    return wl, E.Index.from_workload(wl, dtypes=ALL)


@pytest.mark.parametrize("dt", [E.F32, E.BF16, E.FP8E4M3])
def test_uneven_batch_three_groups(uneven, dt):
    wl, ix = uneven
    assert np.diff(wl.feat_offsets).min() >= 4 and np.diff(wl.feat_offsets).max() <= 128
    ids, sc, offs = ix.topk_workload(wl, scan_dtype=dt, rescore_factor=4)
    torch.cuda.synchronize()
    ids, sc = ids.cpu().numpy().view(np.uint32), sc.cpu().numpy()
    rng = np.random.default_rng(int(dt))
    qs = sorted(set(rng.choice(wl.n_queries, 40, replace=False).tolist()) | {0, 255, 256, 511, 512, 699})
    check(wl, ids, sc, offs, qs)


def test_uneven_batch_equals_queries_run_alone(uneven):
    wl, ix = uneven
    ids, sc, offs = ix.topk_workload(wl)
    ids, sc = ids.cpu().numpy(), sc.cpu().numpy()
    for q in (7, 300, 650):
        a_ids, a_sc, _ = ix.topk_workload(wl, qs=[q])
        lo, hi = offs[q], offs[q + 1]
        assert np.array_equal(a_ids.cpu().numpy(), ids[lo:hi])
        assert np.array_equal(a_sc.cpu().numpy().view(np.uint32), sc[lo:hi].view(np.uint32))


def c4_check_queries(wl, n=64):
    """At least n queries of the 4096: the extremes of K (largest, smallest) and of the feature
    count, the edges of the first and last query groups, then an even spread."""
    F = np.diff(wl.feat_offsets)
    K = wl.k
    pick = {0, 255, 256, 2047, 2048, 3839, 3840, 4095}
    for arr in (K, F):
        pick |= set(np.nonzero(arr == arr.max())[0][:4].tolist())
        pick |= set(np.nonzero(arr == arr.min())[0][:4].tolist())
    pick |= set(np.linspace(0, wl.n_queries - 1, n).astype(int).tolist())
    return sorted(pick)


@pytest.mark.timeout(900)
def test_c4_full_size_checked_queries():
    """4096 queries in one launch over the 10M-ad inventory (BF16 scan, 4 K rescored), in the
    benchmark's launch configuration: autotuned shape, kernels captured in a graph; the eager
    path gives the same bits. At least 64 queries, with K = 2000 and F = 128 among them, are
    checked against the oracle."""
    dev()
    base = W.make("c2")
    wl = W.queries_for(base, "c4")
    ix = E.Index.from_workload(wl, dtypes=1 | (1 << 1))
    U = torch.from_numpy(np.ascontiguousarray(wl.user_emb)).to(dev())
    rep, _ = ix.autotune(U, wl.feat_offsets, wl.feat_keys, wl.k, wl.feat_mult, scan_dtype=E.BF16,
                         rescore_factor=4, reps=1)
    assert ix.launch_shape(E.BF16, wl.n_queries) == rep["best"]
    g = E.Graph()
    ids, sc, offs = ix.topk_workload(wl, scan_dtype=E.BF16, rescore_factor=4, graph=g)
    torch.cuda.synchronize()
    assert offs[-1] == int(wl.k.sum())
    ids, sc = ids.cpu().numpy().view(np.uint32), sc.cpu().numpy()
    qs = c4_check_queries(wl)
    assert len(qs) >= 64
    assert int(wl.k[qs].max()) == 2000 and int(np.diff(wl.feat_offsets)[qs].max()) == 128
    check_batch_vs_oracle(wl, ids, sc, offs, qs=qs, label="c4")
    e_ids, e_sc, _ = ix.topk_workload(wl, scan_dtype=E.BF16, rescore_factor=4)
    assert np.array_equal(e_ids.cpu().numpy().view(np.uint32), ids)
    assert np.array_equal(e_sc.cpu().numpy().view(np.uint32), sc.view(np.uint32))
    g.close()
