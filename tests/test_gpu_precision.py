"""GPU parity of the reduced-precision scans (BF16, FP8-e4m3 with per-ad scales).

The scan ranks ads by approximate scores; the rescore_factor * K best are rescored exactly
in FP32 and the top K returned, with a recall certificate per query (queries that fail it
rerun the FP32 scan). The returned results must therefore meet the same criteria against
the FP64 oracle as the FP32 path: scores within 1e-5, the id set exact up to tolerance ties,
recall@K = 1.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import check_topk

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2511_22460_amd")

ALL = 1 | (1 << 1) | (1 << 2)


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def run(ix, wl, **kw):
    ids, sc, offs = ix.topk_workload(wl, **kw)
    torch.cuda.synchronize()
    return ids.cpu().numpy().view(np.uint32), sc.cpu().numpy(), offs


def check_all(wl, ids, sc, offs, qs=None, exact=False, label=""):
    oix = oracle.Index.of(wl)
    rec = []
    for q in (range(wl.n_queries) if qs is None else qs):
        mult = None if wl.feat_mult is None else wl.query_mults(q)
        d, w, _ = oracle.scores(oix, wl.user_emb[q], wl.query_keys(q), mult)
        a, b = offs[q], offs[q + 1]
        rec.append(check_topk(ids[a:b], sc[a:b], int(wl.k[q]), d + w, exact=exact,
                              label=f"{label} query {q}"))
    assert min(rec) == 1.0


@pytest.fixture(scope="module")
def small():
    dev()
    wl = W.make("c1", n_ads=30_011, dim=64, n_keys=500, lengths=("zipf_draw", 1.2, 5, 8000),
                n_queries=280, feats=(0, 24), key_draw=("uniform",), k=(0, 400))
    return wl, E.Index.from_workload(wl, dtypes=ALL)


@pytest.mark.parametrize("dt", [E.BF16, E.FP8E4M3])
def test_reduced_precision_topk_matches_oracle(small, dt):
    wl, ix = small
    E.set_timing(True)
    ids, sc, offs = run(ix, wl, scan_dtype=dt, rescore_factor=4)
    t = E.last_timings()
    check_all(wl, ids, sc, offs, label=f"dtype {dt}")
    assert t["rescore_ms"] > 0


@pytest.mark.parametrize("dt", [E.BF16, E.FP8E4M3])
def test_failed_certificates_fall_back_to_fp32(small, dt):
    # one candidate per result: the certificate fails for most queries, which are rerun
    wl, ix = small
    E.set_timing(True)
    ids, sc, offs = run(ix, wl, scan_dtype=dt, rescore_factor=1)
    t = E.last_timings()
    assert t["uncertified"] > 0
    check_all(wl, ids, sc, offs, label=f"fallback dtype {dt}")


@pytest.mark.parametrize("dt", [E.BF16, E.FP8E4M3])
def test_rescored_results_equal_the_fp32_scan_bit_for_bit(small, dt):
    # the rescore computes each candidate's dot product with the FP32 scan's own FMA chain
    # and adds the scan's exact cross term, so a certified query returns exactly the FP32
    # scan's ids and score bits (an uncertified one is rerun on the FP32 scan)
    wl, ix = small
    f_ids, f_sc, f_offs = run(ix, wl)
    r_ids, r_sc, r_offs = run(ix, wl, scan_dtype=dt, rescore_factor=4)
    assert np.array_equal(f_offs, r_offs)
    assert np.array_equal(r_ids, f_ids)
    assert np.array_equal(r_sc.view(np.uint32), f_sc.view(np.uint32))


def test_precision_scan_deterministic_and_alone_equals_mix(small):
    wl, ix = small
    a1 = run(ix, wl, scan_dtype=E.FP8E4M3)
    a2 = run(ix, wl, scan_dtype=E.FP8E4M3)
    assert np.array_equal(a1[0], a2[0]) and np.array_equal(a1[1].view(np.uint32), a2[1].view(np.uint32))
    for q in (5, 200):
        s_ids, s_sc, _ = run(ix, wl, qs=[q], scan_dtype=E.FP8E4M3)
        lo, hi = a1[2][q], a1[2][q + 1]
        assert np.array_equal(s_ids, a1[0][lo:hi]) and np.array_equal(s_sc.view(np.uint32), a1[1][lo:hi].view(np.uint32))


@pytest.mark.parametrize("dt,tol", [(E.BF16, 2.0 ** -7), (E.FP8E4M3, 2.0 ** -3)])
def test_approximate_deep_term_error(small, dt, tol):
    # per-dtype error of the scan's deep term against the FP64 oracle, relative to ||u|| ||e||
    wl, ix = small
    U = torch.from_numpy(wl.user_emb[:16]).to(dev())
    nof = np.zeros(17, np.int64)
    deep, wide = ix.score_dense(U, nof, np.zeros(0, np.int32), scan_dtype=dt)
    deep = deep.cpu().numpy().astype(np.float64)
    ref = wl.user_emb[:16].astype(np.float64) @ wl.ad_emb.astype(np.float64).T
    err = np.abs(deep - ref)
    assert err.max() < tol and (wide.cpu() == 0).all()
    st = ix.stats()
    assert st["max_err_bf16"] > 0 and st["max_err_fp8"] > st["max_err_bf16"]


def test_exact_ties_survive_the_approximate_scan():
    wl = W.make("c1", n_ads=20_000, dim=32, n_keys=40, lengths=("zipf_draw", 1.05, 1000, 15000),
                n_queries=8, feats=(4, 16), key_draw=("uniform",), k=(50, 800))
    wl.post_w = np.ones_like(wl.post_w)
    wl.user_emb = np.zeros_like(wl.user_emb)
    ix = E.Index.from_workload(wl, dtypes=ALL)
    for dt in (E.BF16, E.FP8E4M3):
        ids, sc, offs = run(ix, wl, scan_dtype=dt)
        check_all(wl, ids, sc, offs, exact=True, label=f"ties dtype {dt}")


def test_missing_copy_is_unsupported():
    wl = W.make("c1", n_ads=2000, n_keys=20, n_queries=2)
    ix = E.Index.from_workload(wl)
    with pytest.raises(E.EbrError) as ei:
        ix.topk_workload(wl, scan_dtype=E.BF16)
    assert ei.value.status == E.EBR_EUNSUPPORTED


def test_c3_full_size_sampled_queries():
    """The 10M-ad inventory in BF16 and FP8 (+ FP32 master), 256 queries, K = 1000,
    4000 candidates rescored; four sampled queries checked in full."""
    dev()
    wl = W.make("c2")
    ix = E.Index.from_workload(wl, dtypes=ALL)
    for dt in (E.BF16, E.FP8E4M3):
        E.set_timing(True)
        ids, sc, offs = run(ix, wl, scan_dtype=dt, rescore_factor=4)
        check_all(wl, ids, sc, offs, qs=[0, 99, 255], label=f"c3 dtype {dt}")
