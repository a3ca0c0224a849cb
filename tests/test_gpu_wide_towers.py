"""Widened towers: the IPNN concatenation lengthens both the user and the ad vector
(Section 3.2), so the dot product runs at d = 96 and 128 as well as the 64 of the paper's
towers. At these widths query groups hold 128 queries (four consumer waves) and the
reduced-precision copies use the same BF16 operand layout; every path must meet the same
parity bar as at d = 64: FP32 top-K against the FP64 oracle, BF16 / FP8 scans with exact
rescoring returning the FP32 scan's bits, results independent of the batch."""
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


def run(ix, wl, **kw):
    ids, sc, offs = ix.topk_workload(wl, **kw)
    torch.cuda.synchronize()
    return ids.cpu().numpy().view(np.uint32), sc.cpu().numpy(), offs


def check_all(wl, ids, sc, offs, label):
    oix = oracle.Index.of(wl)
    for q in range(wl.n_queries):
        d, w, c = oracle.scores(oix, wl.user_emb[q], wl.query_keys(q), wl.query_mults(q))
        a, b = offs[q], offs[q + 1]
        assert check_topk(ids[a:b], sc[a:b], int(wl.k[q]), d + w, cond_all=c,
                          label=f"{label} query {q}") == 1.0


@pytest.fixture(scope="module", params=[96, 128])
def wide(request):
    dev()
    d = request.param
    # 300 queries: three 128-query groups, the last one ragged; 30,011 ads: a ragged last tile
    wl = W.make("c1", n_ads=30_011, dim=d, n_keys=500, lengths=("zipf_draw", 1.2, 5, 8000),
                n_queries=300, feats=(0, 24), key_draw=("uniform",), k=(0, 400), seed=9000 + d)
    return d, wl, E.Index.from_workload(wl, dtypes=ALL)


def test_fp32_topk(wide):
    d, wl, ix = wide
    ids, sc, offs = run(ix, wl)
    check_all(wl, ids, sc, offs, f"d={d} f32")


@pytest.mark.parametrize("dt", ["bf16", "fp8"])
def test_reduced_precision_topk_and_rescore(wide, dt):
    d, wl, ix = wide
    sd = E.BF16 if dt == "bf16" else E.FP8E4M3
    E.set_timing(True)
    try:
        ids, sc, offs = run(ix, wl, scan_dtype=sd, rescore_factor=4)
        t = E.last_timings()
    finally:
        E.set_timing(False)
    assert t["rescore_ms"] > 0
    check_all(wl, ids, sc, offs, f"d={d} {dt}")
    # the rescore reproduces the FP32 scan's bits (uncertified queries rerun on it)
    f_ids, f_sc, _ = run(ix, wl)
    assert np.array_equal(ids, f_ids)
    assert np.array_equal(sc.view(np.uint32), f_sc.view(np.uint32))


@pytest.mark.parametrize("dt", ["bf16", "fp8"])
def test_failed_certificates_fall_back(wide, dt):
    d, wl, ix = wide
    sd = E.BF16 if dt == "bf16" else E.FP8E4M3
    E.set_timing(True)
    try:
        ids, sc, offs = run(ix, wl, scan_dtype=sd, rescore_factor=1)
        t = E.last_timings()
    finally:
        E.set_timing(False)
    assert t["uncertified"] > 0
    check_all(wl, ids, sc, offs, f"d={d} {dt} fallback")


def test_alone_equals_batch(wide):
    d, wl, ix = wide
    for sd in (E.F32, E.BF16):
        ids, sc, offs = run(ix, wl, scan_dtype=sd)
        for q in (0, 127, 128, 299):
            i1, s1, _ = run(ix, wl, qs=[q], scan_dtype=sd)
            assert np.array_equal(i1, ids[offs[q]:offs[q + 1]])
            assert np.array_equal(s1.view(np.uint32), sc[offs[q]:offs[q + 1]].view(np.uint32))


@pytest.mark.parametrize("dt,tol", [("bf16", 2.0 ** -6), ("fp8", 2.0 ** -2)])
def test_approximate_deep_term_error(wide, dt, tol):
    # per-dtype deep-term error against FP64 products of the FP32 inputs
    d, wl, ix = wide
    sd = E.BF16 if dt == "bf16" else E.FP8E4M3
    U = torch.from_numpy(wl.user_emb[:8]).to(dev())
    deep, _ = ix.score_dense(U, np.zeros(9, np.int64), np.zeros(0, np.int32), scan_dtype=sd)
    ref = wl.user_emb[:8].astype(np.float64) @ wl.ad_emb.astype(np.float64).T
    assert np.abs(deep.cpu().numpy().astype(np.float64) - ref).max() < tol
