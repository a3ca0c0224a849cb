"""ebr_score_topk_noalloc: the top-K entry point that takes its workspace from the library's
fixed device scratch instead of a caller buffer (for callers that cannot allocate). Called
through the C ABI; its results must equal ebr_score_topk's bit for bit, on two calls in a row
(the second smaller, so the scratch holds the first call's contents), and a batch larger
than the scratch must be refused before any device work."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2511_22460_amd")


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def noalloc(ix, wl, scan_dtype=0):
    lib = E.load()
    U = torch.from_numpy(np.ascontiguousarray(wl.user_emb)).to(ix.device)
    b, keep = ix._batch(U, wl.feat_offsets, wl.feat_keys, wl.feat_mult, wl.k, scan_dtype, 4)
    n = int(np.sum(wl.k))
    ids = torch.full((max(1, n),), -1, dtype=torch.int32, device=ix.device)
    sc = torch.full((max(1, n),), float("nan"), dtype=torch.float32, device=ix.device)
    rc = lib.ebr_score_topk_noalloc(ix._h, ctypes.byref(b), ids.data_ptr(), sc.data_ptr(), None)
    torch.cuda.synchronize()
    return rc, ids[:n].cpu().numpy(), sc[:n].cpu().numpy()


def reference(ix, wl, scan_dtype=0):
    ids, sc, _ = ix.topk_workload(wl, scan_dtype=scan_dtype)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), sc.cpu().numpy()


def test_noalloc_matches_the_workspace_entry_point():
    dev()
    wl = W.make("c1", n_ads=30_011, dim=64, n_keys=400, lengths=("zipf_draw", 1.2, 5, 6000),
                n_queries=40, feats=(0, 24), key_draw=("uniform",), k=(0, 400))
    ix = E.Index.from_workload(wl, dtypes=1 | (1 << E.BF16))
    assert E.NOALLOC_SCRATCH_BYTES == 256 << 20
    for sd in (E.F32, E.BF16):
        # first call: the whole batch; second call: a smaller batch on the same scratch
        for sub in (list(range(40)), [3, 17, 29]):
            w = wl.subset(sub)
            rc, ids, sc = noalloc(ix, w, sd)
            assert rc == E.EBR_OK, E.load().ebr_last_error()
            rid, rsc = reference(ix, w, sd)
            assert np.array_equal(ids, rid)
            assert np.array_equal(sc.view(np.uint32), rsc.view(np.uint32))


def test_noalloc_refuses_a_batch_beyond_the_scratch():
    dev()
    wl = W.make("c1", n_ads=30_011, dim=64, n_keys=400, lengths=("zipf_draw", 1.2, 5, 6000),
                n_queries=2400, feats=(0, 8), key_draw=("uniform",), k=(1, 100))
    ix = E.Index.from_workload(wl)
    need = ix.workspace_size(torch.from_numpy(wl.user_emb).to(ix.device), wl.feat_offsets,
                             wl.feat_keys, wl.k, wl.feat_mult)
    assert need > E.NOALLOC_SCRATCH_BYTES
    rc, ids, _ = noalloc(ix, wl)
    assert rc == E.EBR_ENOMEM
    assert b"static scratch" in E.load().ebr_last_error()
    assert (ids == -1).all()
