"""Batch parity against the FP64 oracle for large workloads (test helper).

The oracle's batch entry computes every listed query's top-K (OpenMP over queries); a
query's FP64 scores of all ads are computed only when its id set differs from the oracle's
(parity.check_topk_vs_oracle).
"""
import numpy as np

import oracle
from parity import check_topk_vs_oracle


def check_batch_vs_oracle(wl, ids, sc, offs, qs=None, rel_tol=1e-5, label=""):
    """Every listed query (default: all) against the batch oracle's top-K (OpenMP over
    queries); the full FP64 scores of a query are computed only if its id set differs."""
    qs = list(range(wl.n_queries)) if qs is None else list(qs)
    sub = wl.subset(qs)
    oix = oracle.Index.of(wl)
    o = oracle.topk_batch(oix, sub.user_emb, sub.feat_offsets, sub.feat_keys, sub.k, sub.feat_mult)
    oo = o["offsets"]
    recalls = []
    for i, q in enumerate(qs):
        a, b = offs[q], offs[q + 1]

        def full(q=q):
            mult = None if wl.feat_mult is None else wl.query_mults(q)
            d, w, _ = oracle.scores(oix, wl.user_emb[q], wl.query_keys(q), mult)
            return d + w
        recalls.append(check_topk_vs_oracle(ids[a:b], sc[a:b], int(wl.k[q]), o["ids"][oo[i]:oo[i + 1]],
                                            o["score"][oo[i]:oo[i + 1]], full, rel_tol=rel_tol,
                                            label=f"{label} query {q}"))
    assert min(recalls) == 1.0
    return recalls
