"""Pass criteria for a top-K result against the FP64 oracle.

Scores: every returned ad's FP32 score g(a) is within rel_tol * |s(a)| of the
oracle's FP64 s(a) (or rel_tol * cond(a) in tests built to cancel).
Set: with s_K the oracle's K-th score and delta = 2 * rel_tol * |s_K| (each side
may be off by one tolerance), the result holds K distinct ids, contains every ad
with s > s_K + delta and none with s < s_K - delta; ads inside the band are ties.
Order: sorted by (returned score desc, id asc).
Recall: |G intersect (oracle top-K plus band ties)| / K, the Recall@G_k of
Section 4.1 ("Evaluation metrics") with G = K and the oracle as ground truth.
"""
from __future__ import annotations

import numpy as np


class ParityError(AssertionError):
    pass


def check_topk(ids, scores, k, s_all, *, rel_tol=1e-5, cond_all=None, exact=False, label=""):
    """Check one query's result (ids uint32[k], scores float32[k]) against FP64 scores of all ads.

    s_all: FP64 oracle scores indexed by ad id (length N).
    cond_all: if given, the score tolerance is rel_tol * cond(a) instead of rel_tol * |s(a)|.
    exact: tie band of zero (tests whose scores are exact in FP32): the id set and order
    must equal the oracle's.
    Returns recall@k (band ties count as hits).
    """
    ids = np.asarray(ids).astype(np.int64)
    g = np.asarray(scores, dtype=np.float64)
    s_all = np.asarray(s_all, dtype=np.float64)
    N = len(s_all)
    if len(ids) != k or len(g) != k:
        raise ParityError(f"{label}: expected {k} results, got {len(ids)}")
    if k == 0:
        return 1.0
    if ids.min() < 0 or ids.max() >= N:
        raise ParityError(f"{label}: id out of range")
    if len(np.unique(ids)) != k:
        raise ParityError(f"{label}: duplicate ids")
    s = s_all[ids]
    scale = np.abs(s) if cond_all is None else np.asarray(cond_all, dtype=np.float64)[ids]
    err = np.abs(g - s)
    bad = (g != s) if exact else (err > rel_tol * scale)
    if bad.any():
        i = int(np.argmax(err - rel_tol * scale))
        raise ParityError(f"{label}: score of ad {ids[i]} is {g[i]!r}, oracle {s[i]!r} "
                          f"({int(bad.sum())} of {k} outside tolerance)")
    # order: (score desc, id asc) on the returned scores
    for i in range(k - 1):
        if g[i] < g[i + 1] or (g[i] == g[i + 1] and ids[i] > ids[i + 1]):
            raise ParityError(f"{label}: result not ordered at position {i}")
    # set, with the tie band
    order = np.lexsort((np.arange(N), -s_all))
    s_k = s_all[order[k - 1]]
    delta = 0.0 if exact else 2.0 * rel_tol * abs(s_k)
    must = np.nonzero(s_all > s_k + delta)[0]
    missing = np.setdiff1d(must, ids)
    if len(missing):
        raise ParityError(f"{label}: {len(missing)} ads above the band are missing, "
                          f"e.g. {missing[:5]}")
    low = ids[s < s_k - delta]
    if len(low):
        raise ParityError(f"{label}: {len(low)} returned ads are below the band, e.g. {low[:5]}")
    if exact:
        want = order[:k]
        if not np.array_equal(want, ids):
            raise ParityError(f"{label}: exact-tie result differs from the oracle's ids")
    hits = np.isin(ids, order[:k]) | (np.abs(s - s_k) <= delta)
    return float(hits.sum()) / k


def check_topk_vs_oracle(ids, scores, k, o_ids, o_scores, full_scores, *, rel_tol=1e-5, label=""):
    """check_topk for one query, given the oracle's own top-K (o_ids, o_scores: FP64, ordered by
    (score desc, id asc)) so that the scores of all ads are needed only when the two id sets
    differ. When the sets are equal the set rule holds by itself (the oracle's top-K holds every
    ad above its K-th score, and nothing below it), so scores and order are checked against the
    oracle's values; otherwise full_scores() (FP64 scores of all ads) decides by check_topk.
    Returns recall@k."""
    ids = np.asarray(ids).astype(np.int64)
    g = np.asarray(scores, dtype=np.float64)
    o_ids = np.asarray(o_ids).astype(np.int64)
    if len(ids) != k or len(g) != k or len(o_ids) != k:
        raise ParityError(f"{label}: expected {k} results, got {len(ids)}")
    if k == 0:
        return 1.0
    if len(np.unique(ids)) == k and np.array_equal(np.sort(ids), np.sort(o_ids)):
        s_of = dict(zip(o_ids.tolist(), np.asarray(o_scores, dtype=np.float64).tolist()))
        s = np.array([s_of[a] for a in ids.tolist()])
        err = np.abs(g - s)
        bad = err > rel_tol * np.abs(s)
        if bad.any():
            i = int(np.argmax(err - rel_tol * np.abs(s)))
            raise ParityError(f"{label}: score of ad {ids[i]} is {g[i]!r}, oracle {s[i]!r} "
                              f"({int(bad.sum())} of {k} outside tolerance)")
        for i in range(k - 1):
            if g[i] < g[i + 1] or (g[i] == g[i + 1] and ids[i] > ids[i + 1]):
                raise ParityError(f"{label}: result not ordered at position {i}")
        return 1.0
    return check_topk(ids, scores, k, full_scores(), rel_tol=rel_tol, label=label)
