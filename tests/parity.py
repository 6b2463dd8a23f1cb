"""Comparison of GPU search results with the FP64 oracle.

Tolerance (the reading of "1e-5 relative" for real-valued scores, where a
score near 0 can be a difference of large terms): a GPU score s_gpu of
document i passes when |s_gpu - s_ora| <= 1e-5 * A_i, with A_i the sum of
|q_j * bound| over the terms of the oracle's estimate (for non-negative data
A_i is the score itself, so this is exactly relative). Top-k id sets must be
identical except for documents within that tolerance of the oracle's k-th
score (the band), and the GPU order must agree with the oracle's scores up to
the same tolerance.
"""
import numpy as np

REL = 1e-5


def oracle_topk(scores, ids, k, live=None):
    order = np.lexsort((ids, -scores)) if live is None else None
    if live is not None:
        pos = np.nonzero(live)[0]
        o = np.lexsort((ids[pos], -scores[pos]))
        order = pos[o]
    return order[:k]


def check_query(gpu_ids, gpu_scores, ora_scores, ora_abs, pos_of_id, ids_of_pos, k, live=None, rel=REL,
                what=""):
    """Raise AssertionError with details if the GPU top-k fails the rule."""
    gpu_ids = np.asarray(gpu_ids, dtype=np.int64)
    gpu_scores = np.asarray(gpu_scores, dtype=np.float64)
    O = oracle_topk(ora_scores, ids_of_pos, k, live)
    n_live = len(ora_scores) if live is None else int(np.count_nonzero(live))
    assert len(gpu_ids) == min(k, n_live), "%s count %d vs %d" % (what, len(gpu_ids), min(k, n_live))
    if len(O) == 0:
        return
    gpos = np.array([pos_of_id[int(i)] for i in gpu_ids], dtype=np.int64)
    if live is not None:
        assert np.all(live[gpos]), "%s returned a non-live document" % what
    assert len(set(gpu_ids.tolist())) == len(gpu_ids), "%s duplicate ids" % what
    # (b) every returned score matches the oracle's estimate of that document
    tol = rel * ora_abs[gpos] + 1e-30
    err = np.abs(gpu_scores - ora_scores[gpos])
    bad = np.nonzero(err > tol)[0]
    assert len(bad) == 0, "%s score mismatch at ranks %s: gpu %s oracle %s A %s" % (
        what, bad[:5], gpu_scores[bad[:5]], ora_scores[gpos[bad[:5]]], ora_abs[gpos[bad[:5]]])
    # (c) id sets equal outside the band around the oracle's k-th score
    sk = ora_scores[O[-1]]
    ak = ora_abs[O[-1]]

    def in_band(p):
        return abs(ora_scores[p] - sk) <= rel * max(ora_abs[p], ak) + 1e-30

    oset = set(O.tolist())
    gset = set(gpos.tolist())
    for p in oset - gset:
        assert in_band(p), "%s oracle result (id %d, %.9g) missing from GPU top-k (k-th %.9g)" % (
            what, ids_of_pos[p], ora_scores[p], sk)
    for p in gset - oset:
        assert in_band(p), "%s GPU result (id %d, %.9g) not in oracle top-k (k-th %.9g)" % (
            what, ids_of_pos[p], ora_scores[p], sk)
    # (d) GPU list sorted by its own scores, ties by lower id
    for r in range(len(gpu_ids) - 1):
        a, b = gpu_scores[r], gpu_scores[r + 1]
        assert a > b or (a == b and gpu_ids[r] < gpu_ids[r + 1]), "%s GPU order broken at rank %d" % (what, r)
    # (e) GPU order agrees with the oracle's scores up to tolerance
    for r in range(len(gpos) - 1):
        p, q = gpos[r], gpos[r + 1]
        slack = rel * (ora_abs[p] + ora_abs[q]) + 1e-30
        assert ora_scores[p] >= ora_scores[q] - slack, "%s order vs oracle at rank %d" % (what, r)


def check_batch(gpu_ids, gpu_scores, gpu_counts, oracle_index, queries, k, live=None, rel=REL, what="", rows=None):
    N = oracle_index.N
    ids_of_pos = oracle_index.ids.astype(np.int64)
    pos_of_id = {int(i): p for p, i in enumerate(ids_of_pos)}
    rows = range(queries.rows) if rows is None else rows
    for qi in rows:
        qc, qv = queries.row(qi)
        s, a = oracle_index.score_all(qc, qv)
        c = int(gpu_counts[qi])
        check_query(gpu_ids[qi][:c], gpu_scores[qi][:c], s, a, pos_of_id, ids_of_pos, k, live, rel,
                    "%s q%d" % (what, qi))


def check_rerank_query(gpu_ids, gpu_scores, est, est_abs, exact, exact_abs, ids_of_pos, k, kp, rel=REL, what=""):
    """Alg. 7 result of one query against the oracle's FP64 estimates and exact
    scores of every document. The k' candidates are fixed when no document
    outside the oracle's top-k' lies within tolerance of its k'-th estimate
    (twice the score tolerance, since both sides may round); then the GPU's k
    results must be the oracle's top-k by exact score over those candidates, by
    the rule of check_query. Otherwise the candidate set is open at its edge and
    what still holds is checked: every result is a candidate of some valid
    top-k', its exact score is right, the list is sorted, and no candidate
    that every valid top-k' contains (in the oracle's top-k' and outside the
    edge) beats the GPU's k-th exact score beyond tolerance without being
    returned. Documents
    that share no coordinate with the query score exactly 0 on both sides and
    are ordered by id alike, so they never open the edge. Returns True when
    the query was checked in full."""
    gpu_ids = np.asarray(gpu_ids, dtype=np.int64)
    order = np.lexsort((ids_of_pos, -est))
    V = order[:kp]
    assert len(gpu_ids) == min(k, len(V)), "%s count %d vs %d" % (what, len(gpu_ids), min(k, len(V)))
    if len(V) == 0:
        return True
    skp, akp = est[V[-1]], est_abs[V[-1]]
    near = np.abs(est - skp) <= 2 * rel * np.maximum(est_abs, akp) + 1e-30
    if akp == 0:
        # documents no query coordinate touches score exactly 0 on both sides;
        # among them the lower id wins everywhere, so they fix the set
        near &= est_abs > 0
    outside = np.ones(len(est), bool)
    outside[V] = False
    open_edge = bool(np.any(near & outside))
    if not open_edge:
        ids_V = ids_of_pos[V]
        pos_V = {int(i): p for p, i in enumerate(ids_V)}
        check_query(gpu_ids, gpu_scores, exact[V], exact_abs[V], pos_V, ids_V, k, rel=rel, what=what)
        return True
    pos_of_id = {int(i): p for p, i in enumerate(ids_of_pos)}
    allowed = set(V.tolist()) | set(np.nonzero(near)[0].tolist())
    gpos = np.array([pos_of_id[int(i)] for i in gpu_ids], dtype=np.int64)
    assert len(set(gpos.tolist())) == len(gpos), "%s duplicate ids" % what
    assert all(int(p) in allowed for p in gpos), "%s result outside every valid candidate set" % what
    err = np.abs(np.asarray(gpu_scores, np.float64) - exact[gpos])
    assert np.all(err <= rel * exact_abs[gpos] + 1e-30), "%s exact score mismatch" % what
    for r in range(len(gpu_ids) - 1):
        a, b = gpu_scores[r], gpu_scores[r + 1]
        assert a > b or (a == b and gpu_ids[r] < gpu_ids[r + 1]), "%s order broken at rank %d" % (what, r)
    # The certain candidates (in V and outside the edge) are in every valid
    # top-k', so the GPU scored each of them exactly and kept the k best of its
    # own candidate set: one that beats the GPU's k-th exact score by more than
    # both sides' rounding must have been returned.
    certain = np.setdiff1d(V, np.nonzero(near)[0])
    missing = np.setdiff1d(certain, gpos)
    if len(gpos) and len(missing):
        kth = gpos[-1]
        beat = exact[missing] - exact[kth] > rel * (exact_abs[missing] + exact_abs[kth]) + 1e-30
        assert not np.any(beat), "%s certain candidate (id %d, exact %.9g) beats the GPU's k-th (%.9g) but is " \
            "missing" % (what, ids_of_pos[missing[beat][0]], exact[missing[beat][0]], exact[kth])
    elif len(missing):
        raise AssertionError("%s no results while certain candidates exist" % what)
    return False
