"""The parity checker (tests/parity.py) itself, on the CPU.

Results the oracle computes stand in for a GPU result. A correct one must
pass; the same result with one planted mistake (a better candidate dropped,
a wrong score, a broken order) must fail. The collection holds every vector
twice, under two ids, so every estimate is tied with another document's and
an odd k' always cuts a tied pair: the k'-th estimate's edge is open, which
is the case where only part of Alg. 7's result is fixed.
"""
import numpy as np
import pytest

from oracle import oracle as O
from synth import gen
import parity


@pytest.fixture(scope="module")
def twin():
    w = gen.make_small(5, docs=1500, queries=12)
    d = w.docs
    both = gen.CSR(np.concatenate([d.indptr, d.indptr[1:] + d.indptr[-1]]),
                   np.concatenate([d.coords, d.coords]), np.concatenate([d.vals, d.vals]))
    ora = O.Index(both, w.n, w.m, w.h, w.hash_seed)
    return w, both, ora


def _scores(ora, q, qi):
    qc, qv = q.row(qi)
    est, ea = ora.score_all(qc, qv)
    ex, xa = ora.score_all(qc, qv, exact=True)
    return est, ea, ex, xa


def test_open_edge_accepts_the_oracle_result_and_rejects_a_dropped_candidate(twin):
    w, both, ora = twin
    k, kp = 10, 41
    ids_of_pos = ora.ids.astype(np.int64)
    rids, rsc, _, rcnt = ora.rerank(w.queries, k, kp)
    planted_failures = 0
    for qi in range(w.queries.rows):
        est, ea, ex, xa = _scores(ora, w.queries, qi)
        n = int(rcnt[qi])
        got_ids = rids[qi][:n].astype(np.int64)
        got_sc = rsc[qi][:n].astype(np.float32)
        full = parity.check_rerank_query(got_ids, got_sc, est, ea, ex, xa, ids_of_pos, k, kp, what="q%d" % qi)
        assert not full  # the twin of the k'-th candidate lies just outside
        # plant: drop the best result outside the edge's band and put the best
        # candidate not returned at the end, so membership, scores and order
        # still hold
        order = np.lexsort((ids_of_pos, -est))
        V = order[:kp]
        skp, akp = est[V[-1]], ea[V[-1]]
        near = set(np.nonzero(np.abs(est - skp) <= 2 * parity.REL * np.maximum(ea, akp))[0].tolist())
        drop = next((r for r in range(n) if int(got_ids[r]) not in near), None)
        if drop is None:
            continue
        rest = [p for p in V[np.lexsort((ids_of_pos[V], -ex[V]))] if ids_of_pos[p] not in set(got_ids.tolist())]
        nxt = rest[0]
        keep = np.arange(n) != drop
        bad_ids = np.concatenate([got_ids[keep], [ids_of_pos[nxt]]])
        bad_sc = np.concatenate([got_sc[keep], [np.float32(ex[nxt])]])
        if not (bad_sc[-2] > bad_sc[-1] or (bad_sc[-2] == bad_sc[-1] and bad_ids[-2] < bad_ids[-1])):
            continue
        with pytest.raises(AssertionError, match="certain candidate"):
            parity.check_rerank_query(bad_ids, bad_sc, est, ea, ex, xa, ids_of_pos, k, kp, what="planted q%d" % qi)
        planted_failures += 1
    assert planted_failures >= w.queries.rows - 2


def test_open_edge_rejects_wrong_scores_order_and_outsiders(twin):
    w, both, ora = twin
    k, kp = 10, 41
    ids_of_pos = ora.ids.astype(np.int64)
    rids, rsc, _, rcnt = ora.rerank(w.queries, k, kp)
    est, ea, ex, xa = _scores(ora, w.queries, 0)
    got_ids = rids[0][: rcnt[0]].astype(np.int64)
    got_sc = rsc[0][: rcnt[0]].astype(np.float32)
    wrong = got_sc.copy()
    wrong[3] *= np.float32(1.001)
    with pytest.raises(AssertionError, match="exact score"):
        parity.check_rerank_query(got_ids, wrong, est, ea, ex, xa, ids_of_pos, k, kp)
    swapped_ids, swapped_sc = got_ids.copy(), got_sc.copy()
    swapped_ids[[2, 3]] = swapped_ids[[3, 2]]
    swapped_sc[[2, 3]] = swapped_sc[[3, 2]]
    with pytest.raises(AssertionError, match="order"):
        parity.check_rerank_query(swapped_ids, swapped_sc, est, ea, ex, xa, ids_of_pos, k, kp)
    far = np.lexsort((ids_of_pos, -est))[-1]  # the lowest estimate: in no valid top-k'
    out_ids = np.concatenate([got_ids[:-1], [ids_of_pos[far]]])
    out_sc = np.concatenate([got_sc[:-1], [np.float32(min(ex[far], got_sc[-2]))]])
    with pytest.raises(AssertionError, match="outside every valid candidate set"):
        parity.check_rerank_query(out_ids, out_sc, est, ea, ex, xa, ids_of_pos, k, kp)


def test_fixed_edge_requires_the_oracle_top_k(twin):
    """An even k' keeps both twins of the last pair inside: the candidate set is
    fixed and the result must be the oracle's Alg. 7 top-k."""
    w, both, ora = twin
    k, kp = 10, 40
    ids_of_pos = ora.ids.astype(np.int64)
    rids, rsc, _, rcnt = ora.rerank(w.queries, k, kp)
    fixed = 0
    for qi in range(w.queries.rows):
        est, ea, ex, xa = _scores(ora, w.queries, qi)
        got_ids = rids[qi][: rcnt[qi]].astype(np.int64)
        got_sc = rsc[qi][: rcnt[qi]].astype(np.float32)
        if not parity.check_rerank_query(got_ids, got_sc, est, ea, ex, xa, ids_of_pos, k, kp):
            continue
        fixed += 1
        # the k-th result replaced by the (k+1)-th of the candidates
        order = np.lexsort((ids_of_pos, -est))[:kp]
        byex = order[np.lexsort((ids_of_pos[order], -ex[order]))]
        bad_ids = np.concatenate([got_ids[:-1], [ids_of_pos[byex[k]]]])
        bad_sc = np.concatenate([got_sc[:-1], [np.float32(ex[byex[k]])]])
        if abs(ex[byex[k]] - ex[byex[k - 1]]) <= 1e-5 * (xa[byex[k]] + xa[byex[k - 1]]):
            continue
        with pytest.raises(AssertionError):
            parity.check_rerank_query(bad_ids, bad_sc, est, ea, ex, xa, ids_of_pos, k, kp)
    assert fixed >= w.queries.rows // 2


def test_check_query_rejects_a_dropped_top_result(twin):
    w, both, ora = twin
    ids_of_pos = ora.ids.astype(np.int64)
    pos_of_id = {int(i): p for p, i in enumerate(ids_of_pos)}
    oids, osc, _, ocnt = ora.search(w.queries, 10)
    for qi in range(3):
        s, a = ora.score_all(*w.queries.row(qi))
        parity.check_query(oids[qi], osc[qi].astype(np.float32), s, a, pos_of_id, ids_of_pos, 10)
        order = np.lexsort((ids_of_pos, -s))
        bad_ids = np.concatenate([oids[qi][1:], [ids_of_pos[order[12]]]])
        bad_sc = np.concatenate([osc[qi][1:], [s[order[12]]]]).astype(np.float32)
        with pytest.raises(AssertionError):
            parity.check_query(bad_ids, bad_sc, s, a, pos_of_id, ids_of_pos, 10)
