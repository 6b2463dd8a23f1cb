"""Serving: each search result in the interleaved, continuously batched run is
the result of that search alone against the index state at its position in the
trace (the live set after exactly the preceding inserts and deletes)."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import gen
import parity

pytestmark = pytest.mark.gpu


def _setup(seed=0, prefill=12000, capacity=20000):
    import paper_2301_10622_amd as P

    docs = gen.small_docs(seed, prefill)
    ix = P.Index(1000, 32, 1, capacity=capacity, hash_seed=seed)
    P.load_docs(ix, docs)
    return ix, docs


def _trace(seed, ops, live_ids, next_id, rate):
    tr = gen.serving_trace(seed, ops, live_ids, next_id, rate, ks=(10, 100, 1000))
    csr = gen.trace_csr(tr)
    return tr, csr


def _live_states(docs, tr, csr, sample):
    """Live {id: (coords, vals)} just before each sampled request index."""
    live = {i: docs.row(i) for i in range(docs.rows)}
    out = {}
    want = set(sample)
    for r in range(len(tr["kind"])):
        if r in want:
            out[r] = dict(live)
        kd = tr["kind"][r]
        if kd == 1:
            live[int(tr["ids"][r])] = csr.row(r)
        elif kd == 2:
            del live[int(tr["ids"][r])]
    return out


def _oracle_for(state):
    ids = np.array(sorted(state), dtype=np.uint32)
    rows = [state[int(i)] for i in ids]
    lens = np.array([len(c) for c, _ in rows], dtype=np.int64)
    indptr = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    csr = gen.CSR(indptr, np.concatenate([c for c, _ in rows]).astype(np.uint32),
                  np.concatenate([v for _, v in rows]).astype(np.float32))
    return O.Index(csr, 1000, 32, 1, 0, ids=ids), csr, ids


@pytest.mark.parametrize("qgroup", [1, 2])
def test_serving_results_equal_alone_at_their_snapshot(qgroup):
    """Both the one-query and the grouped (two queries per workgroup) batched
    kernels serve the trace; the results are the same bits as a search alone."""
    import paper_2301_10622_amd as P

    ix, docs = _setup()
    ix.set_schedule(16, 16, 2048, True, qgroup)
    tr, csr = _trace(0, 3000, np.arange(docs.rows), docs.rows, rate=20000.0)
    res_ids, res_sc, res_cnt, lat, rep = ix.serve(tr["kind"], tr["t"], tr["ids"], tr["k"], csr.indptr, csr.coords,
                                                  csr.vals, max_batch=256, max_inflight=3, streams=3, realtime=True,
                                                  budget_bytes=1 << 30)
    kind = tr["kind"]
    sreq = np.nonzero(kind == 0)[0]
    assert rep["searches"] == len(sreq) and rep["rejected"] == 0
    assert rep["inserts"] == int((kind == 1).sum()) and rep["deletes"] == int((kind == 2).sum())
    assert rep["p99_ms"] >= rep["p50_ms"] > 0 and np.all(lat > 0)
    # the index after the run holds exactly the final live set
    final = _live_states(docs, tr, csr, [len(kind) - 1])[len(kind) - 1]
    last = len(kind) - 1
    if kind[last] == 1:
        final[int(tr["ids"][last])] = csr.row(last)
    elif kind[last] == 2:
        del final[int(tr["ids"][last])]
    assert ix.live_count == len(final)
    # sampled searches against the FP64 oracle on their own snapshot
    rng = np.random.default_rng(0)
    pick = sorted(rng.choice(len(sreq), 40, replace=False).tolist())
    states = _live_states(docs, tr, csr, [int(sreq[i]) for i in pick])
    for i in pick:
        r = int(sreq[i])
        ora, _, ids = _oracle_for(states[r])
        qc, qv = csr.row(r)
        s, a = ora.score_all(qc, qv)
        k = int(tr["k"][r])
        pos_of_id = {int(x): p for p, x in enumerate(ids)}
        c = int(res_cnt[i])
        parity.check_query(res_ids[i][:c], res_sc[i][:c], s, a, pos_of_id, ids.astype(np.int64), k,
                           what="serve search %d (request %d)" % (i, r))
    # and a few bit-exactly against the same search alone on a fresh GPU index
    # of that snapshot
    for i in pick[:6]:
        r = int(sreq[i])
        _, snap, ids = _oracle_for(states[r])
        alone = P.Index(1000, 32, 1, capacity=max(len(ids), 1), hash_seed=0)
        # the same container classes as the serving index (whose blocks changed
        # in the session are read from the bitmaps): then the same bits
        P.load_docs(alone, snap, ids=ids, compact=ix.container_classes())
        qc, qv = csr.row(r)
        a_ids, a_sc = alone.search(qc, qv, int(tr["k"][r]))
        c = int(res_cnt[i])
        assert np.array_equal(a_ids, res_ids[i][:c]) and np.array_equal(a_sc, res_sc[i][:c]), i
        alone.close()


def test_serving_overlaps_batches_and_admits_by_budget():
    ix, docs = _setup(1, prefill=8000, capacity=12000)
    tr, csr = _trace(1, 1500, np.arange(docs.rows), docs.rows, rate=1e9)
    # all requests arrive at once: batches queue behind each other and overlap on the device
    _, _, cnt, lat, rep = ix.serve(tr["kind"], tr["t"], tr["ids"], tr["k"], csr.indptr, csr.coords, csr.vals,
                                   max_batch=64, max_inflight=4, streams=4, realtime=False, budget_bytes=1 << 30)
    assert rep["batches"] >= 10 and rep["max_inflight_seen"] >= 2 and rep["rejected"] == 0
    # a budget below one k = 1000 search's workspace (on this small index about 32 KB,
    # k = 100 about 4 KB): those are rejected, the rest run within the budget
    ix2, docs2 = _setup(1, prefill=8000, capacity=12000)
    budget = 20 << 10
    _, _, cnt2, lat2, rep2 = ix2.serve(tr["kind"], tr["t"], tr["ids"], tr["k"], csr.indptr, csr.coords, csr.vals,
                                       max_batch=64, max_inflight=2, streams=2, realtime=False, budget_bytes=budget)
    k1000 = tr["k"][tr["kind"] == 0] == 1000
    assert rep2["rejected"] == int(k1000.sum()) > 0
    assert np.all(cnt2[k1000] == 0xFFFFFFFF) and np.all(cnt2[~k1000] > 0)
    assert 0 < rep2["peak_workspace_bytes"] <= budget


def test_serving_rejects_malformed_traces_without_changes():
    import paper_2301_10622_amd as P

    ix, docs = _setup(2, prefill=1000, capacity=2000)
    before = ix.live_count
    e = np.zeros(0)
    bad = [
        # delete of an id that is not live
        (np.array([2], np.uint8), np.array([0.0]), np.array([99999]), np.array([0]), np.array([0, 0])),
        # insert of a live id
        (np.array([1], np.uint8), np.array([0.0]), np.array([5]), np.array([0]), np.array([0, 1])),
        # unknown kind
        (np.array([7], np.uint8), np.array([0.0]), np.array([0]), np.array([0]), np.array([0, 0])),
    ]
    for kind, t, ids, k, ip in bad:
        with pytest.raises(P.SnnError) as ex:
            ix.serve(kind, t, ids, k, ip, np.array([3] * int(ip[-1]), np.uint32),
                     np.ones(int(ip[-1]), np.float32))
        assert ex.value.status == -1
    assert ix.live_count == before


def test_serving_wide_k_uses_sampled_thresholds_and_keeps_results():
    """A 300,000-document index (74 tiles): batches with k up to 1,000 start
    from sampled thresholds; each search returns the bits of the same search
    run alone in a batch of its k on a schedule too coarse to sample."""
    import paper_2301_10622_amd as P

    docs = gen.small_docs(4, 300_000)
    ix = P.Index(1000, 32, 1, capacity=300_000, hash_seed=4)
    P.load_docs(ix, docs)
    tr = gen.serving_trace(5, 240, np.arange(docs.rows), docs.rows, 1e9, frac_query=1.0, frac_insert=0.0,
                           ks=(10, 100, 1000))
    csr = gen.trace_csr(tr)
    ix.set_schedule(16, 16, 2048, True)
    res_ids, res_sc, res_cnt, lat, rep = ix.serve(tr["kind"], tr["t"], tr["ids"], tr["k"], csr.indptr, csr.coords,
                                                  csr.vals, max_batch=64, max_inflight=3, streams=3, realtime=False,
                                                  budget_bytes=8 << 30)
    assert rep["searches"] == 240 and rep["rejected"] == 0
    ix.set_schedule(16, 64, 2048, True)
    for k in (10, 100, 1000):
        sel = np.nonzero(tr["k"] == k)[0]
        qs = csr.take(sel.tolist())
        ids, sc, cnt = ix.search_batch(qs.indptr, qs.coords, qs.vals, k)
        for j, r in enumerate(sel):
            c = int(res_cnt[r])
            assert c == int(cnt[j]) and np.array_equal(res_ids[r][:c], ids[j][:c]), (k, r)
            assert np.array_equal(res_sc[r][:c], sc[j][:c]), (k, r)
    ix.close()
