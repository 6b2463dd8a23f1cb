"""Parity at the full workload sizes, in the launch configuration the
benchmark times (the autotuned persistent schedule, one batch per launch):
sampled queries of the 1M-document SPLADE-shaped batch (k = 10 and 100, and
the Alg. 7 re-rank with k' = 1000) and of the 4M-document batch of 8,192
queries with nnz 5..400 (k = 100), each checked against the FP64 oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import gen
import parity

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

SAMPLE = 8


def _dev(q):
    import torch

    d = torch.device("cuda:0")
    return (torch.tensor(q.indptr, dtype=torch.int64, device=d), torch.tensor(q.coords.astype(np.int32), device=d),
            torch.tensor(q.vals, device=d))


def _run(ix, t, nq, k, total, kp=None):
    import torch

    stream = torch.cuda.Stream()  # capturable: the batched pass runs as a replayed HIP graph
    with torch.cuda.stream(stream):
        for _ in range(2):  # capture, then replay
            if kp:
                ids, sc, cnt = ix.search_rerank_dev(*t, k, kp, total=total, stream=stream)
            else:
                ids, sc, cnt = ix.search_batch_dev(*t, k, total=total, stream=stream)
    stream.synchronize()
    return ids.cpu().numpy().astype(np.int64), sc.cpu().numpy(), cnt.cpu().numpy()


def _check_sample(ora, q, ids, sc, cnt, k, rows, what):
    ids_of_pos = ora.ids.astype(np.int64)
    pos_of_id = {int(i): p for p, i in enumerate(ids_of_pos)}
    for qi in rows:
        s, a = ora.score_all(*q.row(qi))
        c = int(cnt[qi])
        parity.check_query(ids[qi][:c], sc[qi][:c], s, a, pos_of_id, ids_of_pos, k, what="%s q%d" % (what, qi))


@pytest.fixture(scope="module")
def splade1m():
    import paper_2301_10622_amd as P

    w = gen.make_splade_like(0)
    ix = P.Index(w.n, w.m, w.h, capacity=w.docs.rows, hash_seed=w.hash_seed, forward_store=True)
    P.load_docs(ix, w.docs)
    t = _dev(w.queries)
    sched = ix.autotune(*t, 10, total=int(w.queries.nnz))
    ora = O.Index(w.docs, w.n, w.m, w.h, w.hash_seed)
    yield w, ix, t, ora, sched
    ix.close()


@pytest.mark.parametrize("k", [10, 100])
def test_splade_1m_sampled_queries(splade1m, k):
    w, ix, t, ora, sched = splade1m
    ids, sc, cnt = _run(ix, t, w.queries.rows, k, int(w.queries.nnz))
    assert np.all(cnt == k)
    rows = np.random.default_rng(k).choice(w.queries.rows, SAMPLE, replace=False)
    _check_sample(ora, w.queries, ids, sc, cnt, k, rows, "1M k=%d %s" % (k, sched))


def test_splade_1m_rerank_sampled_queries(splade1m):
    w, ix, t, ora, sched = splade1m
    ids, sc, cnt = _run(ix, t, w.queries.rows, 10, int(w.queries.nnz), kp=1000)
    ids_of_pos = ora.ids.astype(np.int64)
    full = 0
    for qi in np.random.default_rng(3).choice(w.queries.rows, SAMPLE, replace=False):
        qc, qv = w.queries.row(qi)
        est, ea = ora.score_all(qc, qv)
        ex, xa = ora.score_all(qc, qv, exact=True)
        c = int(cnt[qi])
        full += parity.check_rerank_query(ids[qi][:c], sc[qi][:c], est, ea, ex, xa, ids_of_pos, 10, 1000,
                                          what="1M rerank q%d" % qi)
    assert full >= SAMPLE // 2


def test_batch_4m_sampled_queries():
    import paper_2301_10622_amd as P

    w = gen.make_batch(0)
    ix = P.Index(w.n, w.m, w.h, capacity=w.docs.rows, hash_seed=w.hash_seed)
    P.load_docs(ix, w.docs)
    t = _dev(w.queries)
    ix.autotune(*t, 100, total=int(w.queries.nnz))
    ids, sc, cnt = _run(ix, t, w.queries.rows, 100, int(w.queries.nnz))
    ix.close()
    assert np.all(cnt == 100)
    ora = O.Index(w.docs, w.n, w.m, w.h, w.hash_seed)
    # the shortest and the longest query of the batch, and random ones
    nnz = np.diff(w.queries.indptr)
    rows = [int(np.argmin(nnz)), int(np.argmax(nnz))] + list(np.random.default_rng(4).choice(w.queries.rows, 4,
                                                                                             replace=False))
    _check_sample(ora, w.queries, ids, sc, cnt, 100, rows, "4M k=100")
