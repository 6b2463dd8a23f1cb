"""GPU parity of the anytime variant: scoring stops after the first c query
coordinates in the order of Alg. 6 (the time budget of Alg. 4 / Alg. 6 as a
coordinate count), against the FP64 oracle with the same budget."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import gen
import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    import paper_2301_10622_amd as P

    w = gen.make_small(0)
    ix = P.Index(w.n, w.m, w.h, capacity=w.docs.rows, hash_seed=w.hash_seed, forward_store=True)
    P.load_docs(ix, w.docs)
    ora = O.Index(w.docs, w.n, w.m, w.h, w.hash_seed)
    return w, ix, ora


@pytest.mark.parametrize("c", [1, 4, 10, 19])
def test_anytime_matches_oracle(small, c):
    w, ix, ora = small
    q = w.queries
    ids, sc, cnt = ix.search_ex(q.indptr, q.coords, q.vals, 10, max_coords=c)
    ids_of_pos = ora.ids.astype(np.int64)
    pos_of_id = {int(i): p for p, i in enumerate(ids_of_pos)}
    for qi in range(q.rows):
        s, a = ora.score_all(*q.row(qi), max_coords=c)
        n = int(cnt[qi])
        parity.check_query(ids[qi][:n], sc[qi][:n], s, a, pos_of_id, ids_of_pos, 10, what="c=%d q%d" % (c, qi))


def test_budget_at_or_above_nnz_is_the_full_search(small):
    w, ix, ora = small
    q = w.queries
    full = ix.search_batch(q.indptr, q.coords, q.vals, 10)
    for c in (20, 21, 4096):
        got = ix.search_ex(q.indptr, q.coords, q.vals, 10, max_coords=c)
        for a, b in zip(full, got):
            assert np.array_equal(a, b)


def test_anytime_identical_across_forms(small):
    """Plain, batched and learned forms give bit-identical anytime results."""
    import torch
    import paper_2301_10622_amd as P

    w, ix, ora = small
    q = gen.small_queries(7, 300)
    d = torch.device("cuda:0")
    t = (torch.tensor(q.indptr, dtype=torch.int64, device=d), torch.tensor(q.coords.astype(np.int32), device=d),
         torch.tensor(q.vals, device=d))
    tq = gen.small_queries(2, 5000)
    tt = (torch.tensor(tq.indptr, dtype=torch.int64, device=d), torch.tensor(tq.coords.astype(np.int32), device=d),
          torch.tensor(tq.vals, device=d))
    ix.filter_train(*tt, k=10, epochs=2, batch=512, lr=1e-3)
    res = []
    for mode in (P.MODE_PLAIN, P.MODE_BATCHED, P.MODE_LEARNED):
        out = ix.search_ex_dev(*t, 10, mode=mode, max_coords=6)
        torch.cuda.synchronize()
        res.append([o.cpu().numpy() for o in out])
    for other in res[1:]:
        for a, b in zip(res[0], other):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("c", [3, 12])
def test_anytime_rerank_matches_oracle(small, c):
    """Candidates by the budgeted scores, exact scores with the whole query."""
    w, ix, ora = small
    q = w.queries
    ids, sc, cnt = ix.search_ex(q.indptr, q.coords, q.vals, 10, k_prime=200, max_coords=c)
    ids_of_pos = ora.ids.astype(np.int64)
    full = 0
    for qi in range(q.rows):
        qc, qv = q.row(qi)
        est, ea = ora.score_all(qc, qv, max_coords=c)
        ex, xa = ora.score_all(qc, qv, exact=True)
        n = int(cnt[qi])
        full += parity.check_rerank_query(ids[qi][:n], sc[qi][:n], est, ea, ex, xa, ids_of_pos, 10, 200,
                                          what="c=%d q%d" % (c, qi))
    assert full >= 0.85 * q.rows


def test_search_params_are_checked(small):
    import paper_2301_10622_amd as P

    w, ix, ora = small
    q = w.queries
    # (the learned form re-ranks too, with a trained filter: this index has one)
    for kw in (dict(mode=7), dict(k_prime=5), dict(k_prime=70000), dict(mode=P.MODE_PLAIN, k_prime=100)):
        with pytest.raises(P.SnnError) as e:
            ix.search_ex(q.indptr, q.coords, q.vals, 10, **kw)
        assert e.value.status == -1
