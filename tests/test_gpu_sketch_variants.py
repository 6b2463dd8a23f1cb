"""GPU parity of the memory levers: bfloat16 sketches (U rounded up, L down,
the paper's storage precision, Section 4.1) and an upper-only sketch for
non-negative collections (Sinnamon+), against the FP64 oracle built the same
way."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import gen
import parity

pytestmark = pytest.mark.gpu


def _P():
    import paper_2301_10622_amd as P

    return P


def test_bf16_sketch_columns_bit_exact():
    P = _P()
    w = gen.make_small(0, docs=3000, queries=5)
    ix = P.Index(w.n, w.m, w.h, capacity=3000, hash_seed=w.hash_seed, sketch_bf16=True)
    P.load_docs(ix, w.docs)
    for i in np.random.default_rng(0).choice(3000, 200, replace=False):
        c, v = w.docs.row(int(i))
        u, l = ix.read_sketch(int(i))
        ou, ol, _ = O.sketch(c, v, w.m, w.h, w.hash_seed)
        bu = np.array([O.bf16_up(x) for x in ou.astype(np.float32)])
        bl = np.array([O.bf16_down(x) for x in ol.astype(np.float32)])
        assert np.array_equal(u.astype(np.float64), bu) and np.array_equal(l.astype(np.float64), bl), i
    ix.close()


@pytest.mark.parametrize("h,k", [(1, 10), (2, 100)])
def test_bf16_search_matches_oracle_multi_tile(h, k):
    """Signed values, several tiles and a ragged tail."""
    P = _P()
    rng = np.random.default_rng(3 + h)
    docs = gen.sparse_rows(21 + h, 30011, 1500, 1.1, rng.integers(1, 70, 30011), "normal")
    qs = gen.sparse_rows(25 + h, 20, 1500, 1.1, rng.integers(1, 50, 20), "normal")
    ix = P.Index(1500, 24, h, capacity=30011, hash_seed=9, sketch_bf16=True)
    P.load_docs(ix, docs)
    ora = O.Index(docs, 1500, 24, h, 9, bf16=True)
    ids, sc, cnt = ix.search_batch(qs.indptr, qs.coords, qs.vals, k)
    parity.check_batch(ids, sc, cnt, ora, qs, k, what="bf16 h=%d" % h)
    ix.close()


def _nonneg(seed, docs=20000, queries=16):
    rng = np.random.default_rng(seed)
    d = gen.sparse_rows(seed, docs, 3000, 1.05, rng.integers(5, 120, docs), "exp")
    q = gen.sparse_rows(seed + 1, queries, 3000, 1.05, rng.integers(5, 40, queries), "exp")
    return d, q


def test_upper_only_equals_full_sketch_on_nonnegative_data():
    """With q >= 0 the search never reads L, so dropping it changes nothing."""
    P = _P()
    d, q = _nonneg(31)
    full = P.Index(3000, 32, 1, capacity=d.rows, hash_seed=2)
    up = P.Index(3000, 32, 1, capacity=d.rows, hash_seed=2, upper_only=True)
    P.load_docs(full, d)
    P.load_docs(up, d)
    for k in (10, 100):
        a = full.search_batch(q.indptr, q.coords, q.vals, k)
        b = up.search_batch(q.indptr, q.coords, q.vals, k)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    full.close()
    up.close()


def test_upper_only_bf16_matches_oracle_and_rejects_negatives():
    import torch

    P = _P()
    d, q = _nonneg(41)
    ix = P.Index(3000, 32, 1, capacity=d.rows + 10, hash_seed=4, upper_only=True, sketch_bf16=True,
                 forward_store=True)
    P.load_docs(ix, d)
    ora = O.Index(d, 3000, 32, 1, 4, bf16=True)
    ids, sc, cnt = ix.search_batch(q.indptr, q.coords, q.vals, 20)
    parity.check_batch(ids, sc, cnt, ora, q, 20, what="upper-only bf16")
    # re-rank on top: candidates from the bf16 estimates, exact scores from the vectors
    ids, sc, cnt = ix.search_rerank(q.indptr, q.coords, q.vals, 10, 300)
    ids_of_pos = ora.ids.astype(np.int64)
    for qi in range(q.rows):
        qc, qv = q.row(qi)
        est, ea = ora.score_all(qc, qv)
        ex, xa = ora.score_all(qc, qv, exact=True)
        n = int(cnt[qi])
        parity.check_rerank_query(ids[qi][:n], sc[qi][:n], est, ea, ex, xa, ids_of_pos, 10, 300,
                                  what="upper-only bf16 rerank q%d" % qi)
    # negative values have no lower bound to use: rejected on insert and search
    with pytest.raises(P.SnnError) as e:
        ix.insert(10 ** 6, [1, 2], [0.5, -0.25])
    assert e.value.status == -1
    with pytest.raises(P.SnnError):
        ix.search_batch(np.array([0, 2]), np.array([1, 2]), np.array([0.5, -0.25], np.float32), 5)
    dv = torch.device("cuda:0")
    ip = torch.tensor([0, 2, 4], dtype=torch.int64, device=dv)
    qc = torch.tensor([1, 2, 1, 2], dtype=torch.int32, device=dv)
    qv = torch.tensor([0.5, -0.25, 0.5, 0.25], dtype=torch.float32, device=dv)
    ids, sc, cnt = ix.search_batch_dev(ip, qc, qv, 5)
    torch.cuda.synchronize()
    assert int(cnt[0]) == 0 and int(cnt[1]) == 5
    assert ix.last_batch_status()[0] == 1
    ix.close()


@pytest.mark.parametrize("bf16,upper", [(True, False), (False, True), (True, True)])
def test_sketch_variants_every_schedule_same_bits(bf16, upper):
    """The bfloat16 and upper-only sketches under every batched schedule (one,
    two and three queries per workgroup; R = 8 .. 64; persistent or not): the
    same bits as the plain form, and the bfloat16 results against its oracle."""
    P = _P()
    if upper:
        docs, qs = _nonneg(41, docs=30011, queries=24)
        n, m = 3000, 64
    else:
        rng = np.random.default_rng(7)
        docs = gen.sparse_rows(43, 30011, 1500, 1.1, rng.integers(1, 70, 30011), "normal")
        qs = gen.sparse_rows(44, 24, 1500, 1.1, rng.integers(1, 50, 24), "normal")
        n, m = 1500, 24
    ix = P.Index(n, m, 1, capacity=30011, hash_seed=11, sketch_bf16=bf16, upper_only=upper)
    P.load_docs(ix, docs)
    ref = ix.search_ex(qs.indptr, qs.coords, qs.vals, 10, mode=P.MODE_PLAIN)
    for R, Q in ((16, 1), (32, 1), (64, 1), (16, 2), (16, 3), (8, 2), (8, 4)):
        for persistent in (True, False):
            ix.set_schedule(R_plain=max(R, 16), R_batch=R, grid=64 if persistent else 2048, persistent=persistent, qgroup=Q)
            got = ix.search_ex(qs.indptr, qs.coords, qs.vals, 10, mode=P.MODE_BATCHED)
            for a, b in zip(ref, got):
                assert np.array_equal(a, b), (R, Q, persistent)
    if bf16:
        ora = O.Index(docs, n, m, 1, 11, bf16=True)
        parity.check_batch(ref[0], ref[1], ref[2], ora, qs, 10, what="bf16 upper=%s" % upper)
    ix.close()
