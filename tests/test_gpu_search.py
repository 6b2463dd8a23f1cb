"""GPU parity: the HIP path through the C ABI against the FP64 oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import gen
import parity

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2301_10622_amd as P

    return P


@pytest.fixture(scope="module")
def small():
    """The small workload: 10k docs, dim 1,000, m = 32, h = 1, 100 queries of nnz 20."""
    P = _lib()
    w = gen.make_small(0)
    ix = P.Index(w.n, w.m, w.h, capacity=w.docs.rows, hash_seed=w.hash_seed)
    P.load_docs(ix, w.docs)
    ora = O.Index(w.docs, w.n, w.m, w.h, w.hash_seed)
    return w, ix, ora


def test_bucket_table_matches_oracle(small):
    w, ix, _ = small
    assert np.array_equal(ix.bucket_table(), O.bucket_table(w.hash_seed, w.h, w.n, w.m))


def test_bucket_table_h3_matches_oracle():
    P = _lib()
    ix = P.Index(5000, 48, 3, capacity=100, hash_seed=77)
    assert np.array_equal(ix.bucket_table(), O.bucket_table(77, 3, 5000, 48))


def test_sketch_columns_bit_exact(small):
    w, ix, _ = small
    rng = np.random.default_rng(0)
    for i in rng.choice(w.docs.rows, 200, replace=False):
        c, v = w.docs.row(int(i))
        u, l = ix.read_sketch(int(i))
        ou, ol, _ = O.sketch(c, v, w.m, w.h, w.hash_seed)
        assert np.array_equal(u.astype(np.float64), ou) and np.array_equal(l.astype(np.float64), ol), i


def test_search_small_all_queries(small):
    w, ix, ora = small
    ids, sc, cnt = ix.search_batch(w.queries.indptr, w.queries.coords, w.queries.vals, 10)
    parity.check_batch(ids, sc, cnt, ora, w.queries, 10, what="small")


@pytest.mark.parametrize("mode", [0, 1])
def test_search_dev_modes_match_host_batch(small, mode):
    import torch

    P = _lib()
    w, ix, ora = small
    dev = torch.device("cuda:0")
    ip = torch.tensor(w.queries.indptr, dtype=torch.int64, device=dev)
    qc = torch.tensor(w.queries.coords.astype(np.int32), device=dev)
    qv = torch.tensor(w.queries.vals, device=dev)
    ids, sc, cnt = ix.search_batch_dev(ip, qc, qv, 10, mode=mode)
    torch.cuda.synchronize()
    ids = ids.cpu().numpy().astype(np.uint32)
    sc = sc.cpu().numpy()
    cnt = cnt.cpu().numpy()
    hid, hsc, hcnt = ix.search_batch(w.queries.indptr, w.queries.coords, w.queries.vals, 10)
    # same kernels, same per-document accumulation order: bit-identical
    assert np.array_equal(cnt, hcnt) and np.array_equal(ids, hid) and np.array_equal(sc, hsc)


@pytest.mark.parametrize("k", [1, 7, 100, 1000])
def test_search_small_various_k(small, k):
    w, ix, ora = small
    q = w.queries.take(range(0, 100, 9))
    ids, sc, cnt = ix.search_batch(q.indptr, q.coords, q.vals, k)
    parity.check_batch(ids, sc, cnt, ora, q, k, what="k=%d" % k)


def test_single_search_equals_batch_row(small):
    w, ix, _ = small
    qc, qv = w.queries.row(3)
    a_ids, a_sc = ix.search(qc, qv, 10)
    ids, sc, cnt = ix.search_batch(w.queries.indptr, w.queries.coords, w.queries.vals, 10)
    assert np.array_equal(a_ids, ids[3][: cnt[3]]) and np.array_equal(a_sc, sc[3][: cnt[3]])


def _fresh(n, m, h, cap, seed=0):
    P = _lib()
    return P.Index(n, m, h, capacity=cap, hash_seed=seed)


def test_multi_tile_ragged_signed_h2():
    """40,123 docs over several tiles with a ragged tail; h = 2; signed values."""
    P = _lib()
    rng = np.random.default_rng(1)
    docs = gen.sparse_rows(11, 40123, 2000, 1.1, rng.integers(1, 80, 40123), "normal")
    qs = gen.sparse_rows(12, 24, 2000, 1.1, rng.integers(1, 60, 24), "normal")
    ix = _fresh(2000, 24, 2, 40123, seed=3)
    P.load_docs(ix, docs)
    ora = O.Index(docs, 2000, 24, 2, 3)
    for k in (10, 100):
        ids, sc, cnt = ix.search_batch(qs.indptr, qs.coords, qs.vals, k)
        parity.check_batch(ids, sc, cnt, ora, qs, k, what="ragged h2 k=%d" % k)


def test_nonnegative_h3_upper_bound_path():
    P = _lib()
    rng = np.random.default_rng(2)
    docs = gen.sparse_rows(21, 20000, 3000, 1.05, rng.integers(5, 120, 20000), "exp")
    qs = gen.sparse_rows(22, 16, 3000, 1.05, rng.integers(5, 60, 16), "exp")
    ix = _fresh(3000, 64, 3, 20000, seed=9)
    P.load_docs(ix, docs)
    ora = O.Index(docs, 3000, 64, 3, 9)
    ids, sc, cnt = ix.search_batch(qs.indptr, qs.coords, qs.vals, 50)
    parity.check_batch(ids, sc, cnt, ora, qs, 50, what="nonneg h3")


def test_empty_index_and_k_above_live():
    P = _lib()
    ix = _fresh(100, 8, 1, 1000)
    ids, sc = ix.search(np.array([1, 2]), np.array([1.0, -1.0]), 5)
    assert len(ids) == 0
    ix.insert(7, [1, 5], [2.0, 3.0])
    ix.insert(3, [2], [1.5])
    ids, sc = ix.search(np.array([1, 2]), np.array([1.0, -1.0]), 5)
    # doc 7: 1*2 = 2 (no collision possible beyond its own coords in its sketch);
    # doc 3: -1 * lower bound of coordinate 2 = -1.5
    assert list(ids) == [7, 3]
    assert sc[0] >= 2.0 and sc[1] <= -1.5 + 1e-6


def test_untouched_documents_score_zero_and_ties_go_to_lower_id():
    P = _lib()
    ix = _fresh(50, 8, 1, 100)
    # five identical documents (identical scores) with shuffled ids, plus untouched ones
    for i in (40, 12, 33, 5, 27):
        ix.insert(i, [1, 2, 3], [0.5, -1.0, 2.0])
    for i in (90, 80, 70):
        ix.insert(i, [10], [1.0])
    ids, sc = ix.search(np.array([1, 3]), np.array([1.0, 1.0]), 8)
    assert list(ids[:5]) == [5, 12, 27, 33, 40]
    assert np.all(sc[:5] == sc[0]) and list(ids[5:]) == [70, 80, 90] and np.all(sc[5:] == 0)
    # a query with no non-zero value: every document scores 0, lowest ids first
    ids, sc = ix.search(np.array([4]), np.array([0.0]), 4)
    assert list(ids) == [5, 12, 27, 33] and np.all(sc == 0)


def test_malformed_inputs_are_rejected():
    P = _lib()
    ix = _fresh(100, 8, 1, 100)
    ix.insert(1, [1, 2], [1.0, 2.0])
    for c, v in (([100], [1.0]), ([1, 1], [1.0, 2.0]), ([3], [np.nan]), ([3], [np.inf])):
        with pytest.raises(P.SnnError) as e:
            ix.search(np.array(c), np.array(v, dtype=np.float32), 3)
        assert e.value.status == -1
        with pytest.raises(P.SnnError):
            ix.insert(2, c, v)
    with pytest.raises(P.SnnError) as e:
        ix.insert(1, [3], [1.0])
    assert e.value.status == -2
    with pytest.raises(P.SnnError) as e:
        ix.delete(99)
    assert e.value.status == -3
    with pytest.raises(P.SnnError) as e:
        ix.search(np.array([1]), np.array([1.0]), 0)
    assert e.value.status == -1
    assert ix.live_count == 1


@pytest.mark.parametrize("length", [40, 300])
def test_device_batch_flags_duplicates_with_a_zero_value(length):
    """A query that repeats a coordinate is malformed even when one copy holds
    0, in the short (<= 256 entries) and the long preparation path alike; the
    other queries of the batch are unaffected."""
    import torch

    P = _lib()
    w = gen.make_small(1, docs=2000, queries=3)
    ix = P.Index(w.n, w.m, w.h, capacity=w.docs.rows, hash_seed=w.hash_seed)
    P.load_docs(ix, w.docs)
    rng = np.random.default_rng(length)
    c = rng.choice(w.n, length, replace=False).astype(np.uint32)
    v = rng.standard_normal(length).astype(np.float32)
    c[-1] = c[7]
    v[-1] = 0.0  # the duplicate is a zero
    good_c, good_v = w.queries.row(0)
    indptr = np.array([0, len(good_c), len(good_c) + length], dtype=np.int64)
    coords = np.concatenate([good_c, c]).astype(np.int32)
    vals = np.concatenate([good_v, v]).astype(np.float32)
    d = torch.device("cuda:0")
    ids, sc, cnt = ix.search_batch_dev(torch.tensor(indptr, device=d), torch.tensor(coords, device=d),
                                       torch.tensor(vals, device=d), 10, mode=P.MODE_BATCHED, total=len(coords))
    torch.cuda.synchronize()
    cnt = cnt.cpu().numpy()
    inv, _ = ix.last_batch_status()
    assert inv == 1 and cnt[1] == 0 and cnt[0] == 10
    ref_ids, _ = ix.search(good_c, good_v, 10)
    assert np.array_equal(ids.cpu().numpy()[0].astype(np.uint32), ref_ids)
    ix.close()


def test_capacity_full():
    P = _lib()
    ix = _fresh(10, 4, 1, 3)  # rounded up to one full tile internally
    n = 16384
    ix.insert_batch(np.arange(n), np.arange(n + 1), np.zeros(n), np.ones(n))
    with pytest.raises(P.SnnError) as e:
        ix.insert(n, [1], [1.0])
    assert e.value.status == -4
    ix.delete(5)
    ix.insert(n, [1], [1.0])  # reuses the freed slot


def test_streaming_history_equals_fresh_index():
    """Inserts, deletes and re-inserts with slot reuse give the same results as an
    index built from scratch on the live set."""
    P = _lib()
    rng = np.random.default_rng(5)
    pool = gen.sparse_rows(31, 30000, 1000, 1.1, rng.integers(20, 61, 30000), "normal")
    qs = gen.sparse_rows(32, 20, 1000, 1.1, np.full(20, 20), "normal")
    ix = _fresh(1000, 32, 1, 16384, seed=4)
    live = {}
    next_doc = 0
    # bulk load 12k, then a random history of deletes and inserts (the 4,384
    # fresh slots run out in the second step; later inserts reuse freed slots)
    P.load_docs(ix, pool.take(range(12000)), ids=np.arange(12000, dtype=np.uint32) * 3 + 1)
    for i in range(12000):
        live[i * 3 + 1] = i
    next_doc = 12000
    for step in range(6):
        dels = rng.choice(sorted(live), 1500, replace=False)
        ix.delete_batch(dels)
        for d in dels:
            del live[int(d)]
        new_ids = np.arange(2000) + 100000 + step * 5000
        rows = np.arange(next_doc, next_doc + 2000)
        next_doc += 2000
        sub = pool.take(rows)
        ix.insert_batch(new_ids, sub.indptr, sub.coords, sub.vals)
        for i, r in zip(new_ids, rows):
            live[int(i)] = int(r)
        # re-insert a few deleted ids with new vectors
        back = dels[:200]
        rows = np.arange(next_doc, next_doc + 200)
        next_doc += 200
        sub = pool.take(rows)
        ix.insert_batch(back, sub.indptr, sub.coords, sub.vals)
        for i, r in zip(back, rows):
            live[int(i)] = int(r)
    assert ix.live_count == len(live)
    lid = np.array(sorted(live), dtype=np.uint32)
    docs_live = pool.take([live[int(i)] for i in lid])
    ora = O.Index(docs_live, 1000, 32, 1, 4, ids=lid)
    ids, sc, cnt = ix.search_batch(qs.indptr, qs.coords, qs.vals, 25)
    parity.check_batch(ids, sc, cnt, ora, qs, 25, what="streaming")
    # sketches of re-inserted ids hold the new vectors
    for i in lid[:50]:
        c, v = pool.row(live[int(i)])
        u, l = ix.read_sketch(int(i))
        ou, ol, _ = O.sketch(c, v, 32, 1, 4)
        assert np.array_equal(u.astype(np.float64), ou) and np.array_equal(l.astype(np.float64), ol)


def test_update_batches_of_ragged_sizes():
    """Insert and delete batches of sizes below and between multiples of 8 (the
    update kernels split a batch into 8 runs, one per XCD): every live sketch
    column is the oracle's, bit for bit, and searches match the oracle."""
    P = _lib()
    pool = gen.sparse_rows(41, 6000, 1000, 1.1, np.random.default_rng(41).integers(20, 61, 6000), "normal")
    qs = gen.sparse_rows(42, 16, 1000, 1.1, np.full(16, 20), "normal")
    ix = _fresh(1000, 32, 1, 8000, seed=6)
    live = {}
    nxt = 0
    for size in (1, 3, 7, 9, 13, 1001, 4097):
        rows = np.arange(nxt, nxt + size)
        sub = pool.take(rows)
        ids = (rows * 5 + 2).astype(np.uint32)
        ix.insert_batch(ids, sub.indptr, sub.coords, sub.vals)
        live.update({int(i): int(r) for i, r in zip(ids, rows)})
        nxt += size
    rng = np.random.default_rng(43)
    for size in (1, 5, 11, 333):
        dels = rng.choice(sorted(live), size, replace=False)
        ix.delete_batch(dels)
        for d in dels:
            del live[int(d)]
    # refill freed slots with a batch of 349 (not a multiple of 8)
    rows = np.arange(nxt, nxt + 349)
    sub = pool.take(rows)
    ids = (rows * 5 + 2).astype(np.uint32)
    ix.insert_batch(ids, sub.indptr, sub.coords, sub.vals)
    live.update({int(i): int(r) for i, r in zip(ids, rows)})
    assert ix.live_count == len(live)
    lid = np.array(sorted(live), dtype=np.uint32)
    for i in lid:
        c, v = pool.row(live[int(i)])
        u, l = ix.read_sketch(int(i))
        ou, ol, _ = O.sketch(c, v, 32, 1, 6)
        assert np.array_equal(u.astype(np.float64), ou) and np.array_equal(l.astype(np.float64), ol), int(i)
    ora = O.Index(pool.take([live[int(i)] for i in lid]), 1000, 32, 1, 6, ids=lid)
    ids, sc, cnt = ix.search_batch(qs.indptr, qs.coords, qs.vals, 20)
    parity.check_batch(ids, sc, cnt, ora, qs, 20, what="ragged updates")


def test_large_batch_errors_name_the_first_bad_row():
    """Batches large enough to be validated on several host threads report the
    error of the first bad row (a row's id before its vector) and insert nothing."""
    P = _lib()
    ix = _fresh(1000, 32, 1, 20000, seed=7)
    pool = gen.sparse_rows(51, 12000, 1000, 1.1, np.full(12000, 30), "normal")
    ix.insert(5_000_000, [1, 2], [1.0, 2.0])

    def attempt(vec_row, id_row, dup_row=None):
        ids = np.arange(12000, dtype=np.uint32)
        c, v = pool.coords.copy(), pool.vals.copy()
        if vec_row is not None:
            v[pool.indptr[vec_row] + 3] = np.nan
        if dup_row is not None:
            c[pool.indptr[dup_row] + 5] = c[pool.indptr[dup_row] + 9]
        if id_row is not None:
            ids[id_row] = 5_000_000
        with pytest.raises(P.SnnError) as e:
            ix.insert_batch(ids, pool.indptr, c, v)
        assert ix.live_count == 1
        return e.value

    e = attempt(9000, 2000)
    assert e.status == -2 and "already live" in str(e)
    e = attempt(1000, 6000)
    assert e.status == -1 and "non-finite" in str(e)
    e = attempt(11999, None)
    assert e.status == -1 and "non-finite" in str(e)
    e = attempt(None, 11999)
    assert e.status == -2
    e = attempt(7000, None, dup_row=4000)
    assert e.status == -1 and "duplicate coordinate %d" % pool.coords[pool.indptr[4000] + 9] in str(e)
    ix.insert_batch(np.arange(12000, dtype=np.uint32), pool.indptr, pool.coords, pool.vals)
    assert ix.live_count == 12001


@pytest.mark.parametrize("k", [51, 60])
def test_select_around_the_register_cache(k):
    """80 tiles of 4,096 slots: the plain form's per-query select sees at most
    80 k keys, so at k = 51 (at most 4,080) every key is held in registers and
    at k = 60 (up to 4,800, still fewer than 64 per tile on average) most
    queries exceed the 4,096 the registers hold and take the path that reads
    the keys again; both give the batched form's bits and the oracle's top-k."""
    P = _lib()
    docs = gen.small_docs(61, 80 * 4096)
    qs = gen.small_queries(62, 8)
    ix = _fresh(1000, 32, 1, docs.rows, seed=8)
    P.load_docs(ix, docs)
    ix.set_schedule(16, 16, 2048, True, 1)
    import torch

    tens = _dev_batch(qs)
    plain = _dev_search(ix, tens, k, 0)
    work = ix.last_batch_work()
    batched = _dev_search(ix, tens, k, 1)
    for x, y in zip(plain, batched):
        assert np.array_equal(x, y)
    per_query = work["candidates"] / qs.rows
    assert (per_query <= 4096) if k == 51 else (per_query > 4096)
    ora = O.Index(docs, 1000, 32, 1, 8)
    parity.check_batch(plain[0].astype(np.uint32), plain[1], plain[2], ora, qs, k, what="select cache k=%d" % k)


def _dev_batch(q):
    import torch

    dev = torch.device("cuda:0")
    return (torch.tensor(q.indptr, dtype=torch.int64, device=dev),
            torch.tensor(q.coords.astype(np.int32), device=dev), torch.tensor(q.vals, device=dev))


def _dev_search(ix, tensors, k, mode, out=None):
    import torch

    ids, sc, cnt = ix.search_batch_dev(*tensors, k, mode=mode, out=out)
    torch.cuda.synchronize()
    return ids.cpu().numpy().copy(), sc.cpu().numpy().copy(), cnt.cpu().numpy().copy()


def test_all_schedules_give_identical_results(small):
    """Every tile size and launch shape computes the same per-document sums in the
    same order and the same exact selection: results are bit-identical."""
    P = _lib()
    w, ix, ora = small
    t = _dev_batch(w.queries)
    ref = _dev_search(ix, t, 10, P.MODE_PLAIN)
    ref100 = _dev_search(ix, t, 100, P.MODE_PLAIN)
    saved = ix.schedule()
    try:
        for R, Q in ((16, 1), (32, 1), (64, 1), (16, 2), (16, 3), (8, 2), (8, 4)):
            # a 64-workgroup persistent grid: these batches have more items than
            # that (a larger grid would run them one workgroup per item)
            for persistent, grid in ((True, 64), (True, 1024), (False, 2048)):
                ix.set_schedule(R_plain=max(R, 16), R_batch=R, grid=grid, persistent=persistent, qgroup=Q)
                for mode in (P.MODE_PLAIN, P.MODE_BATCHED):
                    for k in (10, 100):
                        got = _dev_search(ix, t, k, mode)
                        want = ref if k == 10 else ref100
                        for a, b in zip(want, got):
                            assert np.array_equal(a, b), (R, Q, persistent, grid, mode, k)
    finally:
        ix.set_schedule(saved["R_plain"], saved["R_batch"], saved["grid"], bool(saved["persistent"]),
                        saved["qgroup"])


def test_graph_replays_match_eager_between_mutations():
    """The batched form replays a captured HIP graph; each replay, with eager work
    and index mutations in between, equals the eager plain path at that state."""
    import torch

    P = _lib()
    w = gen.make_small(3, docs=6000, queries=40)
    stream = torch.cuda.Stream()  # a capturable (non-default) stream, default priority
    torch.cuda.set_stream(stream)
    ix = P.Index(w.n, w.m, w.h, capacity=20000, hash_seed=w.hash_seed, stream=stream)
    P.load_docs(ix, w.docs)
    t = _dev_batch(w.queries)
    dev = torch.device("cuda:0")
    out = (torch.empty((40, 10), dtype=torch.int32, device=dev), torch.empty((40, 10), dtype=torch.float32, device=dev),
           torch.empty(40, dtype=torch.int32, device=dev))
    extra = gen.small_docs(99, 400)
    for it in range(5):
        plain = _dev_search(ix, t, 10, P.MODE_PLAIN)
        got = _dev_search(ix, t, 10, P.MODE_BATCHED, out=out)  # same buffers: graph replay after the first
        for a, b in zip(plain, got):
            assert np.array_equal(a, b), it
        # mutate between replays: delete some docs, insert new ones (slot reuse)
        ix.delete_batch(np.arange(it * 50, it * 50 + 50))
        sub = extra.take(range(it * 80, it * 80 + 80))
        ix.insert_batch(np.arange(80) + 100000 + it * 100, sub.indptr, sub.coords, sub.vals)
    torch.cuda.synchronize()
    torch.cuda.set_stream(torch.cuda.default_stream())


def test_autotune_keeps_results_and_reports_schedule(small):
    P = _lib()
    w, ix, ora = small
    t = _dev_batch(w.queries)
    before = _dev_search(ix, t, 10, P.MODE_BATCHED)
    sch = ix.autotune(*t, 10)
    assert (sch["R_batch"], sch["qgroup"]) in ((16, 1), (32, 1), (64, 1), (16, 2), (16, 3), (8, 4))
    assert sch["R_plain"] in (16, 32, 64) and sch["tried"] == 24
    assert sch["best_ms"] > 0 and sch["best_ms"] <= sch["default_ms"] * 1.5
    after = _dev_search(ix, t, 10, P.MODE_BATCHED)
    for a, b in zip(before, after):
        assert np.array_equal(a, b)


@pytest.fixture(scope="module")
def wide():
    """300,000 documents of the small law: 74 tiles of 4,096 slots, enough for
    the sampled starting thresholds of a wide k."""
    P = _lib()
    w = gen.make_small(5, docs=300_000, queries=16)
    ix = P.Index(w.n, w.m, w.h, capacity=w.docs.rows, hash_seed=w.hash_seed)
    P.load_docs(ix, w.docs)
    yield w, ix
    ix.close()


@pytest.mark.parametrize("k", [256, 1000, 4096])
def test_wide_k_sampled_thresholds_bit_identical(wide, k):
    """k >= tile / 16 with 4,096-slot tiles starts each query from a threshold
    found on a sample of the tiles; with 16,384-slot tiles there are too few
    tiles to sample. Both must return the same bits, and the sampled search
    must hand the selection a few k candidates per query (about 1.5 k plus the
    sample's margin of 32, scaled to the collection), not a share of every
    tile."""
    w, ix = wide
    q = w.queries
    ix.set_schedule(16, 16, 2048, True)
    got = ix.search_batch(q.indptr, q.coords, q.vals, k)
    work = ix.last_batch_work()
    _, fallbacks = ix.last_batch_status()
    ix.set_schedule(16, 64, 2048, True)
    ref = ix.search_batch(q.indptr, q.coords, q.vals, k)
    ix.set_schedule(16, 16, 2048, True)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b), k
    assert fallbacks == 0
    assert 0 < work["candidates"] < q.rows * 8 * k, work


def test_wide_k_sampled_thresholds_match_oracle(wide):
    w, ix = wide
    P = _lib()
    q = w.queries.take(range(4))
    ora = O.Index(w.docs, w.n, w.m, w.h, w.hash_seed)
    ids, sc, cnt = ix.search_batch(q.indptr, q.coords, q.vals, 1000)
    pos_of_id = {i: i for i in range(w.docs.rows)}
    for qi in range(q.rows):
        s, a = ora.score_all(*q.row(qi))
        c = int(cnt[qi])
        parity.check_query(ids[qi][:c], sc[qi][:c], s, a, pos_of_id, np.arange(w.docs.rows), 1000,
                           what="wide k q%d" % qi)


def test_sampled_thresholds_graph_replays_follow_the_live_count():
    """A wide k on a collection with many tiles but few live documents (most
    deleted): the sampled pass's required count is min(k, live), a value the
    captured graph holds, so inserts into freed slots (same tile count) must
    lead to a new graph. Each replay equals the eager plain path."""
    import torch

    P = _lib()
    w = gen.make_small(6, docs=278_528, queries=8)  # every slot used: inserts reuse freed ones
    stream = torch.cuda.Stream()  # a capturable (non-default) stream, default priority
    torch.cuda.set_stream(stream)
    ix = P.Index(w.n, w.m, w.h, capacity=278_528, hash_seed=w.hash_seed, stream=stream)
    P.load_docs(ix, w.docs)
    ix.delete_batch(np.arange(3000, 278_528))
    t = _dev_batch(w.queries)
    dev = torch.device("cuda:0")
    k = 4000
    out = (torch.empty((8, k), dtype=torch.int32, device=dev), torch.empty((8, k), dtype=torch.float32, device=dev),
           torch.empty(8, dtype=torch.int32, device=dev))
    extra = gen.small_docs(77, 6000)
    for it in range(3):
        got = _dev_search(ix, t, k, P.MODE_BATCHED, out=out)
        ref = _dev_search(ix, t, k, P.MODE_PLAIN)
        assert np.all(got[2] == min(k, ix.live_count)), (it, got[2], ix.live_count)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), it
        sub = extra.take(range(it * 2000, it * 2000 + 2000))
        ix.insert_batch(np.arange(2000) + 1_000_000 + it * 2000, sub.indptr, sub.coords, sub.vals)
    torch.cuda.synchronize()
    torch.cuda.set_stream(torch.cuda.default_stream())
    ix.close()


def test_insert_by_word_long_documents_and_partial_words():
    """The word-grouped insert: 4,096 documents of 150-250 coordinates (a full
    posting word of 64 documents holds more (coordinate, bit) pairs than one
    sorting pass takes), then 100 more into the next fresh slots (a partly
    filled word, set with atomics), then 700 deletes and their slots refilled
    (scattered words). Searches from the bitmaps alone and after a compaction
    match the oracle; the sketch columns match bit for bit."""
    P = _lib()
    rng = np.random.default_rng(81)
    docs = gen.sparse_rows(82, 4900, 2000, 1.05, rng.integers(150, 251, 4900), "normal")
    qs = gen.sparse_rows(83, 16, 2000, 1.05, np.full(16, 30), "normal")
    ix = _fresh(2000, 48, 1, 8192, seed=5)
    ids = np.arange(4900, dtype=np.uint32)
    first = docs.take(range(4096))
    ix.insert_batch(ids[:4096], first.indptr, first.coords, first.vals)
    nxt = docs.take(range(4096, 4196))
    ix.insert_batch(ids[4096:4196], nxt.indptr, nxt.coords, nxt.vals)
    gone = np.sort(rng.choice(4196, 700, replace=False)).astype(np.uint32)
    ix.delete_batch(gone)
    refill = docs.take(range(4196, 4896))
    new_ids = np.arange(700, dtype=np.uint32) + 10_000
    ix.insert_batch(new_ids, refill.indptr, refill.coords, refill.vals)
    gone_set = set(gone.tolist())
    live_rows = [r for r in range(4196) if r not in gone_set] + list(range(4196, 4896))
    live_ids = np.concatenate([np.setdiff1d(ids[:4196], gone), new_ids]).astype(np.uint32)
    ora = O.Index(docs.take(live_rows), 2000, 48, 1, 5, ids=live_ids)
    for compact in (False, True):
        if compact:
            ix.compact()
        got = ix.search_batch(qs.indptr, qs.coords, qs.vals, 50)
        parity.check_batch(got[0], got[1], got[2], ora, qs, 50, what="word insert compact=%s" % compact)
    for p in (0, 62, 63, 64, 2000, 3495, 3496, len(live_ids) - 700, len(live_ids) - 1):
        i = int(live_ids[p])
        u, l = ix.read_sketch(i)
        row = live_rows[p]
        ou, ol, _ = O.sketch(*docs.row(row), 48, 1, 5)
        assert np.array_equal(u.astype(np.float64), ou) and np.array_equal(l.astype(np.float64), ol), i
    ix.close()
