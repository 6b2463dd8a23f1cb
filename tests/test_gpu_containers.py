"""Array containers (the sparse-list form of Section 4.1, Notes on
Implementation) next to the posting bitmaps: the classes a compaction picks,
results against the FP64 oracle in every schedule, slots changed after the
compaction (read from the bitmaps) against a fresh compaction with the same
classes, and segments longer than one wave step."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import gen
import parity

pytestmark = pytest.mark.gpu

SCHEDULES = ((16, 1), (32, 1), (64, 1), (16, 2), (16, 3), (8, 2), (8, 4))


def _lib():
    import paper_2301_10622_amd as P

    return P


def _dev(q):
    import torch

    d = torch.device("cuda:0")
    return (torch.tensor(q.indptr, dtype=torch.int64, device=d), torch.tensor(q.coords.astype(np.int32), device=d),
            torch.tensor(q.vals, device=d))


def _run(ix, t, k, mode):
    import torch

    ids, sc, cnt = ix.search_batch_dev(*t, k, mode=mode)
    torch.cuda.synchronize()
    return ids.cpu().numpy().copy(), sc.cpu().numpy().copy(), cnt.cpu().numpy().copy()


def _every_schedule(ix, t, k, what):
    """Results of every schedule and both modes; asserts they are identical and
    returns them."""
    P = _lib()
    saved = ix.schedule()
    ref = None
    try:
        for R, Q in SCHEDULES:
            # persistent on a 64-workgroup grid (fewer workgroups than items)
            for persistent, grid in ((True, 64), (False, 2048)):
                ix.set_schedule(R_plain=max(R, 16), R_batch=R, grid=grid, persistent=persistent, qgroup=Q)
                for mode in (P.MODE_PLAIN, P.MODE_BATCHED):
                    if mode == P.MODE_PLAIN and not persistent:
                        continue
                    got = _run(ix, t, k, mode)
                    if ref is None:
                        ref = got
                    for a, b in zip(ref, got):
                        assert np.array_equal(a, b), (what, R, Q, persistent, mode)
    finally:
        ix.set_schedule(saved["R_plain"], saved["R_batch"], saved["grid"], bool(saved["persistent"]),
                        saved["qgroup"])
    return ref


def _counts(docs, n):
    nzc = docs.coords[docs.vals != 0]
    return np.bincount(nzc, minlength=n)


def test_compaction_classes_follow_the_density_rule():
    """A coordinate gets an array container when its postings cover at most
    1/16 of the used slots (whole 1,024-slot blocks); before any compaction
    every coordinate is a bitmap."""
    P = _lib()
    w = gen.make_small(4, docs=23_000, queries=4)
    ix = P.Index(w.n, w.m, w.h, capacity=w.docs.rows, hash_seed=w.hash_seed)
    P.load_docs(ix, w.docs, compact=False)
    assert not ix.container_classes().any()
    ix.compact()
    used = -(-w.docs.rows // 1024) * 1024
    want = (16 * _counts(w.docs, w.n) <= used).astype(np.uint8)
    got = ix.container_classes()
    assert np.array_equal(got, want)
    assert 0 < got.sum() < w.n  # both kinds occur on this collection
    ix.close()


@pytest.fixture(scope="module")
def multi():
    """60,123 documents of the small-index law: 15 tiles of 4,096 slots, the
    last one ragged; dim 1,000, m = 32, h = 1; 40 queries of nnz 20 (signed
    values)."""
    P = _lib()
    w = gen.make_small(6, docs=60_123, queries=40)
    ix = P.Index(w.n, w.m, w.h, capacity=w.docs.rows + 20_000, hash_seed=w.hash_seed)
    P.load_docs(ix, w.docs)
    ora = O.Index(w.docs, w.n, w.m, w.h, w.hash_seed)
    yield w, ix, ora
    ix.close()


@pytest.mark.parametrize("k", [10, 100])
def test_arrays_match_the_oracle_in_every_schedule(multi, k):
    w, ix, ora = multi
    cls = ix.container_classes()
    # the queries use both kinds of containers
    qc = w.queries.coords
    assert cls[qc].any() and not cls[qc].all()
    res = _every_schedule(ix, _dev(w.queries), k, "arrays k=%d" % k)
    parity.check_batch(res[0].astype(np.uint32), res[1], res[2], ora, w.queries, k, what="arrays k=%d" % k)


def test_stale_blocks_give_the_bits_of_a_fresh_compaction():
    """Deletes, inserts into freed and fresh slots and re-inserts after the
    compaction: the inserted slots are marked changed and read from the
    bitmaps, the deleted ones keep their listed postings; searches give
    exactly the bits of the same index compacted again with the same classes
    (every slot read from arrays), in every schedule; and the oracle's top-k
    of the live set."""
    P = _lib()
    # 47,152 documents in 49,152 slots: the first inserts take the 2,000 fresh
    # slots, the rest reuse freed ones (whose listed postings are stale)
    w = gen.make_small(7, docs=47_152, queries=30)
    pool = gen.small_docs(8, 20_000)
    ix = P.Index(w.n, w.m, w.h, capacity=w.docs.rows, hash_seed=w.hash_seed)
    P.load_docs(ix, w.docs)
    cls = ix.container_classes()
    rng = np.random.default_rng(9)
    live = {i: w.docs.row(i) for i in range(w.docs.rows)}
    nxt = 0
    t = _dev(w.queries)
    for step, k in enumerate((10, 100)):
        # deletes, then inserts (fresh slots while any are left, then freed
        # ones), then re-inserts of deleted ids with new vectors
        dels = rng.choice(sorted(live), 3000, replace=False).astype(np.uint32)
        ix.delete_batch(dels)
        for d in dels:
            del live[int(d)]
        for ids in (np.arange(2500, dtype=np.uint32) + 100_000 + 10_000 * step, dels[:300]):
            sub = pool.take(range(nxt, nxt + len(ids)))
            ix.insert_batch(ids, sub.indptr, sub.coords, sub.vals)
            for i, r in zip(ids, range(nxt, nxt + len(ids))):
                live[int(i)] = pool.row(r)
            nxt += len(ids)
        stale = _every_schedule(ix, t, k, "stale k=%d" % k)
        ix.compact(classes=cls)
        fresh = _every_schedule(ix, t, k, "recompacted k=%d" % k)
        for a, b in zip(stale, fresh):
            assert np.array_equal(a, b), k
    assert np.array_equal(ix.container_classes(), cls)
    lid = np.array(sorted(live), dtype=np.uint32)
    rows = [live[int(i)] for i in lid]
    lens = np.array([len(c) for c, _ in rows], dtype=np.int64)
    ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(lens, out=ptr[1:])
    docs_live = gen.CSR(ptr, np.concatenate([c for c, _ in rows]).astype(np.uint32),
                        np.concatenate([v for _, v in rows]).astype(np.float32))
    ora = O.Index(docs_live, w.n, w.m, w.h, w.hash_seed, ids=lid)
    got = _run(ix, t, 100, P.MODE_BATCHED)
    parity.check_batch(got[0].astype(np.uint32), got[1], got[2], ora, w.queries, 100, what="after mutations")
    ix.close()


def test_stale_blocks_h2_bf16_signed():
    """The same equality with h = 2 mappings, bfloat16 sketches and signed
    values: the bounds stored in the array containers (the h-fold minimum of
    U and maximum of L, as bfloat16) and those the bitmap reading gathers
    from the sketch are the same values, so a mutated index equals its
    recompaction bit for bit, in the schedules h = 2 allows; and the
    bfloat16 oracle's top-k of the live set."""
    P = _lib()
    rng = np.random.default_rng(31)
    n, m, h, seed = 2000, 24, 2, 33
    docs = gen.sparse_rows(32, 15_384, n, 1.1, rng.integers(20, 61, 15_384), "normal")
    pool = gen.sparse_rows(34, 4000, n, 1.1, rng.integers(20, 61, 4000), "normal")
    qs = gen.sparse_rows(35, 20, n, 1.1, np.full(20, 25), "normal")
    ix = P.Index(n, m, h, capacity=docs.rows, hash_seed=seed, sketch_bf16=True)
    P.load_docs(ix, docs)
    cls = ix.container_classes()
    assert cls[qs.coords].any()
    live = {i: docs.row(i) for i in range(docs.rows)}
    dels = rng.choice(sorted(live), 1500, replace=False).astype(np.uint32)
    ix.delete_batch(dels)
    for d in dels:
        del live[int(d)]
    nxt = 0
    for ids in (np.arange(1200, dtype=np.uint32) + 100_000, dels[:200]):  # fresh slots, then freed ones
        sub = pool.take(range(nxt, nxt + len(ids)))
        ix.insert_batch(ids, sub.indptr, sub.coords, sub.vals)
        for i, r in zip(ids, range(nxt, nxt + len(ids))):
            live[int(i)] = pool.row(r)
        nxt += len(ids)
    t = _dev(qs)
    saved = ix.schedule()

    def every(what):
        ref = None
        for R in (16, 32, 64):
            for mode in (P.MODE_PLAIN, P.MODE_BATCHED):
                ix.set_schedule(R_plain=max(R, 16), R_batch=R, grid=64, persistent=True, qgroup=1)
                got = _run(ix, t, 30, mode)
                if ref is None:
                    ref = got
                for a, b in zip(ref, got):
                    assert np.array_equal(a, b), (what, R, mode)
        return ref

    stale = every("stale")
    ix.compact(classes=cls)
    fresh = every("recompacted")
    ix.set_schedule(saved["R_plain"], saved["R_batch"], saved["grid"], bool(saved["persistent"]), saved["qgroup"])
    for a, b in zip(stale, fresh):
        assert np.array_equal(a, b)
    lid = np.array(sorted(live), dtype=np.uint32)
    rows = [live[int(i)] for i in lid]
    lens = np.array([len(c) for c, _ in rows], dtype=np.int64)
    ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(lens, out=ptr[1:])
    docs_live = gen.CSR(ptr, np.concatenate([c for c, _ in rows]).astype(np.uint32),
                        np.concatenate([v for _, v in rows]).astype(np.float32))
    ora = O.Index(docs_live, n, m, h, seed, ids=lid, bf16=True)
    parity.check_batch(fresh[0].astype(np.uint32), fresh[1], fresh[2], ora, qs, 30, what="h2 bf16 after mutations")
    ix.close()


def test_every_coordinate_an_array_long_segments():
    """Classes pinned to arrays for every coordinate: the Zipf head
    coordinates hold hundreds of postings per block, so their segments take
    many wave steps. Oracle parity in every schedule; a mutated (stale) index
    equals its recompaction bit for bit."""
    P = _lib()
    w = gen.make_small(10, docs=20_000, queries=24)
    ix = P.Index(w.n, w.m, w.h, capacity=24_000, hash_seed=w.hash_seed)
    allc = np.ones(w.n, np.uint8)
    P.load_docs(ix, w.docs, compact=allc)
    assert np.array_equal(ix.container_classes(), allc)
    assert _counts(w.docs, w.n).max() > 16 * 64  # some block holds far more than 64 postings
    t = _dev(w.queries)
    ora = O.Index(w.docs, w.n, w.m, w.h, w.hash_seed)
    res = _every_schedule(ix, t, 50, "all arrays")
    parity.check_batch(res[0].astype(np.uint32), res[1], res[2], ora, w.queries, 50, what="all arrays")
    extra = gen.small_docs(11, 3000)
    ix.insert_batch(np.arange(3000, dtype=np.uint32) + 50_000, extra.indptr, extra.coords, extra.vals)
    ix.delete_batch(np.arange(0, 20_000, 7, dtype=np.uint32))
    stale = _every_schedule(ix, t, 50, "all arrays, stale")
    ix.compact(classes=allc)
    fresh = _run(ix, t, 50, P.MODE_BATCHED)
    for a, b in zip(stale, fresh):
        assert np.array_equal(a, b)
    ix.close()


@pytest.mark.parametrize("variant", ["h2_signed", "bf16_upper_h1", "h3_nonneg"])
def test_arrays_with_other_sketches(variant):
    """Array containers with h = 2 on signed data, a bfloat16 upper-only
    sketch, and h = 3 on non-negative data: oracle parity (the bfloat16
    oracle for bfloat16) in every schedule that the sketch allows."""
    P = _lib()
    rng = np.random.default_rng(12)
    if variant == "h2_signed":
        docs = gen.sparse_rows(13, 30_000, 2000, 1.1, rng.integers(20, 61, 30_000), "normal")
        qs = gen.sparse_rows(14, 20, 2000, 1.1, np.full(20, 25), "normal")
        n, m, h, kw = 2000, 24, 2, {}
    elif variant == "bf16_upper_h1":
        docs = gen.sparse_rows(15, 30_000, 2000, 1.1, rng.integers(20, 61, 30_000), "exp")
        qs = gen.sparse_rows(16, 20, 2000, 1.1, np.full(20, 25), "exp")
        n, m, h, kw = 2000, 32, 1, dict(sketch_bf16=True, upper_only=True)
    else:
        docs = gen.sparse_rows(17, 30_000, 3000, 1.05, rng.integers(20, 61, 30_000), "exp")
        qs = gen.sparse_rows(18, 20, 3000, 1.05, np.full(20, 30), "exp")
        n, m, h, kw = 3000, 64, 3, {}
    ix = P.Index(n, m, h, capacity=docs.rows, hash_seed=21, **kw)
    P.load_docs(ix, docs)
    cls = ix.container_classes()
    assert cls[qs.coords].any()
    t = _dev(qs)
    saved = ix.schedule()
    ref = None
    shapes = SCHEDULES if h == 1 else ((16, 1), (32, 1), (64, 1))
    for R, Q in shapes:
        for mode in (P.MODE_PLAIN, P.MODE_BATCHED):
            ix.set_schedule(R_plain=max(R, 16), R_batch=R, grid=64, persistent=True, qgroup=Q)
            got = _run(ix, t, 30, mode)
            if ref is None:
                ref = got
            for a, b in zip(ref, got):
                assert np.array_equal(a, b), (variant, R, Q, mode)
    ix.set_schedule(saved["R_plain"], saved["R_batch"], saved["grid"], bool(saved["persistent"]), saved["qgroup"])
    ora = O.Index(docs, n, m, h, 21, bf16=bool(kw.get("sketch_bf16")))
    parity.check_batch(ref[0].astype(np.uint32), ref[1], ref[2], ora, qs, 30, what=variant)
    ix.close()
