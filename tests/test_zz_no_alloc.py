"""The allocation-free batch search (snn_search_batch_dev_noalloc) against the
device-buffer batch search it mirrors (snn_search_batch_dev), through the C
ABI: identical ids, scores and counts on two calls in a row, the second with a
smaller batch, in both modes it accepts; the first call also against the FP64
oracle. Batches whose workspace exceeds the fixed array, the learned mode and
a wrong current device are rejected with SNN_E_INVALID."""
import gc

import numpy as np
import pytest

import parity
from oracle import oracle as O
from synth import gen

pytestmark = pytest.mark.gpu


def _dev(csr):
    import torch

    return (torch.from_numpy(csr.indptr.astype(np.int64)).cuda(), torch.from_numpy(csr.coords.astype(np.int32)).cuda(),
            torch.from_numpy(csr.vals).cuda())


def _host(t):
    import torch

    torch.cuda.synchronize()
    return tuple(x.cpu().numpy() for x in t)


@pytest.fixture(scope="module")
def small_index():
    import paper_2301_10622_amd as P

    # 30,000 documents: 8 tiles of 4,096 slots, the last one ragged
    w = gen.make_small(5, docs=30_000, queries=300)
    ix = P.Index(w.n, w.m, w.h, capacity=w.docs.rows, hash_seed=w.hash_seed)
    P.load_docs(ix, w.docs)
    yield w, ix
    ix.close()


def _sub(csr, rows):
    ptr = csr.indptr[: rows + 1]
    return gen.CSR(ptr.copy(), csr.coords[: ptr[-1]].copy(), csr.vals[: ptr[-1]].copy())


@pytest.mark.parametrize("mode", [1, 0])
def test_noalloc_equals_the_allocating_entry_point_on_two_calls(small_index, mode):
    import paper_2301_10622_amd as P

    w, ix = small_index
    for rows, k in ((w.queries.rows, 10), (77, 7)):
        q = _sub(w.queries, rows)
        t = _dev(q)
        ref = _host(ix.search_batch_dev(*t, k, mode=mode))
        got = _host(ix.search_batch_dev_noalloc(*t, k, mode=mode))
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), (mode, rows, k)
        if rows == w.queries.rows and mode == P.MODE_BATCHED:
            ora = O.Index(w.docs, w.n, w.m, w.h, w.hash_seed)
            parity.check_batch(got[0], got[1], got[2], ora, q, k, what="noalloc")


def test_noalloc_allocates_nothing_after_its_first_call(small_index):
    import torch

    import paper_2301_10622_amd as P

    w, ix = small_index
    t = _dev(w.queries)
    out = (torch.empty((w.queries.rows, 10), dtype=torch.int32, device="cuda"),
           torch.empty((w.queries.rows, 10), dtype=torch.float32, device="cuda"),
           torch.empty(w.queries.rows, dtype=torch.int32, device="cuda"))
    ix.search_batch_dev_noalloc(*t, 10, out=out)  # the first call on the device looks up the array
    torch.cuda.synchronize()
    # a new index has no workspace of its own; searching it allocates none
    fresh = P.Index(w.n, w.m, w.h, capacity=w.docs.rows, hash_seed=w.hash_seed)
    P.load_docs(fresh, w.docs)
    # no index of an earlier test may be collected (and free its memory)
    # while the device's free memory is compared
    gc.collect()
    gc.disable()
    try:
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for _ in range(3):
            fresh.search_batch_dev_noalloc(*t, 10, out=out)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
    finally:
        gc.enable()
    assert free1 == free0, (free0, free1)
    got = _host(out)
    ref = _host(ix.search_batch_dev(*t, 10))
    fresh.close()
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_noalloc_rejects_what_it_cannot_hold(small_index):
    import paper_2301_10622_amd as P

    w, ix = small_index
    t = _dev(w.queries)
    # 300 queries x 8 tiles x 4,096 candidates x 8 bytes: above the array
    with pytest.raises(P.SnnError) as e:
        ix.search_batch_dev_noalloc(*t, 4096)
    assert e.value.status == -1 and "workspace" in str(e.value)
    with pytest.raises(P.SnnError) as e:
        ix.search_batch_dev_noalloc(*t, 10, mode=P.MODE_LEARNED)
    assert e.value.status == -1
    # a batch that fits still runs after the rejections
    q = _sub(w.queries, 40)
    t = _dev(q)
    ref = _host(ix.search_batch_dev(*t, 100))
    got = _host(ix.search_batch_dev_noalloc(*t, 100))
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
