"""Pins of the FP64 oracle to facts that do not come from the oracle itself.

Each test checks the oracle against the paper (printed tables, theorems,
corollaries), against mathematics (invariants, special cases that reduce to a
textbook computation), or against brute force on tiny inputs. A plausible slip
in the oracle (a dropped term, the wrong bound for a sign, a wrong index, an
off-by-one in the mappings, a wrong tie rule) fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from synth import gen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _table(name, conv=float):
    rows = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        rows.append(tuple(conv(x) for x in line.split()))
    return rows


# --------------------------------------------------------------------------
# the random mappings
# --------------------------------------------------------------------------

def test_splitmix64_published_outputs():
    inc = 0x9E3779B97F4A7C15
    for seed, idx, out in _table("splitmix64_vectors.txt", int):
        assert O.mix64(seed + idx * inc) == out


def test_bucket_table_is_uniform_and_independent_across_mappings():
    # chi-square of pi_0 over m buckets, and pi_0 vs pi_1 agreement ~ 1/m
    n, m, h = 30000, 64, 3
    t = O.bucket_table(7, h, n, m)
    assert t.max() < m
    for o in range(h):
        cnt = np.bincount(t[o], minlength=m)
        chi2 = ((cnt - n / m) ** 2 / (n / m)).sum()
        assert chi2 < 2 * m  # dof m-1; 2m is far in the tail
    agree = (t[0] == t[1]).mean()
    assert abs(agree - 1 / m) < 0.01
    # different seeds give different mappings
    assert (O.bucket_table(8, 1, n, m)[0] != t[0]).mean() > 0.9


# --------------------------------------------------------------------------
# sketching (Alg. 5) and decoding
# --------------------------------------------------------------------------

def test_sketch_member_order_equals_printed_bucket_order():
    rng = np.random.default_rng(0)
    for h in (1, 2, 3):
        for _ in range(20):
            nnz = int(rng.integers(1, 50))
            c = np.sort(rng.choice(200, nnz, replace=False)).astype(np.uint32)
            v = rng.standard_normal(nnz).astype(np.float32)
            a = O.sketch(c, v, 16, h, 3, by_bucket=False)
            b = O.sketch(c, v, 16, h, 3, by_bucket=True)
            for x, y in zip(a, b):
                assert np.array_equal(x, y)


def test_decode_brackets_value_and_recovers_extremes():
    """Theorem 1 per term: lower <= x <= upper; the largest value of a vector is
    recovered exactly from U and the smallest from L (remark after Theorem 2)."""
    rng = np.random.default_rng(1)
    for h in (1, 2, 3):
        for _ in range(200):
            nnz = int(rng.integers(1, 80))
            c = np.sort(rng.choice(1000, nnz, replace=False)).astype(np.uint32)
            v = rng.standard_normal(nnz).astype(np.float32)
            up, lo = O.decode_doc(c, v, 8, h, 11)
            x = v.astype(np.float64)
            assert np.all(up >= x) and np.all(lo <= x)
            assert up[np.argmax(x)] == x.max()
            assert lo[np.argmin(x)] == x.min()


def test_collision_free_documents_decode_exactly():
    m, h, seed = 64, 2, 5
    t = O.bucket_table(seed, h, 5000, m)
    rng = np.random.default_rng(2)
    for _ in range(100):
        used = set()
        coords = []
        for j in rng.permutation(5000):
            b = {int(t[o, j]) for o in range(h)}
            if b & used:
                continue
            used |= b
            coords.append(int(j))
            if len(coords) == 12:
                break
        c = np.sort(np.array(coords, dtype=np.uint32))
        v = rng.standard_normal(len(c)).astype(np.float32)
        up, lo = O.decode_doc(c, v, m, h, seed)
        assert np.array_equal(up, v.astype(np.float64)) and np.array_equal(lo, v.astype(np.float64))


def _sim_decode_errors(m, h, docs=4000, psi=120, n=30000, seed=0):
    """Fraction of active values overestimated by the upper bound, and the mean
    overestimation, for psi uniform coordinates and Uniform[-1,1] values."""
    rng = np.random.default_rng(seed)
    over = 0
    total = 0
    err = 0.0
    for _ in range(docs):
        c = np.sort(rng.choice(n, psi, replace=False)).astype(np.uint32)
        v = rng.uniform(-1, 1, psi).astype(np.float32)
        up, _ = O.decode_doc(c, v, m, h, 12345)
        d = up - v.astype(np.float64)
        over += int((d > 0).sum())
        err += float(d.sum())
        total += psi
    return over / total, err / total


@pytest.mark.parametrize("m", [60, 120, 240])
def test_table1_and_table2_uniform_by_simulation(m):
    t1 = {(int(a), int(b)): c for a, b, c in _table("table1_prob_error.txt")}
    t2 = {(int(a), int(b)): c for a, b, c in _table("table2_expected_error_uniform.txt")}
    for h in (1, 2, 3):
        p, e = _sim_decode_errors(m, h, docs=1500, seed=m * 10 + h)
        assert abs(p - t1[(m, h)]) <= 0.012, (m, h, p)
        assert abs(p - O.prob_error_gaussian(m, h, 119.0)) <= 0.012, (m, h, p)
        assert abs(e - t2[(m, h)]) <= 0.015, (m, h, e)


def test_table1_theorem2_integral_and_corollary_agree():
    """The numeric Theorem 2 integral for Uniform[-1,1] and the Gaussian
    corollary's closed form both reproduce the printed Table 1 row."""
    cdf = lambda a: (a + 1.0) / 2.0
    pdf = lambda a: 0.5
    for m, h, val in _table("table1_prob_error.txt"):
        m, h = int(m), int(h)
        integ = O.prob_error_integral(m, h, 119.0, cdf, pdf, -1.0, 1.0)
        assert abs(integ - val) <= 0.01, (m, h, integ)
        assert abs(O.prob_error_gaussian(m, h, 119.0) - val) <= 0.01


# --------------------------------------------------------------------------
# scoring (Alg. 6) and exact scoring (Eq. 2)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small():
    w = gen.make_small(0, docs=2000, queries=30)
    ix = O.Index(w.docs, w.n, w.m, w.h, w.hash_seed)
    return w, ix


def test_exact_matches_dense_brute_force(small):
    w, ix = small
    D = np.zeros((w.docs.rows, w.n))
    for i in range(w.docs.rows):
        c, v = w.docs.row(i)
        D[i, c] = v
    for qi in range(w.queries.rows):
        qc, qv = w.queries.row(qi)
        q = np.zeros(w.n)
        q[qc] = qv
        s, _ = ix.score_all(qc, qv, exact=True)
        np.testing.assert_allclose(s, D @ q, rtol=1e-12, atol=1e-12)


def test_doc_at_a_time_equals_coordinate_at_a_time(small):
    w, ix = small
    for qi in range(10):
        qc, qv = w.queries.row(qi)
        s, a = ix.score_all(qc, qv)
        for i in range(0, w.docs.rows, 7):
            dc, dv = w.docs.row(i)
            e, ea = O.pair_est(qc, qv, dc, dv, w.m, w.h, w.hash_seed)
            assert e == s[i] and ea == a[i]
            assert O.pair_exact(qc, qv, dc, dv) == ix.score_all(qc, qv, exact=True)[0][i]


def test_theorem1_estimate_never_below_exact_any_sign():
    """Theorem 1 for any query sign: the sequential FP64 sums of the estimate and
    of the exact score walk the same lists in the same order, every estimate term
    is >= its exact term, and rounding is monotone, so est >= exact exactly."""
    rng = np.random.default_rng(3)
    docs = gen.sparse_rows(5, 3000, 300, 1.1, rng.integers(5, 40, 3000), "normal")
    for h in (1, 2, 3):
        ix = O.Index(docs, 300, 8, h, 21)
        qs = gen.sparse_rows(6 + h, 40, 300, 1.1, rng.integers(1, 30, 40), "normal")
        for qi in range(qs.rows):
            qc, qv = qs.row(qi)
            est, _ = ix.score_all(qc, qv)
            ex, _ = ix.score_all(qc, qv, exact=True)
            assert np.all(est >= ex)
            # and it is tight somewhere unless every touched doc collides
            assert np.any(est == ex)


def test_collision_free_index_equals_linscan():
    """With no collisions Sinnamon returns the exact scores (LinScan)."""
    rng = np.random.default_rng(4)
    docs = gen.sparse_rows(9, 500, 100, 1.1, rng.integers(1, 20, 500), "normal")
    m = 4096
    t = O.bucket_table(1, 1, 100, m)[0]
    if len(set(t.tolist())) < 100:  # find a seed with an injective mapping on 100 coords
        for seed in range(2, 200):
            t = O.bucket_table(seed, 1, 100, m)[0]
            if len(set(t.tolist())) == 100:
                break
    else:
        seed = 1
    assert len(set(t.tolist())) == 100
    ix = O.Index(docs, 100, m, 1, seed)
    qs = gen.sparse_rows(10, 20, 100, 1.1, rng.integers(1, 20, 20), "normal")
    for qi in range(qs.rows):
        qc, qv = qs.row(qi)
        assert np.array_equal(ix.score_all(qc, qv)[0], ix.score_all(qc, qv, exact=True)[0])


def test_metamorphic_sign_scale_permutation_untouched(small):
    w, ix = small
    # M1: est(-q, -x) == est(q, x)
    neg = gen.CSR(w.docs.indptr, w.docs.coords, -w.docs.vals)
    ixn = O.Index(neg, w.n, w.m, w.h, w.hash_seed)
    dbl = gen.CSR(w.docs.indptr, w.docs.coords, 2 * w.docs.vals)
    ix2 = O.Index(dbl, w.n, w.m, w.h, w.hash_seed)
    rng = np.random.default_rng(5)
    for qi in range(w.queries.rows):
        qc, qv = w.queries.row(qi)
        s, _ = ix.score_all(qc, qv)
        assert np.array_equal(ixn.score_all(qc, -qv)[0], s)
        # M2: scaling by 2 is exact in binary floating point
        assert np.array_equal(ix.score_all(qc, 2 * qv)[0], 2 * s)
        assert np.array_equal(ix2.score_all(qc, qv)[0], 2 * s)
        # M3: input order of the query's coordinates does not matter
        p = rng.permutation(len(qc))
        assert np.array_equal(ix.score_all(qc[p], qv[p])[0], s)
        # M4: documents sharing no coordinate with q score exactly 0
        touched = np.zeros(w.docs.rows, bool)
        qset = set(qc.tolist())
        for i in range(w.docs.rows):
            touched[i] = bool(qset.intersection(w.docs.row(i)[0].tolist()))
        assert np.all(s[~touched] == 0)


def test_zero_query_values_are_not_coordinates(small):
    w, ix = small
    qc, qv = w.queries.row(0)
    qv2 = qv.copy()
    qv2[::3] = 0
    keep = qv2 != 0
    assert np.array_equal(ix.score_all(qc, qv2)[0], ix.score_all(qc[keep], qv2[keep])[0])


# --------------------------------------------------------------------------
# selection (Alg. 3, FindLargest) with the lower-id tie rule
# --------------------------------------------------------------------------

def _brute_topk(scores, ids, k, live=None):
    items = [(-float(s), int(i), p) for p, (s, i) in enumerate(zip(scores, ids)) if live is None or live[p]]
    items.sort()
    return [p for _, _, p in items[:k]]


def test_find_largest_matches_brute_force_with_ties():
    rng = np.random.default_rng(6)
    for trial in range(200):
        N = int(rng.integers(0, 60))
        k = int(rng.integers(0, 70))
        scores = rng.integers(-3, 4, N).astype(np.float64)  # many ties
        ids = rng.permutation(1000)[:N].astype(np.uint32)
        live = rng.random(N) < 0.8
        got = O.find_largest(scores, k, ids, live)
        assert list(got) == _brute_topk(scores, ids, k, live)


def test_search_returns_all_live_when_k_exceeds_n(small):
    w, ix = small
    ids, sc, ab, cnt = ix.search(w.queries.take([0, 1]), 5000)
    assert list(cnt) == [w.docs.rows, w.docs.rows]
    assert sorted(ids[0][: cnt[0]].tolist()) == list(range(w.docs.rows))


def test_search_equals_score_all_then_select(small):
    w, ix = small
    ids, sc, ab, cnt = ix.search(w.queries, 10, threads=4)
    for qi in range(w.queries.rows):
        qc, qv = w.queries.row(qi)
        s, a = ix.score_all(qc, qv)
        want = _brute_topk(s, np.arange(w.docs.rows), 10)
        assert list(ids[qi]) == want
        assert np.array_equal(sc[qi], s[want]) and np.array_equal(ab[qi], a[want])


# --------------------------------------------------------------------------
# ranking with k' >= k (Alg. 7)
# --------------------------------------------------------------------------

def _dense(w):
    D = np.zeros((w.docs.rows, w.n))
    for i in range(w.docs.rows):
        c, v = w.docs.row(i)
        D[i, c] = v
    return D


def _dense_q(w, qi):
    qc, qv = w.queries.row(qi)
    q = np.zeros(w.n)
    q[qc] = qv
    return qc, qv, q


def test_rerank_equals_brute_force_composition(small):
    """Alg. 7 written out with a dense matrix product and a plain sort: the k'
    best estimates (ties to the lower id), their exact inner products, the k
    best of those. Also returns |q_j x_j| summed over shared coordinates."""
    w, ix = small
    D = _dense(w)
    ids_all = np.arange(w.docs.rows)
    for k, kp in ((10, 10), (10, 57), (5, 300), (25, 1000)):
        ids, sc, ab, cnt = ix.rerank(w.queries, k, kp, threads=4)
        for qi in range(w.queries.rows):
            qc, qv, q = _dense_q(w, qi)
            est, _ = ix.score_all(qc, qv)
            V = _brute_topk(est, ids_all, kp)
            ex = D[V] @ q
            best = [V[p] for p in _brute_topk(ex, np.array(V), k)]
            assert list(ids[qi][: cnt[qi]]) == best, (k, kp, qi)
            np.testing.assert_allclose(sc[qi][: cnt[qi]], D[best] @ q, rtol=1e-12, atol=1e-12)
            np.testing.assert_allclose(ab[qi][: cnt[qi]], np.abs(D[best] * q).sum(axis=1), rtol=1e-12, atol=1e-12)


def test_rerank_of_every_vector_is_exact_search(small):
    """With k' at least the collection size, re-ranking scores every vector
    exactly, so the result is the exact top-k of Eq. 2."""
    w, ix = small
    D = _dense(w)
    ids, sc, ab, cnt = ix.rerank(w.queries, 10, w.docs.rows + 5)
    for qi in range(w.queries.rows):
        _, _, q = _dense_q(w, qi)
        assert list(ids[qi]) == _brute_topk(D @ q, np.arange(w.docs.rows), 10)


def test_rerank_recall_never_drops_as_kprime_grows(small):
    """The candidate sets are nested in k', and a vector of the exact top-k
    that is a candidate stays in the re-ranked top-k, so recall against the
    exact top-k cannot fall as k' grows; at k' = N it is 1."""
    w, ix = small
    D = _dense(w)
    truth = [set(_brute_topk(D @ _dense_q(w, qi)[2], np.arange(w.docs.rows), 10)) for qi in range(w.queries.rows)]
    prev = np.zeros(w.queries.rows)
    for kp in (10, 20, 50, 100, 400, 2000):
        ids, _, _, cnt = ix.rerank(w.queries, 10, kp)
        rec = np.array([len(truth[qi] & set(ids[qi][: cnt[qi]].tolist())) / 10 for qi in range(w.queries.rows)])
        assert np.all(rec >= prev), kp
        prev = rec
    assert np.all(prev == 1.0)


# --------------------------------------------------------------------------
# bfloat16 sketches (the paper's storage precision), U rounded up, L down
# --------------------------------------------------------------------------

def _all_bf16():
    """Every finite bfloat16 value, from all 65,536 bit patterns, sorted."""
    pats = (np.arange(65536, dtype=np.uint32) << 16).view(np.float32)
    return np.unique(pats[np.isfinite(pats)].astype(np.float64))


def test_bf16_rounding_is_the_nearest_bfloat16_above_and_below():
    grid = _all_bf16()
    rng = np.random.default_rng(11)
    xs = np.concatenate([rng.standard_normal(3000), rng.exponential(1.0, 500) * 1e-30,
                         rng.uniform(-1e30, 1e30, 500), grid[rng.integers(0, len(grid), 300)],
                         [1.0, -1.0, 2.0 ** -126, 3.0e38]]).astype(np.float32)
    for x in xs:
        if x == 0:
            continue
        up, dn = O.bf16_up(x), O.bf16_down(x)
        i = np.searchsorted(grid, float(x))  # first grid value >= x
        assert up == grid[i], (x, up, grid[i])
        j = np.searchsorted(grid, float(x), side="right") - 1  # last grid value <= x
        assert dn == grid[j], (x, dn, grid[j])


def test_bf16_sketch_keeps_theorem1_and_rounds_each_bound_outward():
    """Estimates from a bfloat16 sketch are still never below the exact score
    (any sign, h = 1 and 2), never below the float32-sketch estimate for
    non-negative data, and equal to it when every value is a bfloat16."""
    rng = np.random.default_rng(12)
    for h, law in ((1, "normal"), (2, "normal"), (1, "exp")):
        docs = gen.sparse_rows(90 + h, 500, 400, 1.1, rng.integers(10, 50, 500), law)
        qs = gen.sparse_rows(95 + h, 8, 400, 1.1, np.full(8, 30), law)
        b = O.Index(docs, 400, 16, h, 5, bf16=True)
        f = O.Index(docs, 400, 16, h, 5)
        for qi in range(qs.rows):
            qc, qv = qs.row(qi)
            sb, _ = b.score_all(qc, qv)
            sf, _ = f.score_all(qc, qv)
            ex, _ = f.score_all(qc, qv, exact=True)
            assert np.all(sb >= ex - 1e-9)
            if law == "exp":
                assert np.all(sb >= sf - 1e-12) and np.any(sb > sf)
    # values that are bfloat16 already: both sketches hold the same numbers
    docs = gen.sparse_rows(97, 300, 200, 1.1, rng.integers(10, 40, 300), "normal")
    docs.vals[:] = (docs.vals.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)
    docs.vals[docs.vals == 0] = 1.0
    qs = gen.sparse_rows(98, 4, 200, 1.1, np.full(4, 20), "normal")
    b, f = O.Index(docs, 200, 16, 1, 6, bf16=True), O.Index(docs, 200, 16, 1, 6)
    for qi in range(qs.rows):
        qc, qv = qs.row(qi)
        assert np.array_equal(b.score_all(qc, qv)[0], f.score_all(qc, qv)[0])


# --------------------------------------------------------------------------
# anytime scoring: a budget of c coordinates in the order of Alg. 6
# --------------------------------------------------------------------------

def _truncate(qc, qv, c):
    """The c non-zeros of largest |q_j| (ties: lower j), written out directly."""
    nz = [(abs(float(v)), int(j), float(v)) for j, v in zip(qc, qv) if v != 0]
    nz.sort(key=lambda t: (-t[0], t[1]))
    keep = nz[:c]
    return np.array([t[1] for t in keep], np.uint32), np.array([t[2] for t in keep], np.float32)


def test_anytime_budget_scores_the_largest_coordinates_first():
    """Stopping after c coordinates equals scoring the query cut to its c
    entries of largest |q_j| (the order Alg. 6 walks), checked per pair with
    the doc-at-a-time estimate, for signed data and for budgets 0 (all), 1, a
    few, and more than the query has."""
    w = gen.make_small(3, docs=300, queries=6)
    ix = O.Index(w.docs, w.n, w.m, w.h, w.hash_seed)
    for qi in range(w.queries.rows):
        qc, qv = w.queries.row(qi)
        full, _ = ix.score_all(qc, qv)
        for c in (0, 1, 3, 7, 19, 20, 500):
            s, a = ix.score_all(qc, qv, max_coords=c)
            if c == 0 or c >= len(qc):
                assert np.array_equal(s, full)
                continue
            tc, tv = _truncate(qc, qv, c)
            for i in range(0, w.docs.rows, 7):
                dc, dv = w.docs.row(i)
                est = O.pair_est(tc, tv, dc, dv, w.m, w.h, w.hash_seed)
                assert abs(s[i] - est[0]) <= 1e-12 * max(1.0, est[1]), (qi, c, i)


def test_anytime_nonnegative_partial_scores_rise_and_bound_exact():
    """Non-negative data: each further coordinate adds a non-negative term, so
    the anytime score never falls as the budget grows, and it is at least the
    exact inner product over the coordinates processed so far (the upper-bound
    remark of Section 4.2, Theorem 1 applied to the processed part)."""
    rng = np.random.default_rng(8)
    docs = gen.sparse_rows(81, 400, 300, 1.1, rng.integers(5, 40, 400), "exp")
    qs = gen.sparse_rows(82, 5, 300, 1.1, np.full(5, 25), "exp")
    ix = O.Index(docs, 300, 8, 1, 3)
    for qi in range(qs.rows):
        qc, qv = qs.row(qi)
        prev = np.zeros(docs.rows)
        for c in range(1, 26):
            s, _ = ix.score_all(qc, qv, max_coords=c)
            assert np.all(s >= prev - 1e-12)
            tc, tv = _truncate(qc, qv, c)
            ex, _ = ix.score_all(tc, tv, exact=True)
            assert np.all(s >= ex - 1e-12)
            prev = s


def test_anytime_rerank_uses_budgeted_candidates_and_full_exact_scores(small):
    """Alg. 4 / Alg. 7 with a budget: candidates by the budgeted scores, exact
    inner products with the whole query."""
    w, ix = small
    D = _dense(w)
    ids, sc, ab, cnt = ix.rerank(w.queries, 10, 60, max_coords=5)
    for qi in range(w.queries.rows):
        qc, qv, q = _dense_q(w, qi)
        est, _ = ix.score_all(qc, qv, max_coords=5)
        V = _brute_topk(est, np.arange(w.docs.rows), 60)
        best = [V[p] for p in _brute_topk(D[V] @ q, np.array(V), 10)]
        assert list(ids[qi][: cnt[qi]]) == best
        np.testing.assert_allclose(sc[qi][: cnt[qi]], D[best] @ q, rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------
# MLP of the learned filter: gradients against central differences
# --------------------------------------------------------------------------

def test_mlp_gradients_match_central_differences():
    rng = np.random.default_rng(7)
    p = {k: rng.standard_normal(s) * (0.2 if k.startswith("W") else 0.05) for k, s in O.MLP_SHAPES.items()}
    X = rng.standard_normal((6, 256))
    y = rng.standard_normal(6)
    loss, g = O.mlp_loss_grad(X, y, p)
    yh = O.mlp_forward(X, p)
    assert abs(loss - np.mean((yh - y) ** 2)) < 1e-12 * max(1, loss)
    eps = 1e-6
    for name in O.MLP_SHAPES:
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = np.mean((O.mlp_forward(X, p) - y) ** 2)
            flat[idx] = old - eps
            lm = np.mean((O.mlp_forward(X, p) - y) ** 2)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, an)


def test_features_are_linear_in_q_signed_part():
    rng = np.random.default_rng(8)
    c = np.sort(rng.choice(1000, 30, replace=False)).astype(np.uint32)
    v = rng.standard_normal(30).astype(np.float32)
    f = O.features(c, v, 99)
    f2 = O.features(c, 2 * v, 99)
    np.testing.assert_allclose(f2[:128], 2 * f[:128], rtol=0, atol=1e-12)
    np.testing.assert_allclose(f2[128:], 4 * f[128:], rtol=1e-15, atol=1e-12)
    assert abs(f[128:].sum() - float((v.astype(np.float64) ** 2).sum())) < 1e-9
