"""Seeded synthetic sparse vectors for the Sinnamon workloads.

This module only draws inputs. It holds none of the method's arithmetic (no
hashing, no sketching, no scoring), so both the FP64 oracle and the GPU library
can consume what it produces without sharing any code with each other.

Laws (the readings are listed with the workload table in the design notes):

* Coordinates follow a Zipf(s) law over ranks r = 1..n with P(r) proportional to
  r**-s; rank r is coordinate r - 1.
* The distinct coordinates of one vector are a successive weighted sample
  without replacement. Drawing i.i.d. from the Zipf law and keeping the first
  occurrence of every coordinate until psi distinct ones are found is exactly
  that sample (each new coordinate is drawn in proportion to the weight of the
  coordinates not chosen yet), and it is what this module does.
* Values are float64 draws rounded to float32; a value that rounds to exactly 0
  is drawn again, so every stored entry is a non-zero coordinate (the nz()
  definition of Alg. 1 and Alg. 5).
* Coordinates are stored sorted ascending within each vector (CSR).

Every function takes an explicit seed; the same seed gives the same arrays on
any machine (numpy's PCG64).
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Optional

import numpy as np


@dataclasses.dataclass
class CSR:
    """A batch of sparse vectors: row i owns coords[indptr[i]:indptr[i+1]]."""

    indptr: np.ndarray  # int64, len rows + 1
    coords: np.ndarray  # uint32, ascending within a row
    vals: np.ndarray  # float32, non-zero

    @property
    def rows(self) -> int:
        return len(self.indptr) - 1

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def row(self, i: int):
        a, b = int(self.indptr[i]), int(self.indptr[i + 1])
        return self.coords[a:b], self.vals[a:b]

    def take(self, rows) -> "CSR":
        rows = np.asarray(rows, dtype=np.int64)
        lens = (self.indptr[rows + 1] - self.indptr[rows]).astype(np.int64)
        indptr = np.zeros(len(rows) + 1, dtype=np.int64)
        np.cumsum(lens, out=indptr[1:])
        idx = np.concatenate([np.arange(self.indptr[r], self.indptr[r + 1]) for r in rows]) if len(rows) else np.zeros(0, np.int64)
        return CSR(indptr, self.coords[idx].copy(), self.vals[idx].copy())


def zipf_cdf(n: int, s: float) -> np.ndarray:
    w = np.arange(1, n + 1, dtype=np.float64) ** (-float(s))
    c = np.cumsum(w)
    c /= c[-1]
    c[-1] = 1.0
    return c


def _guide_table(cdf: np.ndarray) -> np.ndarray:
    """Guide table for indexed inverse-CDF search (Chen and Asau, 1974)."""
    cells = 4 * len(cdf)
    return np.searchsorted(cdf, np.arange(cells, dtype=np.float64) / cells, side="right").astype(np.int64)


def _inverse_cdf(cdf: np.ndarray, guide: np.ndarray, u: np.ndarray) -> np.ndarray:
    """First index i with cdf[i] > u (same as searchsorted side='right'), clamped to n-1."""
    n = len(cdf)
    cells = len(guide)
    i = guide[np.minimum((u * cells).astype(np.int64), cells - 1)]
    np.minimum(i, n - 1, out=i)
    act = np.nonzero((cdf[i] <= u).ravel())[0]
    flat_i = i.ravel()
    flat_u = u.ravel()
    while len(act):
        flat_i[act] += 1
        np.minimum(flat_i, n - 1, out=flat_i)
        still = (cdf[flat_i[act]] <= flat_u[act]) & (flat_i[act] < n - 1)
        act = act[still]
    return i


def _distinct_rows(rng: np.random.Generator, cdf: np.ndarray, psi: np.ndarray, indptr: np.ndarray) -> np.ndarray:
    """Row i gets the first psi[i] distinct i.i.d. draws from ``cdf``, stored sorted."""
    n = len(cdf)
    guide = _guide_table(cdf)
    out = np.zeros(int(indptr[-1]), dtype=np.uint32)
    order = np.argsort(psi, kind="stable")
    pos = 0
    while pos < len(order):
        # group rows of similar size so the draw matrix is not padded much
        p0 = int(psi[order[pos]])
        lim = max(p0 + 8, int(p0 * 1.25))
        cap = max(1, 4_000_000 // (3 * lim + 64))
        end = int(np.searchsorted(psi[order], lim, side="right"))
        end = min(max(end, pos + 1), pos + cap)
        rows = order[pos:end]
        target = psi[rows].astype(np.int64)
        M = 3 * int(target.max()) + 64
        todo = np.arange(len(rows))
        while len(todo):
            B = len(todo)
            draws = _inverse_cdf(cdf, guide, rng.random((B, M)))
            # sort (coordinate, draw position) pairs packed in one int64 per draw
            key = draws * M + np.arange(M, dtype=np.int64)[None, :]
            key.sort(axis=1)
            sd = key // M
            o = key - sd * M
            first = np.ones_like(sd, dtype=bool)
            first[:, 1:] = sd[:, 1:] != sd[:, :-1]
            fpos = np.where(first, o, M)
            fpos.sort(axis=1)
            t = target[todo]
            kth = fpos[np.arange(B), np.clip(t, 1, M) - 1]
            ok = (t <= M) & (kth < M) & (t > 0)
            ok |= t == 0
            sel = np.nonzero(ok)[0]
            if len(sel):
                keep = first[sel] & (o[sel] <= kth[sel, None]) & (t[sel, None] > 0)
                vals = sd[sel][keep]
                dst_rows = rows[todo[sel]]
                lens = t[sel]
                starts = indptr[dst_rows]
                offs = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
                out[offs + np.arange(int(lens.sum()))] = vals
            todo = todo[~ok]
            M *= 2
        pos = end
    return out


def _values(rng: np.random.Generator, count: int, law: str) -> np.ndarray:
    def draw(c):
        if law == "normal":
            return rng.standard_normal(c)
        if law == "exp":
            return rng.exponential(1.0, c)
        if law == "uniform":
            return rng.uniform(-1.0, 1.0, c)
        raise ValueError(law)

    v = draw(count).astype(np.float32)
    bad = np.nonzero(v == 0)[0]
    while len(bad):
        v[bad] = draw(len(bad)).astype(np.float32)
        bad = bad[v[bad] == 0]
    return v


_CHUNK_ROWS = 65536


def _chunk(args):
    seed, chunk, psi, law, kind, n, zipf_s = args
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, chunk])))
    cdf = np.linspace(1.0 / n, 1.0, n) if kind == "uniform" else zipf_cdf(n, zipf_s)
    indptr = np.zeros(len(psi) + 1, dtype=np.int64)
    np.cumsum(psi, out=indptr[1:])
    coords = _distinct_rows(rng, cdf, psi, indptr)
    vals = _values(rng, len(coords), law)
    return coords, vals


def sparse_rows(seed: int, rows: int, n: int, zipf_s: float, psi: np.ndarray, law: str,
                uniform_coords: bool = False, workers: Optional[int] = None) -> CSR:
    """Rows with psi[i] distinct coordinates each (Zipf or uniform), values by ``law``.

    Rows are drawn in fixed chunks of 65,536 with their own seed stream
    (seed, chunk index), so the result does not depend on ``workers``.
    """
    psi = np.clip(np.asarray(psi, dtype=np.int64), 0, n)
    indptr = np.zeros(rows + 1, dtype=np.int64)
    np.cumsum(psi, out=indptr[1:])
    kind = "uniform" if uniform_coords else "zipf"
    jobs = [(seed, c, psi[a:a + _CHUNK_ROWS], law, kind, n, zipf_s)
            for c, a in enumerate(range(0, rows, _CHUNK_ROWS))]
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    if len(jobs) > 1 and workers > 1:
        # threads, not processes: numpy releases the GIL in the heavy steps, and
        # forked workers do not mix well with profilers attached to the parent
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(min(workers, len(jobs))) as pool:
            parts = list(pool.map(_chunk, jobs))
    else:
        parts = [_chunk(j) for j in jobs]
    coords = np.concatenate([p[0] for p in parts]) if parts else np.zeros(0, np.uint32)
    vals = np.concatenate([p[1] for p in parts]) if parts else np.zeros(0, np.float32)
    return CSR(indptr, coords.astype(np.uint32), vals.astype(np.float32))


def lognormal_counts(rng: np.random.Generator, rows: int, mean: float, sigma: float, n: int) -> np.ndarray:
    """round(LogNormal) with E[X] = mean, clamped to [1, n]."""
    mu = math.log(mean) - 0.5 * sigma * sigma
    return np.clip(np.rint(rng.lognormal(mu, sigma, rows)), 1, n).astype(np.int64)


@dataclasses.dataclass
class Workload:
    name: str
    n: int  # dimensionality
    m: int  # sketch buckets per half
    h: int  # number of random mappings
    hash_seed: int
    k: int
    docs: CSR
    queries: CSR
    ks: tuple = ()


# ---------------------------------------------------------------------------
# The five workloads. Names carry what they are and their sizes.
# ---------------------------------------------------------------------------

def doc_counts_small(rng, rows):  # uniform integer 20..60
    return rng.integers(20, 61, rows)


def make_small(seed: int = 0, docs: int = 10_000, queries: int = 100, query_nnz: int = 20) -> Workload:
    """10k docs, dim 1,000, nnz U{20..60}, Zipf(1.1), N(0,1); m=32, h=1; k=10."""
    n = 1000
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    d = sparse_rows(seed, docs, n, 1.1, doc_counts_small(rng, docs), "normal")
    q = sparse_rows(seed + 1, queries, n, 1.1, np.full(queries, query_nnz), "normal")
    return Workload("small-10k-dim1000", n, 32, 1, seed, 10, d, q, (10,))


def make_splade_like(seed: int = 0, docs: int = 1_000_000, queries: int = 1024) -> Workload:
    """1M docs, dim 30,522, nnz lognormal(mean 120, s 0.5), Zipf(1.05), Exp(1); m=128, h=1."""
    n = 30522
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    d = sparse_rows(seed, docs, n, 1.05, lognormal_counts(rng, docs, 120.0, 0.5, n), "exp")
    rngq = np.random.Generator(np.random.PCG64(seed + 2000))
    q = sparse_rows(seed + 1, queries, n, 1.05, lognormal_counts(rngq, queries, 40.0, 0.5, n), "exp")
    return Workload("splade-like-1m-dim30522", n, 128, 1, seed, 10, d, q, (10, 100))


def uneven_query_counts(rng, rows, lo=5, hi=400):
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), rows))).astype(np.int64)


def bernoulli_counts(rng, rows, psi, n):
    """nnz of vectors whose every coordinate is non-zero with probability psi / n."""
    return rng.binomial(n, psi / n, rows).astype(np.int64)


def make_gaussian(seed: int = 0, psi: int = 100, docs: int = 5_000_000, queries: int = 1000) -> Workload:
    """The real-valued collections of Section 6.5: every coordinate is non-zero
    with probability psi / n (uniform coordinates), values N(0, 1); 5M docs and
    1,000 queries of the same law. G100: psi = 100, n = 10,000, 2m = 74;
    G200: psi = 200, n = 32,000, 2m = 150 (Table 4); h = 1; k = 1,000."""
    n, m = {100: (10_000, 37), 200: (32_000, 75)}[psi]
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    d = sparse_rows(seed, docs, n, 1.0, bernoulli_counts(rng, docs, psi, n), "normal", uniform_coords=True)
    rngq = np.random.Generator(np.random.PCG64(seed + 2000))
    q = sparse_rows(seed + 1, queries, n, 1.0, bernoulli_counts(rngq, queries, psi, n), "normal",
                    uniform_coords=True)
    return Workload("g%d-%dm-dim%d" % (psi, docs // 1_000_000, n), n, m, 1, seed, 1000, d, q, (1000,))


def make_batch(seed: int = 0, docs: int = 4_000_000, queries: int = 8192) -> Workload:
    """Small-workload laws at 4M docs; 8,192 queries with nnz log-uniform 5..400; k=100."""
    n = 1000
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    d = sparse_rows(seed, docs, n, 1.1, doc_counts_small(rng, docs), "normal")
    rngq = np.random.Generator(np.random.PCG64(seed + 2000))
    q = sparse_rows(seed + 1, queries, n, 1.1, uneven_query_counts(rngq, queries), "normal")
    return Workload("batch-4m-dim1000", n, 32, 1, seed, 100, d, q, (100,))


def small_queries(seed: int, count: int, query_nnz: int = 20) -> CSR:
    """Queries with the small workload's law (Zipf(1.1) over dim 1,000, N(0,1))."""
    return sparse_rows(seed, count, 1000, 1.1, np.full(count, query_nnz), "normal")


def serving_queries(seed: int, count: int) -> CSR:
    rng = np.random.Generator(np.random.PCG64(seed + 3000))
    return sparse_rows(seed, count, 1000, 1.1, lognormal_counts(rng, count, 40.0, 0.5, 1000), "normal")


def small_docs(seed: int, count: int) -> CSR:
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    return sparse_rows(seed, count, 1000, 1.1, doc_counts_small(rng, count), "normal")


def serving_trace(seed: int, ops: int, live_ids: np.ndarray, next_id: int, rate_qps: float,
                  frac_query: float = 0.85, frac_insert: float = 0.10, ks=(10, 100, 1000)):
    """Poisson arrivals with an op mix; returns dict of numpy arrays describing the trace.

    kind: 0 = query, 1 = insert, 2 = delete. Inserted docs take fresh ids; deletes
    pick uniformly among ids live at that point of the trace.
    """
    rng = np.random.Generator(np.random.PCG64(seed + 4))
    u = rng.random(ops)
    kind = np.where(u < frac_query, 0, np.where(u < frac_query + frac_insert, 1, 2)).astype(np.int32)
    gaps = rng.exponential(1.0 / rate_qps * frac_query, ops)
    t = np.cumsum(gaps)
    live = list(map(int, live_ids))
    pos = {v: i for i, v in enumerate(live)}
    ids = np.zeros(ops, dtype=np.uint32)
    kk = np.zeros(ops, dtype=np.uint32)
    nid = next_id
    for i in range(ops):
        if kind[i] == 0:
            kk[i] = ks[int(rng.integers(0, len(ks)))]
        elif kind[i] == 1:
            ids[i] = nid
            pos[nid] = len(live)
            live.append(nid)
            nid += 1
        else:
            if not live:
                kind[i] = 0
                kk[i] = ks[0]
                continue
            j = int(rng.integers(0, len(live)))
            v = live[j]
            ids[i] = v
            last = live[-1]
            live[j] = last
            pos[last] = j
            live.pop()
            del pos[v]
    nq = int((kind == 0).sum())
    ni = int((kind == 1).sum())
    queries = serving_queries(seed + 1, nq)
    docs = small_docs(seed + 2, ni)
    return dict(kind=kind, t=t, ids=ids, k=kk, queries=queries, docs=docs)


def trace_csr(tr: dict) -> CSR:
    """Per-request vectors of a serving trace in request order (queries and
    inserted documents; deletes get an empty row)."""
    kind = tr["kind"]
    q, d = tr["queries"], tr["docs"]
    lens = np.zeros(len(kind), dtype=np.int64)
    qi = np.nonzero(kind == 0)[0]
    di = np.nonzero(kind == 1)[0]
    lens[qi] = np.diff(q.indptr)
    lens[di] = np.diff(d.indptr)
    indptr = np.zeros(len(kind) + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    coords = np.zeros(int(indptr[-1]), dtype=np.uint32)
    vals = np.zeros(int(indptr[-1]), dtype=np.float32)
    for rows, src in ((qi, q), (di, d)):
        for j, r in enumerate(rows):
            a, b = int(indptr[r]), int(indptr[r + 1])
            c, v = src.row(j)
            coords[a:b] = c
            vals[a:b] = v
    return CSR(indptr, coords, vals)
