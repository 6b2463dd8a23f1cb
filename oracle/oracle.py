"""ctypes wrapper of the FP64 Sinnamon oracle (``sinnamon_oracle.c``).

TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the GPU library and its Python
binding never do, and the two share no code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sinnamon_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Portable x86-64 level (the library may be built on one host and run on another).
CFLAGS = ["-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        u32, u64, i32, d = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
        P = ctypes.c_void_p
        L.orc_mix64.restype = u64
        L.orc_mix64.argtypes = [u64]
        L.orc_bucket.restype = u32
        L.orc_bucket.argtypes = [u64, u32, u32, u32]
        L.orc_bucket_table.argtypes = [u64, u32, u32, u32, P]
        for f in (L.orc_sketch, L.orc_sketch_by_bucket):
            f.argtypes = [u32, P, P, u32, u32, u64, P, P, P]
        L.orc_decode_doc.argtypes = [u32, P, P, u32, u32, u64, P, P]
        L.orc_pair_est.restype = d
        L.orc_pair_est.argtypes = [u32, P, P, u32, P, P, u32, u32, u64, P]
        L.orc_pair_exact.restype = d
        L.orc_pair_exact.argtypes = [u32, P, P, u32, P, P]
        L.orc_build.restype = P
        L.orc_build.argtypes = [u32, P, P, P, P, u32, u32, u32, u64, u32]
        L.orc_bf16_up.restype = d
        L.orc_bf16_up.argtypes = [ctypes.c_float]
        L.orc_bf16_down.restype = d
        L.orc_bf16_down.argtypes = [ctypes.c_float]
        L.orc_free.argtypes = [P]
        L.orc_postings.restype = u64
        L.orc_postings.argtypes = [P]
        L.orc_score_all.argtypes = [P, u32, P, P, i32, u32, P, P]
        L.orc_find_largest.restype = u32
        L.orc_find_largest.argtypes = [u32, P, P, P, u32, P]
        L.orc_search.argtypes = [P, u32, P, P, P, u32, i32, u32, i32, P, P, P, P]
        L.orc_rerank.argtypes = [P, u32, P, P, P, u32, u32, u32, i32, P, P, P, P]
        L.orc_max_threads.restype = i32
        L.orc_features.argtypes = [u32, P, P, u64, P]
        L.orc_mlp_forward.argtypes = [u32, P, P, P, P, P, P, P, P]
        L.orc_mlp_loss_grad.restype = d
        L.orc_mlp_loss_grad.argtypes = [u32, P, P, P, P, P, P, P, P] + [P] * 6
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint32)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def mix64(z: int) -> int:
    return int(lib().orc_mix64(ctypes.c_uint64(z & 0xFFFFFFFFFFFFFFFF)))


def bucket(seed: int, o: int, j: int, m: int) -> int:
    return int(lib().orc_bucket(seed, o, j, m))


def bucket_table(seed: int, h: int, n: int, m: int) -> np.ndarray:
    out = np.zeros((h, n), dtype=np.uint32)
    lib().orc_bucket_table(seed, h, n, m, _p(out))
    return out


def sketch(coords, vals, m: int, h: int, seed: int, by_bucket: bool = False):
    c, v = _u32(coords), _f32(vals)
    u = np.zeros(m)
    l = np.zeros(m)
    filled = np.zeros(m, dtype=np.uint8)
    f = lib().orc_sketch_by_bucket if by_bucket else lib().orc_sketch
    f(len(c), _p(c), _p(v), m, h, seed, _p(u), _p(l), _p(filled))
    return u, l, filled.astype(bool)


def pair_est(qc, qv, dc, dv, m: int, h: int, seed: int):
    qc, qv, dc, dv = _u32(qc), _f32(qv), _u32(dc), _f32(dv)
    a = np.zeros(1)
    s = lib().orc_pair_est(len(qc), _p(qc), _p(qv), len(dc), _p(dc), _p(dv), m, h, seed, _p(a))
    return float(s), float(a[0])


def pair_exact(qc, qv, dc, dv) -> float:
    qc, qv, dc, dv = _u32(qc), _f32(qv), _u32(dc), _f32(dv)
    return float(lib().orc_pair_exact(len(qc), _p(qc), _p(qv), len(dc), _p(dc), _p(dv)))


def find_largest(scores, k: int, ids=None, live=None) -> np.ndarray:
    """Positions of the k best (score desc, id asc) among live entries (Alg. 3)."""
    sc = np.ascontiguousarray(scores, dtype=np.float64)
    ida = _u32(ids) if ids is not None else None
    lv = np.ascontiguousarray(live, dtype=np.uint8) if live is not None else None
    out = np.zeros(max(k, 1), dtype=np.uint32)
    c = lib().orc_find_largest(len(sc), _p(sc), _p(ida) if ida is not None else None,
                               _p(lv) if lv is not None else None, k, _p(out))
    return out[:c].astype(np.int64)


def decode_doc(coords, vals, m: int, h: int, seed: int):
    """(upper, lower) decode of each of the document's coordinates from its own sketch."""
    c, v = _u32(coords), _f32(vals)
    up = np.zeros(len(c))
    lo = np.zeros(len(c))
    lib().orc_decode_doc(len(c), _p(c), _p(v), m, h, seed, _p(up), _p(lo))
    return up, lo


class Index:
    """Coordinate-at-a-time oracle index over a fixed set of documents."""

    def __init__(self, docs, n: int, m: int, h: int, seed: int, ids: Optional[np.ndarray] = None,
                 bf16: bool = False):
        """bf16: the sketch is stored in bfloat16, U rounded up and L down."""
        self.indptr = np.ascontiguousarray(docs.indptr, dtype=np.int64)
        self.coords = _u32(docs.coords)
        self.vals = _f32(docs.vals)
        self.N = len(self.indptr) - 1
        self.ids = _u32(ids if ids is not None else np.arange(self.N))
        self.n, self.m, self.h, self.seed = n, m, h, seed
        self._h = lib().orc_build(self.N, _p(self.indptr), _p(self.coords), _p(self.vals), _p(self.ids),
                                  n, m, h, seed, 1 if bf16 else 0)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_free(self._h)
            self._h = None

    @property
    def postings(self) -> int:
        return int(lib().orc_postings(self._h))

    def score_all(self, qc, qv, exact: bool = False, max_coords: int = 0):
        """Scores of every document (Alg. 6 estimate or exact); max_coords > 0
        stops after that many coordinates in the sorted order (anytime)."""
        qc, qv = _u32(qc), _f32(qv)
        s = np.zeros(max(self.N, 1))
        a = np.zeros(max(self.N, 1))
        lib().orc_score_all(self._h, len(qc), _p(qc), _p(qv), 1 if exact else 0, max_coords, _p(s), _p(a))
        return s[: self.N], a[: self.N]

    def search(self, queries, k: int, exact: bool = False, threads: int = 1, max_coords: int = 0):
        qp = np.ascontiguousarray(queries.indptr, dtype=np.int64)
        qc, qv = _u32(queries.coords), _f32(queries.vals)
        nq = len(qp) - 1
        ids = np.zeros((nq, max(k, 1)), dtype=np.uint32)
        sc = np.zeros((nq, max(k, 1)))
        ab = np.zeros((nq, max(k, 1)))
        cnt = np.zeros(nq, dtype=np.uint32)
        lib().orc_search(self._h, nq, _p(qp), _p(qc), _p(qv), k, 1 if exact else 0, max_coords, threads,
                         _p(ids), _p(sc), _p(ab), _p(cnt))
        return ids[:, :k], sc[:, :k], ab[:, :k], cnt

    def rerank(self, queries, k: int, kprime: int, threads: int = 1, max_coords: int = 0):
        """Alg. 7 with k' >= k: (ids, exact scores, sum |q_j x_j|, counts);
        max_coords > 0 makes the candidate scoring anytime."""
        qp = np.ascontiguousarray(queries.indptr, dtype=np.int64)
        qc, qv = _u32(queries.coords), _f32(queries.vals)
        nq = len(qp) - 1
        ids = np.zeros((nq, max(k, 1)), dtype=np.uint32)
        sc = np.zeros((nq, max(k, 1)))
        ab = np.zeros((nq, max(k, 1)))
        cnt = np.zeros(nq, dtype=np.uint32)
        lib().orc_rerank(self._h, nq, _p(qp), _p(qc), _p(qv), k, kprime, max_coords, threads, _p(ids), _p(sc), _p(ab),
                         _p(cnt))
        return ids[:, :k], sc[:, :k], ab[:, :k], cnt


def bf16_up(x: float) -> float:
    return float(lib().orc_bf16_up(float(x)))


def bf16_down(x: float) -> float:
    return float(lib().orc_bf16_down(float(x)))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def features(qc, qv, fseed: int) -> np.ndarray:
    qc, qv = _u32(qc), _f32(qv)
    f = np.zeros(256)
    lib().orc_features(len(qc), _p(qc), _p(qv), fseed, _p(f))
    return f


MLP_SHAPES = {"W1": (128, 256), "b1": (128,), "W2": (128, 128), "b2": (128,), "W3": (128,), "b3": (1,)}


def _params(p):
    return [np.ascontiguousarray(p[k], dtype=np.float64).reshape(MLP_SHAPES[k]) for k in MLP_SHAPES]


def mlp_forward(X, p) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    B = X.shape[0]
    ws = _params(p)
    y = np.zeros(B)
    lib().orc_mlp_forward(B, _p(X), *[_p(w) for w in ws], _p(y))
    return y


def mlp_loss_grad(X, y, p):
    X = np.ascontiguousarray(X, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    B = X.shape[0]
    ws = _params(p)
    gs = [np.zeros_like(w) for w in ws]
    loss = lib().orc_mlp_loss_grad(B, _p(X), _p(y), *[_p(w) for w in ws], *[_p(g) for g in gs])
    return float(loss), dict(zip(MLP_SHAPES, gs))


# ---------------------------------------------------------------------------
# Closed forms from the analysis section (used as pins, not by the library).
# ---------------------------------------------------------------------------

def prob_error_gaussian(m: int, h: int, n_minus_1_p: float) -> float:
    """Corollary to Theorem 2: P[upper-bound decode > x] for zero-mean Gaussian values
    (the proof only uses that the value law is continuous)."""
    from math import comb, exp
    b = h * n_minus_1_p / m
    s = 1.0
    for kk in range(1, h + 1):
        s += comb(h, kk) * (-1) ** kk * (1.0 / (kk * b)) * (1.0 - exp(-kk * b))
    return s


def prob_error_integral(m: int, h: int, sum_p: float, cdf, pdf, lo: float, hi: float) -> float:
    """Theorem 2's integral, evaluated numerically for a continuous value law."""
    from scipy import integrate
    f = lambda a: (1.0 - np.exp(-(h / m) * (1.0 - cdf(a)) * sum_p)) ** h * pdf(a)
    return float(integrate.quad(f, lo, hi, limit=200)[0])
