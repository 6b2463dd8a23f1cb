"""Python binding of libsnn.so, the MI355X (gfx950) Sinnamon library.

Argument marshalling only: every step of insert, delete and search runs in the
library's HIP kernels. PyTorch provides device memory and streams for the
device-pointer entry points. The binding fails loudly when the library is not
built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

try:  # load torch first so the library shares torch's HIP runtime in this process
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsnn.so")

SNN_OK = 0
STATUS = {0: "SNN_OK", -1: "SNN_E_INVALID", -2: "SNN_E_EXISTS", -3: "SNN_E_NOT_FOUND", -4: "SNN_E_FULL",
          -5: "SNN_E_NOMEM", -6: "SNN_E_BUSY", -7: "SNN_E_DEVICE"}
MODE_PLAIN, MODE_BATCHED, MODE_LEARNED = 0, 1, 2
FORWARD_STORE = 1  # snn_config.flags: keep the vectors on the device (re-ranking, Alg. 7)
SKETCH_BF16 = 2    # sketch stored in bfloat16, U rounded up and L down
UPPER_ONLY = 4     # no L half (Sinnamon+, non-negative collections)

# every symbol include/snn.h declares (checked by the test suite)
EXPORTS = [
    "snn_create", "snn_destroy", "snn_insert", "snn_insert_batch", "snn_delete", "snn_delete_batch",
    "snn_search", "snn_search_batch", "snn_search_batch_dev", "snn_last_batch_status",
    "snn_last_batch_work", "snn_search_rerank", "snn_search_rerank_dev", "snn_search_ex", "snn_search_ex_dev",
                     "snn_bucket_table",
    "snn_read_sketch", "snn_live_count", "snn_last_error", "snn_profile_enable", "snn_profile_read",
    "snn_profile_read_updates", "snn_autotune", "snn_get_schedule", "snn_set_schedule",
    "snn_filter_train", "snn_filter_features", "snn_filter_predict", "snn_filter_get_params",
    "snn_filter_set_params", "snn_filter_set_delta", "snn_filter_enable", "snn_mlp_loss_grad", "snn_serve_run",
    "snn_search_batch_dev_noalloc", "snn_compact", "snn_container_classes",
]
NOALLOC_SCRATCH_BYTES = 64 << 20
MLP_PARAMS = 49537


class SnnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, str(status)), msg))
        self.status = status


class Schedule(ctypes.Structure):
    _fields_ = [("R_plain", ctypes.c_int32), ("R_batch", ctypes.c_int32), ("grid", ctypes.c_uint32),
                ("persistent", ctypes.c_uint32), ("best_ms", ctypes.c_float), ("default_ms", ctypes.c_float),
                ("tried", ctypes.c_uint32), ("qgroup", ctypes.c_uint32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class FilterParams(ctypes.Structure):
    _fields_ = [("feature_seed", ctypes.c_uint64), ("seed", ctypes.c_uint64), ("k", ctypes.c_uint32),
                ("epochs", ctypes.c_uint32), ("batch", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("holdout", ctypes.c_float), ("target_fallback", ctypes.c_float)]


class FilterReport(ctypes.Structure):
    _fields_ = [("n_train", ctypes.c_uint32), ("n_holdout", ctypes.c_uint32), ("n_unlabelled", ctypes.c_uint32),
                ("steps", ctypes.c_uint32), ("train_mse", ctypes.c_float), ("holdout_mse", ctypes.c_float),
                ("delta", ctypes.c_float), ("holdout_fallback", ctypes.c_float), ("label_ms", ctypes.c_float),
                ("train_ms", ctypes.c_float)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Trace(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("kind", ctypes.c_void_p), ("arrival_s", ctypes.c_void_p),
                ("id", ctypes.c_void_p), ("k", ctypes.c_void_p), ("indptr", ctypes.c_void_p),
                ("coords", ctypes.c_void_p), ("vals", ctypes.c_void_p)]


class ServeParams(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_uint32), ("max_inflight", ctypes.c_uint32), ("streams", ctypes.c_uint32),
                ("realtime", ctypes.c_uint32), ("budget_bytes", ctypes.c_uint64)]


class ServeReport(ctypes.Structure):
    _fields_ = [("searches", ctypes.c_uint32), ("inserts", ctypes.c_uint32), ("deletes", ctypes.c_uint32),
                ("rejected", ctypes.c_uint32), ("batches", ctypes.c_uint32), ("max_batch_seen", ctypes.c_uint32),
                ("max_inflight_seen", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("wall_s", ctypes.c_double),
                ("search_qps", ctypes.c_double), ("p50_ms", ctypes.c_double), ("p90_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("mutation_p50_ms", ctypes.c_double), ("mutation_p99_ms", ctypes.c_double),
                ("peak_workspace_bytes", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class SearchParams(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_uint32), ("k_prime", ctypes.c_uint32), ("max_coords", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class BatchWork(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_uint64), ("candidates_fallback", ctypes.c_uint64),
                ("selects", ctypes.c_uint64), ("selects_fallback", ctypes.c_uint64)]


class Config(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_uint32), ("m", ctypes.c_uint32), ("h", ctypes.c_uint32),
                ("capacity", ctypes.c_uint32), ("hash_seed", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


_lib = None


def lib():
    """Load libsnn.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsnn.so is not built: run __graft_entry__.build() (hipcc for gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        P, u32, u64, i32, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_size_t
        L.snn_create.argtypes = [ctypes.POINTER(Config), P, ctypes.POINTER(P)]
        L.snn_destroy.argtypes = [P]
        L.snn_destroy.restype = None
        L.snn_insert.argtypes = [P, u32, u32, P, P]
        L.snn_insert_batch.argtypes = [P, u32, P, P, P, P]
        L.snn_delete.argtypes = [P, u32]
        L.snn_delete_batch.argtypes = [P, u32, P]
        L.snn_search.argtypes = [P, u32, P, P, u32, P, P, P]
        L.snn_search_batch.argtypes = [P, u32, P, P, P, u32, P, P, P]
        L.snn_search_batch_dev.argtypes = [P, u32, P, u64, P, P, u32, u32, P, P, P, P]
        L.snn_search_batch_dev_noalloc.argtypes = [P, u32, P, u64, P, P, u32, u32, P, P, P, P]
        L.snn_compact.argtypes = [P, P]
        L.snn_container_classes.argtypes = [P, P]
        L.snn_last_batch_status.argtypes = [P, P, P]
        L.snn_search_rerank.argtypes = [P, u32, P, P, P, u32, u32, P, P, P]
        L.snn_search_ex.argtypes = [P, u32, P, P, P, u32, P, P, P, P]
        L.snn_search_ex_dev.argtypes = [P, u32, P, u64, P, P, u32, P, P, P, P, P]
        L.snn_search_rerank_dev.argtypes = [P, u32, P, u64, P, P, u32, u32, P, P, P, P]
        L.snn_last_batch_work.argtypes = [P, P]
        L.snn_bucket_table.argtypes = [P, P]
        L.snn_read_sketch.argtypes = [P, u32, P, P]
        L.snn_profile_enable.argtypes = [P, i32]
        L.snn_profile_read.argtypes = [P, P, P]
        L.snn_profile_read_updates.argtypes = [P, P, P, P, P]
        L.snn_autotune.argtypes = [P, u32, P, u64, P, P, u32, P]
        L.snn_get_schedule.argtypes = [P, P]
        L.snn_set_schedule.argtypes = [P, P]
        L.snn_filter_train.argtypes = [P, u32, P, u64, P, P, P, P]
        L.snn_filter_features.argtypes = [P, u32, P, P, P, P]
        L.snn_filter_predict.argtypes = [P, u32, P, P, P, P]
        L.snn_filter_get_params.argtypes = [P, P]
        L.snn_filter_set_params.argtypes = [P, P, u64, u32]
        L.snn_filter_set_delta.argtypes = [P, ctypes.c_float]
        L.snn_filter_enable.argtypes = [P, i32]
        L.snn_mlp_loss_grad.argtypes = [P, u32, P, P, P, P]
        L.snn_serve_run.argtypes = [P, P, P, P, P, P, P, P]
        L.snn_live_count.argtypes = [P]
        L.snn_live_count.restype = sz
        L.snn_last_error.argtypes = [P]
        L.snn_last_error.restype = ctypes.c_char_p
        for name in ("snn_create", "snn_insert", "snn_insert_batch", "snn_delete", "snn_delete_batch", "snn_search",
                     "snn_search_batch", "snn_search_batch_dev", "snn_last_batch_status",
                     "snn_last_batch_work", "snn_search_rerank", "snn_search_rerank_dev", "snn_search_ex", "snn_search_ex_dev",
    "snn_bucket_table",
                     "snn_read_sketch", "snn_profile_enable", "snn_profile_read", "snn_profile_read_updates", "snn_autotune",
                     "snn_get_schedule", "snn_set_schedule", "snn_filter_train", "snn_filter_features",
                     "snn_filter_predict", "snn_filter_get_params", "snn_filter_set_params", "snn_filter_set_delta",
                     "snn_filter_enable", "snn_mlp_loss_grad", "snn_serve_run", "snn_search_batch_dev_noalloc", "snn_compact",
                     "snn_container_classes"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _tp(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


class Index:
    """A device-resident Sinnamon index (owns its device memory)."""

    def __init__(self, dim: int, m: int, h: int = 1, capacity: int = 1 << 16, hash_seed: int = 0, stream=None,
                 forward_store: bool = False, sketch_bf16: bool = False, upper_only: bool = False):
        L = lib()
        flags = (FORWARD_STORE if forward_store else 0) | (SKETCH_BF16 if sketch_bf16 else 0) | \
            (UPPER_ONLY if upper_only else 0)
        self._cfg = Config(dim, m, h, capacity, hash_seed, flags, 0)
        self.dim, self.m, self.h = dim, m, h
        h_ptr = ctypes.c_void_p()
        if stream is None and torch is not None and torch.cuda.is_available():
            stream = torch.cuda.current_stream()
        self._stream = stream
        st = L.snn_create(ctypes.byref(self._cfg), _stream_handle(stream) if stream is not None else None,
                          ctypes.byref(h_ptr))
        if st != SNN_OK:
            raise SnnError(st, "snn_create failed")
        self._h = h_ptr

    def close(self):
        if getattr(self, "_h", None):
            lib().snn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != SNN_OK:
            raise SnnError(st, lib().snn_last_error(self._h).decode())

    def compact(self, classes=None):
        """snn_compact: array containers for the sparse coordinates (or the
        pinned `classes`, dim bytes, non-zero = array)."""
        if classes is None:
            self._check(lib().snn_compact(self._h, None))
        else:
            c = np.ascontiguousarray(classes, dtype=np.uint8)
            assert c.shape == (self.dim,)
            self._check(lib().snn_compact(self._h, _p(c)))

    def container_classes(self) -> np.ndarray:
        out = np.zeros(self.dim, np.uint8)
        self._check(lib().snn_container_classes(self._h, _p(out)))
        return out

    # ------------------------------------------------------------------ updates
    def insert(self, id: int, coords, vals):
        c = np.ascontiguousarray(coords, dtype=np.uint32)
        v = np.ascontiguousarray(vals, dtype=np.float32)
        self._check(lib().snn_insert(self._h, int(id), len(c), _p(c), _p(v)))

    def insert_batch(self, ids, indptr, coords, vals):
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        ip = np.ascontiguousarray(indptr, dtype=np.uint64)
        c = np.ascontiguousarray(coords, dtype=np.uint32)
        v = np.ascontiguousarray(vals, dtype=np.float32)
        self._check(lib().snn_insert_batch(self._h, len(ids), _p(ids), _p(ip), _p(c), _p(v)))

    def delete(self, id: int):
        self._check(lib().snn_delete(self._h, int(id)))

    def delete_batch(self, ids):
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        self._check(lib().snn_delete_batch(self._h, len(ids), _p(ids)))

    @property
    def live_count(self) -> int:
        return int(lib().snn_live_count(self._h))

    # ------------------------------------------------------------------- search
    def search(self, coords, vals, k: int) -> Tuple[np.ndarray, np.ndarray]:
        c = np.ascontiguousarray(coords, dtype=np.uint32)
        v = np.ascontiguousarray(vals, dtype=np.float32)
        ids = np.zeros(k, np.uint32)
        sc = np.zeros(k, np.float32)
        cnt = np.zeros(1, np.uint32)
        self._check(lib().snn_search(self._h, len(c), _p(c), _p(v), k, _p(ids), _p(sc), _p(cnt)))
        return ids[: cnt[0]], sc[: cnt[0]]

    def search_batch(self, indptr, coords, vals, k: int):
        ip = np.ascontiguousarray(indptr, dtype=np.uint64)
        c = np.ascontiguousarray(coords, dtype=np.uint32)
        v = np.ascontiguousarray(vals, dtype=np.float32)
        nq = len(ip) - 1
        ids = np.zeros((nq, k), np.uint32)
        sc = np.zeros((nq, k), np.float32)
        cnt = np.zeros(nq, np.uint32)
        self._check(lib().snn_search_batch(self._h, nq, _p(ip), _p(c), _p(v), k, _p(ids), _p(sc), _p(cnt)))
        return ids, sc, cnt

    def search_rerank(self, indptr, coords, vals, k: int, k_prime: int):
        """Alg. 7 with k' = k_prime: (ids, exact scores, counts) from host buffers."""
        ip = np.ascontiguousarray(indptr, dtype=np.uint64)
        c = np.ascontiguousarray(coords, dtype=np.uint32)
        v = np.ascontiguousarray(vals, dtype=np.float32)
        nq = len(ip) - 1
        ids = np.zeros((nq, k), np.uint32)
        sc = np.zeros((nq, k), np.float32)
        cnt = np.zeros(nq, np.uint32)
        self._check(lib().snn_search_rerank(self._h, nq, _p(ip), _p(c), _p(v), k, k_prime, _p(ids), _p(sc), _p(cnt)))
        return ids, sc, cnt

    def search_ex(self, indptr, coords, vals, k: int, mode: int = MODE_BATCHED, k_prime: int = 0,
                  max_coords: int = 0):
        """Batch search from host buffers with options: mode, Alg. 7 width k'
        and the anytime coordinate budget. Returns (ids, scores, counts)."""
        ip = np.ascontiguousarray(indptr, dtype=np.uint64)
        c = np.ascontiguousarray(coords, dtype=np.uint32)
        v = np.ascontiguousarray(vals, dtype=np.float32)
        nq = len(ip) - 1
        ids = np.zeros((nq, k), np.uint32)
        sc = np.zeros((nq, k), np.float32)
        cnt = np.zeros(nq, np.uint32)
        prm = SearchParams(mode, k_prime, max_coords, 0)
        self._check(lib().snn_search_ex(self._h, nq, _p(ip), _p(c), _p(v), k, ctypes.byref(prm), _p(ids), _p(sc),
                                        _p(cnt)))
        return ids, sc, cnt

    def search_ex_dev(self, indptr, coords, vals, k: int, mode: int = MODE_BATCHED, k_prime: int = 0,
                      max_coords: int = 0, out=None, stream=None, total: Optional[int] = None):
        """Device tensors in and out, with the options of search_ex."""
        nq = indptr.numel() - 1
        if total is None:
            total = int(coords.numel())
        dev = indptr.device
        if out is None:
            out = (torch.empty((nq, k), dtype=torch.int32, device=dev),
                   torch.empty((nq, k), dtype=torch.float32, device=dev),
                   torch.empty(nq, dtype=torch.int32, device=dev))
        ids, sc, cnt = out
        assert indptr.dtype == torch.int64 and coords.dtype == torch.int32 and vals.dtype == torch.float32
        assert indptr.is_contiguous() and coords.is_contiguous() and vals.is_contiguous()
        assert ids.shape == (nq, k) and sc.shape == (nq, k) and cnt.shape == (nq,)
        prm = SearchParams(mode, k_prime, max_coords, 0)
        self._check(lib().snn_search_ex_dev(self._h, nq, _tp(indptr), int(total), _tp(coords), _tp(vals), k,
                                            ctypes.byref(prm), _tp(ids), _tp(sc), _tp(cnt), _stream_handle(stream)))
        return ids, sc, cnt

    def search_rerank_dev(self, indptr, coords, vals, k: int, k_prime: int, out=None, stream=None,
                          total: Optional[int] = None):
        """Alg. 7 with k' = k_prime on device tensors; outputs (ids, exact scores, counts)."""
        nq = indptr.numel() - 1
        if total is None:
            total = int(coords.numel())
        dev = indptr.device
        if out is None:
            out = (torch.empty((nq, k), dtype=torch.int32, device=dev),
                   torch.empty((nq, k), dtype=torch.float32, device=dev),
                   torch.empty(nq, dtype=torch.int32, device=dev))
        ids, sc, cnt = out
        assert indptr.dtype == torch.int64 and coords.dtype == torch.int32 and vals.dtype == torch.float32
        assert indptr.is_contiguous() and coords.is_contiguous() and vals.is_contiguous()
        assert ids.shape == (nq, k) and sc.shape == (nq, k) and cnt.shape == (nq,)
        self._check(lib().snn_search_rerank_dev(self._h, nq, _tp(indptr), int(total), _tp(coords), _tp(vals), k,
                                                k_prime, _tp(ids), _tp(sc), _tp(cnt), _stream_handle(stream)))
        return ids, sc, cnt

    def search_batch_dev(self, indptr, coords, vals, k: int, mode: int = MODE_BATCHED, out=None, stream=None,
                         total: Optional[int] = None):
        """Device tensors in, device tensors out (ids, scores, counts); enqueued on `stream`.
        `total` = indptr[-1] (read from the tensors when not given)."""
        nq = indptr.numel() - 1
        if total is None:
            total = int(coords.numel())
        dev = indptr.device
        if out is None:
            out = (torch.empty((nq, k), dtype=torch.int32, device=dev),
                   torch.empty((nq, k), dtype=torch.float32, device=dev),
                   torch.empty(nq, dtype=torch.int32, device=dev))
        ids, sc, cnt = out
        assert indptr.dtype == torch.int64 and coords.dtype == torch.int32 and vals.dtype == torch.float32
        assert indptr.is_contiguous() and coords.is_contiguous() and vals.is_contiguous()
        assert ids.shape == (nq, k) and sc.shape == (nq, k) and cnt.shape == (nq,)
        self._check(lib().snn_search_batch_dev(self._h, nq, _tp(indptr), int(total), _tp(coords), _tp(vals), k, mode,
                                               _tp(ids), _tp(sc), _tp(cnt), _stream_handle(stream)))
        return ids, sc, cnt

    def search_batch_dev_noalloc(self, indptr, coords, vals, k: int, mode: int = MODE_BATCHED, out=None,
                                 stream=None, total: Optional[int] = None):
        """search_batch_dev with the workspace in the library's fixed device
        array (snn_search_batch_dev_noalloc): nothing is allocated by the
        call. `out` (ids, scores, counts) must be given when the caller
        cannot allocate either."""
        nq = indptr.numel() - 1
        if total is None:
            total = int(coords.numel())
        dev = indptr.device
        if out is None:
            out = (torch.empty((nq, k), dtype=torch.int32, device=dev),
                   torch.empty((nq, k), dtype=torch.float32, device=dev),
                   torch.empty(nq, dtype=torch.int32, device=dev))
        ids, sc, cnt = out
        assert indptr.dtype == torch.int64 and coords.dtype == torch.int32 and vals.dtype == torch.float32
        assert indptr.is_contiguous() and coords.is_contiguous() and vals.is_contiguous()
        assert ids.shape == (nq, k) and sc.shape == (nq, k) and cnt.shape == (nq,)
        self._check(lib().snn_search_batch_dev_noalloc(self._h, nq, _tp(indptr), int(total), _tp(coords), _tp(vals),
                                                       k, mode, _tp(ids), _tp(sc), _tp(cnt), _stream_handle(stream)))
        return ids, sc, cnt

    def last_batch_status(self):
        inv = ctypes.c_uint32()
        fb = ctypes.c_uint32()
        self._check(lib().snn_last_batch_status(self._h, ctypes.byref(inv), ctypes.byref(fb)))
        return int(inv.value), int(fb.value)

    def last_batch_work(self):
        """Selection work of the last batch: candidates handed to the merge and
        tiles that ran the radix select, main and fallback pass apart."""
        w = BatchWork()
        self._check(lib().snn_last_batch_work(self._h, ctypes.byref(w)))
        return {f: int(getattr(w, f)) for f, _ in BatchWork._fields_}

    # ------------------------------------------------------------- timing
    def profile(self, on: bool = True):
        self._check(lib().snn_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """(summed scoring-kernel milliseconds, launches) since the last read."""
        ms = ctypes.c_double()
        n = ctypes.c_uint32()
        self._check(lib().snn_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)

    def profile_read_updates(self):
        """{insert_ms, insert_docs, delete_ms, delete_docs}: summed kernel time of
        the insert and delete kernels and the documents they covered since the
        last read."""
        ims, dms = ctypes.c_double(), ctypes.c_double()
        idocs, ddocs = ctypes.c_uint64(), ctypes.c_uint64()
        self._check(lib().snn_profile_read_updates(self._h, ctypes.byref(ims), ctypes.byref(idocs),
                                                   ctypes.byref(dms), ctypes.byref(ddocs)))
        return {"insert_ms": float(ims.value), "insert_docs": int(idocs.value),
                "delete_ms": float(dms.value), "delete_docs": int(ddocs.value)}

    # ------------------------------------------------------------- schedule
    def autotune(self, indptr, coords, vals, k: int, total: Optional[int] = None) -> dict:
        """Time candidate schedules on a device-resident batch and keep the fastest."""
        nq = indptr.numel() - 1
        total = int(coords.numel()) if total is None else int(total)
        sch = Schedule()
        self._check(lib().snn_autotune(self._h, nq, _tp(indptr), total, _tp(coords), _tp(vals), k,
                                       ctypes.byref(sch)))
        return sch.as_dict()

    def schedule(self) -> dict:
        sch = Schedule()
        self._check(lib().snn_get_schedule(self._h, ctypes.byref(sch)))
        return sch.as_dict()

    def set_schedule(self, R_plain=16, R_batch=16, grid=2048, persistent=True, qgroup=1):
        sch = Schedule(R_plain, R_batch, grid, 1 if persistent else 0, 0.0, 0.0, 0, qgroup)
        self._check(lib().snn_set_schedule(self._h, ctypes.byref(sch)))

    # ------------------------------------------------------------- learned filter
    def filter_train(self, indptr, coords, vals, k: int = 10, epochs: int = 8, batch: int = 512, lr: float = 1e-3,
                     holdout: float = 0.1, target_fallback: float = 0.05, feature_seed: int = 12345, seed: int = 2,
                     total: Optional[int] = None) -> dict:
        """Train the k-th-score pre-filter on device-resident training queries."""
        nq = indptr.numel() - 1
        total = int(coords.numel()) if total is None else int(total)
        p = FilterParams(feature_seed, seed, k, epochs, batch, lr, holdout, target_fallback)
        rep = FilterReport()
        self._check(lib().snn_filter_train(self._h, nq, _tp(indptr), total, _tp(coords), _tp(vals), ctypes.byref(p),
                                           ctypes.byref(rep)))
        return rep.as_dict()

    def filter_features(self, indptr, coords, vals):
        nq = indptr.numel() - 1
        X = torch.empty((nq, 256), dtype=torch.float32, device=indptr.device)
        self._check(lib().snn_filter_features(self._h, nq, _tp(indptr), _tp(coords), _tp(vals), _tp(X)))
        return X

    def filter_predict(self, indptr, coords, vals):
        nq = indptr.numel() - 1
        y = torch.empty(nq, dtype=torch.float32, device=indptr.device)
        self._check(lib().snn_filter_predict(self._h, nq, _tp(indptr), _tp(coords), _tp(vals), _tp(y)))
        return y

    def filter_get_params(self) -> np.ndarray:
        p = np.zeros(MLP_PARAMS, np.float32)
        self._check(lib().snn_filter_get_params(self._h, _p(p)))
        return p

    def filter_set_params(self, params, feature_seed: int, k: int):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == MLP_PARAMS
        self._check(lib().snn_filter_set_params(self._h, _p(p), feature_seed, k))

    def filter_set_delta(self, delta: float):
        self._check(lib().snn_filter_set_delta(self._h, float(delta)))

    def filter_enable(self, on: bool = True):
        """search / search_batch (host buffers) run the learned form while on."""
        self._check(lib().snn_filter_enable(self._h, 1 if on else 0))

    def mlp_loss_grad(self, X, y):
        """(loss, grad) of the MLP on device feature rows X and targets y."""
        B = X.shape[0]
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device)
        loss = ctypes.c_float()
        self._check(lib().snn_mlp_loss_grad(self._h, B, _tp(X), _tp(y), _tp(g), ctypes.byref(loss)))
        return float(loss.value), g

    # ------------------------------------------------------------- serving
    def serve(self, kind, arrival_s, ids, k, indptr, coords, vals, max_batch=1024, max_inflight=3, streams=3,
              realtime=True, budget_bytes=1 << 30):
        """Run a request trace with continuous batching. Returns (ids, scores,
        counts, latency_ms) per search, in trace order, and the report dict."""
        kind = np.ascontiguousarray(kind, dtype=np.uint8)
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
        idv = np.ascontiguousarray(ids, dtype=np.uint32)
        kv = np.ascontiguousarray(k, dtype=np.uint32)
        ip = np.ascontiguousarray(indptr, dtype=np.uint64)
        c = np.ascontiguousarray(coords, dtype=np.uint32)
        v = np.ascontiguousarray(vals, dtype=np.float32)
        n = len(kind)
        ns = int((kind == 0).sum())
        kmax = int(kv[kind == 0].max()) if ns else 1
        out_ids = np.zeros((ns, kmax), np.uint32)
        out_sc = np.zeros((ns, kmax), np.float32)
        out_cnt = np.zeros(ns, np.uint32)
        lat = np.zeros(ns, np.float64)
        tr = Trace(n, _p(kind).value, _p(arr).value, _p(idv).value, _p(kv).value, _p(ip).value, _p(c).value,
                   _p(v).value)
        pp = ServeParams(max_batch, max_inflight, streams, 1 if realtime else 0, budget_bytes)
        rep = ServeReport()
        self._check(lib().snn_serve_run(self._h, ctypes.byref(tr), ctypes.byref(pp), _p(out_ids), _p(out_sc),
                                        _p(out_cnt), _p(lat), ctypes.byref(rep)))
        return out_ids, out_sc, out_cnt, lat, rep.as_dict()

    # ------------------------------------------------------------- inspection
    def bucket_table(self) -> np.ndarray:
        out = np.zeros((self.h, self.dim), np.uint32)
        self._check(lib().snn_bucket_table(self._h, _p(out)))
        return out

    def read_sketch(self, id: int):
        u = np.zeros(self.m, np.float32)
        l = np.zeros(self.m, np.float32)
        self._check(lib().snn_read_sketch(self._h, int(id), _p(u), _p(l)))
        return u, l


def load_docs(index: Index, docs, ids: Optional[np.ndarray] = None, chunk: int = 1 << 18, compact=True):
    """Insert a CSR batch of documents (ids default to 0..rows-1), then compact
    the lists (compact: True, False, or the pinned classes)."""
    n = docs.rows
    if ids is None:
        ids = np.arange(n, dtype=np.uint32)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        ip = docs.indptr[a:b + 1] - docs.indptr[a]
        c = docs.coords[docs.indptr[a]:docs.indptr[b]]
        v = docs.vals[docs.indptr[a]:docs.indptr[b]]
        index.insert_batch(ids[a:b], ip, c, v)
    if compact is True:
        index.compact()
    elif compact is not False and compact is not None:
        index.compact(classes=compact)
