// Host side of the C ABI (include/snn.h): the slot store, input validation,
// staging of host inputs, and the orchestration of the search kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <system_error>
#include <thread>
#include <unordered_map>
#include <vector>

#include "snn.h"
#include "snn_device.h"
#include "snn_host.h"
#include "snn_mlp.h"

using namespace snn;

static constexpr uint32_t kMaxGridY = 65535;

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
namespace snn {

uint64_t splitmix64_mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

hipError_t DevBuf::ensure(size_t bytes, hipStream_t s) {
  if (bytes <= cap) return hipSuccess;
  if (p) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  size_t want = bytes + bytes / 4 + 4096;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    p = nullptr;
    return e;
  }
  cap = want;
  return hipSuccess;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  cap = 0;
}

hipError_t PinBuf::ensure(size_t bytes, hipStream_t s) {
  if (bytes <= cap) return hipSuccess;
  if (p) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
  }
  size_t want = bytes + bytes / 4 + 4096;
  hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
  if (e != hipSuccess) {
    p = nullptr;
    return e;
  }
  cap = want;
  return hipSuccess;
}

void PinBuf::release() {
  if (p) (void)hipHostFree(p);
  p = nullptr;
  cap = 0;
}

}  // namespace snn

snn_status snn_index::fail(snn_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  err = buf;
  return st;
}

snn_status snn_index::hip_fail(hipError_t e, const char *what) {
  if (e == hipErrorOutOfMemory) return fail(SNN_E_NOMEM, "%s: out of device memory", what);
  return fail(SNN_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(ix, call, what)                 \
  do {                                          \
    hipError_t e__ = (call);                    \
    if (e__ != hipSuccess) return (ix)->hip_fail(e__, what); \
  } while (0)

// Validate one sparse vector; appends its non-zero entries to out_c/out_v.
bool snn_check_vector(snn_index *ix, uint32_t nnz, const uint32_t *c, const float *v, std::vector<uint32_t> *oc,
                      std::vector<float> *ov, VecCheck &vc, const char *what, bool report, uint32_t *nz) {
#define SNN_CHECK_FAIL(...)                           \
  do {                                                \
    if (report) ix->fail(SNN_E_INVALID, __VA_ARGS__); \
    return false;                                     \
  } while (0)
  if (nnz && (!c || !v)) SNN_CHECK_FAIL("%s: null coordinate or value pointer", what);
  const uint32_t dim = ix->cfg.dim;
  const bool upper_only = (ix->cfg.flags & SNN_UPPER_ONLY) != 0;
  if (vc.stamps && vc.stamp.size() != dim) {
    vc.stamp.assign(dim, 0u);
    vc.tag = 0;
  }
  if (vc.stamps && ++vc.tag == 0) {
    std::fill(vc.stamp.begin(), vc.stamp.end(), 0u);
    vc.tag = 1;
  }
  if (!vc.stamps) vc.scratch.clear();
  uint32_t nonzero = 0;
  for (uint32_t t = 0; t < nnz; ++t) {
    if (c[t] >= dim) SNN_CHECK_FAIL("%s: coordinate %u >= dim %u", what, c[t], dim);
    if (!std::isfinite(v[t])) SNN_CHECK_FAIL("%s: non-finite value at coordinate %u", what, c[t]);
    if (upper_only && v[t] < 0.0f)
      SNN_CHECK_FAIL("%s: negative value at coordinate %u (the index keeps no lower bounds)", what, c[t]);
    if (vc.stamps) {
      if (vc.stamp[c[t]] == vc.tag) SNN_CHECK_FAIL("%s: duplicate coordinate %u", what, c[t]);
      vc.stamp[c[t]] = vc.tag;
    } else {
      vc.scratch.push_back(c[t]);
    }
    nonzero += v[t] != 0.0f;
  }
  if (!vc.stamps) {
    std::sort(vc.scratch.begin(), vc.scratch.end());
    for (size_t t = 1; t < vc.scratch.size(); ++t)
      if (vc.scratch[t] == vc.scratch[t - 1]) SNN_CHECK_FAIL("%s: duplicate coordinate %u", what, vc.scratch[t]);
  }
#undef SNN_CHECK_FAIL
  if (oc && ov)
    for (uint32_t t = 0; t < nnz; ++t)
      if (v[t] != 0.0f) {
        oc->push_back(c[t]);
        ov->push_back(v[t]);
      }
  if (nz) *nz = nonzero;
  return true;
}

// Runs f(begin, end) over [0, n) split into contiguous ranges, one per host
// thread (at most 16, at least min_per items each); small n runs inline.
template <class F>
static void par_ranges(uint64_t n, uint64_t min_per, F &&f) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  unsigned T = (unsigned)std::min<uint64_t>(std::min(hw, 16u), n / min_per);
  if (T <= 1) {
    f((uint64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(T - 1);
  for (unsigned t = 1; t < T; ++t) {
    try {
      th.emplace_back([&f, n, t, T] { f(n * t / T, n * (t + 1) / T); });
    } catch (const std::system_error &) {  // no thread to be had: run the range here
      f(n * t / T, n * (t + 1) / T);
    }
  }
  f((uint64_t)0, n / T);
  for (std::thread &x : th) x.join();
}

// memcpy split over host threads (pinned staging of large uploads)
static void par_memcpy(void *dst, const void *src, size_t bytes) {
  const size_t kPiece = (size_t)1 << 20;
  par_ranges((bytes + kPiece - 1) / kPiece, 4, [&](uint64_t a, uint64_t b) {
    const size_t lo = (size_t)a * kPiece, hi = std::min(bytes, (size_t)b * kPiece);
    if (hi > lo) memcpy((char *)dst + lo, (const char *)src + lo, hi - lo);
  });
}

// ---------------------------------------------------------------------------
// create / destroy
// ---------------------------------------------------------------------------
extern "C" snn_status snn_create(const snn_config *cfg, void *hip_stream, snn_index **out) {
  if (!out) return SNN_E_INVALID;
  *out = nullptr;
  if (!cfg || cfg->dim == 0 || cfg->m == 0 || cfg->m > kMaxM || cfg->h == 0 || cfg->h > 4 || cfg->capacity == 0 ||
      cfg->capacity > (1u << 31) || (cfg->flags & ~(SNN_FORWARD_STORE | SNN_SKETCH_BF16 | SNN_UPPER_ONLY)) != 0 ||
      cfg->dim >= (1u << 31))
    return SNN_E_INVALID;
  snn_index *ix = new (std::nothrow) snn_index();
  if (!ix) return SNN_E_NOMEM;
  ix->cfg = *cfg;
  ix->cap = (uint32_t)(((uint64_t)cfg->capacity + kTileMax - 1) / kTileMax * kTileMax);
  ix->W = ix->cap / 64;
  ix->free_slots.init(ix->cap);
  ix->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&ix->device) != hipSuccess) {
    delete ix;
    return SNN_E_DEVICE;
  }
  DevIndex &d = ix->dev;
  d.dim = cfg->dim;
  d.m = cfg->m;
  d.h = cfg->h;
  d.cap = ix->cap;
  d.W = ix->W;
  d.flags = (cfg->flags & SNN_SKETCH_BF16 ? kSketchBf16 : 0u) | (cfg->flags & SNN_UPPER_ONLY ? kUpperOnly : 0u);
  const bool lower = (cfg->flags & SNN_UPPER_ONLY) == 0;
  size_t bits_bytes = (size_t)cfg->dim * ix->W * 8;
  size_t sk_bytes = (size_t)cfg->m * ix->cap * (cfg->flags & SNN_SKETCH_BF16 ? 2 : 4);
  hipError_t e = hipSuccess;
  if ((e = hipMalloc(&d.bits, bits_bytes)) != hipSuccess || (e = hipMalloc(&d.live, (size_t)ix->W * 8)) != hipSuccess ||
      (e = hipMalloc(&d.U, sk_bytes)) != hipSuccess || (lower && (e = hipMalloc(&d.L, sk_bytes)) != hipSuccess) ||
      (e = hipMalloc(&d.slot2id, (size_t)ix->cap * 4)) != hipSuccess ||
      (e = hipMalloc(&d.bucket, (size_t)cfg->h * cfg->dim * 4)) != hipSuccess ||
      (e = hipMalloc(&d.stale, (size_t)(ix->cap >> 10) * 4)) != hipSuccess) {
    snn_status st = e == hipErrorOutOfMemory ? SNN_E_NOMEM : SNN_E_DEVICE;
    snn_destroy(ix);
    return st;
  }
  // zero bitmaps and sketches; slot2id = reserved id
  if (hipMemsetAsync(d.bits, 0, bits_bytes, ix->stream) != hipSuccess ||
      hipMemsetAsync(d.live, 0, (size_t)ix->W * 8, ix->stream) != hipSuccess ||
      hipMemsetAsync(d.U, 0, sk_bytes, ix->stream) != hipSuccess ||
      (lower && hipMemsetAsync(d.L, 0, sk_bytes, ix->stream) != hipSuccess) ||
      launch_fill_u32(d.slot2id, 0xFFFFFFFFu, ix->cap, ix->stream) != hipSuccess ||
      launch_fill_u32(d.stale, 0u, ix->cap >> 10, ix->stream) != hipSuccess) {
    snn_destroy(ix);
    return SNN_E_DEVICE;
  }
  // the random mappings pi_o(j) = mix64(mix64(seed + o) ^ j) mod m
  std::vector<uint32_t> tab((size_t)cfg->h * cfg->dim);
  for (uint32_t o = 0; o < cfg->h; ++o) {
    const uint64_t so = splitmix64_mix(cfg->hash_seed + o);
    for (uint32_t j = 0; j < cfg->dim; ++j)
      tab[(size_t)o * cfg->dim + j] = (uint32_t)(splitmix64_mix(so ^ (uint64_t)j) % cfg->m);
  }
  if (hipMemcpyAsync(d.bucket, tab.data(), tab.size() * 4, hipMemcpyHostToDevice, ix->stream) != hipSuccess ||
      hipStreamSynchronize(ix->stream) != hipSuccess) {
    snn_destroy(ix);
    return SNN_E_DEVICE;
  }
  ix->slot_id.assign(ix->cap, 0xFFFFFFFFu);
  ix->fwd.resize(ix->cap);
  if (cfg->flags & SNN_FORWARD_STORE) {
    ix->has_fwd = true;
    ix->fwd_roff.assign(ix->cap, 0);
    ix->fwd_rlog.assign(ix->cap, 0);
    ix->fwd_free.resize(64);
    if (hipMalloc(&ix->fw.off, (size_t)ix->cap * 8) != hipSuccess ||
        hipMalloc(&ix->fw.len, (size_t)ix->cap * 4) != hipSuccess ||
        launch_fill_u32(ix->fw.len, 0u, ix->cap, ix->stream) != hipSuccess ||
        launch_fill_u32((uint32_t *)ix->fw.off, 0u, (size_t)ix->cap * 2, ix->stream) != hipSuccess ||
        rerank_init() != hipSuccess || hipStreamSynchronize(ix->stream) != hipSuccess) {
      snn_destroy(ix);
      return SNN_E_NOMEM;
    }
  }
  ix->tune_init();
  *out = ix;
  return SNN_OK;
}

extern "C" void snn_destroy(snn_index *ix) {
  if (!ix) return;
  if (ix->stream) (void)hipStreamSynchronize(ix->stream);
  else (void)hipDeviceSynchronize();
  ix->release_extras();
  DevIndex &d = ix->dev;
  if (d.bits) (void)hipFree(d.bits);
  if (d.live) (void)hipFree(d.live);
  if (d.U) (void)hipFree(d.U);
  if (d.L) (void)hipFree(d.L);
  if (d.slot2id) (void)hipFree(d.slot2id);
  if (d.bucket) (void)hipFree(d.bucket);
  if (d.stale) (void)hipFree(d.stale);
  ix->lists_seg.release();
  ix->lists_post.release();
  ix->lists_pu.release();
  ix->lists_pl.release();
  ix->crow.release();
  if (ix->fw.ent) (void)hipFree(ix->fw.ent);
  if (ix->fw.off) (void)hipFree(ix->fw.off);
  if (ix->fw.len) (void)hipFree(ix->fw.len);
  ix->up.release();
  ix->pin.release();
  ix->wsp.release();
  delete ix;
}

extern "C" size_t snn_live_count(const snn_index *ix) { return ix ? ix->live : 0; }

extern "C" const char *snn_last_error(const snn_index *ix) {
  if (!ix) return "null index";
  return ix->err.c_str();
}

// ---------------------------------------------------------------------------
// insert / delete
// ---------------------------------------------------------------------------
// Forward-store regions for n documents about to be written to `slots`
// (document r has ptr[r + 1] - ptr[r] entries). A slot keeps its region while
// the new document fits; otherwise the region goes to the free list of its
// size class and the document gets one of size 2^ceil(log2(len)) (at least 16
// entries), from that class's free list or from the top of the store. The
// store grows (doubling, contents copied) before any placement changes, so a
// failed allocation leaves the index as it was.
snn_status snn_index::fwd_place(const uint32_t *slots, const uint64_t *ptr, size_t n, uint64_t *doc_off) {
  auto lg_of = [](uint64_t len) {
    uint32_t lg = 4;
    while ((1ull << lg) < len) ++lg;
    return lg;
  };
  uint64_t worst = fwd_top;
  for (size_t r = 0; r < n; ++r) worst += 1ull << lg_of(ptr[r + 1] - ptr[r]);
  if (worst > fwd_cap || !fw.ent) {
    const uint64_t want = std::max<uint64_t>(std::max<uint64_t>(worst, fwd_cap * 2), (uint64_t)1 << 20);
    uint2 *p = nullptr;
    HIP_TRY(this, hipMalloc(&p, want * 8), "forward store");
    if (fw.ent) {
      hipError_t e = hipDeviceSynchronize();  // in-flight searches may still read the old store
      if (e == hipSuccess && fwd_top) e = hipMemcpy(p, fw.ent, fwd_top * 8, hipMemcpyDeviceToDevice);
      if (e != hipSuccess) {
        (void)hipFree(p);
        return hip_fail(e, "forward store growth");
      }
      (void)hipFree(fw.ent);
    }
    fw.ent = p;
    fwd_cap = want;
    graphs.clear();  // captured launches hold the old address
  }
  for (size_t r = 0; r < n; ++r) {
    const uint64_t len = ptr[r + 1] - ptr[r];
    const uint32_t s = slots[r];
    if (fwd_rlog[s] && (1ull << fwd_rlog[s]) >= len) {
      doc_off[r] = fwd_roff[s];
      continue;
    }
    if (fwd_rlog[s]) fwd_free[fwd_rlog[s]].push_back(fwd_roff[s]);
    const uint32_t lg = lg_of(len);
    uint64_t off;
    if (!fwd_free[lg].empty()) {
      off = fwd_free[lg].back();
      fwd_free[lg].pop_back();
    } else {
      off = fwd_top;
      fwd_top += 1ull << lg;
    }
    fwd_roff[s] = off;
    fwd_rlog[s] = lg;
    doc_off[r] = off;
  }
  return SNN_OK;
}

snn_status snn_index::upload_and_insert(const std::vector<uint32_t> &slots, const std::vector<uint32_t> &ids,
                                        const std::vector<uint64_t> &indptr, const std::vector<uint32_t> &coords,
                                        const std::vector<float> &vals, size_t r0, size_t r1) {
  const size_t n = r1 - r0;
  const uint64_t e0 = indptr[r0], e1 = indptr[r1];
  const size_t ne = (size_t)(e1 - e0);
  std::vector<uint64_t> doc_off;
  if (has_fwd) {
    doc_off.resize(n);
    snn_status st = fwd_place(slots.data() + r0, indptr.data() + r0, n, doc_off.data());
    if (st != SNN_OK) return st;
  }
  const size_t bytes = n * 4 * 2 + (n + 1) * 8 + ne * 8 + n * 8 + 64;
  HIP_TRY(this, pin.ensure(bytes, stream), "insert staging");
  HIP_TRY(this, up.ensure(bytes, stream), "insert upload");
  char *hp = (char *)pin.p;
  size_t o_slots = 0, o_ids = n * 4, o_ptr = (o_ids + n * 4 + 7) / 8 * 8, o_c = o_ptr + (n + 1) * 8, o_v = o_c + ne * 4;
  memcpy(hp + o_slots, slots.data() + r0, n * 4);
  memcpy(hp + o_ids, ids.data() + r0, n * 4);
  uint64_t *ip = (uint64_t *)(hp + o_ptr);
  for (size_t r = 0; r <= n; ++r) ip[r] = indptr[r0 + r] - e0;
  par_memcpy(hp + o_c, coords.data() + e0, ne * 4);
  par_memcpy(hp + o_v, vals.data() + e0, ne * 4);
  const size_t o_off = (o_v + ne * 4 + 7) / 8 * 8;
  if (has_fwd) memcpy(hp + o_off, doc_off.data(), n * 8);
  char *dp = (char *)up.p;
  HIP_TRY(this, hipMemcpyAsync(dp, hp, has_fwd ? o_off + n * 8 : o_v + ne * 4, hipMemcpyHostToDevice, stream),
          "insert copy");
  HIP_TRY(this, prof_update(0, (uint32_t)n, false), "event");
  HIP_TRY(this,
          launch_insert(dev, (uint32_t)n, (uint32_t *)(dp + o_slots), (uint32_t *)(dp + o_ids),
                        (uint64_t *)(dp + o_ptr), (uint32_t *)(dp + o_c), (float *)(dp + o_v), fw,
                        has_fwd ? (uint64_t *)(dp + o_off) : nullptr, stream),
          "insert kernel");
  HIP_TRY(this, prof_update(0, (uint32_t)n, true), "event");
  HIP_TRY(this, hipStreamSynchronize(stream), "insert sync");
  return SNN_OK;
}

extern "C" snn_status snn_insert_batch(snn_index *ix, uint32_t n, const uint32_t *ids, const uint64_t *indptr,
                                       const uint32_t *coords, const float *vals) {
  if (!ix) return SNN_E_INVALID;
  if (n == 0) return SNN_OK;
  if (!ids || !indptr) return ix->fail(SNN_E_INVALID, "insert: null ids or indptr");
  // Validate everything first (all-or-nothing). The error reported is the one
  // of the first bad row, with a row's id checked before its vector: the ids
  // in order on this thread, the vectors on several.
  uint32_t r_id = n;
  snn_status id_st = SNN_OK;
  {
    IdMap seen;
    seen.reserve(n);
    for (uint32_t r = 0; r < n && r_id == n; ++r) {
      if (ids[r] == 0xFFFFFFFFu) {
        id_st = ix->fail(SNN_E_INVALID, "insert: id 0xFFFFFFFF is reserved");
      } else if (ix->id2slot.contains(ids[r])) {
        id_st = ix->fail(SNN_E_EXISTS, "insert: id %u is already live", ids[r]);
      } else if (seen.contains(ids[r])) {
        id_st = ix->fail(SNN_E_INVALID, "insert: id %u twice in one batch", ids[r]);
      } else {
        seen.put(ids[r], r);
      }
      if (id_st != SNN_OK) r_id = r;
    }
  }
  const uint64_t dim = ix->cfg.dim;
  std::vector<uint64_t> optr((size_t)n + 1, 0);  // non-zeros per row, then their offsets
  std::atomic<uint32_t> r_vec{r_id};             // first row with a bad vector
  par_ranges(r_id, 1024, [&](uint64_t a, uint64_t b) {
    VecCheck vc;
    vc.stamps = b - a >= 256 && dim <= ((uint64_t)1 << 20);
    for (uint64_t r = a; r < b; ++r) {
      if (r >= r_vec.load(std::memory_order_relaxed)) return;  // an earlier row failed
      uint32_t nz = 0;
      const bool ok = indptr[r + 1] >= indptr[r] && indptr[r + 1] - indptr[r] <= dim &&
                      snn_check_vector(ix, (uint32_t)(indptr[r + 1] - indptr[r]), coords + indptr[r],
                                       vals + indptr[r], nullptr, nullptr, vc, "insert", false, &nz);
      if (!ok) {
        uint32_t cur = r_vec.load(std::memory_order_relaxed);
        while ((uint32_t)r < cur && !r_vec.compare_exchange_weak(cur, (uint32_t)r)) {
        }
        return;
      }
      optr[r + 1] = nz;
    }
  });
  const uint32_t r_bad = r_vec.load();
  if (r_bad < r_id) {  // the first bad row has a good id: say what is wrong with its vector
    if (indptr[r_bad + 1] < indptr[r_bad]) return ix->fail(SNN_E_INVALID, "insert: indptr not monotone");
    const uint64_t len = indptr[r_bad + 1] - indptr[r_bad];
    if (len > dim) return ix->fail(SNN_E_INVALID, "insert: vector with more entries than dim");
    VecCheck vc;
    snn_check_vector(ix, (uint32_t)len, coords + indptr[r_bad], vals + indptr[r_bad], nullptr, nullptr, vc, "insert");
    return SNN_E_INVALID;
  }
  if (r_id < n) return id_st;
  size_t avail = ix->free_slots.size() + (ix->cap - ix->next_fresh);
  if (n > avail) return ix->fail(SNN_E_FULL, "insert: %u vectors but only %zu free slots", n, avail);
  // the non-zero entries, packed
  for (uint32_t r = 0; r < n; ++r) optr[r + 1] += optr[r];
  std::vector<uint32_t> oc(optr[n]);
  std::vector<float> ov(optr[n]);
  par_ranges(n, 1024, [&](uint64_t a, uint64_t b) {
    for (uint64_t r = a; r < b; ++r) {
      uint64_t o = optr[r];
      for (uint64_t e = indptr[r]; e < indptr[r + 1]; ++e)
        if (vals[e] != 0.0f) {
          oc[o] = coords[e];
          ov[o] = vals[e];
          ++o;
        }
    }
  });
  // assign slots: freed columns (Section 4.3) and fresh ones, in the pool's order
  std::vector<uint32_t> slot_of(n);
  std::vector<uint32_t> vid(ids, ids + n);
  for (uint32_t r = 0; r < n; ++r) slot_of[r] = ix->free_slots.take(ix->next_fresh, ix->cap, ix->array_coords > 0);
  // upload in chunks of at most ~16M entries
  const size_t kChunk = (size_t)16 << 20;
  size_t r0 = 0;
  while (r0 < n) {
    size_t r1 = r0 + 1;
    while (r1 < n && optr[r1 + 1] - optr[r0] <= kChunk && r1 - r0 < (1u << 20)) ++r1;
    snn_status st = ix->upload_and_insert(slot_of, vid, optr, oc, ov, r0, r1);
    if (st != SNN_OK) return st;  // device error: the index is no longer consistent
    r0 = r1;
  }
  ix->id2slot.reserve(ix->id2slot.size() + n);
  for (uint32_t r = 0; r < n; ++r) {
    const uint32_t s = slot_of[r];
    ix->id2slot.put(ids[r], s);
    ix->slot_id[s] = ids[r];
  }
  par_ranges(n, 1024, [&](uint64_t a, uint64_t b) {  // distinct slots: distinct vectors
    for (uint64_t r = a; r < b; ++r) ix->fwd[slot_of[r]].assign(oc.begin() + optr[r], oc.begin() + optr[r + 1]);
  });
  ix->live += n;
  ix->mutations++;
  return SNN_OK;
}

extern "C" snn_status snn_insert(snn_index *ix, uint32_t id, uint32_t nnz, const uint32_t *coords, const float *vals) {
  uint64_t ip[2] = {0, nnz};
  return snn_insert_batch(ix, 1, &id, ip, coords, vals);
}

extern "C" snn_status snn_delete_batch(snn_index *ix, uint32_t n, const uint32_t *ids) {
  if (!ix) return SNN_E_INVALID;
  if (n == 0) return SNN_OK;
  if (!ids) return ix->fail(SNN_E_INVALID, "delete: null ids");
  std::vector<uint32_t> slots(n);
  IdMap seen;
  seen.reserve(n);
  for (uint32_t r = 0; r < n; ++r) {
    const uint32_t *it = ix->id2slot.find(ids[r]);
    if (!it) return ix->fail(SNN_E_NOT_FOUND, "delete: id %u is not live", ids[r]);
    if (seen.contains(ids[r])) return ix->fail(SNN_E_INVALID, "delete: id %u twice in one batch", ids[r]);
    seen.put(ids[r], r);
    slots[r] = *it;
  }
  std::vector<uint64_t> ptr(n + 1, 0);
  std::vector<uint32_t> co;
  for (uint32_t r = 0; r < n; ++r) {
    const auto &f = ix->fwd[slots[r]];
    co.insert(co.end(), f.begin(), f.end());
    ptr[r + 1] = co.size();
  }
  snn_status st = ix->upload_and_delete(slots, ptr, co, 1, 1);
  if (st != SNN_OK) return st;
  for (uint32_t r = 0; r < n; ++r) {
    const uint32_t s = slots[r];
    ix->id2slot.erase(ids[r]);
    ix->slot_id[s] = 0xFFFFFFFFu;
    ix->fwd[s].clear();
    ix->fwd[s].shrink_to_fit();
    ix->free_slots.release(s);
  }
  ix->live -= n;
  ix->mutations++;
  return SNN_OK;
}

snn_status snn_index::upload_and_delete(const std::vector<uint32_t> &slots, const std::vector<uint64_t> &ptr,
                                        const std::vector<uint32_t> &co, int clear_bits, int clear_live) {
  const size_t n = slots.size(), ne = co.size();
  const size_t bytes = n * 4 + 8 + (n + 1) * 8 + ne * 4 + 64;
  HIP_TRY(this, pin.ensure(bytes, stream), "delete staging");
  HIP_TRY(this, up.ensure(bytes, stream), "delete upload");
  char *hp = (char *)pin.p;
  size_t o_ptr = (n * 4 + 7) / 8 * 8, o_c = o_ptr + (n + 1) * 8;
  memcpy(hp, slots.data(), n * 4);
  memcpy(hp + o_ptr, ptr.data(), (n + 1) * 8);
  if (ne) memcpy(hp + o_c, co.data(), ne * 4);
  char *dp = (char *)up.p;
  HIP_TRY(this, hipMemcpyAsync(dp, hp, o_c + ne * 4, hipMemcpyHostToDevice, stream), "delete copy");
  HIP_TRY(this, prof_update(1, (uint32_t)n, false), "event");
  HIP_TRY(this,
          launch_delete(dev, (uint32_t)n, (uint32_t *)dp, (uint64_t *)(dp + o_ptr), (uint32_t *)(dp + o_c), clear_bits,
                        clear_live, stream),
          "delete kernel");
  HIP_TRY(this, prof_update(1, (uint32_t)n, true), "event");
  HIP_TRY(this, hipStreamSynchronize(stream), "delete sync");
  return SNN_OK;
}

extern "C" snn_status snn_delete(snn_index *ix, uint32_t id) { return snn_delete_batch(ix, 1, &id); }

// ---------------------------------------------------------------------------
// search
// ---------------------------------------------------------------------------

// Device workspace for one batch: prepared entries, per-query state, tile
// candidates. Laid out in one allocation.
// kt: candidates a tile keeps per query; kprime > 0: the re-rank's buffers too.
// ext (nullable): a caller region of ext_bytes (256-byte aligned) that holds
// every buffer instead, so that nothing is allocated; a batch that needs more
// is rejected.
snn_status snn_index::prepare_workspace(uint32_t nq, uint64_t total, uint32_t kt, uint32_t tiles, uint32_t kprime,
                                        uint32_t ksample, SearchWs &w, Workspace &W, hipStream_t stream, char *ext,
                                        size_t ext_bytes) {
  const uint32_t h = cfg.h;
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  size_t o = 0;
  const size_t o_cnt = o; o += al((size_t)nq * 4);
  const size_t o_status = o; o += al((size_t)nq * 4);
  const size_t o_thr = o; o += al((size_t)nq * 4);
  const size_t o_fb = o; o += al((size_t)nq * 4);
  const size_t o_keff = o; o += al((size_t)nq * 4);
  const size_t o_j = o; o += al((size_t)total * 4 + 64);  // the grouped kernel reads up to 16 entries past a list
  const size_t o_q = o; o += al((size_t)total * 4);
  const size_t o_b = o; o += al((size_t)total * 4 * h);
  const size_t o_nd = o; o += al((size_t)nq * 4);
  const size_t o_cr = o; o += al((size_t)total * 4);
  const size_t o_cc = o; o += al((size_t)nq * tiles * 4);
  const size_t o_queue = o; o += al(64 * 4);
  const size_t o_qlist = o; o += al((size_t)nq * 4);
  const size_t o_nlist = o; o += al(4);
  const size_t o_stats = o; o += al(32);
  const size_t o_nz = o; o += al((size_t)nq * 4);
  const size_t o_sthr = o; o += al((size_t)nq * 4);
  const size_t ks = ksample <= kMaxK ? ksample : 0;  // larger samples select into the re-rank buffers
  const size_t o_ssi = o; o += al((size_t)nq * ks * 4);
  const size_t o_sss = o; o += al((size_t)nq * ks * 4);
  const size_t o_ssc = o; o += al((size_t)nq * 4);
  const size_t cand_bytes = (size_t)nq * tiles * kt * 8 + 64;
  const size_t kp = kprime;
  const size_t cslot_bytes = kprime ? (size_t)nq * tiles * kt * 4 + 64 : 0;
  const size_t o_keys = kprime ? al((size_t)nq * kp * 12 + (size_t)nq * 4) : 0;
  const size_t rr_bytes = kprime ? o_keys + (size_t)nq * kp * 8 + 256 : 0;
  char *p, *pc, *ps = nullptr, *pr = nullptr;
  if (ext) {
    const size_t need = al(o) + al(cand_bytes) + al(cslot_bytes) + al(rr_bytes);
    if (need > ext_bytes)
      return fail(SNN_E_INVALID, "search: the batch needs %zu bytes of workspace, more than the %zu of the region",
                  need, ext_bytes);
    p = ext;
    pc = p + al(o);
    if (kprime) {
      ps = pc + al(cand_bytes);
      pr = ps + al(cslot_bytes);
    }
  } else {
    HIP_TRY(this, W.ws.ensure(o, stream), "search workspace");
    HIP_TRY(this, W.cand.ensure(cand_bytes, stream), "candidate buffer");
    if (kprime) {
      HIP_TRY(this, W.cslot.ensure(cslot_bytes, stream), "candidate slots");
      HIP_TRY(this, W.rr.ensure(rr_bytes, stream), "re-rank candidates");
      ps = (char *)W.cslot.p;
      pr = (char *)W.rr.p;
    }
    p = (char *)W.ws.p;
    pc = (char *)W.cand.p;
  }
  w.cnt = (uint32_t *)(p + o_cnt);
  w.status = (uint32_t *)(p + o_status);
  w.thr = (uint32_t *)(p + o_thr);
  w.fallback = (uint32_t *)(p + o_fb);
  w.keff = (uint32_t *)(p + o_keff);
  w.j = (uint32_t *)(p + o_j);
  w.q = (float *)(p + o_q);
  w.b = (uint32_t *)(p + o_b);
  w.nd = (uint32_t *)(p + o_nd);
  w.cr = (uint32_t *)(p + o_cr);
  w.cand_cnt = (uint32_t *)(p + o_cc);
  w.queue = (uint32_t *)(p + o_queue);
  w.qlist = (uint32_t *)(p + o_qlist);
  w.nlist = (uint32_t *)(p + o_nlist);
  w.stats = (unsigned long long *)(p + o_stats);
  w.nz_full = (uint32_t *)(p + o_nz);
  w.sthr = (uint32_t *)(p + o_sthr);
  w.ss_ids = (uint32_t *)(p + o_ssi);
  w.ss_sc = (float *)(p + o_sss);
  w.ss_cnt = (uint32_t *)(p + o_ssc);
  w.cand = (uint64_t *)pc;
  w.cslot = w.rr_ids = w.rr_slot = w.rr_cnt = nullptr;
  w.rr_sc = nullptr;
  w.rk = nullptr;
  if (kprime) {
    w.cslot = (uint32_t *)ps;
    w.rr_ids = (uint32_t *)pr;
    w.rr_sc = (float *)(w.rr_ids + (size_t)nq * kp);
    w.rr_slot = (uint32_t *)(w.rr_sc + (size_t)nq * kp);
    w.rr_cnt = w.rr_slot + (size_t)nq * kp;
    w.rk = (uint64_t *)(pr + o_keys);
  }
  return SNN_OK;
}

// Enqueue the selection of each query's top-k over all of its tile groups.
snn_status snn_index::enqueue_merge(const SearchWs &w, const MergeJob &j, hipStream_t s) {
  SelectArgs m{};
  m.groups_in = j.in ? 1u : j.tiles;
  m.in_stride = j.in_stride;
  m.kmax = j.k;
  m.kq = j.kq;
  m.keff = j.keff;
  m.in = j.in ? j.in : w.cand;
  m.in_cnt = j.in ? j.in_cnt : w.cand_cnt;
  m.status = w.status;
  m.qlist = j.qlist;
  m.nlist = j.nlist;
  m.emitted = j.emitted;
  m.in_slot = j.slots ? w.cslot : nullptr;
  m.res_ids = j.res_ids;
  m.res_scores = j.res_scores;
  m.res_cnt = j.res_cnt;
  m.res_slots = j.res_slots;
  m.fallback = j.set_fallback ? w.fallback : nullptr;
  for (uint32_t c0 = 0; c0 < j.nqm; c0 += kMaxGridY) {
    m.q0 = j.q0 + c0;
    m.nq = std::min<uint32_t>(kMaxGridY, j.nqm - c0);
    HIP_TRY(this, launch_select(m, j.sorted, s), "select kernel");
  }
  return SNN_OK;
}

// Enqueue one batched or plain search. The device work is: query preparation,
// threshold initialisation, the scoring + selection tiles, the select of each
// query's top-k over its tiles, and with k' > k the exact re-rank and the final
// select. Starting thresholds come from a learned-filter pass (features, MLP)
// or, for a wide k, from a first pass over a sample of the tiles; the queries
// that then kept fewer than min(k, live) candidates run the tiles and select
// again without one, all on the device.
// ev (nullable): events around the tile launches (main pass, fallback pass).
snn_status snn_index::enqueue_search(const SearchPlan &p, const SearchOpts &o, hipStream_t s, hipEvent_t *ev) {
  const SearchWs &w = p.w;
  const LearnedPass *lp = o.learned;
  QueryDesc qd{p.d_ptr, w.cnt, w.nd, w.status, w.j, w.q, w.b, w.cr, o.ebase};
  if (lp) {
    HIP_TRY(this, launch_features(p.nq, p.d_ptr, p.d_c, p.d_v, lp->table, lp->dim, lp->X, s), "feature kernel");
    HIP_TRY(this,
            launch_mlp_fwd(p.nq, lp->X, nullptr, lp->Pb, lp->yhat, nullptr, 0.0f, nullptr, nullptr, nullptr, nullptr,
                           nullptr, nullptr, s),
            "mlp forward");
    HIP_TRY(this, launch_threshold(p.nq, lp->yhat, lp->delta, lp->keff_value, lp->thr, lp->keff, s), "threshold");
  }
  HIP_TRY(this, launch_prep(dev, qd, p.nq, p.d_c, p.d_v, o.max_coords, w.nz_full, (const uint32_t *)crow.p, s),
          "prep kernel");
  HIP_TRY(this, launch_fill_u32((uint32_t *)w.stats, 0u, 8, s), "stats fill");
  TileArgs a{};
  a.ix = dev;
  a.qd = qd;
  a.nq = p.nq;
  a.tiles = p.tiles;
  a.kmax = p.kt;
  a.kq = o.kq;
  a.thr = w.thr;
  a.cand = w.cand;
  a.cand_cnt = w.cand_cnt;
  a.queue = w.queue;
  a.xcds = 8;
  a.qseq = o.qseq;
  a.vis = vis;
  a.dirty = dirty;
  a.nselect = w.stats + 2;
  const bool rerank = o.rerank_k != 0;
  a.cand_slot = rerank ? w.cslot : nullptr;
  MergeJob mj;
  mj.tiles = p.tiles;
  mj.k = p.k;
  mj.in_stride = p.kt;
  mj.kq = o.kq;
  mj.res_ids = rerank ? w.rr_ids : p.d_ids;
  mj.res_scores = rerank ? w.rr_sc : p.d_sc;
  mj.res_cnt = rerank ? w.rr_cnt : p.d_cnt;
  mj.res_slots = rerank ? w.rr_slot : nullptr;
  mj.slots = rerank;
  mj.sorted = !rerank;
  mj.emitted = w.stats;
  mj.set_fallback = true;
  if (p.mode == SNN_MODE_PLAIN) {
    HIP_TRY(this, launch_fill_u32(w.thr, 0u, p.nq, s), "thr fill");
    for (uint32_t q = 0; q < p.nq; ++q) {
      a.q0 = q;
      hipEvent_t e0 = prof_on ? prof_event() : nullptr;
      if (e0) HIP_TRY(this, hipEventRecord(e0, s), "event");
      HIP_TRY(this, launch_tiles_latency(a, p.R, s), "tile kernel");
      if (e0) {
        hipEvent_t e1 = prof_event();
        HIP_TRY(this, hipEventRecord(e1, s), "event");
        prof_events.push_back(e0);
        prof_events.push_back(e1);
      }
      mj.q0 = q;
      mj.nqm = 1;
      snn_status st = enqueue_merge(w, mj, s);
      if (st != SNN_OK) return st;
    }
    return SNN_OK;
  }
  // one batched tile pass: the persistent grid or one workgroup per item
  auto tiles_pass = [&](hipEvent_t e0, hipEvent_t e1) -> snn_status {
    a.q0 = 0;
    if (p.persistent) HIP_TRY(this, launch_fill_u32(w.queue, 0u, 64, s), "queue fill");
    if (e0) HIP_TRY(this, hipEventRecord(e0, s), "event");
    if (p.qgroup > 1) {
      // several queries per workgroup; the non-persistent grid covers query groups
      const uint32_t ng = (p.nq + p.qgroup - 1) / p.qgroup;
      if (p.persistent) {
        HIP_TRY(this, launch_tiles_grouped(a, p.R, p.qgroup, true, p.grid, 0, s), "grouped tile kernel");
      } else {
        for (uint32_t c0 = 0; c0 < ng; c0 += kMaxGridY) {
          a.q0 = c0;
          HIP_TRY(this, launch_tiles_grouped(a, p.R, p.qgroup, false, 0, std::min<uint32_t>(kMaxGridY, ng - c0), s),
                  "grouped tile kernel");
        }
      }
    } else if (p.persistent) {
      HIP_TRY(this, launch_tiles_persistent(a, p.R, p.grid, s), "persistent tile kernel");
    } else {
      for (uint32_t c0 = 0; c0 < p.nq; c0 += kMaxGridY) {
        a.q0 = c0;
        HIP_TRY(this, launch_tiles(a, p.R, std::min<uint32_t>(kMaxGridY, p.nq - c0), s), "tile kernel");
      }
    }
    if (e1) HIP_TRY(this, hipEventRecord(e1, s), "event");
    return SNN_OK;
  };
  snn_status st = SNN_OK;
  // Starting thresholds and the count each query must keep: from the learned
  // filter, or, when k' exceeds a tile, from a first pass over a sample of the
  // tiles (the lowest score among the k_s best there); queries that keep fewer
  // candidates run again without a threshold, so the results never change.
  const uint32_t *thr_init = o.thr_init, *keff = o.keff;
  if (lp) {
    thr_init = lp->thr;
    keff = lp->keff;
  } else if (p.tiles_s) {
    HIP_TRY(this, launch_fill_u32(w.thr, 0u, p.nq, s), "thr fill");
    // one k for every query here: a tile keeps at most kmax candidates per
    // query (the stride of this pass), whatever the query's own k. That is
    // four times a sampled tile's share of the k_s best (at least 32), not
    // k_s: the lowest of the k_s best of what the tiles keep is the sample's
    // own k_s-th best unless one tile held more of them than that, and then it
    // is lower, which only lets more documents through the main pass (what the
    // tiles keep is a subset of the sample; with fewer than k_s of them there
    // is no threshold). The tile selects and the sample's select get cheaper.
    a.tiles = p.tiles_s;
    const uint32_t share = (uint32_t)std::max<uint64_t>(32u, (4ull * p.k_s + p.tiles_s - 1) / p.tiles_s);
    a.kmax = std::min(std::min(p.k_s, p.kt), share);
    a.kq = nullptr;
    a.nselect = nullptr;
    st = tiles_pass(nullptr, nullptr);
    if (st != SNN_OK) return st;
    MergeJob m1 = mj;
    m1.tiles = p.tiles_s;
    m1.k = p.k_s;
    m1.in_stride = a.kmax;
    m1.kq = nullptr;
    m1.emitted = nullptr;
    m1.set_fallback = false;
    m1.q0 = 0;
    m1.nqm = p.nq;
    if (p.k_s <= kMaxK) {  // into the sample buffers, unsorted: only their lowest score is used
      m1.res_ids = w.ss_ids;
      m1.res_scores = w.ss_sc;
      m1.res_cnt = w.ss_cnt;
      m1.res_slots = nullptr;
      m1.slots = false;
      m1.sorted = false;
    }  // else (re-rank with a very wide k'): unsorted, into the re-rank buffers
    st = enqueue_merge(w, m1, s);
    if (st != SNN_OK) return st;
    // the select wrote each query's k_s results at stride k_s
    HIP_TRY(this, launch_sample_thr(p.nq, p.k_s, p.k_s, m1.res_scores, m1.res_cnt, w.sthr, s), "sample threshold");
    HIP_TRY(this, launch_keff(p.nq, o.kq, p.k, (uint32_t)std::min<size_t>(p.k, live), w.keff, s), "keff");
    a.tiles = p.tiles;
    a.kmax = p.kt;
    a.kq = o.kq;
    a.nselect = w.stats + 2;
    thr_init = w.sthr;
    keff = w.keff;
  }
  if (thr_init) {
    HIP_TRY(this, launch_copy_u32(w.thr, thr_init, p.nq, s), "thr init");
  } else {
    HIP_TRY(this, launch_fill_u32(w.thr, 0u, p.nq, s), "thr fill");
  }
  mj.keff = keff;
  st = tiles_pass(ev ? ev[0] : nullptr, ev ? ev[1] : nullptr);
  if (st != SNN_OK) return st;
  mj.q0 = 0;
  mj.nqm = p.nq;
  st = enqueue_merge(w, mj, s);
  if (st != SNN_OK) return st;
  if (thr_init && keff) {
    // the queries that kept fewer than keff candidates, again with no threshold
    HIP_TRY(this, launch_fallback_list(p.nq, w.fallback, w.qlist, w.nlist, w.thr, s), "fallback list");
    a.qlist = w.qlist;
    a.nlist = w.nlist;
    a.nselect = w.stats + 3;
    st = tiles_pass(ev ? ev[2] : nullptr, ev ? ev[3] : nullptr);
    if (st != SNN_OK) return st;
    a.qlist = a.nlist = nullptr;
    MergeJob mf = mj;
    mf.keff = nullptr;
    mf.set_fallback = false;
    mf.qlist = w.qlist;
    mf.nlist = w.nlist;
    mf.emitted = w.stats + 1;
    st = enqueue_merge(w, mf, s);
    if (st != SNN_OK) return st;
  }
  if (rerank) {
    RerankArgs r{};
    r.fw = fw;
    r.qd = qd;
    r.kprime = p.k;
    r.hash_cap = o.hash_cap;
    r.cand_ids = w.rr_ids;
    r.cand_slots = w.rr_slot;
    r.cand_cnt = w.rr_cnt;
    r.nz_full = w.nz_full;
    r.keys = w.rk;
    HIP_TRY(this, launch_rerank(r, p.nq, s), "re-rank kernel");
    // the k best of the k' exact scores, in order
    MergeJob fin;
    fin.k = o.rerank_k;
    fin.sorted = true;
    fin.in = w.rk;
    fin.in_cnt = w.rr_cnt;
    fin.in_stride = p.k;
    fin.res_ids = p.d_ids;
    fin.res_scores = p.d_sc;
    fin.res_cnt = p.d_cnt;
    fin.q0 = 0;
    fin.nqm = p.nq;
    st = enqueue_merge(w, fin, s);
    if (st != SNN_OK) return st;
  }
  return SNN_OK;
}

snn_status snn_index::plan_search(uint32_t nq, const uint64_t *d_ptr, uint64_t total, const uint32_t *d_c,
                                  const float *d_v, uint32_t k, int mode, uint32_t *d_ids, float *d_sc,
                                  uint32_t *d_cnt, SearchPlan &p, const SearchOpts &o, hipStream_t s) {
  p.nq = nq;
  p.d_ptr = d_ptr;
  p.total = total;
  p.d_c = d_c;
  p.d_v = d_v;
  p.k = k;
  p.mode = mode;
  p.d_ids = d_ids;
  p.d_sc = d_sc;
  p.d_cnt = d_cnt;
  p.R = mode == SNN_MODE_PLAIN ? tune.R_plain : tune.R_batch;
  // grouped tiles address entries with 32-bit positions
  p.qgroup = mode == SNN_MODE_PLAIN || cfg.h != 1 || total - o.ebase > 0xFFFFFFF0ull ? 1 : tune.qgroup;
  if (p.qgroup == 1 && p.R < 16) p.R = 16;  // the one-query kernels are built for R >= 16
  p.persistent = mode != SNN_MODE_PLAIN && tune.persistent;
  p.grid = tune.grid;
  const uint32_t tile_docs = (uint32_t)kBlock * p.R;
  p.tiles = (next_fresh + tile_docs - 1) / tile_docs;
  if (p.tiles == 0) return SNN_OK;
  // A batch with no more (query group, tile) items than the persistent grid
  // has workgroups gains nothing from the work queues (each workgroup would
  // take at most one item), and the emptied queues would still cost every
  // workgroup a round of atomics on them: it runs one workgroup per item.
  if (p.persistent && (uint64_t)((nq + p.qgroup - 1) / p.qgroup) * p.tiles <= p.grid) p.persistent = false;
  p.kt = std::min<uint32_t>(k, tile_docs);
  // A wide k (k' of Alg. 7 when re-ranking; a sixteenth of a tile or more): a
  // tile's own selection keeps the tile's k best, a large share of it (all of
  // it when k reaches the tile), so a query hands the selection about
  // tiles x min(k, tile) candidates. A first pass over the first
  // tiles / kSampleStride tiles selects the k_s best there, k_s chosen so that
  // about 1.5 k documents of the whole collection (plus 32 of the sample's
  // documents' worth, a margin for small samples) score at least the lowest of
  // them: k_s is a count of a random sample, whose relative spread is about
  // 1 / sqrt(k_s), 2-9% here, so fewer than k pass only many spreads away (a
  // slot range holds a random sample of the collection's documents; when it
  // does not, more queries run the no-threshold pass, nothing else).
  // With per-query k the batch k sets k_s: a lower threshold is still valid.
  p.tiles_s = p.k_s = 0;
  if (mode == SNN_MODE_BATCHED && !o.thr_init && (uint64_t)k * 16 >= tile_docs && p.tiles >= 4 * kSampleStride) {
    const uint32_t ts = p.tiles / kSampleStride;
    const uint64_t ks = (3ull * k * ts + 2ull * p.tiles - 1) / (2ull * p.tiles) + 32;
    if (ks < k) {
      p.tiles_s = ts;
      p.k_s = (uint32_t)ks;
    }
  }
  return prepare_workspace(nq, total - o.ebase, p.kt, p.tiles, o.rerank_k ? k : 0, p.k_s, p.w, o.wsp ? *o.wsp : wsp,
                           s, o.ext_ws, o.ext_ws_bytes);
}

snn_status snn_index::run_search(uint32_t nq, const uint64_t *d_ptr, uint64_t total, const uint32_t *d_c,
                                 const float *d_v, uint32_t k, int mode, uint32_t *d_ids, float *d_sc,
                                 uint32_t *d_cnt, hipStream_t s, const SearchOpts &o) {
  SearchPlan p;
  snn_status st = plan_search(nq, d_ptr, total, d_c, d_v, k, mode, d_ids, d_sc, d_cnt, p, o, s);
  if (st != SNN_OK) return st;
  if (p.tiles == 0) {  // nothing was ever inserted: no results
    last_status = nullptr;
    last_stats = nullptr;
    last_nlist = nullptr;
    HIP_TRY(this, launch_fill_u32(d_cnt, 0u, nq, s), "fill");
    return SNN_OK;
  }
  last_ws = p.w;
  last_status = p.w.status;
  last_stats = p.w.stats;
  last_nlist = o.learned || p.tiles_s ? p.w.nlist : nullptr;
  // graphs need a capturable stream (the legacy default stream is not one);
  // timed (profiled) passes launch eagerly so events can bracket the tile kernel
  if (mode == SNN_MODE_PLAIN || !use_graphs || s == nullptr || prof_on || o.no_graph) {
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    const int nev = prof_on && mode != SNN_MODE_PLAIN ? (o.learned || p.tiles_s ? 4 : 2) : 0;
    for (int i = 0; i < nev; ++i) ev[i] = prof_event();
    st = enqueue_search(p, o, s, nev ? ev : nullptr);
    for (int i = 0; i < nev; ++i) prof_events.push_back(ev[i]);
    return st;
  }
  // batched forms replay a captured HIP graph of the whole pass
  GraphKey key{};
  key.nq = nq; key.total = total; key.k = k; key.mode = mode; key.R = p.R; key.grid = p.grid;
  key.qgroup = (uint32_t)p.qgroup;
  key.persistent = p.persistent; key.tiles = p.tiles; key.prof = false;
  key.ptr = d_ptr; key.c = d_c; key.v = d_v; key.ids = d_ids; key.sc = d_sc; key.cnt = d_cnt;
  key.thr = o.thr_init; key.kq = o.kq; key.keff = o.keff; key.stream = s;
  Workspace &W = o.wsp ? *o.wsp : wsp;
  key.ws = W.ws.p; key.cand = W.cand.p; key.qseq = o.qseq; key.ebase = o.ebase;
  key.rerank_k = o.rerank_k;
  key.max_coords = o.max_coords;
  key.hash_cap = o.hash_cap;
  key.cslot = W.cslot.p;
  key.rr = W.rr.p;
  key.fwd = fw.ent;
  // the sampled pass's required counts, min(k, live), are kernel arguments
  key.skeff = p.tiles_s ? (uint32_t)std::min<size_t>(k, live) : 0u;
  if (const LearnedPass *lp = o.learned) {
    key.lX = lp->X; key.ly = lp->yhat; key.lthr = lp->thr; key.lkeff = lp->keff; key.lPb = lp->Pb;
    key.ltab = lp->table; key.lkeff_v = lp->keff_value;
    memcpy(&key.ldelta, &lp->delta, 4);
  }
  GraphEntry *g = graphs.find(key);
  if (!g) {
    GraphEntry e;
    e.key = key;
    hipGraph_t graph = nullptr;
    HIP_TRY(this, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "graph capture");
    snn_status est = enqueue_search(p, o, s, nullptr);
    hipError_t ce = hipStreamEndCapture(s, &graph);
    if (est != SNN_OK || ce != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      e.release();
      if (est != SNN_OK) return est;
      return hip_fail(ce, "graph capture");
    }
    hipError_t ie = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      e.release();
      return hip_fail(ie, "graph instantiate");
    }
    g = graphs.insert(e);
  }
  HIP_TRY(this, hipGraphLaunch(g->exec, s), "graph launch");
  return SNN_OK;
}

// LDS hash slots the re-rank kernel needs for queries of at most `max_nnz`
// entries: a power of two at least 8 times that (a table at most 1/8 full, so
// probes nearly always end in the first bucket) up to 4,096 slots (32 KB, three
// workgroups per CU), else at least twice that (at most half full).
static uint32_t rerank_hash_cap(uint64_t max_nnz) {
  uint64_t ub = std::min<uint64_t>(max_nnz, (uint64_t)kPrepCap);
  uint32_t cap = 64;
  while (cap < 8 * ub && cap < 4096) cap <<= 1;
  while (cap < 2 * ub) cap <<= 1;
  return cap;
}

// Arguments every search form shares: k, the mode, the re-rank width and the
// anytime budget.
static snn_status check_params(snn_index *ix, uint32_t k, const snn_search_params &p) {
  if (k == 0 || k > kMaxK) return ix->fail(SNN_E_INVALID, "search: k must be in 1..%u", kMaxK);
  if (p.mode > SNN_MODE_LEARNED) return ix->fail(SNN_E_INVALID, "search: unknown mode %u", p.mode);
  if (p.reserved != 0) return ix->fail(SNN_E_INVALID, "search: reserved field must be 0");
  if (p.k_prime != 0) {
    if (p.k_prime < k) return ix->fail(SNN_E_INVALID, "re-rank: need k <= k' (k = %u, k' = %u)", k, p.k_prime);
    if (!ix->has_fwd) return ix->fail(SNN_E_INVALID, "re-rank: the index has no forward store (SNN_FORWARD_STORE)");
    if (p.k_prime > kMaxKPrime) return ix->fail(SNN_E_INVALID, "re-rank: k' must be <= %u", kMaxKPrime);
    if (p.mode == SNN_MODE_PLAIN)
      return ix->fail(SNN_E_INVALID, "re-rank: runs in SNN_MODE_BATCHED or SNN_MODE_LEARNED");
  }
  return SNN_OK;
}

// One device-resident batch: validated arguments, then the chosen form.
static snn_status search_dev(snn_index *ix, uint32_t nq, const uint64_t *indptr, uint64_t total,
                             const uint32_t *coords, const float *vals, uint32_t k, const snn_search_params &p,
                             uint64_t max_nnz, uint32_t *out_ids, float *out_scores, uint32_t *out_counts,
                             hipStream_t s) {
  ix->last_nq = nq;
  ix->last_mode = p.mode;
  if (p.mode == SNN_MODE_LEARNED) {
    // with k' > k the filter's threshold starts the selection of the k' candidates
    const uint32_t kb = p.k_prime ? p.k_prime : k;
    return ix->search_learned(nq, indptr, total, coords, vals, kb, p.max_coords, p.k_prime ? k : 0u,
                              p.k_prime ? rerank_hash_cap(max_nnz) : 0u, out_ids, out_scores, out_counts, s);
  }
  SearchOpts o;
  o.max_coords = p.max_coords;
  uint32_t kb = k;
  if (p.k_prime != 0) {
    o.rerank_k = k;
    o.hash_cap = rerank_hash_cap(max_nnz);
    kb = p.k_prime;
  }
  return ix->run_search(nq, indptr, total, coords, vals, kb, (int)p.mode, out_ids, out_scores, out_counts, s, o);
}

// Host-buffer batch search: validate, stage, search, read back.
static snn_status search_host(snn_index *ix, uint32_t nq, const uint64_t *indptr, const uint32_t *coords,
                              const float *vals, uint32_t k, const snn_search_params &sp, uint32_t *out_ids,
                              float *out_scores, uint32_t *out_counts) {
  snn_status st = check_params(ix, k, sp);
  if (st != SNN_OK) return st;
  if (nq == 0) return SNN_OK;
  if (!indptr || !out_ids || !out_scores || !out_counts) return ix->fail(SNN_E_INVALID, "search: null pointer");
  VecCheck vc;
  uint64_t max_len = 0;
  for (uint32_t r = 0; r < nq; ++r) {
    if (indptr[r + 1] < indptr[r]) return ix->fail(SNN_E_INVALID, "search: indptr not monotone");
    uint64_t len = indptr[r + 1] - indptr[r];
    if (len > (uint64_t)kPrepCap) return ix->fail(SNN_E_INVALID, "search: a query has more than %d entries", kPrepCap);
    max_len = std::max(max_len, len);
    if (!snn_check_vector(ix, (uint32_t)len, coords + indptr[r], vals + indptr[r], nullptr, nullptr, vc, "search"))
      return SNN_E_INVALID;
  }
  const uint64_t total = indptr[nq];
  hipStream_t s = ix->stream;
  const size_t in_bytes = ((size_t)(nq + 1) * 8 + total * 8 + 255) / 256 * 256 + 256;
  const size_t out_bytes = (size_t)nq * k * 8 + (size_t)nq * 4 + 64;
  HIP_TRY(ix, ix->pin.ensure(in_bytes + out_bytes, s), "search staging");
  HIP_TRY(ix, ix->up.ensure(in_bytes + out_bytes, s), "search upload");
  char *hp = (char *)ix->pin.p, *dp = (char *)ix->up.p;
  const size_t o_c = (size_t)(nq + 1) * 8, o_v = o_c + total * 4, o_out = (o_v + total * 4 + 255) / 256 * 256;
  memcpy(hp, indptr, (size_t)(nq + 1) * 8);
  // the kernels index entries from 0: rebase the offsets
  uint64_t base = indptr[0];
  for (uint32_t r = 0; r <= nq; ++r) ((uint64_t *)hp)[r] -= base;
  if (total - base) {
    memcpy(hp + o_c, coords + base, (total - base) * 4);
    memcpy(hp + o_v, vals + base, (total - base) * 4);
  }
  HIP_TRY(ix, hipMemcpyAsync(dp, hp, o_v + (total - base) * 4, hipMemcpyHostToDevice, s), "search copy");
  uint32_t *d_ids = (uint32_t *)(dp + o_out);
  float *d_sc = (float *)(d_ids + (size_t)nq * k);
  uint32_t *d_cnt = (uint32_t *)(d_sc + (size_t)nq * k);
  st = search_dev(ix, nq, (uint64_t *)dp, total - base, (uint32_t *)(dp + o_c), (float *)(dp + o_v), k, sp, max_len,
                  d_ids, d_sc, d_cnt, s);
  if (st != SNN_OK) return st;
  HIP_TRY(ix, hipMemcpyAsync(hp + o_out, d_ids, out_bytes - 64, hipMemcpyDeviceToHost, s), "search readback");
  HIP_TRY(ix, hipStreamSynchronize(s), "search sync");
  const uint32_t *h_ids = (const uint32_t *)(hp + o_out);
  const float *h_sc = (const float *)(h_ids + (size_t)nq * k);
  const uint32_t *h_cnt = (const uint32_t *)(h_sc + (size_t)nq * k);
  memcpy(out_ids, h_ids, (size_t)nq * k * 4);
  memcpy(out_scores, h_sc, (size_t)nq * k * 4);
  memcpy(out_counts, h_cnt, (size_t)nq * 4);
  return SNN_OK;
}

// Device-buffer entry: the common checks of the _dev calls.
static snn_status search_dev_entry(snn_index *ix, uint32_t nq, const uint64_t *indptr, uint64_t total,
                                   const uint32_t *coords, const float *vals, uint32_t k, const snn_search_params &p,
                                   uint32_t *out_ids, float *out_scores, uint32_t *out_counts, void *stream) {
  snn_status st = check_params(ix, k, p);
  if (st != SNN_OK) return st;
  if (nq == 0) return ix->fail(SNN_E_INVALID, "search: nq must be > 0");
  if (!indptr || !out_ids || !out_scores || !out_counts || (total && (!coords || !vals)))
    return ix->fail(SNN_E_INVALID, "search: null pointer");
  hipStream_t s = stream ? (hipStream_t)stream : ix->stream;
  // no query holds more entries than the batch (the host does not read indptr)
  return search_dev(ix, nq, indptr, total, coords, vals, k, p, total, out_ids, out_scores, out_counts, s);
}

// The device-buffer search with every workspace buffer carved from the
// caller's region `ext` of `ext_bytes`: no device allocation and no HIP graph
// (the work is enqueued kernel by kernel, so a capturing caller records it).
snn_status snn_search_dev_in_region(snn_index *ix, uint32_t nq, const uint64_t *indptr, uint64_t total,
                                    const uint32_t *coords, const float *vals, uint32_t k, uint32_t mode,
                                    uint32_t *out_ids, float *out_scores, uint32_t *out_counts, void *stream,
                                    char *ext, size_t ext_bytes) {
  const snn_search_params p{mode, 0, 0, 0};
  snn_status st = check_params(ix, k, p);
  if (st != SNN_OK) return st;
  if (mode == SNN_MODE_LEARNED)
    return ix->fail(SNN_E_INVALID, "search: the allocation-free form runs SNN_MODE_PLAIN or SNN_MODE_BATCHED");
  if (nq == 0) return ix->fail(SNN_E_INVALID, "search: nq must be > 0");
  if (!indptr || !out_ids || !out_scores || !out_counts || (total && (!coords || !vals)))
    return ix->fail(SNN_E_INVALID, "search: null pointer");
  hipStream_t s = stream ? (hipStream_t)stream : ix->stream;
  ix->last_nq = nq;
  ix->last_mode = mode;
  SearchOpts o;
  o.ext_ws = ext;
  o.ext_ws_bytes = ext_bytes;
  o.no_graph = true;
  return ix->run_search(nq, indptr, total, coords, vals, k, (int)mode, out_ids, out_scores, out_counts, s, o);
}

extern "C" snn_status snn_search_batch(snn_index *ix, uint32_t nq, const uint64_t *indptr, const uint32_t *coords,
                                       const float *vals, uint32_t k, uint32_t *out_ids, float *out_scores,
                                       uint32_t *out_counts) {
  if (!ix) return SNN_E_INVALID;
  // with the filter enabled the same search runs the learned form (same results)
  const uint32_t mode = ix->filter_on ? SNN_MODE_LEARNED : SNN_MODE_BATCHED;
  return search_host(ix, nq, indptr, coords, vals, k, snn_search_params{mode, 0, 0, 0}, out_ids, out_scores,
                     out_counts);
}

extern "C" snn_status snn_search_rerank(snn_index *ix, uint32_t nq, const uint64_t *indptr, const uint32_t *coords,
                                        const float *vals, uint32_t k, uint32_t k_prime, uint32_t *out_ids,
                                        float *out_scores, uint32_t *out_counts) {
  if (!ix) return SNN_E_INVALID;
  if (k_prime == 0) return ix->fail(SNN_E_INVALID, "re-rank: k' must be >= k");
  return search_host(ix, nq, indptr, coords, vals, k, snn_search_params{SNN_MODE_BATCHED, k_prime, 0, 0}, out_ids,
                     out_scores, out_counts);
}

extern "C" snn_status snn_search_ex(snn_index *ix, uint32_t nq, const uint64_t *indptr, const uint32_t *coords,
                                    const float *vals, uint32_t k, const snn_search_params *params,
                                    uint32_t *out_ids, float *out_scores, uint32_t *out_counts) {
  if (!ix) return SNN_E_INVALID;
  if (!params) return ix->fail(SNN_E_INVALID, "search: null params");
  return search_host(ix, nq, indptr, coords, vals, k, *params, out_ids, out_scores, out_counts);
}

extern "C" snn_status snn_search_rerank_dev(snn_index *ix, uint32_t nq, const uint64_t *indptr, uint64_t total,
                                            const uint32_t *coords, const float *vals, uint32_t k, uint32_t k_prime,
                                            uint32_t *out_ids, float *out_scores, uint32_t *out_counts, void *stream) {
  if (!ix) return SNN_E_INVALID;
  if (k_prime == 0) return ix->fail(SNN_E_INVALID, "re-rank: k' must be >= k");
  return search_dev_entry(ix, nq, indptr, total, coords, vals, k, snn_search_params{SNN_MODE_BATCHED, k_prime, 0, 0},
                          out_ids, out_scores, out_counts, stream);
}

extern "C" snn_status snn_search_ex_dev(snn_index *ix, uint32_t nq, const uint64_t *indptr, uint64_t total,
                                        const uint32_t *coords, const float *vals, uint32_t k,
                                        const snn_search_params *params, uint32_t *out_ids, float *out_scores,
                                        uint32_t *out_counts, void *stream) {
  if (!ix) return SNN_E_INVALID;
  if (!params) return ix->fail(SNN_E_INVALID, "search: null params");
  return search_dev_entry(ix, nq, indptr, total, coords, vals, k, *params, out_ids, out_scores, out_counts, stream);
}

extern "C" snn_status snn_search(snn_index *ix, uint32_t nnz, const uint32_t *coords, const float *vals, uint32_t k,
                                 uint32_t *out_ids, float *out_scores, uint32_t *out_count) {
  uint64_t ip[2] = {0, nnz};
  return snn_search_batch(ix, 1, ip, coords, vals, k, out_ids, out_scores, out_count);
}

extern "C" snn_status snn_search_batch_dev(snn_index *ix, uint32_t nq, const uint64_t *indptr, uint64_t total,
                                           const uint32_t *coords, const float *vals, uint32_t k, uint32_t mode,
                                           uint32_t *out_ids, float *out_scores, uint32_t *out_counts, void *stream) {
  if (!ix) return SNN_E_INVALID;
  return search_dev_entry(ix, nq, indptr, total, coords, vals, k, snn_search_params{mode, 0, 0, 0}, out_ids,
                          out_scores, out_counts, stream);
}

extern "C" snn_status snn_last_batch_status(snn_index *ix, uint32_t *invalid_queries, uint32_t *fallbacks) {
  if (!ix) return SNN_E_INVALID;
  uint32_t inv = 0;
  uint32_t fb = 0;
  if (ix->last_nq && ix->last_status) {
    std::vector<uint32_t> st(ix->last_nq);
    HIP_TRY(ix, hipDeviceSynchronize(), "sync");
    HIP_TRY(ix, hipMemcpy(st.data(), ix->last_status, (size_t)ix->last_nq * 4, hipMemcpyDeviceToHost), "status readback");
    for (uint32_t v : st) inv += v != 0;
    if (ix->last_nlist)
      HIP_TRY(ix, hipMemcpy(&fb, ix->last_nlist, 4, hipMemcpyDeviceToHost), "fallback count readback");
  }
  if (invalid_queries) *invalid_queries = inv;
  if (fallbacks) *fallbacks = fb;
  return SNN_OK;
}

extern "C" snn_status snn_last_batch_work(snn_index *ix, snn_batch_work *out) {
  if (!ix || !out) return SNN_E_INVALID;
  unsigned long long c[4] = {0, 0, 0, 0};
  if (ix->last_nq && ix->last_stats) {
    HIP_TRY(ix, hipDeviceSynchronize(), "sync");
    HIP_TRY(ix, hipMemcpy(c, ix->last_stats, 32, hipMemcpyDeviceToHost), "work counters readback");
  }
  out->candidates = c[0];
  out->candidates_fallback = c[1];
  out->selects = c[2];
  out->selects_fallback = c[3];
  return SNN_OK;
}

extern "C" snn_status snn_bucket_table(snn_index *ix, uint32_t *out) {
  if (!ix || !out) return SNN_E_INVALID;
  HIP_TRY(ix, hipMemcpy(out, ix->dev.bucket, (size_t)ix->cfg.h * ix->cfg.dim * 4, hipMemcpyDeviceToHost), "bucket readback");
  return SNN_OK;
}

extern "C" snn_status snn_read_sketch(snn_index *ix, uint32_t id, float *u, float *l) {
  if (!ix || !u || !l) return SNN_E_INVALID;
  const uint32_t *it = ix->id2slot.find(id);
  if (!it) return ix->fail(SNN_E_NOT_FOUND, "read_sketch: id %u is not live", id);
  const uint32_t s = *it;
  HIP_TRY(ix, hipStreamSynchronize(ix->stream), "sync");
  const uint32_t m = ix->cfg.m;
  if (ix->cfg.flags & SNN_SKETCH_BF16) {
    std::vector<uint16_t> hu(m, 0), hl(m, 0);
    HIP_TRY(ix, hipMemcpy2D(hu.data(), 2, (uint16_t *)ix->dev.U + s, (size_t)ix->cap * 2, 2, m, hipMemcpyDeviceToHost),
            "U readback");
    if (ix->dev.L)
      HIP_TRY(ix,
              hipMemcpy2D(hl.data(), 2, (uint16_t *)ix->dev.L + s, (size_t)ix->cap * 2, 2, m, hipMemcpyDeviceToHost),
              "L readback");
    for (uint32_t b = 0; b < m; ++b) {
      const uint32_t ub = (uint32_t)hu[b] << 16, lb = (uint32_t)hl[b] << 16;
      memcpy(&u[b], &ub, 4);
      memcpy(&l[b], &lb, 4);
    }
    return SNN_OK;
  }
  HIP_TRY(ix, hipMemcpy2D(u, 4, ix->dev.U + s, (size_t)ix->cap * 4, 4, m, hipMemcpyDeviceToHost), "U readback");
  if (ix->dev.L)
    HIP_TRY(ix, hipMemcpy2D(l, 4, ix->dev.L + s, (size_t)ix->cap * 4, 4, m, hipMemcpyDeviceToHost), "L readback");
  else
    for (uint32_t b = 0; b < m; ++b) l[b] = 0.0f;
  return SNN_OK;
}

hipEvent_t snn_index::prof_event() {
  if (!prof_pool.empty()) {
    hipEvent_t e = prof_pool.back();
    prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// While profiling, one event on the index's stream before (end = false) or
// after (end = true) an update kernel.
hipError_t snn_index::prof_update(int which, uint32_t docs, bool end) {
  if (!prof_on) return hipSuccess;
  hipEvent_t e = prof_event();
  if (!e) return hipErrorOutOfMemory;
  hipError_t r = hipEventRecord(e, stream);
  if (r != hipSuccess) {
    prof_pool.push_back(e);
    return r;
  }
  prof_upd[which].push_back(e);
  if (end) prof_upd_docs[which].push_back(docs);
  return hipSuccess;
}

extern "C" snn_status snn_profile_read_updates(snn_index *ix, double *insert_ms, uint64_t *insert_docs,
                                               double *delete_ms, uint64_t *delete_docs) {
  if (!ix) return SNN_E_INVALID;
  double ms_out[2] = {0, 0};
  uint64_t docs_out[2] = {0, 0};
  for (int w = 0; w < 2; ++w) {
    std::vector<hipEvent_t> &ev = ix->prof_upd[w];
    for (size_t i = 0; i + 1 < ev.size(); i += 2) {
      HIP_TRY(ix, hipEventSynchronize(ev[i + 1]), "event sync");
      float ms = 0;
      HIP_TRY(ix, hipEventElapsedTime(&ms, ev[i], ev[i + 1]), "event time");
      ms_out[w] += ms;
    }
    for (uint32_t d : ix->prof_upd_docs[w]) docs_out[w] += d;
    for (hipEvent_t e : ev) ix->prof_pool.push_back(e);
    ev.clear();
    ix->prof_upd_docs[w].clear();
  }
  if (insert_ms) *insert_ms = ms_out[0];
  if (insert_docs) *insert_docs = docs_out[0];
  if (delete_ms) *delete_ms = ms_out[1];
  if (delete_docs) *delete_docs = docs_out[1];
  return SNN_OK;
}

extern "C" snn_status snn_profile_enable(snn_index *ix, int on) {
  if (!ix) return SNN_E_INVALID;
  ix->prof_on = on != 0;
  return SNN_OK;
}

extern "C" snn_status snn_profile_read(snn_index *ix, double *tile_ms, uint32_t *launches) {
  if (!ix) return SNN_E_INVALID;
  double total = 0;
  uint32_t n = 0;
  for (size_t i = 0; i + 1 < ix->prof_events.size(); i += 2) {
    HIP_TRY(ix, hipEventSynchronize(ix->prof_events[i + 1]), "event sync");
    float ms = 0;
    HIP_TRY(ix, hipEventElapsedTime(&ms, ix->prof_events[i], ix->prof_events[i + 1]), "event time");
    total += ms;
    ++n;
  }
  for (hipEvent_t e : ix->prof_events) ix->prof_pool.push_back(e);
  ix->prof_events.clear();
  total += ix->prof_accum_ms;
  n += ix->prof_accum_n;
  ix->prof_accum_ms = 0;
  ix->prof_accum_n = 0;
  if (tile_ms) *tile_ms = total;
  if (launches) *launches = n;
  return SNN_OK;
}
