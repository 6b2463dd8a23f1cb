// Host-side state of one index (the opaque snn_index of include/snn.h).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <set>
#include <string>
#include <unordered_map>
#include <vector>

#include "snn.h"
#include "snn_device.h"

namespace snn {

uint64_t splitmix64_mix(uint64_t z);

// grow-only device buffer; growing synchronises the stream before freeing
struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
  hipError_t ensure(size_t bytes, hipStream_t s);
  void release();
};

struct PinBuf {
  void *p = nullptr;
  size_t cap = 0;
  hipError_t ensure(size_t bytes, hipStream_t s);
  void release();
};

// Device buffers of one in-flight search batch.
struct Workspace {
  DevBuf ws, cand;
  DevBuf cslot, rr;  // re-rank: candidate slots, the selected k' candidates
  void release() {
    ws.release();
    cand.release();
    cslot.release();
    rr.release();
  }
};

struct SearchWs {
  uint32_t *cnt = nullptr, *status = nullptr, *thr = nullptr, *fallback = nullptr, *keff = nullptr;
  uint32_t *j = nullptr, *b = nullptr;
  uint32_t *nd = nullptr, *cr = nullptr;  // bitmap-entry counts; array rows of the other entries
  float *q = nullptr;
  uint32_t *cand_cnt = nullptr, *queue = nullptr;
  uint64_t *cand = nullptr;
  uint32_t *qlist = nullptr, *nlist = nullptr;  // learned filter: the queries that fall back
  uint32_t *nz_full = nullptr;                  // [nq] whole non-zero count of each prepared query
  uint32_t *sthr = nullptr;                     // [nq] starting thresholds from a sample of the tiles
  uint32_t *ss_ids = nullptr, *ss_cnt = nullptr;  // the sample pass's selection (k_s <= 4,096), unsorted
  float *ss_sc = nullptr;
  uint32_t *cslot = nullptr;  // re-rank: slot of each candidate
  uint32_t *rr_ids = nullptr, *rr_slot = nullptr, *rr_cnt = nullptr;  // re-rank: the k' selected candidates
  float *rr_sc = nullptr;
  uint64_t *rk = nullptr;                       // re-rank: their exact-score keys
  unsigned long long *stats = nullptr;          // candidates emitted, selecting tiles (main, fallback pass)
};

// A search whose k' exceeds a tile samples one tile in kSampleStride for its
// starting thresholds.
constexpr uint32_t kSampleStride = 16;

// Launch schedule of the search kernels (set by the autotuner).
struct Tune {
  int R_plain = 16;      // registers (64-doc groups) per lane, plain mode
  int R_batch = 16;      // same, batched mode
  bool persistent = true;
  uint32_t grid = 2048;  // persistent grid
  int qgroup = 1;        // queries per batched workgroup (h = 1)
};

// External id -> slot: open addressing with linear probing over a power-of-two
// table (at most half full), erase by backward shift, so no tombstones. The
// id 0xFFFFFFFF is reserved by the API and marks an empty cell.
class IdMap {
 public:
  static constexpr uint32_t kEmpty = 0xFFFFFFFFu;
  size_t size() const { return n_; }
  void reserve(size_t want) {
    size_t cap = 16;
    while (cap < 2 * want) cap <<= 1;
    if (cap > keys_.size()) rehash(cap);
  }
  const uint32_t *find(uint32_t id) const {
    if (keys_.empty()) return nullptr;
    for (size_t i = slot_of(id);; i = (i + 1) & mask_) {
      if (keys_[i] == id) return &vals_[i];
      if (keys_[i] == kEmpty) return nullptr;
    }
  }
  bool contains(uint32_t id) const { return find(id) != nullptr; }
  // inserts or overwrites
  void put(uint32_t id, uint32_t slot) {
    if (2 * (n_ + 1) > keys_.size()) rehash(keys_.empty() ? 16 : 2 * keys_.size());
    size_t i = slot_of(id);
    while (keys_[i] != kEmpty && keys_[i] != id) i = (i + 1) & mask_;
    if (keys_[i] == kEmpty) ++n_;
    keys_[i] = id;
    vals_[i] = slot;
  }
  // false when absent
  bool erase(uint32_t id) {
    if (keys_.empty()) return false;
    size_t i = slot_of(id);
    while (keys_[i] != id) {
      if (keys_[i] == kEmpty) return false;
      i = (i + 1) & mask_;
    }
    // shift later members of the probe run back into the hole
    for (size_t j = (i + 1) & mask_;; j = (j + 1) & mask_) {
      if (keys_[j] == kEmpty) break;
      const size_t home = slot_of(keys_[j]);
      // j's entry may move to i when its home is not within (i, j] cyclically
      if (((j - home) & mask_) >= ((j - i) & mask_)) {
        keys_[i] = keys_[j];
        vals_[i] = vals_[j];
        i = j;
      }
    }
    keys_[i] = kEmpty;
    --n_;
    return true;
  }
  template <typename F>
  void for_each(F f) const {
    for (size_t i = 0; i < keys_.size(); ++i)
      if (keys_[i] != kEmpty) f(keys_[i], vals_[i]);
  }

 private:
  size_t slot_of(uint32_t id) const { return (size_t)((id * 0x9E3779B97F4A7C15ull) >> 32) & mask_; }
  void rehash(size_t cap) {
    std::vector<uint32_t> ok, ov;
    ok.swap(keys_);
    ov.swap(vals_);
    keys_.assign(cap, kEmpty);
    vals_.assign(cap, 0);
    mask_ = cap - 1;
    n_ = 0;
    for (size_t i = 0; i < ok.size(); ++i)
      if (ok[i] != kEmpty) put(ok[i], ov[i]);
  }
  std::vector<uint32_t> keys_, vals_;
  size_t mask_ = 0, n_ = 0;
};

// Free slots, grouped by 1,024-slot block, and the order in which inserts take
// them. Every insert marks its block stale (until the next compaction the
// block's array-container coordinates are read from the posting bitmaps), and
// a mirror of those marks is kept here. Before any compaction has built array
// containers, freed slots are reused first and fresh ones taken after them
// (Section 4.3). Once array containers exist, an insert goes where it costs
// least: a free slot of a block already stale, then a fresh slot (the tail
// blocks), and only then a free slot of a clean block -- the one with the most
// free slots, which then counts as stale for the slots after it.
class SlotPool {
 public:
  void init(uint32_t cap) {
    nblk_ = cap >> 10;
    free_.assign(nblk_, {});
    stale_.assign(nblk_, 0);
    stale_free_.clear();
    clean_.clear();
    count_ = 0;
  }
  size_t size() const { return count_; }
  bool is_stale(uint32_t blk) const { return stale_[blk] != 0; }

  void release(uint32_t slot) {
    const uint32_t b = slot >> 10;
    auto &f = free_[b];
    if (stale_[b]) {
      if (f.empty()) stale_free_.insert(b);
    } else {
      if (!f.empty()) clean_.erase({(uint32_t)f.size(), b});
      clean_.insert({(uint32_t)f.size() + 1, b});
    }
    f.push_back(slot);
    ++count_;
  }

  // The slot of the next insert; the caller has checked that one is left
  // (size() > 0 or next_fresh < cap). arrays: array containers exist.
  uint32_t take(uint32_t &next_fresh, uint32_t cap, bool arrays) {
    if (!stale_free_.empty()) return pop(*stale_free_.begin());
    if ((arrays || clean_.empty()) && next_fresh < cap) {
      const uint32_t s = next_fresh++;
      mark_stale(s >> 10);
      return s;
    }
    const uint32_t b = clean_.rbegin()->second;
    mark_stale(b);
    return pop(b);
  }

  // after a compaction: no block is stale
  void clear_stale() {
    for (uint32_t b : stale_free_) clean_.insert({(uint32_t)free_[b].size(), b});
    stale_free_.clear();
    std::fill(stale_.begin(), stale_.end(), (uint8_t)0);
  }

 private:
  void mark_stale(uint32_t b) {
    if (stale_[b]) return;
    stale_[b] = 1;
    if (!free_[b].empty()) {
      clean_.erase({(uint32_t)free_[b].size(), b});
      stale_free_.insert(b);
    }
  }
  uint32_t pop(uint32_t b) {  // b is stale with free slots
    auto &f = free_[b];
    const uint32_t s = f.back();
    f.pop_back();
    if (f.empty()) stale_free_.erase(b);
    --count_;
    return s;
  }
  uint32_t nblk_ = 0;
  std::vector<std::vector<uint32_t>> free_;
  std::vector<uint8_t> stale_;
  std::set<uint32_t> stale_free_;                       // stale blocks with free slots
  std::set<std::pair<uint32_t, uint32_t>> clean_;       // (free slots, block) of clean blocks
  size_t count_ = 0;
};

struct LearnedFilter;   // learned k-th-score pre-filter (kernels_mlp.hip)

// Device state of a learned-filter pass: feature table and bf16 weights, per-query
// features, prediction, threshold keys and required counts.
struct LearnedPass {
  const uint32_t *table = nullptr;
  const uint16_t *Pb = nullptr;
  float *X = nullptr, *yhat = nullptr;
  uint32_t *thr = nullptr, *keff = nullptr;
  float delta = 0.0f;
  uint32_t keff_value = 0, dim = 0;
};

// Optional per-query inputs of a search (device arrays of nq entries).
struct SearchOpts {
  const LearnedPass *learned = nullptr;  // filtered pass with a device-side plain fallback
  uint32_t rerank_k = 0;                 // > 0: the batch k is k' of Alg. 7 and this many are returned
  uint32_t hash_cap = 0;                 // re-rank: LDS hash slots per query
  uint32_t max_coords = 0;               // anytime budget: coordinates scored per query (0 = all)
  const uint32_t *thr_init = nullptr;  // initial inclusive threshold keys (learned filter)
  const uint32_t *kq = nullptr;        // per-query k (<= the batch k)
  const uint32_t *keff = nullptr;      // count below which the filter check reports a fallback
  const uint32_t *qseq = nullptr;      // serving: per-query sequence numbers (snapshot visibility)
  uint64_t ebase = 0;                  // indptr value of the batch's first entry
  Workspace *wsp = nullptr;            // buffers (null: the index's own)
  char *ext_ws = nullptr;              // caller region that holds every buffer instead (nothing allocated)
  size_t ext_ws_bytes = 0;
  bool no_graph = false;
};

// One selection pass over the tile candidates of queries q0 .. q0 + nqm
// (or of the listed queries, when qlist is set).
struct MergeJob {
  uint32_t q0 = 0, nqm = 0, tiles = 0, k = 0;
  const uint32_t *kq = nullptr, *keff = nullptr;
  uint32_t *res_ids = nullptr, *res_cnt = nullptr, *res_slots = nullptr;
  bool slots = false;  // carry the candidates' slots (cslot) to the results
  bool sorted = true;  // results in key order (k <= 4,096); else any order (re-rank candidates)
  // input: the tile candidates (in == null) or one group per query
  const uint64_t *in = nullptr;
  const uint32_t *in_cnt = nullptr;
  uint32_t in_stride = 0;
  float *res_scores = nullptr;
  const uint32_t *qlist = nullptr, *nlist = nullptr;
  unsigned long long *emitted = nullptr;
  bool set_fallback = false;
};

struct SearchPlan {
  uint32_t nq = 0, k = 0, tiles = 0, grid = 0;
  uint32_t kt = 0;  // candidates one tile keeps per query: min(k, slots per tile)
  // k above a tile (re-rank): a first pass over tiles_s tiles selects the k_s
  // best there, whose lowest score starts the threshold of the full pass
  uint32_t tiles_s = 0, k_s = 0;
  int mode = 0, R = 16, qgroup = 1;
  bool persistent = false;
  uint64_t total = 0;
  const uint64_t *d_ptr = nullptr;
  const uint32_t *d_c = nullptr;
  const float *d_v = nullptr;
  uint32_t *d_ids = nullptr, *d_cnt = nullptr;
  float *d_sc = nullptr;
  SearchWs w;
};

struct GraphKey {
  uint32_t nq, k, mode, R, grid, tiles, qgroup;
  uint64_t total;
  bool persistent, prof;
  const void *ptr, *c, *v, *ids, *sc, *cnt, *thr, *kq, *keff, *ws, *cand, *qseq;
  const void *lX, *ly, *lthr, *lkeff, *lPb, *ltab;
  uint32_t ldelta, lkeff_v, rerank_k, hash_cap, max_coords;
  uint32_t skeff;  // sampled starting thresholds: the count cap min(k, live) the graph holds (0: none)
  const void *cslot, *rr, *fwd;
  uint64_t ebase;
  hipStream_t stream;
  bool operator==(const GraphKey &o) const {
    return nq == o.nq && k == o.k && mode == o.mode && R == o.R && grid == o.grid && tiles == o.tiles &&
           qgroup == o.qgroup &&
           lX == o.lX && ly == o.ly && lthr == o.lthr && lkeff == o.lkeff && lPb == o.lPb && ltab == o.ltab &&
           ldelta == o.ldelta && lkeff_v == o.lkeff_v && rerank_k == o.rerank_k && hash_cap == o.hash_cap &&
           max_coords == o.max_coords && skeff == o.skeff &&
           cslot == o.cslot && rr == o.rr && fwd == o.fwd &&
           total == o.total && persistent == o.persistent && prof == o.prof && ptr == o.ptr && c == o.c &&
           v == o.v && ids == o.ids && sc == o.sc && cnt == o.cnt && thr == o.thr && kq == o.kq && keff == o.keff &&
           ws == o.ws && cand == o.cand && qseq == o.qseq && ebase == o.ebase &&
           stream == o.stream;
  }
};

struct GraphEntry {
  GraphKey key{};
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    exec = nullptr;
    ev0 = ev1 = nullptr;
  }
};

// A few instantiated graphs, most recent last.
struct GraphCache {
  std::vector<GraphEntry> e;
  GraphEntry *find(const GraphKey &k) {
    for (auto &x : e)
      if (x.key == k) return &x;
    return nullptr;
  }
  GraphEntry *insert(const GraphEntry &g) {
    if (e.size() >= 8) {
      e.front().release();
      e.erase(e.begin());
    }
    e.push_back(g);
    return &e.back();
  }
  void clear() {
    for (auto &x : e) x.release();
    e.clear();
  }
};

}  // namespace snn

void snn_filter_release(struct snn_index *ix);
// Device-buffer search with the workspace in the caller's region (snn_api.cpp).
snn_status snn_search_dev_in_region(struct snn_index *ix, uint32_t nq, const uint64_t *indptr, uint64_t total,
                                    const uint32_t *coords, const float *vals, uint32_t k, uint32_t mode,
                                    uint32_t *out_ids, float *out_scores, uint32_t *out_counts, void *stream,
                                    char *ext, size_t ext_bytes);
// Working state of the duplicate-coordinate check: a sort of the coordinates,
// or, over many vectors of a moderate dimension, one stamp per coordinate (the
// tag of the last vector that held it), so each vector costs O(nnz).
struct VecCheck {
  std::vector<uint32_t> scratch;
  std::vector<uint32_t> stamp;
  uint32_t tag = 0;
  bool stamps = false;
};
// Validates one vector (coordinates < dim, finite values, no duplicate
// coordinates, no negative values without an L half). On success appends its
// non-zero entries to *oc / *ov when given and stores their count in *nz when
// given. On failure records the reason with ix->fail when `report` (only then
// is ix written, so unreported checks may run on several threads).
bool snn_check_vector(struct snn_index *ix, uint32_t nnz, const uint32_t *c, const float *v,
                      std::vector<uint32_t> *oc, std::vector<float> *ov, VecCheck &vc, const char *what,
                      bool report = true, uint32_t *nz = nullptr);

struct snn_index {
  snn_config cfg{};
  uint32_t cap = 0, W = 0;
  int device = -1;  // the device current at snn_create, which holds the index
  hipStream_t stream = nullptr;
  snn::DevIndex dev{};
  snn::DevForward fw{};  // forward store (SNN_FORWARD_STORE)

  // slot store
  snn::IdMap id2slot;
  std::vector<uint32_t> slot_id;             // external id per slot (0xFFFFFFFF = free)
  std::vector<std::vector<uint32_t>> fwd;    // coordinates of the document in each slot
  snn::SlotPool free_slots;                  // freed columns and the order inserts take them
  // forward store (SNN_FORWARD_STORE): device entries dev.fwd[0 .. fwd_cap), of
  // which [0, fwd_top) have been handed out. Each slot owns a region of a
  // power-of-two size; a region too small for a new document goes to the free
  // list of its size class.
  bool has_fwd = false;
  uint64_t fwd_top = 0, fwd_cap = 0;
  std::vector<uint64_t> fwd_roff;
  std::vector<uint32_t> fwd_rlog;                    // log2 region size per slot (0: none)
  std::vector<std::vector<uint64_t>> fwd_free;       // by log2 size
  uint32_t next_fresh = 0;                   // slots [0, next_fresh) have been used
  size_t live = 0;
  uint64_t mutations = 0;

  // array containers (snn_compact): crow [dim] (null before the first
  // compaction), seg and post; the class of every coordinate (1: array)
  snn::DevBuf crow, lists_seg, lists_post, lists_pu, lists_pl;
  std::vector<uint8_t> classes;
  uint32_t list_rows = 0;
  uint64_t list_postings = 0;
  uint32_t array_coords = 0;  // coordinates of class 1

  // buffers
  snn::DevBuf up;
  snn::Workspace wsp;
  uint64_t *vis = nullptr, *dirty = nullptr;  // serving snapshot state (allocated by snn_serve_run)
  snn::PinBuf pin;
  snn::SearchWs last_ws;
  uint32_t last_nq = 0, last_mode = 0;
  const uint32_t *last_status = nullptr;  // device: per-query status of the last batch
  const uint32_t *last_nlist = nullptr;   // device: fallback count of the last learned batch
  const unsigned long long *last_stats = nullptr;  // device: selection work of the last batch
  snn::Tune tune;
  snn::LearnedFilter *filter = nullptr;
  bool filter_on = false;  // snn_filter_enable: the host-buffer searches run the learned form

  std::string err;

  snn::GraphCache graphs;
  bool use_graphs = true;
  float tune_best_ms = 0, tune_default_ms = 0;
  uint32_t tune_tried = 0;
  snn_schedule last_sched{};

  // kernel timing (snn_profile_*)
  bool prof_on = false;
  double prof_accum_ms = 0;
  uint32_t prof_accum_n = 0;
  std::vector<hipEvent_t> prof_events;  // pairs (start, end) recorded since the last read
  std::vector<hipEvent_t> prof_pool;
  // (start, end) pairs around the insert and the delete kernels, and the
  // documents each pair covered, recorded since the last read
  std::vector<hipEvent_t> prof_upd[2];
  std::vector<uint32_t> prof_upd_docs[2];
  hipEvent_t prof_event();
  hipError_t prof_update(int which, uint32_t docs, bool end);

  snn_status fail(snn_status st, const char *fmt, ...);
  snn_status hip_fail(hipError_t e, const char *what);

  snn_status fwd_place(const uint32_t *slots, const uint64_t *ptr, size_t n, uint64_t *doc_off);
  snn_status upload_and_insert(const std::vector<uint32_t> &slots, const std::vector<uint32_t> &ids,
                               const std::vector<uint64_t> &indptr, const std::vector<uint32_t> &coords,
                               const std::vector<float> &vals, size_t r0, size_t r1);
  snn_status upload_and_delete(const std::vector<uint32_t> &slots, const std::vector<uint64_t> &ptr,
                               const std::vector<uint32_t> &co, int clear_bits, int clear_live);
  snn_status prepare_workspace(uint32_t nq, uint64_t total, uint32_t kt, uint32_t tiles, uint32_t kprime, uint32_t ksample,
                               snn::SearchWs &w, snn::Workspace &W, hipStream_t s, char *ext, size_t ext_bytes);
  snn_status enqueue_merge(const snn::SearchWs &w, const snn::MergeJob &j, hipStream_t s);
  snn_status plan_search(uint32_t nq, const uint64_t *d_ptr, uint64_t total, const uint32_t *d_c, const float *d_v,
                         uint32_t k, int mode, uint32_t *d_ids, float *d_sc, uint32_t *d_cnt, snn::SearchPlan &p,
                         const snn::SearchOpts &o, hipStream_t s);
  snn_status enqueue_search(const snn::SearchPlan &p, const snn::SearchOpts &o, hipStream_t s, hipEvent_t *ev);
  snn_status run_search(uint32_t nq, const uint64_t *d_ptr, uint64_t total, const uint32_t *d_c, const float *d_v,
                        uint32_t k, int mode, uint32_t *d_ids, float *d_sc, uint32_t *d_cnt, hipStream_t s,
                        const snn::SearchOpts &o);
  snn_status search_learned(uint32_t nq, const uint64_t *d_ptr, uint64_t total, const uint32_t *d_c,
                            const float *d_v, uint32_t k, uint32_t max_coords, uint32_t rerank_k, uint32_t hash_cap,
                            uint32_t *d_ids, float *d_sc, uint32_t *d_cnt, hipStream_t s);
  snn_status compact(const uint8_t *pinned);
  void tune_init();
  void release_extras();
};
