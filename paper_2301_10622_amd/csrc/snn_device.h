// Device-side data layout and kernel entry points of the Sinnamon library.
//
// Layout in HBM (one index):
//   bits     uint64 [dim][W]      posting bitmaps: the bit of slot s in row j is set
//                                 when the document in slot s has coordinate j in
//                                 nz(x) (the id-only inverted index I[j] of Section
//                                 4.1, stored as a bitmap over slots; W = cap / 64;
//                                 bit order post_word / post_bit below)
//   live     uint64 [W]           bit of slot s (order slot_word / slot_bit) set
//                                 when slot s holds a live document
//   U, L     float  [m][cap]      the sketch matrix halves, one contiguous row per
//                                 bucket (the transposed layout of Section 4.1);
//                                 bfloat16 with SNN_SKETCH_BF16, no L with
//                                 SNN_UPPER_ONLY
//   slot2id  uint32 [cap]         external id of the document in each slot
//   bucket   uint32 [h][dim]      the random mappings pi_o(j)
//   fwd      uint2  [entries]     forward store (optional, DevForward): (coordinate,
//                                 value bits) of each document, the vector storage S
//                                 of Alg. 7; per slot its first entry (uint64) and
//                                 entry count (uint32)
//   crow     uint32 [dim]         array-container row of each coordinate, or kNoRow
//                                 (bitmap container only); set by a compaction
//   seg      uint32 [rows][nblk+1] per array row and 1,024-slot block, the first entry
//                                 of the block's segment in `post` (the row's last
//                                 entry closes it)
//   post     uint16 [entries]     the posting slots of array rows, as offsets inside
//                                 their block, in any order within a segment
//   pu, pl   float  [entries]     per array posting (coordinate j, slot s), the bounds
//                                 the sketch gives: min_o U[pi_o(j)][s] and
//                                 max_o L[pi_o(j)][s] (bfloat16 with SNN_SKETCH_BF16,
//                                 no pl with SNN_UPPER_ONLY), copied at the compaction
//   stale    uint32 [nblk]        non-zero for a block with a slot inserted (or a live
//                                 slot's postings cleared) since the last compaction:
//                                 its array segments are out of date, the bitmaps
//                                 never are (a slot deleted whole keeps its listed
//                                 postings; it is not live, so its score is unused)
//
// Containers (the id lists of Section 4.1, Notes on Implementation, held the
// way Roaring holds them): every coordinate keeps its posting bitmap, which
// insert and delete update in place; a compaction gives each coordinate of
// density at most 1/16 an array container as well -- per 1,024-slot block the
// block offsets of its postings -- so that scoring it costs work per posting
// rather than per slot. A block changed after the compaction is marked stale
// and read from the bitmaps.
//
// Lane l of a wave owns slots 4l .. 4l+3 of each 256-slot group it covers, so
// it reads their 4 sketch values with one load and no lane ever contends with
// another for a score. The live and dirty bitmaps are interleaved by group so
// that a 64-bit word is a wavefront lane mask: in group g (slots 256g ..
// 256g+255), word 4g + i has bit l set for slot 256g + 4l + i. The posting
// bitmaps are lane-major inside each block of 1,024 slots (4 groups): the 16
// bits of lane l -- slot 256g + 4l + i of the block at bit 4g + i -- form the
// block's 16-bit chunk l, so a wave reads its lanes' bits of one coordinate
// with a 2-byte load per lane (128 contiguous bytes) and many coordinates'
// bits can be in flight at once in vector registers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snn {

constexpr int kWaves = 4;               // waves per workgroup
constexpr int kBlock = 64 * kWaves;      // threads per workgroup
constexpr uint32_t kTileMax = 16384;     // largest tile (docs); capacity is a multiple
constexpr int kPrepCap = 4096;           // max non-zeros of one query
constexpr uint32_t kMaxK = 4096;        // largest k of a sorted result
constexpr uint32_t kMaxKPrime = 65536;  // largest k' of the re-rank (Alg. 7)
constexpr uint32_t kMaxM = 1024;        // largest m: the insert folds a column's 2m buckets in LDS

struct DevIndex {
  uint64_t *bits;
  uint64_t *live;
  float *U;
  float *L;
  uint32_t *slot2id;
  uint32_t *bucket;
  uint32_t *stale;       // [nblk] blocks changed since the last compaction
  const uint32_t *seg;   // [rows][nblk + 1] array containers (null before any compaction)
  const uint16_t *post;
  const void *pu, *pl;   // [entries] bounds of the array postings (float, or bfloat16 bits)
  uint32_t dim, m, h, cap, W;
  uint32_t flags;     // kSketchBf16 | kUpperOnly
};
constexpr uint32_t kNoRow = 0xFFFFFFFFu;  // crow of a coordinate with a bitmap container only
constexpr uint32_t kSketchBf16 = 2u;  // U and L rows hold bfloat16 (U rounded up, L down)
constexpr uint32_t kUpperOnly = 4u;   // no L half: non-negative collections (Sinnamon+)

// Forward store (optional), kept out of DevIndex: the scoring kernel's
// argument block stays small, which keeps its register use (and occupancy)
// where it is without one.
struct DevForward {
  uint2 *ent;        // (coordinate, value bits) entries; null without a forward store
  uint64_t *off;     // [cap] first entry of each slot's document
  uint32_t *len;     // [cap] its number of entries
};

// Prepared queries (Alg. 6 first steps): entry i < cnt[q] of query q sits at
// qptr[q] + i. The entries are the query's first cnt[q] coordinates in the
// order |q_j| descending, ties by lower j; with h = 1 they are then stored by
// sketch row (b), ties in that order, so that a document's terms are added row
// by row whichever kernel scores it.
struct QueryDesc {
  const uint64_t *qptr;  // [nq + 1] (the caller's CSR offsets; entry e sits at e - ebase below)
  uint32_t *cnt;         // [nq] non-zero entries after preparation
  uint32_t *nd;          // [nq] of those, the leading entries scored from bitmap containers; the
                         // rest (array containers) follow in the order of Alg. 6
  uint32_t *status;      // [nq] 0 = ok, else malformed
  uint32_t *j;           // [total]
  float *q;              // [total]
  uint32_t *b;           // [total * h] the buckets pi_o(j); with h = 1 the sketch row
                         // (pi_0(j) << 1) | (q_j < 0), i.e. the bucket and the U / L half
  uint32_t *cr;          // [total] array-container row of each entry past nd
  uint64_t ebase;        // qptr value of the first entry held in j, q, b
};

struct TileArgs {
  DevIndex ix;
  QueryDesc qd;
  uint32_t nq;        // queries in the batch
  uint32_t q0;        // first query of this launch
  uint32_t tiles;     // active tiles (covering slots below the high-water mark)
  uint32_t kmax;      // candidate stride per (query, tile)
  const uint32_t *kq; // per-query k (nullable: kmax for all)
  uint32_t *thr;      // [nq] shared inclusive lower bound on the k-th key (0 = none)
  uint64_t *cand;     // [nq][tiles][kmax]
  uint32_t *cand_cnt; // [nq][tiles]
  // persistent schedule
  uint32_t *queue;    // [8] per-XCD work counters (zeroed before launch)
  uint32_t xcds;      // number of per-XCD queues
  // snapshot visibility while serving (qseq null: every live slot is visible)
  const uint32_t *qseq;   // [nq] sequence number of each query
  const uint64_t *vis;    // [cap] (insert seq << 32) | delete seq
  const uint64_t *dirty;  // bitmap, slot layout of `live`: slot changed during the session
  // query list (nullable): the launch covers queries qlist[0 .. *nlist), a count
  // written on the device by an earlier kernel of the same stream
  const uint32_t *qlist;
  const uint32_t *nlist;
  uint32_t *cand_slot;    // [nq][tiles][kmax] slot of each candidate (nullable)
  unsigned long long *nselect;  // += 1 per tile that ran the radix select (nullable)
};

// Final selection of each query's top-k over all of its tile groups.
struct SelectArgs {
  uint32_t nq;
  uint32_t q0;
  uint32_t groups_in;   // candidate groups per query (tiles)
  uint32_t in_stride;   // stride of a group
  uint32_t kmax;        // k, and the stride of a result row
  const uint32_t *kq;   // per-query k (nullable)
  const uint32_t *keff; // per-query required count for the filter check (nullable)
  const uint64_t *in;     // [nq][groups_in][in_stride] keys
  const uint32_t *in_cnt; // [nq][groups_in]
  uint32_t *res_ids;    // [nq][kmax]
  float *res_scores;
  uint32_t *res_cnt;    // [nq]
  uint32_t *fallback;   // [nq] set to 1 when fewer than keff candidates survived
  const uint32_t *status; // [nq] malformed queries produce 0 results
  const uint32_t *qlist;  // query list (nullable), as in TileArgs
  const uint32_t *nlist;
  unsigned long long *emitted; // nullable: += candidates read
  const uint32_t *in_slot;     // candidate slots, layout of `in` (nullable)
  uint32_t *res_slots;         // [nq][kmax] slots of the results (with in_slot)
};

// live / dirty bitmaps: word and bit of a slot
__host__ __device__ inline uint32_t slot_word(uint32_t slot) { return ((slot >> 8) << 2) | (slot & 3u); }
__host__ __device__ inline uint32_t slot_bit(uint32_t slot) { return (slot >> 2) & 63u; }
// posting bitmaps: word and bit of a slot inside a row (block slot >> 10, lane
// l = (slot >> 2) & 63 in word l / 4 at bits 16 (l % 4) + 4g + i)
__host__ __device__ inline uint32_t post_word(uint32_t slot) { return ((slot >> 10) << 4) | ((slot >> 4) & 15u); }
__host__ __device__ inline uint32_t post_bit(uint32_t slot) {
  return (((slot >> 2) & 3u) << 4) | (((slot >> 8) & 3u) << 2) | (slot & 3u);
}

// order-preserving float -> uint32 map (negative floats reversed); 0 never occurs for finite x
__host__ __device__ inline uint32_t ord_key(float x) {
  uint32_t b = __builtin_bit_cast(uint32_t, x);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__host__ __device__ inline float key_value(uint32_t k) {
  uint32_t b = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __builtin_bit_cast(float, b);
}

// launchers (return hipError_t of the launch)
hipError_t launch_insert(const DevIndex &ix, uint32_t n, const uint32_t *slots, const uint32_t *ids,
                         const uint64_t *indptr, const uint32_t *coords, const float *vals, const DevForward &fw,
                         const uint64_t *doc_off, hipStream_t s);
hipError_t launch_serve_mark(uint64_t *vis, uint64_t *dirty, uint32_t n, const uint32_t *slots,
                             const uint32_t *seqs, int is_insert, hipStream_t s);
hipError_t launch_serve_init(uint64_t *vis, uint64_t *dirty, const uint64_t *live, uint32_t cap, hipStream_t s);
hipError_t launch_delete(const DevIndex &ix, uint32_t n, const uint32_t *slots, const uint64_t *indptr,
                         const uint32_t *coords, int clear_bits, int clear_live, hipStream_t s);
// max_coords: anytime budget (0 = every coordinate); nz_full (nullable): whole counts;
// crow (nullable): array-container rows (none: every entry is scored from bitmaps)
hipError_t launch_prep(const DevIndex &ix, QueryDesc qd, uint32_t nq, const uint32_t *coords, const float *vals,
                       uint32_t max_coords, uint32_t *nz_full, const uint32_t *crow, hipStream_t s);
// compaction: postings per coordinate (cnt[dim]), then the array containers of
// the coordinates with a row (crow[j] != kNoRow, rows in rbase order)
hipError_t launch_count_rows(const DevIndex &ix, uint32_t *cnt, hipStream_t s);
hipError_t launch_build_lists(const DevIndex &ix, uint32_t nrows, const uint32_t *row_coord, const uint64_t *rbase,
                              uint32_t *seg, uint16_t *post, void *pu, void *pl, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t value, size_t n, hipStream_t s);
hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, size_t n, hipStream_t s);
hipError_t launch_tiles(const TileArgs &a, int R, uint32_t nq_launch, hipStream_t s);
// one query (a.q0) alone, latency-first (the plain form)
hipError_t launch_tiles_latency(const TileArgs &a, int R, hipStream_t s);
hipError_t launch_tiles_persistent(const TileArgs &a, int R, uint32_t grid, hipStream_t s);
// h = 1: Q queries per workgroup, one sketch-row load for all of them; the
// non-persistent form launches (tiles, ng_launch) groups from group a.q0
hipError_t launch_tiles_grouped(const TileArgs &a, int R, int Q, bool persistent, uint32_t grid, uint32_t ng_launch,
                                hipStream_t s);
// the top-k of each query straight from all its candidate groups (radix select);
// sorted: the k <= 4,096 results in key order (no slots); unsorted: the k' <=
// 65,536 candidates of the re-rank in any order, with their slots
hipError_t launch_select(const SelectArgs &a, bool sorted, hipStream_t s);
// Alg. 7: exact scores of the selected k' candidates of each query, as keys
// ord(score) << 32 | (0xFFFFFFFF - id); the k best are then selected.
struct RerankArgs {
  DevForward fw;
  QueryDesc qd;
  uint32_t q0;              // first query of this launch
  uint32_t kprime;          // stride of the candidate and key rows
  uint32_t hash_cap;        // LDS hash slots for the query (power of two > 2 * max nnz)
  const uint32_t *cand_ids;   // [nq][kprime]
  const uint32_t *cand_slots; // [nq][kprime]
  const uint32_t *cand_cnt;   // [nq]
  const uint32_t *nz_full;    // [nq] non-zeros of each prepared query (all of them, whatever the budget)
  uint64_t *keys;             // [nq][kprime] out: exact-score keys
};
hipError_t launch_rerank(const RerankArgs &a, uint32_t nq, hipStream_t s);
hipError_t rerank_init();  // allows the re-rank kernel its largest LDS footprint

hipError_t launch_fallback_list(uint32_t nq, const uint32_t *flags, uint32_t *qlist, uint32_t *nlist, uint32_t *thr,
                                hipStream_t s);
// keff[q] = min(kq ? kq[q] : kmax, cap)
hipError_t launch_keff(uint32_t nq, const uint32_t *kq, uint32_t kmax, uint32_t cap, uint32_t *keff, hipStream_t s);
// thr[q] = ord(lowest of the ks scores sc[q][0 .. ks)) when cnt[q] >= ks, else 0
hipError_t launch_sample_thr(uint32_t nq, uint32_t ks, uint32_t stride, const float *sc, const uint32_t *cnt,
                             uint32_t *thr, hipStream_t s);

}  // namespace snn
