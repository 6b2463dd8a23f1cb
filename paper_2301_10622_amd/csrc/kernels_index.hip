// Index-update kernels (insert: Alg. 5; delete: Section 4.3) and query
// preparation (the first steps of Alg. 6).
#include "snn_device.h"

namespace snn {

// ---------------------------------------------------------------------------
// Insert (Alg. 5). One wavefront per document; workgroup b takes document
// (b mod 8) * ceil(n / 8) + b / 8, so each XCD (workgroups go to the 8 XCDs in
// turn) inserts one contiguous run of the batch. Batches fill consecutive
// slots, so the 4-byte column entries of neighbouring slots, which share
// 128-byte lines of every sketch row, meet in one XCD's L2 instead of eight.
// (A fixed grid looping over the run is slower: the barrier between two
// documents makes each wave wait for its stores, which a finished wave leaves
// in flight.) For each document:
//   1. every (coordinate, mapping) pair folds its value into its bucket's
//      running max and min, kept in LDS as order-preserving integer keys so
//      plain integer atomics give the exact float max/min in any order;
//   2. the column `slot` of U and L is written whole (buckets no coordinate
//      maps to get 0), so a reused column holds no trace of its last owner;
//   3. the slot's bit is set in the posting bitmap of every coordinate, in the
//      live bitmap, and slot2id records the external id;
//   4. with a forward store, the document's (coordinate, value) pairs are
//      copied to its region (doc_off, placed by the host).
// The caller guarantees the slot's old postings were cleared before (delete).
// The slot's block is marked stale: until the next compaction, searches read
// its postings from the bitmaps.
// ---------------------------------------------------------------------------

// Document of workgroup b in an update launch over n documents (8 * ceil(n / 8)
// workgroups; those past the last document do nothing).
__device__ __forceinline__ uint32_t upd_doc(uint32_t n) {
  return (blockIdx.x & 7u) * ((n + 7u) / 8u) + (blockIdx.x >> 3);
}
inline uint32_t upd_grid(uint32_t n) { return 8u * ((n + 7u) / 8u); }
constexpr uint32_t kUpdMaxDocs = 1u << 28;  // per launch; keeps the grid below 2^31

// Directed rounding of a float32 to bfloat16 (its upper 16 bits): dropping the
// low bits moves a value toward zero, so rounding up a positive value (down a
// negative one) takes the next bfloat16 away from zero.
__device__ __forceinline__ uint16_t bf16_round(float x, bool up) {
  const uint32_t b = __builtin_bit_cast(uint32_t, x);
  uint32_t t = b >> 16;
  if ((b & 0xFFFFu) != 0u && ((x > 0.0f) == up)) t += 1u;
  return (uint16_t)t;
}

// Steps 1, 2 and 4 above for document d (with `postings`, step 3's posting
// bits too, one atomic each), a wave per document; umax / umin are the wave's
// m LDS keys each. Every wave of the workgroup calls it the same number of
// times (a wave without a document passes active = false), since it holds
// workgroup barriers.
__device__ __forceinline__ void insert_doc(const DevIndex &ix, bool active, uint32_t d,
                                           const uint32_t *__restrict__ slots, const uint32_t *__restrict__ ids,
                                           const uint64_t *__restrict__ indptr, const uint32_t *__restrict__ coords,
                                           const float *__restrict__ vals, const DevForward &fw,
                                           const uint64_t *__restrict__ doc_off, uint32_t *umax, uint32_t *umin,
                                           bool postings) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t m = ix.m, h = ix.h;
  for (uint32_t b = lane; b < m; b += 64) {
    umax[b] = 0u;           // below every finite key
    umin[b] = 0xFFFFFFFFu;  // above every finite key
  }
  __syncthreads();
  uint64_t e0 = 0, e1 = 0;
  uint32_t slot = 0;
  if (active) {
    e0 = indptr[d];
    e1 = indptr[d + 1];
    slot = slots[d];
    const uint64_t pbit = 1ull << post_bit(slot);
    const size_t pword = post_word(slot);
    for (uint64_t e = e0 + lane; e < e1; e += 64) {
      const uint32_t j = coords[e];
      const float v = vals[e];
      if (v == 0.0f) continue;  // not in nz(x)
      const uint32_t key = ord_key(v);
      for (uint32_t o = 0; o < h; ++o) {
        const uint32_t b = ix.bucket[(size_t)o * ix.dim + j];
        atomicMax(&umax[b], key);
        atomicMin(&umin[b], key);
      }
      if (postings) atomicOr((unsigned long long *)&ix.bits[(size_t)j * ix.W + pword], (unsigned long long)pbit);
    }
  }
  __syncthreads();
  if (!active) return;
  const bool bf = (ix.flags & kSketchBf16) != 0, lower = (ix.flags & kUpperOnly) == 0;
  for (uint32_t b = lane; b < m; b += 64) {
    const uint32_t a = umax[b], c = umin[b];
    const float u = a ? key_value(a) : 0.0f;
    const float l = (c != 0xFFFFFFFFu) ? key_value(c) : 0.0f;
    const size_t at = (size_t)b * ix.cap + slot;
    if (bf) {
      ((uint16_t *)ix.U)[at] = bf16_round(u, true);
      if (lower) ((uint16_t *)ix.L)[at] = bf16_round(l, false);
    } else {
      ix.U[at] = u;
      if (lower) ix.L[at] = l;
    }
  }
  if (doc_off) {
    const uint64_t o = doc_off[d];
    for (uint64_t e = e0 + lane; e < e1; e += 64)
      fw.ent[o + (e - e0)] = make_uint2(coords[e], __builtin_bit_cast(uint32_t, vals[e]));
    if (lane == 0) {
      fw.off[slot] = o;
      fw.len[slot] = (uint32_t)(e1 - e0);
    }
  }
  if (lane == 0) {
    ix.slot2id[slot] = ids[d];
    atomicOr((unsigned long long *)&ix.live[slot_word(slot)], (unsigned long long)(1ull << slot_bit(slot)));
    ix.stale[slot >> 10] = 1u;  // the block's array containers no longer list all its postings
  }
}

__global__ __launch_bounds__(64) void k_insert(DevIndex ix, uint32_t n, const uint32_t *__restrict__ slots,
                                               const uint32_t *__restrict__ ids,
                                               const uint64_t *__restrict__ indptr,
                                               const uint32_t *__restrict__ coords,
                                               const float *__restrict__ vals, DevForward fw,
                                               const uint64_t *__restrict__ doc_off) {
  extern __shared__ uint32_t ins_lds[];  // 2m words: running max keys, then min keys
  const uint32_t d = upd_doc(n);
  if (d >= n) return;
  insert_doc(ix, true, d, slots, ids, indptr, coords, vals, fw, doc_off, ins_lds, ins_lds + ix.m, true);
}

hipError_t launch_insert(const DevIndex &ix, uint32_t n, const uint32_t *slots, const uint32_t *ids,
                         const uint64_t *indptr, const uint32_t *coords, const float *vals, const DevForward &fw,
                         const uint64_t *doc_off, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (n > kUpdMaxDocs || ix.m > kMaxM) return hipErrorInvalidValue;
  if ((doc_off != nullptr) != (fw.ent != nullptr)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_insert, dim3(upd_grid(n)), dim3(64), 2u * ix.m * sizeof(uint32_t), s, ix, n, slots, ids,
                     indptr, coords, vals, fw, doc_off);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Delete (Section 4.3): clear the slot's bit in the posting bitmap of each of
// its coordinates and/or in the live bitmap. The sketch column stays as is.
// One wavefront per document, with the insert's per-XCD runs.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_delete(DevIndex ix, uint32_t n, const uint32_t *__restrict__ slots,
                                               const uint64_t *__restrict__ indptr,
                                               const uint32_t *__restrict__ coords, int clear_bits,
                                               int clear_live) {
  const uint32_t d = upd_doc(n);
  if (d >= n) return;
  const uint32_t slot = slots[d];
  const uint64_t pmask = ~(1ull << post_bit(slot));
  const size_t pword = post_word(slot);
  if (clear_bits) {
    for (uint64_t e = indptr[d] + threadIdx.x; e < indptr[d + 1]; e += 64)
      atomicAnd((unsigned long long *)&ix.bits[(size_t)coords[e] * ix.W + pword], (unsigned long long)pmask);
    // A slot deleted whole keeps its listed array postings: with its live bit
    // clear its score is never selected, and the insert that reuses it marks
    // the block stale. Postings cleared from a live slot make it stale now.
    if (threadIdx.x == 0 && !clear_live) ix.stale[slot >> 10] = 1u;
  }
  if (clear_live && threadIdx.x == 0)
    atomicAnd((unsigned long long *)&ix.live[slot_word(slot)], (unsigned long long)~(1ull << slot_bit(slot)));
}

hipError_t launch_delete(const DevIndex &ix, uint32_t n, const uint32_t *slots, const uint64_t *indptr,
                         const uint32_t *coords, int clear_bits, int clear_live, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (n > kUpdMaxDocs) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_delete, dim3(upd_grid(n)), dim3(64), 0, s, ix, n, slots, indptr, coords, clear_bits,
                     clear_live);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Compaction: array containers (Section 4.1, Notes on Implementation: the
// lists are held as Roaring holds them, an array of offsets where a block is
// sparse). k_count_rows counts each coordinate's postings; the host picks the
// coordinates that get an array container and their place in `post`;
// k_build_lists then writes, per such coordinate and 1,024-slot block, the
// segment start and the block offsets of the set bits.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_count_rows(DevIndex ix, uint32_t *__restrict__ cnt) {
  __shared__ uint32_t red[4];
  const uint32_t j = blockIdx.x;
  const uint64_t *row = ix.bits + (size_t)j * ix.W;
  uint32_t c = 0;
  for (uint32_t w = threadIdx.x; w < ix.W; w += blockDim.x) c += (uint32_t)__popcll(row[w]);
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) cnt[j] = red[0] + red[1] + red[2] + red[3];
}

hipError_t launch_count_rows(const DevIndex &ix, uint32_t *cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_count_rows, dim3(ix.dim), dim3(256), 0, s, ix, cnt);
  return hipGetLastError();
}

constexpr uint32_t kListChunk = 2048;  // blocks per pass of k_build_lists (8 per thread)

// One workgroup per array row r (coordinate row_coord[r]): segment starts
// seg[r][b] = rbase[r] + postings of the row in blocks before b, and
// seg[r][nblk] = rbase[r] + the row's count; the postings of block b go to
// post[seg[r][b] ..] as block offsets, lane l's set bits in bit order, and
// the bounds of each posting to pu / pl at the same place: the sketch's
// bounds for coordinate j at the slot (Alg. 6), the smallest of its h upper
// entries and the largest of its h lower entries, folded in mapping order
// with fminf / fmaxf as the scoring kernels fold them.
__global__ __launch_bounds__(256) void k_build_lists(DevIndex ix, const uint32_t *__restrict__ row_coord,
                                                     const uint64_t *__restrict__ rbase, uint32_t *__restrict__ seg,
                                                     uint16_t *__restrict__ post, void *__restrict__ pu,
                                                     void *__restrict__ pl) {
  __shared__ uint32_t cb[kListChunk];
  __shared__ uint32_t wsum[4];
  const uint32_t r = blockIdx.x;
  const uint32_t j = row_coord[r];
  const uint32_t nblk = ix.cap >> 10;
  const uint64_t *row = ix.bits + (size_t)j * ix.W;
  uint32_t *sr = seg + (size_t)r * (nblk + 1);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool bf = (ix.flags & kSketchBf16) != 0, lower = (ix.flags & kUpperOnly) == 0;
  uint64_t carry = rbase[r];
  for (uint32_t b0 = 0; b0 < nblk; b0 += kListChunk) {
    const uint32_t nb = min(kListChunk, nblk - b0);
    // postings per block, 8 consecutive blocks per thread
    uint32_t loc[8], tot = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t i = threadIdx.x * 8u + (uint32_t)k;
      uint32_t c = 0;
      if (i < nb) {
        const uint64_t *w = row + (size_t)(b0 + i) * 16u;
#pragma unroll
        for (int x = 0; x < 16; ++x) c += (uint32_t)__popcll(w[x]);
      }
      loc[k] = c;
      tot += c;
    }
    // exclusive scan of the per-thread totals: in the wave, then over the waves
    uint32_t inc = tot;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t ex = inc - tot;
    for (int w = 0; w < wave; ++w) ex += wsum[w];
    const uint32_t chunk_total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t i = threadIdx.x * 8u + (uint32_t)k;
      if (i < nb) {
        cb[i] = ex;
        sr[b0 + i] = (uint32_t)(carry + ex);
      }
      ex += loc[k];
    }
    __syncthreads();
    // offsets: a wave per block, each lane its 16-bit chunk of the block
    for (uint32_t i = (uint32_t)wave; i < nb; i += 4u) {
      const uint32_t bits = ((const uint16_t *)(row + (size_t)(b0 + i) * 16u))[lane];
      const uint32_t c = (uint32_t)__popc(bits);
      uint32_t pinc = c;
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(pinc, o);
        if (lane >= o) pinc += y;
      }
      uint64_t at = carry + cb[i] + (pinc - c);
      uint32_t b = bits;
      while (b) {
        const uint32_t x = (uint32_t)__builtin_ctz(b);
        b &= b - 1u;
        const uint32_t off = 256u * (x >> 2) + 4u * (uint32_t)lane + (x & 3u);
        const size_t slot = ((size_t)(b0 + i) << 10) + off;
        post[at] = (uint16_t)off;
        float u = 0.0f, l = 0.0f;
        for (uint32_t o = 0; o < ix.h; ++o) {
          const size_t a = (size_t)ix.bucket[(size_t)o * ix.dim + j] * ix.cap + slot;
          const float uo = bf ? __builtin_bit_cast(float, (uint32_t)((const uint16_t *)ix.U)[a] << 16) : ix.U[a];
          u = o ? __builtin_fminf(u, uo) : uo;
          if (lower) {
            const float lo = bf ? __builtin_bit_cast(float, (uint32_t)((const uint16_t *)ix.L)[a] << 16) : ix.L[a];
            l = o ? __builtin_fmaxf(l, lo) : lo;
          }
        }
        if (bf) {
          ((uint16_t *)pu)[at] = (uint16_t)(__builtin_bit_cast(uint32_t, u) >> 16);
          if (lower) ((uint16_t *)pl)[at] = (uint16_t)(__builtin_bit_cast(uint32_t, l) >> 16);
        } else {
          ((float *)pu)[at] = u;
          if (lower) ((float *)pl)[at] = l;
        }
        ++at;
      }
    }
    carry += chunk_total;
    __syncthreads();  // cb and wsum are reused by the next chunk
  }
  if (threadIdx.x == 0) sr[nblk] = (uint32_t)carry;
}

hipError_t launch_build_lists(const DevIndex &ix, uint32_t nrows, const uint32_t *row_coord, const uint64_t *rbase,
                              uint32_t *seg, uint16_t *post, void *pu, void *pl, hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_build_lists, dim3(nrows), dim3(256), 0, s, ix, row_coord, rbase, seg, post, pu, pl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Serving snapshots. vis[slot] packs (insert seq << 32) | delete seq in one
// 64-bit word, written and read whole, so a query never sees a torn pair; a
// query with sequence t sees the slot iff insert seq < t < delete seq. Only
// slots whose dirty bit is set are checked; every slot that is free when a
// session starts is dirty from the start, deleted slots become dirty when the
// delete is applied.
// ---------------------------------------------------------------------------
__global__ void k_serve_init(uint64_t *vis, uint64_t *dirty, const uint64_t *live, uint32_t cap) {
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < cap; s += gridDim.x * blockDim.x) {
    const bool lv = (live[slot_word(s)] >> slot_bit(s)) & 1ull;
    vis[s] = lv ? 0x00000000FFFFFFFFull : 0xFFFFFFFF00000000ull;  // live: always seen; free: never
  }
  for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < cap / 64; w += gridDim.x * blockDim.x)
    dirty[w] = ~live[w];
}

hipError_t launch_serve_init(uint64_t *vis, uint64_t *dirty, const uint64_t *live, uint32_t cap, hipStream_t s) {
  hipLaunchKernelGGL(k_serve_init, dim3(1024), dim3(256), 0, s, vis, dirty, live, cap);
  return hipGetLastError();
}

__global__ void k_serve_mark(uint64_t *vis, uint64_t *dirty, uint32_t n, const uint32_t *slots, const uint32_t *seqs,
                             int is_insert) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t s = slots[i];
  const uint64_t old = vis[s];
  vis[s] = is_insert ? (((uint64_t)seqs[i] << 32) | 0xFFFFFFFFull) : ((old & 0xFFFFFFFF00000000ull) | seqs[i]);
  atomicOr((unsigned long long *)&dirty[slot_word(s)], (unsigned long long)(1ull << slot_bit(s)));
}

hipError_t launch_serve_mark(uint64_t *vis, uint64_t *dirty, uint32_t n, const uint32_t *slots, const uint32_t *seqs,
                             int is_insert, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_serve_mark, dim3((n + 255) / 256), dim3(256), 0, s, vis, dirty, n, slots, seqs, is_insert);
  return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint32_t blocks = (uint32_t)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, value, n);
  return hipGetLastError();
}

__global__ void k_copy_u32(uint32_t *d, const uint32_t *s, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint32_t blocks = (uint32_t)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_copy_u32, dim3(blocks), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Query preparation (Alg. 6, first steps). One workgroup per query:
//   drop zero values (nz), reject coordinates >= dim, non-finite values,
//   duplicate coordinates and, without an L half, negative values, sort by |q_j| descending with ties to the lower j
//   (the order Alg. 6 walks the coordinates in), and look up the h buckets
//   K = {pi_o(j)} of every coordinate. cnt[q], the number of coordinates the
//   scoring walks, is cut to max_coords when that is smaller (the anytime
//   budget; every entry is still written), and nz_full[q] (nullable) gets the
//   whole count for the exact re-rank.
//   With h = 1 the cnt scored entries are then stored by sketch row (bucket,
//   then sign: U before L), ties in the order above. That is the order in
//   which every search form adds a query's terms, so a kernel that walks
//   several queries' entries row by row, loading each row once for all of
//   them, adds each document's terms in the same order as one query alone,
//   and every form gives bit-identical scores. At T = infinity the order of
//   the additions changes rounding only; which coordinates are scored is
//   still decided by the Alg. 6 order.
// Sort keys are 64-bit: high word ~|q|bits (ascending = |q| descending), low
// word (j << 1) | sign, so equal magnitudes fall back to the lower coordinate.
// ---------------------------------------------------------------------------
__device__ inline void bitonic_sort_u64_asc(uint64_t *s, int n) {
  for (int size = 2; size <= n; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int i = threadIdx.x; i < (n >> 1); i += blockDim.x) {
        const int lo = 2 * stride * (i / stride) + (i % stride);
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint64_t a = s[lo], b = s[hi];
        if ((a > b) == up) {
          s[lo] = b;
          s[hi] = a;
        }
      }
    }
  __syncthreads();
}

// Scoring order of the scored entries (the first min(nz, max_coords) in the
// Alg. 6 order): those of coordinates with a bitmap container only come first
// -- with h = 1 by sketch row, ties in the Alg. 6 order; with h > 1 in the
// Alg. 6 order -- then those with an array container (crow[j] != kNoRow), in
// the Alg. 6 order; the entries past the budget follow. nd[q] counts the first
// kind; cr[e] holds the array row of each entry of the second.
__device__ __forceinline__ uint32_t prep_row(const DevIndex &ix, const uint32_t *crow, uint32_t j, uint32_t sign,
                                             bool scored) {
  if (!scored) return 0x7FFFFFFFu;
  if (crow && crow[j] != kNoRow) return 0x7FFFFFFEu;
  return ix.h == 1 ? (ix.bucket[j] << 1) | sign : 0u;
}

__global__ __launch_bounds__(256) void k_prep(DevIndex ix, QueryDesc qd, const uint32_t *__restrict__ coords,
                                              const float *__restrict__ vals, uint32_t max_coords,
                                              uint32_t *__restrict__ nz_full, const uint32_t *__restrict__ crow) {
  __shared__ uint64_t keys[kPrepCap];
  __shared__ uint32_t bad;
  __shared__ uint32_t nz;
  __shared__ uint32_t ndense;
  const uint32_t q = blockIdx.x;
  const uint64_t e0 = qd.qptr[q];
  const uint64_t len64 = qd.qptr[q + 1] - e0;
  if (threadIdx.x == 0) {
    bad = len64 > (uint64_t)kPrepCap ? 1u : 0u;
    nz = 0;
    ndense = 0;
  }
  __syncthreads();
  if (bad) {
    if (threadIdx.x == 0) {
      qd.cnt[q] = 0;
      qd.nd[q] = 0;
      qd.status[q] = 1;
      if (nz_full) nz_full[q] = 0;
    }
    return;
  }
  const int len = (int)len64;
  if (len <= 256) {
    // short queries: rank counting instead of sorting. Keys of distinct
    // coordinates are distinct; equal coordinates are duplicates.
    __shared__ uint32_t sj[256];
    __shared__ uint64_t okey[256];
    const int t = threadIdx.x;
    uint64_t key = ~0ull;
    uint32_t j = 0xFFFFFFFFu, vb = 0;
    if (t < len) {
      j = coords[e0 + t];
      vb = __builtin_bit_cast(uint32_t, vals[e0 + t]);
      const uint32_t ab = vb & 0x7FFFFFFFu;
      if (j >= ix.dim || ab >= 0x7F800000u) atomicOr(&bad, 1u);
      if ((ix.flags & kUpperOnly) && ab != 0u && (vb >> 31)) atomicOr(&bad, 1u);  // no L to bound it
      if (ab != 0u) {
        atomicAdd(&nz, 1u);
        key = ((uint64_t)(~ab) << 32) | ((uint64_t)(j & 0x7FFFFFFFu) << 1) | (uint64_t)(vb >> 31);
      }
      keys[t] = key;
      sj[t] = j;
    }
    __syncthreads();
    uint32_t rank = 0;
    if (t < len) {
      for (int x = 0; x < len; ++x) {
        if (x != t && sj[x] == j) atomicOr(&bad, 1u);
        rank += keys[x] < key ? 1u : 0u;
      }
    }
    __syncthreads();  // `bad` and `nz` are final
    // scoring order (prep_row), by (row, rank)
    const uint32_t scored = min(nz, max_coords);
    uint64_t ok = ~0ull;
    uint32_t row = 0x7FFFFFFFu;
    if (t < len && !bad && key != ~0ull) {
      row = prep_row(ix, crow, j, vb >> 31, rank < scored);
      ok = ((uint64_t)row << 32) | rank;
      if (row < 0x7FFFFFFEu) atomicAdd(&ndense, 1u);
    }
    if (t < len) okey[t] = ok;
    __syncthreads();
    if (t < len && !bad && key != ~0ull) {
      uint32_t pos = 0;
      for (int x = 0; x < len; ++x) pos += okey[x] < ok ? 1u : 0u;
      const uint64_t e = e0 - qd.ebase + pos;
      qd.j[e] = j;
      qd.q[e] = vals[e0 + t];
      if (ix.h == 1) qd.b[e] = (ix.bucket[j] << 1) | (vb >> 31);  // the sketch row: bucket, then U / L
      else
        for (uint32_t o = 0; o < ix.h; ++o) qd.b[e * ix.h + o] = ix.bucket[(size_t)o * ix.dim + j];
      if (row == 0x7FFFFFFEu) qd.cr[e] = crow[j];
    }
    if (t == 0) {
      qd.cnt[q] = bad ? 0u : min(nz, max_coords);
      qd.nd[q] = bad ? 0u : ndense;
      qd.status[q] = bad ? 1u : 0u;
      if (nz_full) nz_full[q] = bad ? 0u : nz;
    }
    return;
  }
  int n = 1;
  while (n < len) n <<= 1;
  // validation, the non-zero count, and the coordinates of every entry (zero
  // values included, as in the short path) for the duplicate check
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    uint64_t key = ~0ull;
    if (i < len) {
      const uint32_t j = coords[e0 + i];
      const float v = vals[e0 + i];
      const uint32_t vb = __builtin_bit_cast(uint32_t, v);
      const uint32_t ab = vb & 0x7FFFFFFFu;
      if (j >= ix.dim || ab >= 0x7F800000u) atomicOr(&bad, 1u);
      if ((ix.flags & kUpperOnly) && ab != 0u && (vb >> 31)) atomicOr(&bad, 1u);  // no L to bound it
      if (ab != 0u) atomicAdd(&nz, 1u);
      key = (uint64_t)j;
    }
    keys[i] = key;
  }
  __syncthreads();
  // duplicate check: sort the coordinates alone, then compare neighbours
  {
    bitonic_sort_u64_asc(keys, n);
    for (int i = threadIdx.x; i + 1 < n; i += blockDim.x)
      if (keys[i] != ~0ull && keys[i] == keys[i + 1]) atomicOr(&bad, 1u);
    __syncthreads();
  }
  if (bad) {
    if (threadIdx.x == 0) {
      qd.cnt[q] = 0;
      qd.nd[q] = 0;
      qd.status[q] = 1;
      if (nz_full) nz_full[q] = 0;
    }
    return;
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    uint64_t key = ~0ull;
    if (i < len) {
      const uint32_t j = coords[e0 + i];
      const uint32_t vb = __builtin_bit_cast(uint32_t, vals[e0 + i]);
      const uint32_t ab = vb & 0x7FFFFFFFu;
      if (ab != 0u) key = ((uint64_t)(~ab) << 32) | ((uint64_t)j << 1) | (uint64_t)(vb >> 31);
    }
    keys[i] = key;
  }
  bitonic_sort_u64_asc(keys, n);
  const uint32_t cnt = nz;
  // scoring order (prep_row): sort (row, rank)
  __shared__ uint64_t okeys[kPrepCap];
  const uint32_t scored = min(cnt, max_coords);
  for (uint32_t i = threadIdx.x; i < (uint32_t)n; i += blockDim.x) {
    uint64_t ok = ~0ull;
    if (i < cnt) {
      const uint32_t lo = (uint32_t)keys[i];
      const uint32_t row = prep_row(ix, crow, lo >> 1, lo & 1u, i < scored);
      ok = ((uint64_t)row << 32) | i;
      if (row < 0x7FFFFFFEu) atomicAdd(&ndense, 1u);
    }
    okeys[i] = ok;
  }
  bitonic_sort_u64_asc(okeys, n);
  for (uint32_t p = threadIdx.x; p < cnt; p += blockDim.x) {
    const uint64_t ok = okeys[p];
    const uint64_t k = keys[(uint32_t)ok];
    const uint32_t ab = ~(uint32_t)(k >> 32);
    const uint32_t lo = (uint32_t)k;
    const uint32_t j = lo >> 1;
    const uint32_t vb = ab | ((lo & 1u) << 31);
    const uint64_t e = e0 - qd.ebase + p;
    qd.j[e] = j;
    qd.q[e] = __builtin_bit_cast(float, vb);
    if (ix.h == 1) qd.b[e] = (ix.bucket[j] << 1) | (vb >> 31);  // the sketch row: bucket, then U / L
    else
      for (uint32_t o = 0; o < ix.h; ++o) qd.b[e * ix.h + o] = ix.bucket[(size_t)o * ix.dim + j];
    if ((uint32_t)(ok >> 32) == 0x7FFFFFFEu) qd.cr[e] = crow[j];
  }
  if (threadIdx.x == 0) {
    qd.cnt[q] = min(cnt, max_coords);
    qd.nd[q] = ndense;
    qd.status[q] = 0;
    if (nz_full) nz_full[q] = cnt;
  }
}

hipError_t launch_prep(const DevIndex &ix, QueryDesc qd, uint32_t nq, const uint32_t *coords, const float *vals,
                       uint32_t max_coords, uint32_t *nz_full, const uint32_t *crow, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prep, dim3(nq), dim3(256), 0, s, ix, qd, coords, vals, max_coords ? max_coords : 0xFFFFFFFFu,
                     nz_full, crow);
  return hipGetLastError();
}

}  // namespace snn
