// Search kernels: Sinnamon scoring (Alg. 6, T = infinity) fused with a
// per-tile top-k selection, and the merge of tile candidates into the final
// top-k (Alg. 3 / Alg. 7 with k' = k).
//
// A workgroup owns one (query, doc tile) pair. The tile is 256 * R consecutive
// slots, R / 4 groups of 256 per wave; in a group lane l owns the 4 adjacent
// slots 4l .. 4l+3. For each query coordinate j, in the order of Alg. 6, each
// lane reads its own posting bits of j -- the posting bitmaps are lane-major,
// so that is one 2-byte load per lane and 1,024-slot block, and the bits of
// several coordinates are fetched together to share one memory latency. A lane
// with any of its 4 slots on the list reads their 4 bounds from sketch row
// pi(j) -- min over the U rows if q_j > 0, max over the L rows otherwise --
// with one 16-byte load, and adds q_j * bound for the slots whose bit is set
// (q_j under the sign-extended bit, so no branches). A lane with none loads
// from an out-of-range buffer offset, which returns 0 without touching memory,
// so one vector memory instruction serves 256 slots. Scores never leave
// registers.
//
// Selection keys are ord(score) << 32 | (0xFFFFFFFF - id), so a larger key
// means a higher score, then a lower id. The tile first finds the k-th largest
// 32-bit score key by a most-significant-bit-first binary radix select built on
// wavefront ballots and popcounts (one workgroup reduction per bit, stopping as
// soon as the selected set has exactly k members), resolves ties at the k-th
// score by the lower id the same way, and writes at most k candidates. It then
// raises the query's shared threshold to its k-th key: no document below it can
// be in the global top-k, so later tiles keep fewer candidates.
#include <type_traits>

#include "snn_device.h"

namespace snn {

constexpr uint32_t kBufFlags = 0x00020000u;  // raw buffer resource, 32-bit data format
constexpr int kOob = (int)0x80000000u;         // buffer offset past every range: load returns 0
constexpr int kChunk = 4;  // query entries whose posting bits are fetched together

// Sketch rows hold float32 or, with SNN_SKETCH_BF16, bfloat16 values: a lane's
// 4 slots of a 256-slot group are 16 or 8 consecutive bytes.
template <bool kBf16>
struct Elem {
  static constexpr int kBytes = kBf16 ? 2 : 4;
  static constexpr int kLane = 4 * kBytes;   // bytes per lane and group
  static constexpr int kGroup = 64 * kLane;  // bytes per group
};

// The bounds of a lane's 4 slots in one group of a sketch row; 0 for an
// out-of-range offset (no memory is touched then). A bfloat16 is the upper
// half of a float32, so widening is a shift.
template <bool kBf16>
__device__ __forceinline__ void load4(__amdgpu_buffer_rsrc_t rs, int off, float (&v)[4]) {
  if constexpr (kBf16) {
    const uint32_t w0 = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
    const uint32_t w1 = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 4, 0, 0);
    v[0] = __builtin_bit_cast(float, w0 << 16);
    v[1] = __builtin_bit_cast(float, w0 & 0xFFFF0000u);
    v[2] = __builtin_bit_cast(float, w1 << 16);
    v[3] = __builtin_bit_cast(float, w1 & 0xFFFF0000u);
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      v[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off + 4 * i, 0, 0));
  }
}

// Buffer resource over the wave's slots of row b of U (q_j > 0) or L.
template <bool kBf16, int G>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const DevIndex &ix, bool upper, uint32_t b,
                                                           uint32_t wslot0) {
  const char *p = (const char *)(upper ? ix.U : ix.L) + ((size_t)b * ix.cap + wslot0) * Elem<kBf16>::kBytes;
  return __builtin_amdgcn_make_buffer_rsrc((void *)p, 0, G * Elem<kBf16>::kGroup, kBufFlags);
}

// Read-only arrays are read through the constant address space: with a
// wave-uniform address the loads become scalar loads (s_load), so query entries
// and the live / dirty words land in SGPRs (the latter drive lane masks directly).
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T *p) {
  return (cptr<T>)(p);
}

// Posting bits of one coordinate for the lane's slots in the wave's G groups:
// bit 4r + i <-> slot wslot0 + 256r + 4 lane + i. The bitmaps are lane-major in
// blocks of 1,024 slots, so this is one 2-byte load per lane and block.
template <int G>
struct LaneBits {
  using type = typename std::conditional<(G <= 8), uint32_t, uint64_t>::type;
};

template <int G>
__device__ __forceinline__ typename LaneBits<G>::type lane_bits(const DevIndex &ix, uint32_t j, uint32_t wslot0,
                                                                int lane) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void *)(ix.bits + (size_t)j * ix.W), 0, ix.W * 8u, kBufFlags);
  const int off = (int)((wslot0 >> 10) * 128u) + lane * 2;
  if constexpr (G <= 4) {
    // G = 2: the wave covers half a block, the bits of groups 2 and 3 when it
    // starts at the second half
    const uint32_t c = __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0);
    return c >> ((wslot0 >> 6) & 8u);
  } else {
    typename LaneBits<G>::type b = 0;
#pragma unroll
    for (int k = 0; k < G / 4; ++k)
      b |= (typename LaneBits<G>::type)__builtin_amdgcn_raw_buffer_load_b16(rs, off + 128 * k, 0, 0) << (16 * k);
    return b;
  }
}

// the 4 bits of group r
template <typename T>
__device__ __forceinline__ bool group_bits(T b, int r) {
  return ((b >> (4 * r)) & (T)15) != 0;
}

// q_j where bit x is set, +0 elsewhere (bits of q_j under a sign-extended bit)
template <typename T>
__device__ __forceinline__ float masked_q(T b, int x, uint32_t qbits) {
  const uint32_t w = x < 32 ? (uint32_t)b : (uint32_t)((uint64_t)b >> 32);
  const uint32_t m = (uint32_t)((int32_t)(w << (31 - (x & 31))) >> 31);
  return __builtin_bit_cast(float, m & qbits);
}

struct SelShared {
  uint32_t red[2][kWaves];
  uint32_t emit;
  uint32_t item;
};

__device__ __forceinline__ uint32_t wg_sum(uint32_t v, SelShared &sh, int &par) {
  if ((threadIdx.x & 63) == 0) sh.red[par][threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t s = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) s += sh.red[par][w];
  par ^= 1;
  return s;
}

__device__ __forceinline__ uint64_t uniform64(uint64_t w) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)w);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(w >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// k-th largest of the workgroup's keys (k >= 1, at least k keys non-zero).
// Returns the threshold T. exact = true: {key >= T} has exactly k members.
// exact = false: T is the k-th largest key itself, {key > T} has k - need
// members and need >= 1 of the keys equal to T are still to be chosen.
template <int R>
__device__ uint32_t select_kth(const uint32_t (&key)[R], uint32_t k, SelShared &sh, int &par, bool &exact,
                               uint32_t &need_out) {
  uint32_t prefix = 0, need = k;
  for (int bit = 31; bit >= 0; --bit) {
    const uint32_t hm = 0xFFFFFFFFu << bit;
    const uint32_t want = prefix | (1u << bit);
    uint32_t c = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) c += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64((key[r] & hm) == want));
    c = wg_sum(c, sh, par);
    if (c >= need) {
      prefix = want;
      if (c == need) {
        exact = true;
        need_out = 0;
        return prefix;
      }
    } else {
      need -= c;
    }
  }
  exact = false;
  need_out = need;
  return prefix;
}

template <int R>
__device__ __forceinline__ uint32_t count_pred(const bool (&p)[R]) {
  uint32_t c = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) c += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(p[r]));
  return c;
}

// Slot layout inside a 256-slot group (see snn_device.h): lane l owns slots
// 4l .. 4l+3; live / dirty word i of the group has bit l set for slot 4l + i.
// Register index x = 4r + i of a lane is slot wslot0 + 256r + 4l + i.
template <int R>
__device__ __forceinline__ uint32_t slot_of(uint32_t wslot0, int x, int lane) {
  return wslot0 + 256u * (uint32_t)(x >> 2) + 4u * (uint32_t)lane + (uint32_t)(x & 3);
}

template <int R>
__device__ void finish(const TileArgs &a, uint32_t q, uint32_t t, const float (&acc)[R], SelShared &sh);

// ---------------- entries with array containers ----------------
// A query's entries past nd[q] belong to coordinates whose postings are also
// held as per-block offset lists (array containers). For each such entry and
// each 1,024-slot block of the wave, the wave reads the block's segment -- at
// most 64 offsets per step, one per lane -- gathers each listed slot's bound
// and adds q_j * bound into that slot's score in LDS: work per posting, not
// per slot. The entries go in the Alg. 6 order; within one entry the listed
// slots are distinct, so no two lanes touch one score, and the wave's LDS
// operations complete in issue order. In a block changed since the last
// compaction (stale) the same entries are read from the posting bitmaps and
// the same terms added in the same order, so both give identical bits. The
// LDS sums are added to the register scores at the end, one add per slot.

// One bound of a slot: q > 0 reads min_o U[pi_o(j)][slot], q < 0 max_o L[...].
// kH1: h = 1, where the prepared row (bucket << 1 | q < 0) names the half.
template <bool kBf16, bool kH1>
__device__ __forceinline__ float gather_bound(const DevIndex &ix, cptr<uint32_t> qb, uint64_t e, uint32_t h,
                                              bool upper, uint32_t slot) {
  auto one = [&](uint32_t row, bool up) -> float {
    const size_t at = (size_t)row * ix.cap + slot;
    if constexpr (kBf16) {
      const uint16_t x = ((const uint16_t *)(up ? ix.U : ix.L))[at];
      return __builtin_bit_cast(float, (uint32_t)x << 16);
    } else {
      return (up ? ix.U : ix.L)[at];
    }
  };
  if (kH1 || h == 1) {
    const uint32_t b = qb[e];  // (bucket << 1) | (q < 0)
    return one(b >> 1, (b & 1u) == 0u);
  }
  float v = one(qb[e * h], upper);
  for (uint32_t o = 1; o < h; ++o) {
    const float x = one(qb[e * h + o], upper);
    v = upper ? __builtin_fminf(v, x) : __builtin_fmaxf(v, x);
  }
  return v;
}

// sp: the wave's 256 G scores in LDS (slot wslot0 + x at sp[x]); sets them to
// the sums of the terms of entries [e_begin, e_end).
//
// The segment bounds of up to 64 entries in the block are read at once, lane t
// holding entry t's (one vector load each). Their postings, entry after entry,
// form one list of `total` postings, which the wave takes 64 at a time: lane l
// takes posting p0 + l, finds its entry by a binary search over the lanes'
// exclusive prefix sums of the segment lengths, and loads the offset and the
// posting's bound, which the compaction stored beside it (so no sketch row is
// gathered from). A wave step thus serves several short segments with
// contiguous loads. The adds of a step then go entry by entry (one round per
// distinct entry among its lanes), so each score takes its terms in entry
// order. A stale block gathers the bounds from the sketch instead; for a slot
// unchanged since the compaction they are the stored values.
template <int R, bool kBf16, bool kH1>
__device__ void score_arrays(const TileArgs &a, uint64_t e_begin, uint64_t e_end, uint32_t wslot0, float *sp) {
  constexpr int G = R / 4;
  constexpr uint32_t kSpan = 256u * G;  // slots of the wave
  constexpr int CH = 8;                 // entries whose loads are in flight together
  const uint32_t lane = threadIdx.x & 63;
  const DevIndex &ix = a.ix;
  const cptr<uint32_t> qj = as_const(a.qd.j);
  const cptr<float> qq = as_const(a.qd.q);
  const cptr<uint32_t> qb = as_const(a.qd.b);
  const uint32_t h = ix.h;
  const uint32_t nblk1 = (ix.cap >> 10) + 1u;
#pragma unroll
  for (int r = 0; r < G; ++r) *(float4 *)(sp + 256 * r + 4 * lane) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  __builtin_amdgcn_wave_barrier();
  // blocks of the wave: G / 4 whole blocks, or (G = 2) half of one
  constexpr uint32_t nb = G >= 4 ? (uint32_t)(G / 4) : 1u;
  for (uint32_t bi = 0; bi < nb; ++bi) {
    const uint32_t blk = (wslot0 >> 10) + bi;
    const uint32_t bslot0 = blk << 10;                           // first slot of the block
    const uint32_t lo = wslot0 > bslot0 ? wslot0 - bslot0 : 0u;  // the wave's part of the block
    const uint32_t hi = min(lo + kSpan, 1024u);
    float *spb = sp + (bslot0 + lo - wslot0);  // spb[o - lo]: block offset o, for lo <= o < hi
    // one term: the bound of the slot at block offset o, into its score
    auto add = [&](uint64_t e, float q, uint32_t o) {
      if (o >= lo && o < hi) {
        const float v = gather_bound<kBf16, kH1>(ix, qb, e, h, q > 0.0f, bslot0 + o);
        spb[o - lo] = __builtin_fmaf(q, v, spb[o - lo]);
      }
    };
    if (as_const(ix.stale)[blk] == 0u) {
      for (uint64_t eb = e_begin; eb < e_end; eb += 64) {
        const uint32_t ne = (uint32_t)min((uint64_t)64, e_end - eb);
        // lane t: entry eb + t's segment start, length and value
        uint32_t vs0 = 0, vn = 0;
        float vq = 0.0f;
        if (lane < ne) {
          const size_t rb = (size_t)a.qd.cr[eb + lane] * nblk1 + blk;
          vs0 = ix.seg[rb];
          vn = ix.seg[rb + 1] - vs0;
          vq = qq[eb + lane];
        }
        // exclusive prefix sum of the lengths over the lanes, and the total
        uint32_t incl = vn;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const uint32_t y = __shfl_up(incl, d, 64);
          if ((int)lane >= d) incl += y;
        }
        const uint32_t excl = incl - vn;
        const uint32_t total = __builtin_amdgcn_readlane(incl, 63);
        // S wave steps at a time: their searches, offset and bound loads are
        // all issued before the first add, so the steps share their latencies
        constexpr int S = R >= 32 ? 4 : 3;  // 4 where the wave spans several blocks
        for (uint32_t p0 = 0; p0 < total; p0 += 64u * S) {
          uint32_t t[S], o[S];
          float q[S], v[S];
#pragma unroll
          for (int k = 0; k < S; ++k) t[k] = 0;
          // entry of posting p: the last lane u with excl(u) <= p (a lane with
          // an empty segment shares the next lane's excl, so u's segment is
          // not empty when p < total)
#pragma unroll
          for (uint32_t d = 32; d >= 1; d >>= 1) {
#pragma unroll
            for (int k = 0; k < S; ++k) {
              const uint32_t ex = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((t[k] + d) << 2), (int)excl);
              if (ex <= p0 + 64u * k + lane) t[k] += d;
            }
          }
#pragma unroll
          for (int k = 0; k < S; ++k) {
            const uint32_t p = p0 + 64u * k + lane;
            const uint32_t s0t = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(t[k] << 2), (int)vs0);
            const uint32_t ext = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(t[k] << 2), (int)excl);
            q[k] = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute((int)(t[k] << 2), __builtin_bit_cast(int, vq)));
            const uint32_t at = s0t + (p - ext);
            o[k] = 0xFFFFu;
            v[k] = 0.0f;
            if (p < total) {
              o[k] = (uint32_t)ix.post[at];
              // the posting's bound, stored beside it: U's side for q > 0, L's for q < 0
              const void *src = q[k] > 0.0f ? ix.pu : ix.pl;
              if constexpr (kBf16)
                v[k] = __builtin_bit_cast(float, (uint32_t)((const uint16_t *)src)[at] << 16);
              else
                v[k] = ((const float *)src)[at];
            }
          }
          // adds, one entry per round, in entry order
#pragma unroll
          for (int k = 0; k < S; ++k) {
            const bool mine = o[k] >= lo && o[k] < hi;
            uint64_t rem = __builtin_amdgcn_ballot_w64(mine);
            while (rem) {
              const uint32_t tf = __builtin_amdgcn_readlane(t[k], (uint32_t)__builtin_ctzll(rem));
              const uint64_t grp = __builtin_amdgcn_ballot_w64(t[k] == tf) & rem;
              if (mine && t[k] == tf) spb[o[k] - lo] = __builtin_fmaf(q[k], v[k], spb[o[k] - lo]);
              __builtin_amdgcn_wave_barrier();
              rem &= ~grp;
            }
          }
        }
      }
    } else {
      // stale block: the same terms from the posting bitmaps; lane l owns
      // block offsets 256g + 4l + i, at bit 4g + i of its 16-bit chunk. CH
      // entries at a time: their bits, then the bound of each lane's first
      // listed slot of every entry, are requested together; the adds go entry
      // by entry, a lane's further slots of an entry right after its first
      const uint16_t *bw = (const uint16_t *)(ix.bits + ((size_t)blk << 4)) + lane;  // row j: bw[j * 4W]
      for (uint64_t e = e_begin; e < e_end; e += CH) {
        uint32_t bits[CH], o1[CH];
        float qv[CH], v1[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const bool in = e + k < e_end;
          const uint64_t ek = in ? e + k : e;
          qv[k] = qq[ek];
          bits[k] = in ? (uint32_t)bw[(size_t)qj[ek] * ix.W * 4u] : 0u;
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const uint32_t x = (uint32_t)__builtin_ctz(bits[k] | 0x10000u);
          o1[k] = bits[k] ? 256u * (x >> 2) + 4u * lane + (x & 3u) : 0xFFFFu;
          const bool mine = o1[k] >= lo && o1[k] < hi;
          v1[k] = mine ? gather_bound<kBf16, kH1>(ix, qb, e + k, h, qv[k] > 0.0f, bslot0 + o1[k]) : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          if (o1[k] >= lo && o1[k] < hi) spb[o1[k] - lo] = __builtin_fmaf(qv[k], v1[k], spb[o1[k] - lo]);
          uint32_t rest = bits[k] & (bits[k] - 1u);
          while (rest) {
            const uint32_t x = (uint32_t)__builtin_ctz(rest);
            rest &= rest - 1u;
            add(e + k, qv[k], 256u * (x >> 2) + 4u * lane + (x & 3u));
          }
          __builtin_amdgcn_wave_barrier();
        }
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// acc += the wave's LDS sums (one add per slot)
template <int R>
__device__ __forceinline__ void fold_arrays(const float *sp, float (&acc)[R]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < R / 4; ++r) {
    const float4 x = *(const float4 *)(sp + 256 * r + 4 * lane);
    acc[4 * r + 0] += x.x;
    acc[4 * r + 1] += x.y;
    acc[4 * r + 2] += x.z;
    acc[4 * r + 3] += x.w;
  }
}

template <int R, bool kBf16>
__device__ void tile_body(const TileArgs &a, uint32_t q, uint32_t t, SelShared &sh, float *sp) {
  constexpr int G = R / 4;  // 256-slot groups per wave
  using LB = typename LaneBits<G>::type;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t wslot0 = t * (uint32_t)(kBlock * R) + (uint32_t)wave * 256u * G;
  const DevIndex &ix = a.ix;

  if (as_const(a.qd.status)[q] != 0u) {  // malformed query: no candidates
    if (threadIdx.x == 0) a.cand_cnt[(size_t)q * a.tiles + t] = 0;
    return;
  }

  // ---------------- scoring (Alg. 6) ----------------
  // For each group the lane loads its 4 slots' bounds with one 16-byte load
  // (out of range, so zeros and no memory traffic, when none of them is on the
  // list) and adds q_j * bound for the slots whose bit is set; absent slots add
  // (+0) * bound, an exact no-op.
  float acc[R];
#pragma unroll
  for (int x = 0; x < R; ++x) acc[x] = 0.0f;

  const uint64_t e0 = as_const(a.qd.qptr)[q] - a.qd.ebase;
  const uint32_t ne = as_const(a.qd.cnt)[q];
  const uint32_t nd = as_const(a.qd.nd)[q];  // entries scored from bitmaps; the rest from arrays
  const uint32_t h = ix.h;
  const cptr<uint32_t> qj = as_const(a.qd.j);
  const cptr<float> qq = as_const(a.qd.q);
  const cptr<uint32_t> qb = as_const(a.qd.b);
  // Two coordinates at a time: their loads are issued together, so one memory
  // round trip serves both; the adds still go in coordinate order, so every
  // document's sum is the same as one at a time. A second coordinate past the
  // end of the list has no bits and adds nothing.
  auto score_two = [&](uint32_t c, LB ba, uint32_t c2, LB bb) {
    const float qa = qq[e0 + c], qbv = qq[e0 + c2];
    const uint32_t qab = __builtin_bit_cast(uint32_t, qa), qbb = __builtin_bit_cast(uint32_t, qbv);
    const __amdgpu_buffer_rsrc_t ra = row_rsrc<kBf16, G>(ix, qa > 0.0f, qb[e0 + c] >> 1, wslot0);
    const __amdgpu_buffer_rsrc_t rb = row_rsrc<kBf16, G>(ix, qbv > 0.0f, qb[e0 + c2] >> 1, wslot0);
#pragma unroll
    for (int r = 0; r < G; ++r) {
      const int lo = r * Elem<kBf16>::kGroup + lane * Elem<kBf16>::kLane;
      const int offa = group_bits(ba, r) ? lo : kOob;
      const int offb = group_bits(bb, r) ? lo : kOob;
      float va[4], vb[4];
      load4<kBf16>(ra, offa, va);
      load4<kBf16>(rb, offb, vb);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float x = __builtin_fmaf(masked_q(ba, 4 * r + i, qab), va[i], acc[4 * r + i]);
        acc[4 * r + i] = __builtin_fmaf(masked_q(bb, 4 * r + i, qbb), vb[i], x);
      }
    }
  };
  // h > 1: least upper bound (q > 0) or greatest lower bound over the h rows;
  // unused mappings repeat row 0, which leaves the min / max unchanged (four
  // loads always: skipping them by h was slower, 18.9 against 13.6 ms per
  // 1,024-query step at h = 2)
  auto score_multi = [&](uint32_t c, LB bw) {
    const float qv = qq[e0 + c];
    const uint32_t qbits = __builtin_bit_cast(uint32_t, qv);
    const bool upper = qv > 0.0f;
    __amdgpu_buffer_rsrc_t rs[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      const uint32_t oo = (uint32_t)o < h ? (uint32_t)o : 0u;
      rs[o] = row_rsrc<kBf16, G>(ix, upper, qb[(e0 + c) * h + oo], wslot0);
    }
#pragma unroll
    for (int r = 0; r < G; ++r) {
      const int off = group_bits(bw, r) ? r * Elem<kBf16>::kGroup + lane * Elem<kBf16>::kLane : kOob;
      float v[4];
      load4<kBf16>(rs[0], off, v);
#pragma unroll
      for (int o = 1; o < 4; ++o) {
        float x[4];
        load4<kBf16>(rs[o], off, x);
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = upper ? __builtin_fminf(v[i], x[i]) : __builtin_fmaxf(v[i], x[i]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[4 * r + i] = __builtin_fmaf(masked_q(bw, 4 * r + i, qbits), v[i], acc[4 * r + i]);
    }
  };
  // The posting bits of kChunk coordinates are fetched together (one 2-byte
  // load per lane and 1,024-slot block each), so their memory latency is paid
  // once per chunk rather than once per coordinate.
  LB cb[kChunk];
  for (uint32_t c = 0; c < nd;) {
    if (c % kChunk == 0) {
#pragma unroll
      for (int k = 0; k < kChunk; ++k) cb[k] = lane_bits<G>(ix, qj[e0 + min(c + (uint32_t)k, nd - 1u)], wslot0, lane);
    }
    if (h == 1) {
      const bool two = c + 1u < nd;
      score_two(c, cb[0], two ? c + 1u : c, two ? cb[1] : (LB)0);
      c += 2;
#pragma unroll
      for (int k = 0; k + 2 < kChunk; ++k) cb[k] = cb[k + 2];
    } else {
      score_multi(c, cb[0]);
      c += 1;
#pragma unroll
      for (int k = 0; k + 1 < kChunk; ++k) cb[k] = cb[k + 1];
    }
  }
  if (nd < ne) {
    score_arrays<R, kBf16, false>(a, e0 + nd, e0 + ne, wslot0, sp + wave * 64 * R);
    fold_arrays<R>(sp + wave * 64 * R, acc);
  }

  finish<R>(a, q, t, acc, sh);
}

// Selection and emission of one (query, tile) item from its scores.
template <int R>
__device__ void finish(const TileArgs &a, uint32_t q, uint32_t t, const float (&acc)[R], SelShared &sh) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t wslot0 = t * (uint32_t)(kBlock * R) + (uint32_t)wave * 64u * R;
  const uint32_t wword0 = wslot0 >> 6;
  const DevIndex &ix = a.ix;
  const uint32_t kq = a.kq ? as_const(a.kq)[q] : a.kmax;
  uint32_t *ccnt = a.cand_cnt + (size_t)q * a.tiles + t;
  uint64_t *cout = a.cand + ((size_t)q * a.tiles + t) * a.kmax;
  // ---------------- selection keys ----------------
  uint32_t key[R];
  const cptr<uint64_t> lw = as_const(ix.live) + wword0;
  const uint32_t thr0 = __hip_atomic_load(&a.thr[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t thr = __builtin_amdgcn_readfirstlane(thr0);
#pragma unroll
  for (int x = 0; x < R; ++x) {
    const bool lv = __builtin_amdgcn_inverse_ballot_w64(lw[x]);  // word 4r + i <-> register 4r + i
    const float s = acc[x] == 0.0f ? 0.0f : acc[x];  // -0 -> +0
    const uint32_t kk = ord_key(s);
    key[x] = (lv && kk >= thr) ? kk : 0u;
  }
  if (a.qseq) {
    // serving snapshot: a slot changed during the session is seen only if it was
    // inserted before the query and not deleted before it
    const uint32_t tq = as_const(a.qseq)[q];
    const cptr<uint64_t> dw = as_const(a.dirty) + wword0;
#pragma unroll
    for (int x = 0; x < R; ++x) {
      if (key[x] != 0u && __builtin_amdgcn_inverse_ballot_w64(dw[x])) {
        const uint64_t v = __hip_atomic_load(const_cast<uint64_t *>(&a.vis[slot_of<R>(wslot0, x, lane)]),
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t ins = (uint32_t)(v >> 32), del = (uint32_t)v;
        if (!(ins < tq && tq < del)) key[x] = 0u;
      }
    }
  }
  int par = 0;
  uint32_t nvalid;
  {
    uint32_t c = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) c += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(key[r] != 0u));
    nvalid = wg_sum(c, sh, par);
  }

  // Emission rule: mode 0 keeps every valid key; mode 1 keeps key >= T;
  // mode 2 keeps key > T and, among key == T, the ids whose id key >= T2.
  int mode = 0;
  uint32_t T = 0, T2 = 0;
  uint32_t idk[R];
#pragma unroll
  for (int r = 0; r < R; ++r) idk[r] = 0u;
  if (nvalid > kq) {
    bool exact;
    uint32_t need;
    T = select_kth<R>(key, kq, sh, par, exact, need);
    mode = 1;
    if (!exact) {
      uint32_t c = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) c += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(key[r] == T));
      const uint32_t nt = wg_sum(c, sh, par);
      if (nt != need) {
        // ties at the k-th score: keep the `need` lowest ids among them
#pragma unroll
        for (int r = 0; r < R; ++r)
          idk[r] = key[r] == T ? (0xFFFFFFFFu - ix.slot2id[slot_of<R>(wslot0, r, lane)]) : 0u;
        bool ex2;
        uint32_t need2;
        T2 = select_kth<R>(idk, need, sh, par, ex2, need2);
        mode = 2;
      }
    }
  }

  // ---------------- emit candidates ----------------
  if (threadIdx.x == 0) sh.emit = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool e = mode == 0 ? key[r] != 0u
                             : (mode == 1 ? key[r] >= T : (key[r] > T || (key[r] == T && idk[r] >= T2)));
    const uint64_t mask = __builtin_amdgcn_ballot_w64(e);
    if (mask == 0) continue;
    uint32_t basepos = 0;
    if (lane == 0) basepos = atomicAdd(&sh.emit, (uint32_t)__popcll(mask));
    basepos = __builtin_amdgcn_readfirstlane(basepos);
    if (e) {
      const uint32_t pos = basepos + (uint32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
      const uint32_t slot = slot_of<R>(wslot0, r, lane);
      const uint32_t id = ix.slot2id[slot];
      cout[pos] = ((uint64_t)key[r] << 32) | (uint64_t)(0xFFFFFFFFu - id);
      if (a.cand_slot) a.cand_slot[((size_t)q * a.tiles + t) * a.kmax + pos] = slot;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *ccnt = sh.emit;
    if (mode != 0 && T > thr) atomicMax(&a.thr[q], T);
    if (mode != 0 && a.nselect) atomicAdd(a.nselect, 1ull);
  }
}

// Q queries on one tile (h = 1). Each query's scored entries are stored by
// sketch row (k_prep), so the workgroup walks the Q lists together, row by
// row: a row of U (or L) is loaded once for every query that has a coordinate
// in it, and each query adds its terms in its own stored order, the order one
// query alone uses. Scores of the Q queries stay in registers; each then goes
// through the same selection as a single query.
template <int R, bool kBf16, int Q>
__device__ void tile_group(const TileArgs &a, uint32_t grp, uint32_t t, uint32_t nq_eff, SelShared &sh, float *sp) {
  constexpr int G = R / 4;
  static_assert(G <= 4, "grouped tiles cover at most one 1,024-slot block per wave");
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t wslot0 = t * (uint32_t)(kBlock * R) + (uint32_t)wave * 256u * G;
  const DevIndex &ix = a.ix;
  const cptr<uint32_t> qj = as_const(a.qd.j);
  const cptr<float> qq = as_const(a.qd.q);
  const cptr<uint32_t> qb = as_const(a.qd.b);
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  // per query: the cursor into its list and the list's end (32-bit entry
  // positions: the host keeps a grouped batch below 2^32 entries), the sketch
  // row of the entry under the cursor (none past the end) and the posting bits
  // of the next entries, fetched kChunk at a time (cb[i][0] is the cursor's)
  uint32_t qid[Q], row[Q], left[Q], cur[Q], end[Q], aend[Q];
  uint32_t cb[Q][kChunk];
  auto refill = [&](int i) {
    // the chunk's coordinates in one scalar load (the entry array is padded by
    // kChunk entries); entries past the list's end fetch the first entry's
    // bits again and are never used
    uint32_t js[kChunk];
#pragma unroll
    for (int c = 0; c < kChunk; ++c) js[c] = qj[cur[i] + (uint32_t)c];
#pragma unroll
    for (int c = 0; c < kChunk; ++c)
      cb[i][c] = lane_bits<G>(ix, cur[i] + (uint32_t)c < end[i] ? js[c] : js[0], wslot0, lane);
    left[i] = kChunk;
  };
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const uint32_t slot = grp * (uint32_t)Q + (uint32_t)i;
    qid[i] = kNone;
    cur[i] = end[i] = aend[i] = 0;
    left[i] = 0;
    if (slot < nq_eff) {
      const uint32_t q = a.qlist ? as_const(a.qlist)[slot] : slot;
      qid[i] = q;
      if (as_const(a.qd.status)[q] == 0u) {
        cur[i] = (uint32_t)(as_const(a.qd.qptr)[q] - a.qd.ebase);
        end[i] = cur[i] + as_const(a.qd.nd)[q];     // bitmap entries, walked by row below
        aend[i] = cur[i] + as_const(a.qd.cnt)[q];   // array entries [end, aend) after them
      }
    }
    row[i] = kNone;
    if (cur[i] < end[i]) {
      row[i] = qb[cur[i]];
      refill(i);
    }
  }
  float acc[Q][R];
#pragma unroll
  for (int i = 0; i < Q; ++i)
#pragma unroll
    for (int x = 0; x < R; ++x) acc[i][x] = 0.0f;
  for (;;) {
    uint32_t rmin = kNone;
#pragma unroll
    for (int i = 0; i < Q; ++i) rmin = min(rmin, row[i]);
    if (rmin == kNone) break;
    // the row's bounds for the wave's slots, read densely: one 16-byte (8-byte)
    // load per lane and group
    const char *rp = (const char *)((rmin & 1u) == 0u ? ix.U : ix.L) +
                     ((size_t)(rmin >> 1) * ix.cap + wslot0) * Elem<kBf16>::kBytes;
    float v[G][4];
#pragma unroll
    for (int r = 0; r < G; ++r) {
      if constexpr (kBf16) {
        const uint2 x = ((const uint2 *)rp)[r * 64 + lane];
        v[r][0] = __builtin_bit_cast(float, x.x << 16);
        v[r][1] = __builtin_bit_cast(float, x.x & 0xFFFF0000u);
        v[r][2] = __builtin_bit_cast(float, x.y << 16);
        v[r][3] = __builtin_bit_cast(float, x.y & 0xFFFF0000u);
      } else {
        const float4 x = ((const float4 *)rp)[r * 64 + lane];
        v[r][0] = x.x;
        v[r][1] = x.y;
        v[r][2] = x.z;
        v[r][3] = x.w;
      }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      while (row[i] == rmin) {
        const uint32_t qbits = __builtin_bit_cast(uint32_t, qq[cur[i]]);
        const uint32_t bw = cb[i][0];
#pragma unroll
        for (int r = 0; r < G; ++r)
#pragma unroll
          for (int k = 0; k < 4; ++k)
            acc[i][4 * r + k] = __builtin_fmaf(masked_q(bw, 4 * r + k, qbits), v[r][k], acc[i][4 * r + k]);
#pragma unroll
        for (int c = 0; c + 1 < kChunk; ++c) cb[i][c] = cb[i][c + 1];
        ++cur[i];
        row[i] = kNone;
        if (cur[i] < end[i]) {
          row[i] = qb[cur[i]];
          if (--left[i] == 0) refill(i);
        }
      }
    }
  }
  // each query's array entries (the cursor stopped at its bitmap entries'
  // end), one query at a time through the wave's LDS scores
#pragma unroll 1
  for (int i = 0; i < Q; ++i) {
    uint32_t b = cur[0], en = aend[0];
#pragma unroll
    for (int ii = 1; ii < Q; ++ii)
      if (ii == i) {
        b = cur[ii];
        en = aend[ii];
      }
    if (b < en) {
      score_arrays<R, kBf16, true>(a, b, en, wslot0, sp + wave * 64 * R);
#pragma unroll
      for (int ii = 0; ii < Q; ++ii)
        if (ii == i) fold_arrays<R>(sp + wave * 64 * R, acc[ii]);
    }
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (qid[i] == kNone) continue;
    if (as_const(a.qd.status)[qid[i]] != 0u) {  // malformed query: no candidates
      if (threadIdx.x == 0) a.cand_cnt[(size_t)qid[i] * a.tiles + t] = 0;
      continue;
    }
    finish<R>(a, qid[i], t, acc[i], sh);
  }
}

// One query alone (the plain form): its 256 R-slot tiles fill only part of the
// device, so the time of a tile is the length of its chain of memory round
// trips, not throughput. This body keeps a whole chunk in flight at once: the
// bounds of the chunk's PC entries are loaded together, with the posting bits
// of the next chunk, and then applied in entry order (the same terms, added in
// the same order as tile_body). h = 1 only; registers are plentiful here.
template <int R, bool kBf16>
__device__ void tile_body_latency(const TileArgs &a, uint32_t q, uint32_t t, SelShared &sh, float *sp) {
  constexpr int G = R / 4;
  constexpr int PC = 4;  // entries per chunk
  using LB = typename LaneBits<G>::type;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t wslot0 = t * (uint32_t)(kBlock * R) + (uint32_t)wave * 256u * G;
  const DevIndex &ix = a.ix;
  if (as_const(a.qd.status)[q] != 0u) {  // malformed query: no candidates
    if (threadIdx.x == 0) a.cand_cnt[(size_t)q * a.tiles + t] = 0;
    return;
  }
  float acc[R];
#pragma unroll
  for (int x = 0; x < R; ++x) acc[x] = 0.0f;
  const uint64_t e0 = as_const(a.qd.qptr)[q] - a.qd.ebase;
  const uint32_t ne = as_const(a.qd.cnt)[q];
  const uint32_t nd = as_const(a.qd.nd)[q];  // entries scored from bitmaps; the rest from arrays
  const cptr<uint32_t> qj = as_const(a.qd.j);
  const cptr<float> qq = as_const(a.qd.q);
  const cptr<uint32_t> qb = as_const(a.qd.b);
  LB cb[PC];
#pragma unroll
  for (int k = 0; k < PC; ++k) cb[k] = nd ? lane_bits<G>(ix, qj[e0 + min((uint32_t)k, nd - 1u)], wslot0, lane) : (LB)0;
  for (uint32_t c0 = 0; c0 < nd; c0 += PC) {
    LB nb[PC];
    const bool more = c0 + PC < nd;
#pragma unroll
    for (int k = 0; k < PC; ++k)
      nb[k] = more ? lane_bits<G>(ix, qj[e0 + min(c0 + PC + (uint32_t)k, nd - 1u)], wslot0, lane) : (LB)0;
    float v[PC][G][4];
    uint32_t qbits[PC];
#pragma unroll
    for (int k = 0; k < PC; ++k) {
      const uint32_t c = min(c0 + (uint32_t)k, nd - 1u);  // past the end: a repeat with no bits
      const LB bk = c0 + (uint32_t)k < nd ? cb[k] : (LB)0;
      cb[k] = bk;
      const float qv = qq[e0 + c];
      qbits[k] = __builtin_bit_cast(uint32_t, qv);
      const __amdgpu_buffer_rsrc_t rs = row_rsrc<kBf16, G>(ix, qv > 0.0f, qb[e0 + c] >> 1, wslot0);
#pragma unroll
      for (int r = 0; r < G; ++r)
        load4<kBf16>(rs, group_bits(bk, r) ? r * Elem<kBf16>::kGroup + lane * Elem<kBf16>::kLane : kOob, v[k][r]);
    }
    // every load of the chunk is issued before the first add (the scheduler
    // would otherwise trade this overlap for registers)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < PC; ++k)
#pragma unroll
      for (int r = 0; r < G; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          acc[4 * r + i] = __builtin_fmaf(masked_q(cb[k], 4 * r + i, qbits[k]), v[k][r][i], acc[4 * r + i]);
#pragma unroll
    for (int k = 0; k < PC; ++k) cb[k] = nb[k];
  }
  if (nd < ne) {
    score_arrays<R, kBf16, true>(a, e0 + nd, e0 + ne, wslot0, sp + wave * 64 * R);
    fold_arrays<R>(sp + wave * 64 * R, acc);
  }
  finish<R>(a, q, t, acc, sh);
}

template <int R, bool kBf16>
__device__ __forceinline__ void one_item(const TileArgs &a, SelShared &sh, float *sp) {
  uint32_t q = a.q0 + blockIdx.y;
  if (a.qlist) {
    if (q >= *as_const(a.nlist)) return;
    q = as_const(a.qlist)[q];
  }
  tile_body<R, kBf16>(a, q, blockIdx.x, sh, sp);
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_tiles(TileArgs a) {
  __shared__ SelShared sh;
  __shared__ __align__(16) float sp[kWaves * 64 * R];
  one_item<R, false>(a, sh, sp);
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_tiles_bf16(TileArgs a) {
  __shared__ SelShared sh;
  __shared__ __align__(16) float sp[kWaves * 64 * R];
  one_item<R, true>(a, sh, sp);
}

// the plain form: query a.q0 alone, one workgroup per tile (R = 64 keeps the
// throughput body: a chunk of its bounds would not fit the registers)
template <int R, bool kBf16>
__global__ __launch_bounds__(kBlock) void k_tiles_latency(TileArgs a) {
  __shared__ SelShared sh;
  __shared__ __align__(16) float sp[kWaves * 64 * R];
  if (R <= 32 && a.ix.h == 1) tile_body_latency<R, kBf16>(a, a.q0, blockIdx.x, sh, sp);
  else tile_body<R, kBf16>(a, a.q0, blockIdx.x, sh, sp);
}

// Persistent form: a fixed grid pulls (query, tile) items from per-XCD queues.
// Workgroups are dispatched round-robin over the XCDs, so workgroup b runs on
// XCD b % xcds; queue x holds the tiles t with t % xcds == x, tile-major, so
// the workgroups of one XCD work through one tile's bitmap and sketch slices
// for many queries while those slices sit in that XCD's L2. A drained queue
// steals from the others; every workgroup exits once all queues are drained.
template <int R, bool kBf16>
__device__ __forceinline__ void persistent_items(const TileArgs &a, SelShared &sh, float *sp) {
  const uint32_t X = a.xcds;
  const uint32_t home = blockIdx.x % X;
  const uint32_t nq = a.qlist ? *as_const(a.nlist) : a.nq;
  if (nq == 0) return;  // an empty query list: no queue traffic at all
  for (uint32_t step = 0; step < X; ++step) {
    const uint32_t x = (home + step) % X;
    const uint32_t tiles_x = a.tiles > x ? (a.tiles - x + X - 1) / X : 0u;
    const uint32_t items = tiles_x * nq;
    for (;;) {
      __syncthreads();
      if (threadIdx.x == 0) sh.item = atomicAdd(&a.queue[x], 1u);
      __syncthreads();
      const uint32_t it = sh.item;
      if (it >= items) break;
      const uint32_t t = x + X * (it / nq);
      const uint32_t q = a.qlist ? as_const(a.qlist)[it % nq] : it % nq;
      tile_body<R, kBf16>(a, q, t, sh, sp);
    }
  }
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_tiles_persistent(TileArgs a) {
  __shared__ SelShared sh;
  __shared__ __align__(16) float sp[kWaves * 64 * R];
  persistent_items<R, false>(a, sh, sp);
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_tiles_persistent_bf16(TileArgs a) {
  __shared__ SelShared sh;
  __shared__ __align__(16) float sp[kWaves * 64 * R];
  persistent_items<R, true>(a, sh, sp);
}

// Grouped forms: items are (query group, tile); group g holds the queries
// g * Q .. g * Q + Q - 1 of the batch (or of the query list).
template <int R, bool kBf16, int Q>
__global__ __launch_bounds__(kBlock) void k_tiles_grouped(TileArgs a) {
  __shared__ SelShared sh;
  __shared__ __align__(16) float sp[kWaves * 64 * R];
  const uint32_t nq = a.qlist ? *as_const(a.nlist) : a.nq;
  const uint32_t grp = a.q0 + blockIdx.y;
  if (grp * (uint32_t)Q >= nq) return;
  tile_group<R, kBf16, Q>(a, grp, blockIdx.x, nq, sh, sp);
}

// Waves per SIMD the persistent grouped kernel is built for: left to the
// compiler. (Before the array containers, R = 16 with two queries was built
// for 8 waves at 64 VGPRs, 2.4% faster than 7; with the array path that cap
// spills in the scoring loop, and 6 waves are 7% faster than 8.)
template <int R, bool kBf16, int Q>
struct GroupedWaves {
  static constexpr int value = 1;
};

template <int R, bool kBf16, int Q>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(GroupedWaves<R, kBf16, Q>::value)))
void k_tiles_persistent_grouped(TileArgs a) {
  __shared__ SelShared sh;
  __shared__ __align__(16) float sp[kWaves * 64 * R];
  const uint32_t X = a.xcds;
  const uint32_t home = blockIdx.x % X;
  const uint32_t nq = a.qlist ? *as_const(a.nlist) : a.nq;
  if (nq == 0) return;  // an empty query list: no queue traffic at all
  const uint32_t ng = (nq + Q - 1) / Q;
  for (uint32_t step = 0; step < X; ++step) {
    const uint32_t x = (home + step) % X;
    const uint32_t tiles_x = a.tiles > x ? (a.tiles - x + X - 1) / X : 0u;
    const uint32_t items = tiles_x * ng;
    for (;;) {
      __syncthreads();
      if (threadIdx.x == 0) sh.item = atomicAdd(&a.queue[x], 1u);
      __syncthreads();
      const uint32_t it = sh.item;
      if (it >= items) break;
      tile_group<R, kBf16, Q>(a, it % ng, x + X * (it / ng), nq, sh, sp);
    }
  }
}

template <int R, int Q>
static void launch_grouped_rq(const TileArgs &a, bool bf, bool persistent, uint32_t grid, uint32_t ng_launch,
                              hipStream_t s) {
  if (persistent) {
    if (bf) hipLaunchKernelGGL((k_tiles_persistent_grouped<R, true, Q>), dim3(grid), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_tiles_persistent_grouped<R, false, Q>), dim3(grid), dim3(kBlock), 0, s, a);
  } else {
    if (bf) hipLaunchKernelGGL((k_tiles_grouped<R, true, Q>), dim3(a.tiles, ng_launch), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_tiles_grouped<R, false, Q>), dim3(a.tiles, ng_launch), dim3(kBlock), 0, s, a);
  }
}

hipError_t launch_tiles_grouped(const TileArgs &a, int R, int Q, bool persistent, uint32_t grid, uint32_t ng_launch,
                                hipStream_t s) {
  if (a.ix.h != 1) return hipErrorInvalidValue;
  const bool bf = (a.ix.flags & kSketchBf16) != 0;
  if (R == 16 && Q == 2) launch_grouped_rq<16, 2>(a, bf, persistent, grid, ng_launch, s);
  else if (R == 16 && Q == 3) launch_grouped_rq<16, 3>(a, bf, persistent, grid, ng_launch, s);
  else if (R == 8 && Q == 2) launch_grouped_rq<8, 2>(a, bf, persistent, grid, ng_launch, s);
  else if (R == 8 && Q == 4) launch_grouped_rq<8, 4>(a, bf, persistent, grid, ng_launch, s);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_tiles(const TileArgs &a, int R, uint32_t nq_launch, hipStream_t s) {
  dim3 grid(a.tiles, nq_launch);
  const bool bf = (a.ix.flags & kSketchBf16) != 0;
  switch (R) {
    case 16: hipLaunchKernelGGL(bf ? k_tiles_bf16<16> : k_tiles<16>, grid, dim3(kBlock), 0, s, a); break;
    case 32: hipLaunchKernelGGL(bf ? k_tiles_bf16<32> : k_tiles<32>, grid, dim3(kBlock), 0, s, a); break;
    case 64: hipLaunchKernelGGL(bf ? k_tiles_bf16<64> : k_tiles<64>, grid, dim3(kBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int R>
static void launch_latency_r(const TileArgs &a, bool bf, hipStream_t s) {
  if (bf) hipLaunchKernelGGL((k_tiles_latency<R, true>), dim3(a.tiles), dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL((k_tiles_latency<R, false>), dim3(a.tiles), dim3(kBlock), 0, s, a);
}

hipError_t launch_tiles_latency(const TileArgs &a, int R, hipStream_t s) {
  const bool bf = (a.ix.flags & kSketchBf16) != 0;
  switch (R) {
    case 16: launch_latency_r<16>(a, bf, s); break;
    case 32: launch_latency_r<32>(a, bf, s); break;
    case 64: launch_latency_r<64>(a, bf, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_tiles_persistent(const TileArgs &a, int R, uint32_t grid, hipStream_t s) {
  const bool bf = (a.ix.flags & kSketchBf16) != 0;
  switch (R) {
    case 16:
      hipLaunchKernelGGL(bf ? k_tiles_persistent_bf16<16> : k_tiles_persistent<16>, dim3(grid), dim3(kBlock), 0, s, a);
      break;
    case 32:
      hipLaunchKernelGGL(bf ? k_tiles_persistent_bf16<32> : k_tiles_persistent<32>, dim3(grid), dim3(kBlock), 0, s, a);
      break;
    case 64:
      hipLaunchKernelGGL(bf ? k_tiles_persistent_bf16<64> : k_tiles_persistent<64>, dim3(grid), dim3(kBlock), 0, s, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace snn
