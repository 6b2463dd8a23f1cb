// Ranking with k' >= k (Alg. 7), first half: the k' candidates of each query,
// chosen by their Sinnamon scores, are fetched from the forward store and
// scored with the exact inner product of Eq. 2. The k best by exact score
// (ties by the lower external id) are then picked by the select kernel.
//
// One workgroup of 8 waves per (query, share of its candidates); a small batch
// spreads each query's candidates over several workgroups. The query's
// non-zeros (all of them, whatever the anytime budget of the scoring) go into
// an open-addressing hash table in LDS (coordinate -> value) of 4-slot
// buckets: one probe reads the 4 coordinates of a bucket at once (16 bytes)
// and, on a match, the value next to them. The table is at most 1/8 full where
// the space allows (at most 1/2 always), so a document entry, present in the
// query or not, nearly always costs one probe whatever the dimensionality.
//
// Each wave takes 64 candidates at a time: lane l fetches the slot,
// forward-store offset and length of candidate l, and the wave sorts the 64 by
// length. It then scores them 8 at a time in that order, so the 8 have similar
// lengths: its 64 lanes read 64 consecutive (coordinate, value) entries of each
// of the 8 documents per step (coalesced 512-byte reads, all 8 in flight) and
// sum q_j * x_j in FP32. A fixed tree of cross-lane adds (DPP moves within
// rows, then the four row sums) finishes each sum, so the result does not
// depend on timing. Each exact score leaves as a 64-bit key
// ord(score) << 32 | (0xFFFFFFFF - id).
#include <algorithm>

#include "snn_device.h"

namespace snn {

constexpr int kRrWaves = 8;
constexpr int kRrStep = 8;  // candidates a wave scores at once
constexpr int kRrLk = 4;    // hash lookups a lane has in flight
constexpr int kRrBlock = 64 * kRrWaves;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;  // no coordinate reaches 2^31

// lane `src` (the same in every lane) of v
__device__ __forceinline__ uint32_t lane_u32(uint32_t v, int src) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, src);
}

template <int kCtrl>
__device__ __forceinline__ float dpp_add(float x) {
  return x + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kCtrl, 0xF, 0xF, false));
}

// Sum of the wave's 64 values, in a fixed order and the same in every lane:
// pairs (lanes 2i, 2i + 1), then quads, then halves of 8 lanes and of 16 by
// DPP moves within each row of 16 lanes, then the four rows' sums as
// (row 0 + row 1) + (row 2 + row 3). Each step adds two equal-sized partial
// sums, so every lane of a group holds the same bits.
__device__ __forceinline__ float wave_sum(float x) {
  x = dpp_add<0xB1>(x);   // quad_perm [1, 0, 3, 2]
  x = dpp_add<0x4E>(x);   // quad_perm [2, 3, 0, 1]
  x = dpp_add<0x141>(x);  // row_half_mirror: the other quad of the 8
  x = dpp_add<0x140>(x);  // row_mirror: the other 8 of the row
  const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 0));
  const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 16));
  const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 32));
  const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 48));
  return (r0 + r1) + (r2 + r3);
}

__global__ __launch_bounds__(kRrBlock) void k_rerank(RerankArgs a) {
  extern __shared__ uint4 lds4[];
  uint32_t *lds = (uint32_t *)lds4;
  // bucket b: coordinates at lds[8b .. 8b + 3], their values at lds[8b + 4 .. 8b + 7];
  // slot s is entry s & 3 of bucket s >> 2, and probing runs through the slots in order
  const uint32_t cap = a.hash_cap, mask = cap - 1u, bmask = cap / 4u - 1u;
  const uint32_t shift = 32u - (uint32_t)__builtin_ctz(cap / 4u);
  const uint32_t q = a.q0 + blockIdx.x;
  const uint32_t n = a.cand_cnt[q];
  const uint32_t ne = a.qd.status[q] ? 0u : a.nz_full[q];  // the exact score uses every coordinate
  const uint64_t e0 = a.qd.qptr[q] - a.qd.ebase;
  const int tid = threadIdx.x;
  if (2u * ne > cap) return;  // the launcher sizes the table for every query; never taken
  // this workgroup's share [lo, hi) of the query's candidates
  const uint32_t share = ((n + gridDim.y - 1) / gridDim.y + 63u) & ~63u;
  const uint32_t lo = blockIdx.y * share, hi = min(n, lo + share);
  if (lo >= hi) return;

  // the query as a hash table: linear probing from the first slot of the
  // coordinate's bucket. Nothing is removed, so every slot from there to a
  // stored coordinate is taken, and a probe can stop at the first bucket with
  // a free slot.
  for (uint32_t i = tid; i < cap / 4u; i += kRrBlock) lds4[2u * i] = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
  __syncthreads();
  for (uint32_t i = tid; i < ne; i += kRrBlock) {
    const uint32_t j = a.qd.j[e0 + i];
    const float v = a.qd.q[e0 + i];
    uint32_t h = ((j * 0x9E3779B1u) >> shift) * 4u;
    for (;;) {
      const uint32_t at = 8u * (h >> 2) + (h & 3u);
      const uint32_t prev = atomicCAS(&lds[at], kEmpty, j);
      if (prev == kEmpty) {
        lds[at + 4u] = __builtin_bit_cast(uint32_t, v);
        break;
      }
      if (prev == j) break;  // coordinates of a valid query are distinct
      h = (h + 1u) & mask;
    }
  }
  __syncthreads();
  // bit i set where slot i of the bucket holds j
  auto match = [](const uint4 &kj, uint32_t j) {
    return (uint32_t)(kj.x == j) | (uint32_t)(kj.y == j) << 1 | (uint32_t)(kj.z == j) << 2 |
           (uint32_t)(kj.w == j) << 3;
  };
  // the value of coordinate j in the query, 0 where absent: kRrLk lookups at
  // a time, their first buckets' reads in flight together; slots fill in
  // order, so a bucket with a free slot ends a probe, and the walk on to the
  // next bucket is rare
  auto lookup = [&](const uint32_t *j, float *out) {
    uint32_t b[kRrLk], m[kRrLk];
    uint4 kj[kRrLk];
#pragma unroll
    for (int u = 0; u < kRrLk; ++u) {
      b[u] = (j[u] * 0x9E3779B1u) >> shift;
      kj[u] = lds4[2u * b[u]];
    }
#pragma unroll
    for (int u = 0; u < kRrLk; ++u) {
      m[u] = match(kj[u], j[u]);
      uint32_t w = kj[u].w;
      while (m[u] == 0u && w != kEmpty) {
        b[u] = (b[u] + 1u) & bmask;
        const uint4 k2 = lds4[2u * b[u]];
        m[u] = match(k2, j[u]);
        w = k2.w;
      }
    }
#pragma unroll
    for (int u = 0; u < kRrLk; ++u) {
      const float v = __builtin_bit_cast(float, lds[8u * b[u] + 4u + (m[u] ? (uint32_t)__builtin_ctz(m[u]) : 0u)]);
      out[u] = m[u] ? v : 0.0f;
    }
  };

  // exact inner products of this workgroup's share of the candidates
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform, so the per-step values below stay scalar
  const size_t cbase = (size_t)q * a.kprime;
  for (uint32_t base = lo + (uint32_t)wave * 64u; base < hi; base += (uint32_t)kRrBlock) {
    const uint32_t c = base + (uint32_t)lane;
    uint32_t id = 0, len = 0;
    uint64_t off = 0;
    if (c < hi) {
      const uint32_t slot = a.cand_slots[cbase + c];
      id = a.cand_ids[cbase + c];
      off = a.fw.off[slot];
      len = a.fw.len[slot];
    }
    const uint32_t here = min(64u, hi - base);
    // the chunk's candidates in order of length (a bitonic sort of
    // length << 6 | lane over the wave, the lanes past the end last), so the
    // kRrStep scored together have similar lengths and few lanes idle
    uint32_t skey = c < hi ? (min(len, (1u << 26) - 1u) << 6) | (uint32_t)lane : 0xFFFFFFFFu;
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        const uint32_t other = (uint32_t)__shfl_xor((int)skey, j, 64);
        const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
        skey = keep_min ? min(skey, other) : max(skey, other);
      }
    }
    // kRrStep candidates at a time, so their entries' loads are in flight
    // together; each candidate's sum is formed exactly as alone (lane l adds
    // entries l, l + 64, ... in order, then the tree of cross-lane adds)
    for (uint32_t t0 = 0; t0 < here; t0 += kRrStep) {
      uint64_t o[kRrStep];
      uint32_t ln[kRrStep], src[kRrStep];
      float acc[kRrStep];
      uint32_t lmax = 0;
#pragma unroll
      for (int u = 0; u < kRrStep; ++u) {
        const uint32_t t = t0 + (uint32_t)u;
        src[u] = t < here ? lane_u32(skey, (int)t) & 63u : 64u;
        const int sl = (int)(src[u] & 63u);
        o[u] = ((uint64_t)lane_u32((uint32_t)(off >> 32), sl) << 32) | lane_u32((uint32_t)off, sl);
        ln[u] = t < here ? lane_u32(len, sl) : 0u;
        lmax = max(lmax, ln[u]);
        acc[u] = 0.0f;
      }
      for (uint32_t eb = 0; eb < lmax; eb += 64u) {
        const uint32_t e = eb + (uint32_t)lane;
        uint32_t ej[kRrStep];
        float ev[kRrStep], qv[kRrStep] = {};
#pragma unroll
        for (int u = 0; u < kRrStep; ++u) {
          const uint2 en = e < ln[u] ? a.fw.ent[o[u] + e] : make_uint2(0u, 0u);
          ej[u] = en.x;
          ev[u] = __builtin_bit_cast(float, en.y);
        }
#pragma unroll
        for (int u0 = 0; u0 < kRrStep; u0 += kRrLk) {
          uint32_t gmax = 0;
#pragma unroll
          for (int u = u0; u < u0 + kRrLk; ++u) gmax = max(gmax, ln[u]);
          if (eb < gmax) lookup(ej + u0, qv + u0);  // else every lane of the group is past its end
        }
#pragma unroll
        for (int u = 0; u < kRrStep; ++u)
          if (e < ln[u]) acc[u] = __builtin_fmaf(qv[u], ev[u], acc[u]);
      }
#pragma unroll
      for (int u = 0; u < kRrStep; ++u) {
        acc[u] = wave_sum(acc[u]);
        if ((uint32_t)lane == src[u]) {
          const float s = acc[u] == 0.0f ? 0.0f : acc[u];  // -0 -> +0
          a.keys[cbase + c] = ((uint64_t)ord_key(s) << 32) | (uint64_t)(0xFFFFFFFFu - id);
        }
      }
    }
  }
}

hipError_t rerank_init() {
  // the largest table: 8,192 slots, 64 KB of LDS
  return hipFuncSetAttribute((const void *)k_rerank, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
}

hipError_t launch_rerank(const RerankArgs &a, uint32_t nq, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  if (a.kprime == 0 || a.kprime > kMaxKPrime || a.hash_cap < 64 || a.hash_cap > 8192 ||
      (a.hash_cap & (a.hash_cap - 1)) || !a.fw.ent || !a.keys)
    return hipErrorInvalidValue;
  const size_t lds = (size_t)a.hash_cap * 8;
  // workgroups per query: about 2,048 in all for batches below 2,048 queries
  // (more than the device holds at once, in shares small enough that the last
  // workgroups to start end soon after the rest), and at least 128 candidates
  // each (one query of k' = 1,000: 7 workgroups; of k' = 20,000: 156)
  const uint32_t by_grid = std::max<uint32_t>(1u, 2048u / nq);
  const uint32_t by_work = std::max<uint32_t>(1u, a.kprime / 128u);
  const uint32_t splits = std::min<uint32_t>(256u, std::min(by_grid, by_work));
  for (uint32_t c0 = 0; c0 < nq; c0 += 65535u) {
    RerankArgs b = a;
    b.q0 = a.q0 + c0;
    hipLaunchKernelGGL(k_rerank, dim3(std::min<uint32_t>(65535u, nq - c0), splits), dim3(kRrBlock), lds, s, b);
  }
  return hipGetLastError();
}

}  // namespace snn
