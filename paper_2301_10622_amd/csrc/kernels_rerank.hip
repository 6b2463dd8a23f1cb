// Ranking with k' >= k (Alg. 7), first half: the k' candidates of each query,
// chosen by their Sinnamon scores, are fetched from the forward store and
// scored with the exact inner product of Eq. 2. The k best by exact score
// (ties by the lower external id) are then picked by the select kernel.
//
// One workgroup of 8 waves per (query, share of its candidates); a small batch
// spreads each query's candidates over several workgroups. The query's non-zeros (all of them,
// whatever the anytime budget of the scoring) go into an open-addressing hash
// table in LDS (coordinate -> value), so a document entry costs one LDS probe
// whatever the dimensionality. Each wave takes 64 candidates at a time: lane l
// fetches the slot, forward-store offset and length of candidate l, then the
// wave walks the candidates one after another, its 64 lanes reading 64
// consecutive (coordinate, value) entries of the document per step
// (coalesced 512-byte reads) and summing q_j * x_j in FP32; a fixed butterfly
// of cross-lane adds finishes each sum, so the result does not depend on
// timing. Each exact score leaves as a 64-bit key
// ord(score) << 32 | (0xFFFFFFFF - id).
#include <algorithm>

#include "snn_device.h"

namespace snn {

constexpr int kRrWaves = 8;
constexpr int kRrStep = 8;  // candidates a wave scores at once
constexpr int kRrBlock = 64 * kRrWaves;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;  // no coordinate reaches 2^31

__device__ __forceinline__ uint32_t shfl_u32(uint32_t v, int src) {
  return (uint32_t)__shfl((int)v, src, 64);
}

__global__ __launch_bounds__(kRrBlock) void k_rerank(RerankArgs a) {
  extern __shared__ uint32_t lds[];
  const uint32_t cap = a.hash_cap, mask = cap - 1u;
  const uint32_t shift = 32u - (uint32_t)__builtin_ctz(cap);
  uint32_t *hk = lds;                      // [cap] coordinates
  float *hv = (float *)(lds + cap);        // [cap] values
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

  // the query as a hash table: linear probing, at most half full
  for (uint32_t i = tid; i < cap; i += kRrBlock) hk[i] = kEmpty;
  __syncthreads();
  for (uint32_t i = tid; i < ne; i += kRrBlock) {
    const uint32_t j = a.qd.j[e0 + i];
    const float v = a.qd.q[e0 + i];
    uint32_t h = (j * 0x9E3779B1u) >> shift;
    for (;;) {
      const uint32_t prev = atomicCAS(&hk[h], kEmpty, j);
      if (prev == kEmpty) {
        hv[h] = v;
        break;
      }
      if (prev == j) break;  // coordinates of a valid query are distinct
      h = (h + 1u) & mask;
    }
  }
  __syncthreads();
  auto lookup = [&](uint32_t j) -> float {
    uint32_t h = (j * 0x9E3779B1u) >> shift;
    for (;;) {
      const uint32_t kj = hk[h];
      if (kj == j) return hv[h];
      if (kj == kEmpty) return 0.0f;
      h = (h + 1u) & mask;
    }
  };

  // exact inner products of this workgroup's share of the candidates
  const int lane = tid & 63, wave = tid >> 6;
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
    // kRrStep candidates at a time, so their entries' loads are in flight
    // together; each candidate's sum is formed exactly as alone (lane l adds
    // entries l, l + 64, ... in order, then the butterfly)
    for (uint32_t t0 = 0; t0 < here; t0 += kRrStep) {
      uint64_t o[kRrStep];
      uint32_t ln[kRrStep];
      float acc[kRrStep];
      uint32_t lmax = 0;
#pragma unroll
      for (int u = 0; u < kRrStep; ++u) {
        const uint32_t t = t0 + (uint32_t)u;
        const int src = t < here ? (int)t : 0;
        o[u] = ((uint64_t)shfl_u32((uint32_t)(off >> 32), src) << 32) | shfl_u32((uint32_t)off, src);
        ln[u] = t < here ? shfl_u32(len, src) : 0u;
        lmax = max(lmax, ln[u]);
        acc[u] = 0.0f;
      }
      for (uint32_t e = (uint32_t)lane; e < lmax; e += 64u) {
        uint2 en[kRrStep];
#pragma unroll
        for (int u = 0; u < kRrStep; ++u) en[u] = e < ln[u] ? a.fw.ent[o[u] + e] : make_uint2(0u, 0u);
#pragma unroll
        for (int u = 0; u < kRrStep; ++u)
          if (e < ln[u]) acc[u] = __builtin_fmaf(lookup(en[u].x), __builtin_bit_cast(float, en[u].y), acc[u]);
      }
#pragma unroll
      for (int u = 0; u < kRrStep; ++u) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) acc[u] += __shfl_xor(acc[u], d, 64);
        if ((uint32_t)lane == t0 + (uint32_t)u && t0 + (uint32_t)u < here) {
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
  // workgroups per query: enough to fill the device for small batches, and at
  // least 128 candidates each (one query of k' = 1,000: 7 workgroups; of
  // k' = 20,000: 156)
  const uint32_t by_grid = std::max<uint32_t>(1u, 1024u / nq);
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
