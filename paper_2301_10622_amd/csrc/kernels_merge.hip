// Merge of the per-tile candidates of each query into its final top-k
// (selection of Alg. 3 / Alg. 7 with k' = k, over the tile winners).
#include "snn_device.h"

namespace snn {

constexpr uint32_t kRankMax = 1024;  // lists up to this size are ordered by rank counting

template <typename T>
using cptr = const __attribute__((address_space(4))) T *;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T *p) {
  return (cptr<T>)(p);
}

// ---------------------------------------------------------------------------
// Merge: one workgroup takes up to `fanin` candidate groups of one query,
// sorts them by key descending in LDS (bitonic), and keeps the k best. The last
// level writes (id, score) results; earlier levels write a smaller group list.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_merge(MergeArgs a) {
  __shared__ uint64_t s[kMergeCap];
  __shared__ uint32_t off[257];
  const uint32_t q = a.q0 + blockIdx.y;
  const uint32_t g = blockIdx.x;
  const uint32_t g0 = g * a.fanin;
  const uint32_t g1 = min(g0 + a.fanin, a.groups_in);
  const uint32_t ng = g1 > g0 ? g1 - g0 : 0u;
  const uint32_t kq = a.kq ? as_const(a.kq)[q] : a.kmax;
  // offsets of each input group inside the LDS list (fanin <= 256): block scan
  const uint32_t myc = threadIdx.x < ng ? as_const(a.in_cnt)[(size_t)q * a.groups_in + g0 + threadIdx.x] : 0u;
  off[threadIdx.x + 1] = myc;
  if (threadIdx.x == 0) off[0] = 0;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {
    const uint32_t v = (int)threadIdx.x + 1 - d >= 1 ? off[threadIdx.x + 1 - d] : 0u;
    __syncthreads();
    off[threadIdx.x + 1] += v;
    __syncthreads();
  }
  const uint32_t M = off[ng];
  int n = 1;
  while (n < (int)M) n <<= 1;
  // gather: element e belongs to the last group whose offset is <= e
  const uint64_t *src0 = a.in + ((size_t)q * a.groups_in + g0) * a.kmax;
  for (uint32_t e = threadIdx.x; e < M; e += blockDim.x) {
    uint32_t lo = 0, hi = ng;  // off[lo] <= e < off[hi]
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (off[mid] <= e) lo = mid;
      else hi = mid;
    }
    s[e] = src0[(size_t)lo * a.kmax + (e - off[lo])];
  }
  const bool bad = a.status && a.status[q] != 0u;
  const uint32_t keep = bad ? 0u : min(M, kq);
  if (M <= (uint32_t)kRankMax) {
    // small lists: the keys are distinct (one per document), so each key's
    // rank is the number of larger keys; the k best go straight to their place
    __syncthreads();
    uint64_t *dst = a.groups_out > 1 ? a.out + ((size_t)q * a.groups_out + g) * a.kmax : nullptr;
    uint32_t *ids = a.res_ids + (size_t)q * a.kmax;
    float *sc = a.res_scores + (size_t)q * a.kmax;
    for (uint32_t e = threadIdx.x; e < M; e += blockDim.x) {
      const uint64_t key = s[e];
      uint32_t rank = 0;
      for (uint32_t x = 0; x < M; ++x) rank += s[x] > key ? 1u : 0u;
      if (rank < keep) {
        if (dst) {
          dst[rank] = key;
        } else {
          ids[rank] = 0xFFFFFFFFu - (uint32_t)key;
          sc[rank] = key_value((uint32_t)(key >> 32));
        }
      }
    }
    if (threadIdx.x == 0) {
      if (dst) {
        a.out_cnt[(size_t)q * a.groups_out + g] = keep;
      } else {
        a.res_cnt[q] = keep;
        if (a.fallback) a.fallback[q] = (!bad && a.keff && M < a.keff[q]) ? 1u : 0u;
      }
    }
    return;
  }
  for (int e = (int)M + threadIdx.x; e < n; e += blockDim.x) s[e] = 0ull;
  // bitonic sort, descending
  for (int size = 2; size <= n; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int i = threadIdx.x; i < (n >> 1); i += blockDim.x) {
        const int lo = 2 * stride * (i / stride) + (i % stride);
        const int hi = lo + stride;
        const bool down = (lo & size) == 0;
        const uint64_t x = s[lo], y = s[hi];
        if ((x < y) == down) {
          s[lo] = y;
          s[hi] = x;
        }
      }
    }
  __syncthreads();
  if (a.groups_out > 1) {
    uint64_t *dst = a.out + ((size_t)q * a.groups_out + g) * a.kmax;
    for (uint32_t e = threadIdx.x; e < keep; e += blockDim.x) dst[e] = s[e];
    if (threadIdx.x == 0) a.out_cnt[(size_t)q * a.groups_out + g] = keep;
  } else {
    uint32_t *ids = a.res_ids + (size_t)q * a.kmax;
    float *sc = a.res_scores + (size_t)q * a.kmax;
    for (uint32_t e = threadIdx.x; e < keep; e += blockDim.x) {
      const uint64_t key = s[e];
      ids[e] = 0xFFFFFFFFu - (uint32_t)key;
      sc[e] = key_value((uint32_t)(key >> 32));
    }
    if (threadIdx.x == 0) {
      a.res_cnt[q] = keep;
      if (a.fallback) a.fallback[q] = (!bad && a.keff && M < a.keff[q]) ? 1u : 0u;
    }
  }
}

hipError_t launch_merge(const MergeArgs &a, hipStream_t s) {
  if (a.fanin > 256 || (uint64_t)a.fanin * a.kmax > (uint64_t)kMergeCap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_merge, dim3(a.groups_out, a.nq), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace snn
