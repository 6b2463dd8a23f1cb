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
// With kPay the candidates' slots travel with their keys (the re-rank input).
template <bool kPay>
__global__ __launch_bounds__(256) void k_merge(MergeArgs a) {
  __shared__ uint64_t s[kMergeCap];
  __shared__ uint32_t ps[kPay ? kMergeCap : 1];
  __shared__ uint32_t off[257];
  uint32_t q = a.q0 + blockIdx.y;
  if (a.qlist) {
    if (q >= *as_const(a.nlist)) return;
    q = as_const(a.qlist)[q];
  }
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
  if (a.emitted && threadIdx.x == 0 && M) atomicAdd(a.emitted, (unsigned long long)M);
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
    if (kPay) ps[e] = a.in_slot[((size_t)q * a.groups_in + g0 + lo) * a.kmax + (e - off[lo])];
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
          if (kPay) a.out_slot[((size_t)q * a.groups_out + g) * a.kmax + rank] = ps[e];
        } else {
          ids[rank] = 0xFFFFFFFFu - (uint32_t)key;
          sc[rank] = key_value((uint32_t)(key >> 32));
          if (kPay) a.res_slots[(size_t)q * a.kmax + rank] = ps[e];
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
          if (kPay) {
            const uint32_t t = ps[lo];
            ps[lo] = ps[hi];
            ps[hi] = t;
          }
        }
      }
    }
  __syncthreads();
  if (a.groups_out > 1) {
    uint64_t *dst = a.out + ((size_t)q * a.groups_out + g) * a.kmax;
    for (uint32_t e = threadIdx.x; e < keep; e += blockDim.x) {
      dst[e] = s[e];
      if (kPay) a.out_slot[((size_t)q * a.groups_out + g) * a.kmax + e] = ps[e];
    }
    if (threadIdx.x == 0) a.out_cnt[(size_t)q * a.groups_out + g] = keep;
  } else {
    uint32_t *ids = a.res_ids + (size_t)q * a.kmax;
    float *sc = a.res_scores + (size_t)q * a.kmax;
    for (uint32_t e = threadIdx.x; e < keep; e += blockDim.x) {
      const uint64_t key = s[e];
      ids[e] = 0xFFFFFFFFu - (uint32_t)key;
      sc[e] = key_value((uint32_t)(key >> 32));
      if (kPay) a.res_slots[(size_t)q * a.kmax + e] = ps[e];
    }
    if (threadIdx.x == 0) {
      a.res_cnt[q] = keep;
      if (a.fallback) a.fallback[q] = (!bad && a.keff && M < a.keff[q]) ? 1u : 0u;
    }
  }
}

hipError_t launch_merge(const MergeArgs &a, hipStream_t s) {
  if (a.fanin > 256 || (uint64_t)a.fanin * a.kmax > (uint64_t)kMergeCap) return hipErrorInvalidValue;
  const bool pay = a.in_slot != nullptr;
  if (pay && (a.groups_out > 1 ? a.out_slot == nullptr : a.res_slots == nullptr)) return hipErrorInvalidValue;
  if (pay) hipLaunchKernelGGL(k_merge<true>, dim3(a.groups_out, a.nq), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_merge<false>, dim3(a.groups_out, a.nq), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fallback list of the learned filter: one workgroup compacts the queries whose
// filtered merge kept fewer than the required candidates, in query order, into
// qlist[0 .. *nlist), and clears their shared thresholds for the plain pass.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fallback_list(uint32_t nq, const uint32_t *__restrict__ flags,
                                                       uint32_t *__restrict__ qlist, uint32_t *__restrict__ nlist,
                                                       uint32_t *__restrict__ thr) {
  __shared__ uint32_t cnt[256];
  __shared__ uint32_t base;
  if (threadIdx.x == 0) base = 0;
  for (uint32_t c0 = 0; c0 < nq; c0 += 256) {
    const uint32_t q = c0 + threadIdx.x;
    const uint32_t f = (q < nq && flags[q]) ? 1u : 0u;
    cnt[threadIdx.x] = f;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
      const uint32_t v = threadIdx.x >= (unsigned)d ? cnt[threadIdx.x - d] : 0u;
      __syncthreads();
      cnt[threadIdx.x] += v;
      __syncthreads();
    }
    if (f) {
      qlist[base + cnt[threadIdx.x] - 1] = q;
      thr[q] = 0u;
    }
    __syncthreads();
    if (threadIdx.x == 255) base += cnt[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) *nlist = base;
}

hipError_t launch_fallback_list(uint32_t nq, const uint32_t *flags, uint32_t *qlist, uint32_t *nlist, uint32_t *thr,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_fallback_list, dim3(1), dim3(256), 0, s, nq, flags, qlist, nlist, thr);
  return hipGetLastError();
}

}  // namespace snn
