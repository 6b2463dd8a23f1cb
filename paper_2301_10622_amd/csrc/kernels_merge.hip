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
// Select: the final top-k of one query straight from all of its tile groups,
// for large k where sorting every candidate would dominate. One workgroup per
// query finds the k-th largest 64-bit key by most-significant-digit radix
// select: each pass builds a 4,096-bin histogram (12-bit digits) of the keys
// that share the prefix found so far and picks the bin holding the k-th key;
// it stops once a bin holds exactly the keys still needed (normally after the
// three passes that fix the 32-bit score; ties at the k-th score go on into
// the id bits). The keys at or above the found prefix are then exactly the k
// best; only they are sorted (bitonic, at most 4,096 in LDS).
// ---------------------------------------------------------------------------
constexpr int kSelBlock = 512;
constexpr int kSelWaves = kSelBlock / 64;
constexpr int kSelBins = 4096;

template <bool kPay>
__global__ __launch_bounds__(kSelBlock) void k_select(MergeArgs a) {
  __shared__ uint32_t hist[kSelBins];
  __shared__ uint32_t part[kSelBlock];
  __shared__ uint64_t sel[kMaxK];
  __shared__ uint32_t sels[kPay ? kMaxK : 1];
  __shared__ uint32_t sh_bin, sh_need, sh_pos;
  uint32_t q = a.q0 + blockIdx.y;
  if (a.qlist) {
    if (q >= *as_const(a.nlist)) return;
    q = as_const(a.qlist)[q];
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t G = a.groups_in;
  const uint32_t *cnts = a.in_cnt + (size_t)q * G;
  const uint64_t *base = a.in + (size_t)q * G * a.kmax;
  const uint32_t kq = a.kq ? as_const(a.kq)[q] : a.kmax;
  const bool bad = a.status && a.status[q] != 0u;
  // every key of the query: wave w walks groups w, w + 8, ..., its lanes the group's keys
  auto for_each = [&](auto f) {
    for (uint32_t g = (uint32_t)wave; g < G; g += kSelWaves) {
      const uint32_t c = cnts[g];
      const uint64_t *src = base + (size_t)g * a.kmax;
      for (uint32_t e = (uint32_t)lane; e < c; e += 64) f(src[e], g, e);
    }
  };
  // M = number of candidates
  uint32_t mine = 0;
  for (uint32_t g = (uint32_t)tid; g < G; g += kSelBlock) mine += cnts[g];
  part[tid] = mine;
  __syncthreads();
  for (int d = kSelBlock / 2; d > 0; d >>= 1) {
    if (tid < d) part[tid] += part[tid + d];
    __syncthreads();
  }
  const uint32_t M = part[0];
  __syncthreads();
  if (a.emitted && tid == 0 && M) atomicAdd(a.emitted, (unsigned long long)M);
  const uint32_t keep = bad ? 0u : min(M, kq);
  uint64_t T = 0;  // the result is every key >= T
  if (keep > 0 && keep < M) {
    uint64_t P = 0;
    int pb = 0;
    uint32_t need = keep;
    for (;;) {
      const int d = min(12, 64 - pb);
      const uint32_t nb = 1u << d;
      for (uint32_t i = tid; i < nb; i += kSelBlock) hist[i] = 0u;
      __syncthreads();
      for_each([&](uint64_t key, uint32_t, uint32_t) {
        if (pb == 0 || (key >> (64 - pb)) == P)
          atomicAdd(&hist[(uint32_t)(key >> (64 - pb - d)) & (nb - 1u)], 1u);
      });
      __syncthreads();
      // counts above each thread's 8 bins (suffix scan), then the bin that
      // holds the need-th largest key
      const uint32_t per = (nb + kSelBlock - 1) / kSelBlock;
      const uint32_t b0 = (uint32_t)tid * per;
      uint32_t s = 0;
      for (uint32_t b = b0; b < b0 + per && b < nb; ++b) s += hist[b];
      part[tid] = s;
      __syncthreads();
      for (int off = 1; off < kSelBlock; off <<= 1) {
        const uint32_t v = tid + off < kSelBlock ? part[tid + off] : 0u;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
      }
      uint32_t above = part[tid] - s;
      for (int b = (int)min(b0 + per, nb) - 1; b >= (int)b0; --b) {
        const uint32_t h = hist[b];
        if (above < need && above + h >= need) {
          sh_bin = (uint32_t)b;
          sh_need = need - above;
        }
        above += h;
      }
      __syncthreads();
      const uint32_t bin = sh_bin;
      const uint32_t in_bin = hist[bin];
      need = sh_need;
      P = (P << d) | bin;
      pb += d;
      __syncthreads();
      if (in_bin == need || pb == 64) {
        T = pb == 64 ? P : (P << (64 - pb));
        break;
      }
    }
  }
  // the keep best keys (with their slots), then sorted
  if (tid == 0) sh_pos = 0;
  __syncthreads();
  if (keep > 0) {
    for_each([&](uint64_t key, uint32_t g, uint32_t e) {
      if (key >= T) {
        const uint32_t pos = atomicAdd(&sh_pos, 1u);
        sel[pos] = key;
        if (kPay) sels[pos] = a.in_slot[((size_t)q * G + g) * a.kmax + e];
      }
    });
  }
  __syncthreads();
  uint32_t np = 1;
  while (np < keep) np <<= 1;
  for (uint32_t i = keep + tid; i < np; i += kSelBlock) sel[i] = 0ull;
  for (uint32_t size = 2; size <= np; size <<= 1)
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (uint32_t i = tid; i < (np >> 1); i += kSelBlock) {
        const uint32_t lo = 2 * stride * (i / stride) + (i % stride);
        const uint32_t hi = lo + stride;
        const bool down = (lo & size) == 0;
        const uint64_t x = sel[lo], y = sel[hi];
        if ((x < y) == down) {
          sel[lo] = y;
          sel[hi] = x;
          if (kPay) {
            const uint32_t t = sels[lo];
            sels[lo] = sels[hi];
            sels[hi] = t;
          }
        }
      }
    }
  __syncthreads();
  uint32_t *ids = a.res_ids + (size_t)q * a.kmax;
  float *sc = a.res_scores + (size_t)q * a.kmax;
  for (uint32_t r = tid; r < keep; r += kSelBlock) {
    const uint64_t key = sel[r];
    ids[r] = 0xFFFFFFFFu - (uint32_t)key;
    sc[r] = key_value((uint32_t)(key >> 32));
    if (kPay) a.res_slots[(size_t)q * a.kmax + r] = sels[r];
  }
  if (tid == 0) {
    a.res_cnt[q] = keep;
    if (a.fallback) a.fallback[q] = (!bad && a.keff && M < a.keff[q]) ? 1u : 0u;
  }
}

hipError_t launch_select(const MergeArgs &a, hipStream_t s) {
  if (a.kmax > kMaxK || a.groups_out != 1 || !a.res_ids || !a.res_scores || !a.res_cnt) return hipErrorInvalidValue;
  const bool pay = a.in_slot != nullptr;
  if (pay && a.res_slots == nullptr) return hipErrorInvalidValue;
  if (pay) hipLaunchKernelGGL(k_select<true>, dim3(1, a.nq), dim3(kSelBlock), 0, s, a);
  else hipLaunchKernelGGL(k_select<false>, dim3(1, a.nq), dim3(kSelBlock), 0, s, a);
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
