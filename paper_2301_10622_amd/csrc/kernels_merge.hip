// Merge of the per-tile candidates of each query into its final top-k
// (selection of Alg. 3 / Alg. 7 over the tile winners), and the fallback list
// of the learned filter.
#include <algorithm>

#include "snn_device.h"

namespace snn {

template <typename T>
using cptr = const __attribute__((address_space(4))) T *;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T *p) {
  return (cptr<T>)(p);
}

// ---------------------------------------------------------------------------
// Select: the final top-k of one query straight from all of its tile groups,
// without sorting every candidate (a query can have k keys from each of
// hundreds of tiles; at k = 4,096 the whole collection). One workgroup per
// query finds the k-th largest 64-bit key by most-significant-digit radix
// select: each pass builds a 4,096-bin histogram (12-bit digits) of the keys
// that share the prefix found so far and picks the bin holding the k-th key;
// it stops once a bin holds exactly the keys still needed (normally after the
// three passes that fix the 32-bit score; ties at the k-th score go on into
// the id bits). The keys at or above the found prefix are then exactly the k
// best. kSorted: only they are sorted (bitonic, at most 4,096 in LDS) and
// written in order; otherwise (the k' candidates of the re-rank, up to 65,536)
// they are written in the order found, with their slots.
// ---------------------------------------------------------------------------
constexpr int kSelBlock = 512;  // threads of a select workgroup (1,024 for small batches)
constexpr int kSelBins = 4096;
constexpr uint32_t kSelScanMax = 2048;  // groups whose key offsets fit in LDS
constexpr int kSelCache = 8;             // keys per thread held in registers (4,096 or 8,192 per query)
constexpr int kSelU = 4;                 // keys of a group per lane in flight (large groups)
// keys copied to LDS after the first radix pass: 1,024, or 4,096 in the form
// launched for a sorted top-k with k above 512 (more LDS, one workgroup per CU)
template <bool kBig>
constexpr uint32_t sel_cmp() { return kBig ? 4096u : 1024u; }

// Inclusive prefix sum of v over the workgroup's threads, and the total: a
// shuffle scan inside each wave, then the kW wave totals through LDS (two
// barriers, where a scan over the threads in LDS takes two per doubling).
template <int kW>
__device__ __forceinline__ uint32_t sel_scan(uint32_t v, uint32_t *wsum, uint32_t &total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  uint32_t off = 0, t = 0;
#pragma unroll
  for (int w = 0; w < kW; ++w) {
    const uint32_t sw = wsum[w];
    off += w < wave ? sw : 0u;
    t += sw;
  }
  __syncthreads();  // wsum is free for the next scan
  total = t;
  return x + off;
}

template <bool kPay, bool kSorted, bool kBig, int kB>
__global__ __launch_bounds__(kB) void k_select(SelectArgs a) {
  constexpr int kWv = kB / 64;  // waves of the workgroup
  constexpr uint32_t kSelCmp = sel_cmp<kBig>();
  __shared__ uint32_t hist[kSelBins];
  __shared__ uint32_t wsum[kWv];
  __shared__ uint64_t sel[kSorted ? kMaxK : 1];
  __shared__ uint32_t sels[kPay && kSorted ? kMaxK : 1];
  __shared__ uint32_t sh_bin, sh_need, sh_pos;
  __shared__ uint32_t goff[kSelScanMax + 1];  // first key of each group among all the query's keys
  // after the first radix pass: the keys at or above the bin found, when few
  __shared__ uint64_t cmp_key[kSelCmp];
  __shared__ uint32_t cmp_g[kSelCmp], cmp_e[kSelCmp];
  __shared__ uint32_t cmp_n;
  uint32_t q = a.q0 + blockIdx.y;
  if (a.qlist) {
    if (q >= *as_const(a.nlist)) return;
    q = as_const(a.qlist)[q];
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t G = a.groups_in;
  const uint32_t *cnts = a.in_cnt + (size_t)q * G;
  const uint64_t *base = a.in + (size_t)q * G * a.in_stride;
  const uint32_t kq = a.kq ? as_const(a.kq)[q] : a.kmax;
  const bool bad = a.status && a.status[q] != 0u;
  // M = number of candidates; with at most kSelScanMax groups also each
  // group's first key in the concatenation of all groups (thread t sums the
  // groups t * per .. t * per + per - 1, then a scan over the threads)
  const bool scan = G <= kSelScanMax;
  const uint32_t gper = (G + kB - 1) / kB;
  uint32_t mine = 0;
  if (scan) {
    for (uint32_t g = (uint32_t)tid * gper; g < min(G, ((uint32_t)tid + 1) * gper); ++g) mine += cnts[g];
  } else {
    for (uint32_t g = (uint32_t)tid; g < G; g += kB) mine += cnts[g];
  }
  uint32_t M;
  const uint32_t incl = sel_scan<kWv>(mine, wsum, M);
  if (scan) {
    uint32_t o = incl - mine;
    for (uint32_t g = (uint32_t)tid * gper; g < min(G, ((uint32_t)tid + 1) * gper); ++g) {
      goff[g] = o;
      o += cnts[g];
    }
    if (tid == 0) goff[G] = M;
  }
  __syncthreads();
  // Every key of the query. Small groups (fewer than 64 keys on average), or
  // fewer groups than twice the waves (one long group: the k' exact scores of
  // a re-rank): the threads stride over the concatenated keys and find each
  // key's group by binary search in goff, so no lane or wave idles; otherwise
  // wave w walks groups w, w + 8, ..., its lanes the group's keys.
  const bool flat = scan && (M < 64u * G || G < 2u * kWv);
  // At most kSelCache keys per thread: read them (and their groups) once into
  // registers and serve every pass from there.
  const bool cached = flat && M <= (uint32_t)(kSelCache * kB);
  uint64_t ck[kSelCache];
  uint32_t cg[kSelCache], ce[kSelCache];
  if (cached) {
#pragma unroll
    for (int u = 0; u < kSelCache; ++u) {
      const uint32_t i = (uint32_t)tid + (uint32_t)u * kB;
      ck[u] = 0;
      cg[u] = ce[u] = 0;
      if (i < M) {
        uint32_t lo = 0, hi = G;  // goff[lo] <= i < goff[hi]
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (goff[mid] <= i) lo = mid;
          else hi = mid;
        }
        cg[u] = lo;
        ce[u] = i - goff[lo];
        ck[u] = base[(size_t)lo * a.in_stride + ce[u]];
      }
    }
  }
  bool compacted = false;
  auto for_each = [&](auto f) {
    if (compacted) {
      const uint32_t n = cmp_n;
      for (uint32_t i = (uint32_t)tid; i < n; i += kB) f(cmp_key[i], cmp_g[i], cmp_e[i]);
    } else if (cached) {
#pragma unroll
      for (int u = 0; u < kSelCache; ++u)
        if ((uint32_t)tid + (uint32_t)u * kB < M) f(ck[u], cg[u], ce[u]);
    } else if (flat) {
      constexpr int U = 4;  // keys in flight per thread
      for (uint32_t i0 = (uint32_t)tid; i0 < M; i0 += U * kB) {
        uint64_t kk[U];
        uint32_t gg[U], ee[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t i = i0 + (uint32_t)u * kB;
          gg[u] = ee[u] = 0;
          kk[u] = 0;
          if (i < M) {
            uint32_t lo = 0, hi = G;  // goff[lo] <= i < goff[hi]
            while (hi - lo > 1) {
              const uint32_t mid = (lo + hi) >> 1;
              if (goff[mid] <= i) lo = mid;
              else hi = mid;
            }
            gg[u] = lo;
            ee[u] = i - goff[lo];
            kk[u] = base[(size_t)lo * a.in_stride + ee[u]];
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (i0 + (uint32_t)u * kB < M) f(kk[u], gg[u], ee[u]);
      }
    } else {
      // two groups at a time and kSelU keys of each per lane, so 2 kSelU
      // loads are in flight per lane
      for (uint32_t g = (uint32_t)wave; g < G; g += 2 * kWv) {
        const uint32_t g2 = g + kWv;
        const uint32_t c1 = scan ? goff[g + 1] - goff[g] : cnts[g];
        const uint32_t c2 = g2 < G ? (scan ? goff[g2 + 1] - goff[g2] : cnts[g2]) : 0u;
        const uint64_t *s1 = base + (size_t)g * a.in_stride;
        const uint64_t *s2 = base + (size_t)g2 * a.in_stride;
        for (uint32_t e0 = (uint32_t)lane; e0 < max(c1, c2); e0 += 64u * kSelU) {
          uint64_t k1[kSelU], k2[kSelU];
#pragma unroll
          for (int u = 0; u < kSelU; ++u) {
            const uint32_t e = e0 + 64u * (uint32_t)u;
            k1[u] = e < c1 ? s1[e] : 0ull;
            k2[u] = e < c2 ? s2[e] : 0ull;
          }
#pragma unroll
          for (int u = 0; u < kSelU; ++u) {
            const uint32_t e = e0 + 64u * (uint32_t)u;
            if (e < c1) f(k1[u], g, e);
            if (e < c2) f(k2[u], g2, e);
          }
        }
      }
    }
  };
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
      for (uint32_t i = tid; i < nb; i += kB) hist[i] = 0u;
      __syncthreads();
      for_each([&](uint64_t key, uint32_t, uint32_t) {
        if (pb == 0 || (key >> (64 - pb)) == P)
          atomicAdd(&hist[(uint32_t)(key >> (64 - pb - d)) & (nb - 1u)], 1u);
      });
      __syncthreads();
      // counts above each thread's 8 bins (suffix scan), then the bin that
      // holds the need-th largest key
      const uint32_t per = (nb + kB - 1) / kB;
      const uint32_t b0 = (uint32_t)tid * per;
      uint32_t s = 0;
      for (uint32_t b = b0; b < b0 + per && b < nb; ++b) s += hist[b];
      uint32_t tot;
      const uint32_t pre = sel_scan<kWv>(s, wsum, tot);
      uint32_t above = tot - pre;  // keys in the bins of the threads after this one
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
      // The keys whose first pb bits are at least P (the keep - need above the
      // bin and the in_bin in it) hold every key still to be decided and every
      // key to emit. When they are few, one more read copies them to LDS and
      // the remaining passes and the emission work from there.
      if (!cached && !compacted && (keep - need) + in_bin <= kSelCmp) {
        if (tid == 0) cmp_n = 0;
        __syncthreads();
        for_each([&](uint64_t key, uint32_t g, uint32_t e) {
          if ((key >> (64 - pb)) >= P) {
            const uint32_t pos = atomicAdd(&cmp_n, 1u);
            cmp_key[pos] = key;
            cmp_g[pos] = g;
            cmp_e[pos] = e;
          }
        });
        __syncthreads();
        compacted = true;
      }
    }
  }
  // the keep best keys (with their slots)
  if (tid == 0) sh_pos = 0;
  __syncthreads();
  uint32_t *ids = a.res_ids + (size_t)q * a.kmax;
  float *sc = a.res_scores + (size_t)q * a.kmax;
  if (keep > 0) {
    for_each([&](uint64_t key, uint32_t g, uint32_t e) {
      if (key >= T) {
        const uint32_t pos = atomicAdd(&sh_pos, 1u);
        const uint32_t slot = kPay ? a.in_slot[((size_t)q * G + g) * a.in_stride + e] : 0u;
        if (kSorted) {
          sel[pos] = key;
          if (kPay) sels[pos] = slot;
        } else {
          ids[pos] = 0xFFFFFFFFu - (uint32_t)key;
          sc[pos] = key_value((uint32_t)(key >> 32));
          if (kPay) a.res_slots[(size_t)q * a.kmax + pos] = slot;
        }
      }
    });
  }
  __syncthreads();
  if (!kSorted) {
    if (tid == 0) {
      a.res_cnt[q] = keep;
      if (a.fallback) a.fallback[q] = (!bad && a.keff && M < a.keff[q]) ? 1u : 0u;
    }
    return;
  }
  uint32_t np = 1;
  while (np < keep) np <<= 1;
  for (uint32_t i = keep + tid; i < np; i += kB) sel[i] = 0ull;
  for (uint32_t size = 2; size <= np; size <<= 1)
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (uint32_t i = tid; i < (np >> 1); i += kB) {
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
  for (uint32_t r = tid; r < keep; r += kB) {
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

template <int kB>
static void launch_select_b(const SelectArgs &a, bool sorted, bool pay, hipStream_t s) {
  if (sorted && !pay && a.kmax > 512)
    hipLaunchKernelGGL((k_select<false, true, true, kB>), dim3(1, a.nq), dim3(kB), 0, s, a);
  else if (sorted && !pay)
    hipLaunchKernelGGL((k_select<false, true, false, kB>), dim3(1, a.nq), dim3(kB), 0, s, a);
  else if (!sorted && pay)
    hipLaunchKernelGGL((k_select<true, false, false, kB>), dim3(1, a.nq), dim3(kB), 0, s, a);
  else if (a.kmax > 512)  // unsorted without slots: the sampled pass's threshold
    hipLaunchKernelGGL((k_select<false, false, true, kB>), dim3(1, a.nq), dim3(kB), 0, s, a);
  else
    hipLaunchKernelGGL((k_select<false, false, false, kB>), dim3(1, a.nq), dim3(kB), 0, s, a);
}

hipError_t launch_select(const SelectArgs &a, bool sorted, hipStream_t s) {
  if (a.kmax == 0 || a.in_stride == 0 || !a.res_ids || !a.res_scores || !a.res_cnt) return hipErrorInvalidValue;
  if (sorted ? a.kmax > kMaxK : a.kmax > kMaxKPrime) return hipErrorInvalidValue;
  const bool pay = a.in_slot != nullptr;
  if (pay != (a.res_slots != nullptr)) return hipErrorInvalidValue;
  // a batch of at most as many queries as CUs gets 1,024-thread workgroups:
  // one workgroup per query works alone on its CU
  if (a.nq <= 256) launch_select_b<1024>(a, sorted, pay, s);
  else launch_select_b<kSelBlock>(a, sorted, pay, s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Starting threshold of a search whose k' exceeds a tile (Alg. 7): the lowest
// score among the ks best of a sample of the tiles, as an inclusive score key;
// 0 (no threshold) when the sample held fewer than ks candidates. One
// workgroup per query.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sample_thr(uint32_t ks, uint32_t stride, const float *__restrict__ sc,
                                                    const uint32_t *__restrict__ cnt, uint32_t *__restrict__ thr) {
  __shared__ float red[256];
  const uint32_t q = blockIdx.x;
  const uint32_t c = cnt[q];
  float m = __builtin_inff();
  for (uint32_t i = threadIdx.x; i < c; i += 256) m = fminf(m, sc[(size_t)q * stride + i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (threadIdx.x < (unsigned)d) red[threadIdx.x] = fminf(red[threadIdx.x], red[threadIdx.x + d]);
    __syncthreads();
  }
  if (threadIdx.x == 0) thr[q] = (c >= ks && ks > 0) ? ord_key(red[0]) : 0u;
}

hipError_t launch_sample_thr(uint32_t nq, uint32_t ks, uint32_t stride, const float *sc, const uint32_t *cnt,
                             uint32_t *thr, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  if (ks > stride) return hipErrorInvalidValue;
  for (uint32_t q0 = 0; q0 < nq; q0 += 65535u) {
    const uint32_t n = std::min<uint32_t>(65535u, nq - q0);
    hipLaunchKernelGGL(k_sample_thr, dim3(n), dim3(256), 0, s, ks, stride, sc + (size_t)q0 * stride, cnt + q0,
                       thr + q0);
  }
  return hipGetLastError();
}

// keff[q] = min(k of query q, cap): the candidates query q must keep so that a
// starting threshold cannot have cut its top-k
__global__ __launch_bounds__(256) void k_keff(uint32_t nq, const uint32_t *__restrict__ kq, uint32_t kmax,
                                              uint32_t cap, uint32_t *__restrict__ keff) {
  const uint32_t q = blockIdx.x * 256 + threadIdx.x;
  if (q < nq) keff[q] = min(kq ? kq[q] : kmax, cap);
}

hipError_t launch_keff(uint32_t nq, const uint32_t *kq, uint32_t kmax, uint32_t cap, uint32_t *keff, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_keff, dim3((nq + 255) / 256), dim3(256), 0, s, nq, kq, kmax, cap, keff);
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
