// Learned k-th-score pre-filter: hashed query features, the 256-128-128-1 MLP
// (bf16 weights, fp32 accumulation) forward, backward and Adam kernels, the
// per-query threshold, and the compaction of queries that must fall back to
// the plain path.
//
// The filter is not part of the paper. It predicts ln(s_k), the log of the k-th
// Sinnamon score a query gets, and turns the prediction into a threshold tau
// that initialises the selection's running threshold (theta of Alg. 3, which
// otherwise starts at minus infinity). If at least k documents reach tau, the
// k-th score is >= tau, so every top-k member passes and the result equals the
// plain one; otherwise the query is re-run on the plain path.
//
// Parameter vector layout (fp32 masters, bf16 compute copies, gradients and
// Adam moments all share it): W1[128][256] | b1[128] | W2[128][128] | b2[128] |
// W3[128] | b3[1], weights row-major [out][in].
#include "snn_device.h"
#include "snn_mlp.h"

namespace snn {

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

// round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------------------
// Features: f[g(j)] += xi(j) * q_j (first 128), f[128 + g(j)] += q_j^2 (last
// 128); table[j] = g(j) | (xi(j) < 0) << 31. Thread t owns feature t and adds
// the query's entries in input order, so the sums are deterministic.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_features(uint32_t nq, const uint64_t *__restrict__ qptr,
                                                  const uint32_t *__restrict__ coords, const float *__restrict__ vals,
                                                  const uint32_t *__restrict__ table, uint32_t dim,
                                                  float *__restrict__ X) {
  __shared__ uint32_t sg[512];
  __shared__ float sv[512];
  const uint32_t q = blockIdx.x;
  const uint64_t e0 = qptr[q], e1 = qptr[q + 1];
  const int t = threadIdx.x;
  const uint32_t mine = (uint32_t)(t & 127);
  const bool sq = t >= 128;
  float acc = 0.0f;
  for (uint64_t c0 = e0; c0 < e1; c0 += 512) {
    const uint32_t n = (uint32_t)min<uint64_t>(512, e1 - c0);
    __syncthreads();
    for (uint32_t i = t; i < n; i += 256) {
      const uint32_t j = coords[c0 + i];
      const float v = vals[c0 + i];
      const bool ok = j < dim && v != 0.0f;
      sg[i] = ok ? table[j] : 0xFFFFFFFFu;  // 0xFFFFFFFF: no feature
      sv[i] = v;
    }
    __syncthreads();
    for (uint32_t i = 0; i < n; ++i) {
      const uint32_t g = sg[i];
      if (g == 0xFFFFFFFFu || (g & 127u) != mine) continue;
      const float v = sv[i];
      acc += sq ? v * v : ((g >> 31) ? -v : v);
    }
  }
  X[(size_t)q * kFeat + t] = acc;
}

hipError_t launch_features(uint32_t nq, const uint64_t *qptr, const uint32_t *coords, const float *vals,
                           const uint32_t *table, uint32_t dim, float *X, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3(nq), dim3(256), 0, s, nq, qptr, coords, vals, table, dim, X);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Forward (and, for training, the per-sample backward quantities).
// One workgroup: kQT samples. rows[b] selects the sample's feature row (null:
// identity). With y != null it also computes dy = 2 (yhat - y) / B_total,
// d2 = relu'(z2) * dy * W3 and d1 = relu'(z1) * W2^T d2, and saves h1, h2, d1,
// d2 and dy for the weight-gradient kernel.
// ---------------------------------------------------------------------------
constexpr int kQT = 16;

__global__ __launch_bounds__(256) void k_mlp_fwd(uint32_t B, const float *__restrict__ X, const uint32_t *__restrict__ rows,
                                                 const uint16_t *__restrict__ Pb, float *__restrict__ yhat,
                                                 const float *__restrict__ y, float inv_btotal, float *__restrict__ H1,
                                                 float *__restrict__ H2, float *__restrict__ D1, float *__restrict__ D2,
                                                 float *__restrict__ DY, float *__restrict__ loss) {
  __shared__ float x[kQT][kFeat];
  __shared__ float h1[kQT][kHid];
  __shared__ float h2[kQT][kHid];
  __shared__ float d2[kQT][kHid];
  __shared__ float dyv[kQT];
  const int t = threadIdx.x;
  const uint32_t b0 = blockIdx.x * kQT;
  const uint32_t nb = min<uint32_t>(kQT, B - b0);
  for (int i = t; i < kQT * kFeat; i += 256) {
    const int bb = i / kFeat, f = i % kFeat;
    float v = 0.0f;
    if ((uint32_t)bb < nb) {
      const uint32_t r = rows ? rows[b0 + bb] : b0 + bb;
      v = X[(size_t)r * kFeat + f];
    }
    x[bb][f] = v;
  }
  __syncthreads();
  const uint16_t *W1 = Pb + kOffW1, *W2 = Pb + kOffW2, *W3 = Pb + kOffW3;
  const int o = t & 127, half = t >> 7;  // output unit, which 8 samples
  {
    float acc[8];
    const float bias = bf16_to_f32(Pb[kOffB1 + o]);
#pragma unroll
    for (int s = 0; s < 8; ++s) acc[s] = bias;
    for (int i = 0; i < kFeat; ++i) {
      const float w = bf16_to_f32(W1[o * kFeat + i]);
#pragma unroll
      for (int s = 0; s < 8; ++s) acc[s] = __builtin_fmaf(w, x[half * 8 + s][i], acc[s]);
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) h1[half * 8 + s][o] = acc[s] > 0.0f ? acc[s] : 0.0f;
  }
  __syncthreads();
  {
    float acc[8];
    const float bias = bf16_to_f32(Pb[kOffB2 + o]);
#pragma unroll
    for (int s = 0; s < 8; ++s) acc[s] = bias;
    for (int i = 0; i < kHid; ++i) {
      const float w = bf16_to_f32(W2[o * kHid + i]);
#pragma unroll
      for (int s = 0; s < 8; ++s) acc[s] = __builtin_fmaf(w, h1[half * 8 + s][i], acc[s]);
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) h2[half * 8 + s][o] = acc[s] > 0.0f ? acc[s] : 0.0f;
  }
  __syncthreads();
  if (t < kQT) {
    float acc = bf16_to_f32(Pb[kOffB3]);
    for (int i = 0; i < kHid; ++i) acc = __builtin_fmaf(bf16_to_f32(W3[i]), h2[t][i], acc);
    if ((uint32_t)t < nb) {
      yhat[b0 + t] = acc;
      if (y) {
        const float e = acc - y[b0 + t];
        dyv[t] = 2.0f * e * inv_btotal;
        atomicAdd(loss, e * e);
      }
    } else {
      dyv[t] = 0.0f;
    }
  }
  if (!y) return;
  __syncthreads();
  // d2 = relu'(z2) * dy * W3 ; save h1, h2, d2, dy
  for (int i = t; i < kQT * kHid; i += 256) {
    const int bb = i / kHid, u = i % kHid;
    const float g = h2[bb][u] > 0.0f ? dyv[bb] * bf16_to_f32(W3[u]) : 0.0f;
    d2[bb][u] = g;
    if ((uint32_t)bb < nb) {
      H1[(size_t)(b0 + bb) * kHid + u] = h1[bb][u];
      H2[(size_t)(b0 + bb) * kHid + u] = h2[bb][u];
      D2[(size_t)(b0 + bb) * kHid + u] = g;
    }
  }
  if (t < kQT && (uint32_t)t < nb) DY[b0 + t] = dyv[t];
  __syncthreads();
  // d1[u] = relu'(z1[u]) * sum_o W2[o][u] d2[o]
  {
    const int u = t & 127;
    float acc[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) acc[s] = 0.0f;
    for (int oo = 0; oo < kHid; ++oo) {
      const float w = bf16_to_f32(W2[oo * kHid + u]);
#pragma unroll
      for (int s = 0; s < 8; ++s) acc[s] = __builtin_fmaf(w, d2[half * 8 + s][oo], acc[s]);
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int bb = half * 8 + s;
      if ((uint32_t)bb < nb) D1[(size_t)(b0 + bb) * kHid + u] = h1[bb][u] > 0.0f ? acc[s] : 0.0f;
    }
  }
}

hipError_t launch_mlp_fwd(uint32_t B, const float *X, const uint32_t *rows, const uint16_t *Pb, float *yhat,
                          const float *y, float inv_btotal, float *H1, float *H2, float *D1, float *D2, float *DY,
                          float *loss, hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_fwd, dim3((B + kQT - 1) / kQT), dim3(256), 0, s, B, X, rows, Pb, yhat, y, inv_btotal, H1,
                     H2, D1, D2, DY, loss);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Weight gradients: one thread per parameter, summing over the batch in order
// (deterministic, no atomics).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_wgrad(uint32_t B, const float *__restrict__ X, const uint32_t *__restrict__ rows,
                                                   const float *__restrict__ H1, const float *__restrict__ H2,
                                                   const float *__restrict__ D1, const float *__restrict__ D2,
                                                   const float *__restrict__ DY, float *__restrict__ G) {
  const uint32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p >= (uint32_t)kParams) return;
  float acc = 0.0f;
  if (p < (uint32_t)kOffB1) {  // W1[o][i] = sum_b d1[b][o] x[b][i]
    const uint32_t o = p / kFeat, i = p % kFeat;
    for (uint32_t b = 0; b < B; ++b) {
      const uint32_t r = rows ? rows[b] : b;
      acc = __builtin_fmaf(D1[(size_t)b * kHid + o], X[(size_t)r * kFeat + i], acc);
    }
  } else if (p < (uint32_t)kOffW2) {  // b1
    const uint32_t o = p - kOffB1;
    for (uint32_t b = 0; b < B; ++b) acc += D1[(size_t)b * kHid + o];
  } else if (p < (uint32_t)kOffB2) {  // W2[o][i] = sum_b d2[b][o] h1[b][i]
    const uint32_t q = p - kOffW2, o = q / kHid, i = q % kHid;
    for (uint32_t b = 0; b < B; ++b) acc = __builtin_fmaf(D2[(size_t)b * kHid + o], H1[(size_t)b * kHid + i], acc);
  } else if (p < (uint32_t)kOffW3) {  // b2
    const uint32_t o = p - kOffB2;
    for (uint32_t b = 0; b < B; ++b) acc += D2[(size_t)b * kHid + o];
  } else if (p < (uint32_t)kOffB3) {  // W3[i] = sum_b dy[b] h2[b][i]
    const uint32_t i = p - kOffW3;
    for (uint32_t b = 0; b < B; ++b) acc = __builtin_fmaf(DY[b], H2[(size_t)b * kHid + i], acc);
  } else {  // b3
    for (uint32_t b = 0; b < B; ++b) acc += DY[b];
  }
  G[p] = acc;
}

hipError_t launch_mlp_wgrad(uint32_t B, const float *X, const uint32_t *rows, const float *H1, const float *H2,
                            const float *D1, const float *D2, const float *DY, float *G, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_wgrad, dim3((kParams + 255) / 256), dim3(256), 0, s, B, X, rows, H1, H2, D1, D2, DY, G);
  return hipGetLastError();
}

// Adam on the fp32 masters, then refresh the bf16 compute copies.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ P, uint16_t *__restrict__ Pb,
                                              const float *__restrict__ G, float *__restrict__ M,
                                              float *__restrict__ V, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const uint32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p >= (uint32_t)kParams) return;
  const float g = G[p];
  const float m = b1 * M[p] + (1.0f - b1) * g;
  const float v = b2 * V[p] + (1.0f - b2) * g * g;
  M[p] = m;
  V[p] = v;
  const float w = P[p] - lr * (m / c1) / (sqrtf(v / c2) + eps);
  P[p] = w;
  Pb[p] = f32_to_bf16(w);
}

hipError_t launch_adam(float *P, uint16_t *Pb, const float *G, float *M, float *V, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, P, Pb, G, M, V, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

__global__ void k_to_bf16(const float *__restrict__ P, uint16_t *__restrict__ Pb, uint32_t n) {
  const uint32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p < n) Pb[p] = f32_to_bf16(P[p]);
}

hipError_t launch_to_bf16(const float *P, uint16_t *Pb, uint32_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3((n + 255) / 256), dim3(256), 0, s, P, Pb, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Labels: y = ln(s_k) from the plain method's k-th score when the query has k
// results and s_k > 0, else NaN (no label).
// ---------------------------------------------------------------------------
__global__ void k_labels(uint32_t nq, uint32_t k, const float *__restrict__ scores, const uint32_t *__restrict__ cnt,
                         float *__restrict__ y) {
  const uint32_t q = blockIdx.x * 256 + threadIdx.x;
  if (q >= nq) return;
  const float s = cnt[q] >= k ? scores[(size_t)q * k + k - 1] : 0.0f;
  y[q] = s > 0.0f ? logf(s) : __builtin_nanf("");
}

hipError_t launch_labels(uint32_t nq, uint32_t k, const float *scores, const uint32_t *cnt, float *y, hipStream_t s) {
  hipLaunchKernelGGL(k_labels, dim3((nq + 255) / 256), dim3(256), 0, s, nq, k, scores, cnt, y);
  return hipGetLastError();
}

// thr[q] = ord(tau) with tau = exp(yhat - delta): the inclusive starting
// threshold of the selection. tau not a positive finite number: no threshold
// (thr 0) when it is 0 or NaN, everything filtered out (forcing the fallback)
// when it is +inf. keff[q] = min(k, live): the count the filter must reach.
__global__ void k_threshold(uint32_t nq, const float *__restrict__ yhat, float delta, uint32_t keff,
                            uint32_t *__restrict__ thr, uint32_t *__restrict__ ke) {
  const uint32_t q = blockIdx.x * 256 + threadIdx.x;
  if (q >= nq) return;
  const float tau = expf(yhat[q] - delta);
  uint32_t t = 0;
  if (tau > 0.0f && tau < __builtin_inff()) t = ord_key(tau);
  else if (tau == __builtin_inff()) t = 0xFFFFFFFFu;
  thr[q] = t;
  ke[q] = keff;
}

hipError_t launch_threshold(uint32_t nq, const float *yhat, float delta, uint32_t keff, uint32_t *thr, uint32_t *ke,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_threshold, dim3((nq + 255) / 256), dim3(256), 0, s, nq, yhat, delta, keff, thr, ke);
  return hipGetLastError();
}

}  // namespace snn
