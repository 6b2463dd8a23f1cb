// Shapes and parameter layout of the learned filter's MLP (256 -> 128 -> 128 -> 1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snn {

constexpr int kFeat = 256;
constexpr int kHid = 128;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHid * kFeat;  // 32768
constexpr int kOffW2 = kOffB1 + kHid;          // 32896
constexpr int kOffB2 = kOffW2 + kHid * kHid;   // 49280
constexpr int kOffW3 = kOffB2 + kHid;          // 49408
constexpr int kOffB3 = kOffW3 + kHid;          // 49536
constexpr int kParams = kOffB3 + 1;            // 49537

hipError_t launch_features(uint32_t nq, const uint64_t *qptr, const uint32_t *coords, const float *vals,
                           const uint32_t *table, uint32_t dim, float *X, hipStream_t s);
hipError_t launch_mlp_fwd(uint32_t B, const float *X, const uint32_t *rows, const uint16_t *Pb, float *yhat,
                          const float *y, float inv_btotal, float *H1, float *H2, float *D1, float *D2, float *DY,
                          float *loss, hipStream_t s);
hipError_t launch_mlp_wgrad(uint32_t B, const float *X, const uint32_t *rows, const float *H1, const float *H2,
                            const float *D1, const float *D2, const float *DY, float *G, hipStream_t s);
hipError_t launch_adam(float *P, uint16_t *Pb, const float *G, float *M, float *V, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);
hipError_t launch_to_bf16(const float *P, uint16_t *Pb, uint32_t n, hipStream_t s);
hipError_t launch_labels(uint32_t nq, uint32_t k, const float *scores, const uint32_t *cnt, float *y, hipStream_t s);
hipError_t launch_threshold(uint32_t nq, const float *yhat, float delta, uint32_t keff, uint32_t *thr, uint32_t *ke,
                            hipStream_t s);

}  // namespace snn
