// Host orchestration of the learned k-th-score pre-filter: feature table,
// labelling with the plain search, training with the MLP kernels, calibration
// of the margin delta, and the filtered search with its plain fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <vector>

#include "snn_host.h"
#include "snn_mlp.h"

using namespace snn;

namespace snn {

struct LearnedFilter {
  bool ready = false;
  uint64_t fseed = 0;
  uint32_t k = 10;
  float delta = 0.0f;
  bool table_ok = false;
  uint32_t adam_t = 0;
  DevBuf P, Pb, M, V, G, table;
  DevBuf X, yhat, thr, keff;                                          // search scratch
  DevBuf tX, ty, trow, tyrow, H1, H2, D1, D2, DY, loss, tmpy;        // training scratch
  void release() {
    for (DevBuf *b : {&P, &Pb, &M, &V, &G, &table, &X, &yhat, &thr, &keff, &tX, &ty, &trow, &tyrow, &H1, &H2, &D1,
                      &D2, &DY, &loss, &tmpy})
      b->release();
  }
};

}  // namespace snn

#define HIP_TRY(ix, call, what)                                \
  do {                                                         \
    hipError_t e__ = (call);                                   \
    if (e__ != hipSuccess) return (ix)->hip_fail(e__, what);   \
  } while (0)

static LearnedFilter *filter_of(snn_index *ix) {
  if (!ix->filter) ix->filter = new LearnedFilter();
  return ix->filter;
}

static snn_status ensure_table(snn_index *ix, LearnedFilter *f, uint64_t fseed) {
  if (f->table_ok && f->fseed == fseed) return SNN_OK;
  const uint32_t n = ix->cfg.dim;
  std::vector<uint32_t> t(n);
  const uint64_t s0 = splitmix64_mix(fseed), s1 = splitmix64_mix(fseed + 1);
  for (uint32_t j = 0; j < n; ++j) {
    const uint32_t g = (uint32_t)(splitmix64_mix(s0 ^ (uint64_t)j) % 128u);
    const uint32_t neg = (uint32_t)(splitmix64_mix(s1 ^ (uint64_t)j) >> 63);
    t[j] = g | (neg << 31);
  }
  HIP_TRY(ix, f->table.ensure((size_t)n * 4, ix->stream), "filter table");
  HIP_TRY(ix, hipMemcpyAsync(f->table.p, t.data(), (size_t)n * 4, hipMemcpyHostToDevice, ix->stream), "table copy");
  HIP_TRY(ix, hipStreamSynchronize(ix->stream), "table sync");
  f->fseed = fseed;
  f->table_ok = true;
  return SNN_OK;
}

static snn_status ensure_params(snn_index *ix, LearnedFilter *f) {
  hipStream_t s = ix->stream;
  HIP_TRY(ix, f->P.ensure(kParams * 4, s), "params");
  HIP_TRY(ix, f->Pb.ensure(kParams * 2, s), "params");
  HIP_TRY(ix, f->M.ensure(kParams * 4, s), "params");
  HIP_TRY(ix, f->V.ensure(kParams * 4, s), "params");
  HIP_TRY(ix, f->G.ensure(kParams * 4, s), "params");
  return SNN_OK;
}

static snn_status load_params(snn_index *ix, LearnedFilter *f, const float *host) {
  hipStream_t s = ix->stream;
  snn_status st = ensure_params(ix, f);
  if (st != SNN_OK) return st;
  HIP_TRY(ix, hipMemcpyAsync(f->P.p, host, kParams * 4, hipMemcpyHostToDevice, s), "params copy");
  HIP_TRY(ix, launch_to_bf16((float *)f->P.p, (uint16_t *)f->Pb.p, kParams, s), "bf16");
  HIP_TRY(ix, launch_fill_u32((uint32_t *)f->M.p, 0u, kParams, s), "adam m");
  HIP_TRY(ix, launch_fill_u32((uint32_t *)f->V.p, 0u, kParams, s), "adam v");
  HIP_TRY(ix, hipStreamSynchronize(s), "params sync");
  f->adam_t = 0;
  return SNN_OK;
}

static snn_status features(snn_index *ix, LearnedFilter *f, uint32_t nq, const uint64_t *ptr, const uint32_t *c,
                           const float *v, float *X, hipStream_t s) {
  HIP_TRY(ix, launch_features(nq, ptr, c, v, (const uint32_t *)f->table.p, ix->cfg.dim, X, s), "feature kernel");
  return SNN_OK;
}

extern "C" snn_status snn_filter_set_params(snn_index *ix, const float *params, uint64_t feature_seed, uint32_t k) {
  if (!ix || !params || k == 0 || k > kMaxK) return SNN_E_INVALID;
  LearnedFilter *f = filter_of(ix);
  snn_status st = ensure_table(ix, f, feature_seed);
  if (st != SNN_OK) return st;
  st = load_params(ix, f, params);
  if (st != SNN_OK) return st;
  f->k = k;
  f->ready = true;
  return SNN_OK;
}

extern "C" snn_status snn_filter_get_params(snn_index *ix, float *params) {
  if (!ix || !params) return SNN_E_INVALID;
  LearnedFilter *f = ix->filter;
  if (!f || !f->ready) return ix->fail(SNN_E_INVALID, "filter: no parameters");
  std::vector<uint16_t> b(kParams);
  HIP_TRY(ix, hipStreamSynchronize(ix->stream), "sync");
  HIP_TRY(ix, hipMemcpy(b.data(), f->Pb.p, kParams * 2, hipMemcpyDeviceToHost), "params readback");
  for (int p = 0; p < kParams; ++p) {
    const uint32_t u = (uint32_t)b[p] << 16;
    memcpy(&params[p], &u, 4);
  }
  return SNN_OK;
}

extern "C" snn_status snn_filter_set_delta(snn_index *ix, float delta) {
  if (!ix) return SNN_E_INVALID;
  LearnedFilter *f = filter_of(ix);
  f->delta = delta;
  return SNN_OK;
}

extern "C" snn_status snn_filter_enable(snn_index *ix, int on) {
  if (!ix) return SNN_E_INVALID;
  if (on && (!ix->filter || !ix->filter->ready))
    return ix->fail(SNN_E_INVALID, "filter: no trained filter (call snn_filter_train or snn_filter_set_params)");
  ix->filter_on = on != 0;
  return SNN_OK;
}

extern "C" snn_status snn_filter_features(snn_index *ix, uint32_t nq, const uint64_t *indptr, const uint32_t *coords,
                                          const float *vals, float *out_features) {
  if (!ix || !indptr || !out_features) return SNN_E_INVALID;
  LearnedFilter *f = ix->filter;
  if (!f || !f->table_ok) return ix->fail(SNN_E_INVALID, "filter: no feature table");
  return features(ix, f, nq, indptr, coords, vals, out_features, ix->stream);
}

static snn_status predict(snn_index *ix, LearnedFilter *f, uint32_t nq, const uint64_t *ptr, const uint32_t *c,
                          const float *v, float *yhat, hipStream_t s) {
  HIP_TRY(ix, f->X.ensure((size_t)nq * kFeat * 4, s), "features");
  snn_status st = features(ix, f, nq, ptr, c, v, (float *)f->X.p, s);
  if (st != SNN_OK) return st;
  HIP_TRY(ix,
          launch_mlp_fwd(nq, (float *)f->X.p, nullptr, (uint16_t *)f->Pb.p, yhat, nullptr, 0.0f, nullptr, nullptr,
                         nullptr, nullptr, nullptr, nullptr, s),
          "mlp forward");
  return SNN_OK;
}

extern "C" snn_status snn_filter_predict(snn_index *ix, uint32_t nq, const uint64_t *indptr, const uint32_t *coords,
                                         const float *vals, float *out_yhat) {
  if (!ix || !indptr || !out_yhat) return SNN_E_INVALID;
  LearnedFilter *f = ix->filter;
  if (!f || !f->ready) return ix->fail(SNN_E_INVALID, "filter: not trained");
  return predict(ix, f, nq, indptr, coords, vals, out_yhat, ix->stream);
}

// ---------------------------------------------------------------------------
// gradient of the MSE on a given batch (checks the training kernels)
// ---------------------------------------------------------------------------
static snn_status ensure_train_bufs(snn_index *ix, LearnedFilter *f, uint32_t B) {
  hipStream_t s = ix->stream;
  HIP_TRY(ix, f->H1.ensure((size_t)B * kHid * 4, s), "act");
  HIP_TRY(ix, f->H2.ensure((size_t)B * kHid * 4, s), "act");
  HIP_TRY(ix, f->D1.ensure((size_t)B * kHid * 4, s), "act");
  HIP_TRY(ix, f->D2.ensure((size_t)B * kHid * 4, s), "act");
  HIP_TRY(ix, f->DY.ensure((size_t)B * 4, s), "act");
  HIP_TRY(ix, f->tmpy.ensure((size_t)B * 4, s), "act");
  HIP_TRY(ix, f->loss.ensure(256, s), "loss");
  return SNN_OK;
}

extern "C" snn_status snn_mlp_loss_grad(snn_index *ix, uint32_t B, const float *X, const float *y, float *grad,
                                        float *loss) {
  if (!ix || !X || !y || !grad || B == 0) return SNN_E_INVALID;
  LearnedFilter *f = ix->filter;
  if (!f || !f->ready) return ix->fail(SNN_E_INVALID, "filter: no parameters");
  hipStream_t s = ix->stream;
  snn_status st = ensure_train_bufs(ix, f, B);
  if (st != SNN_OK) return st;
  HIP_TRY(ix, launch_fill_u32((uint32_t *)f->loss.p, 0u, 1, s), "loss fill");
  HIP_TRY(ix,
          launch_mlp_fwd(B, X, nullptr, (uint16_t *)f->Pb.p, (float *)f->tmpy.p, y, 1.0f / (float)B, (float *)f->H1.p,
                         (float *)f->H2.p, (float *)f->D1.p, (float *)f->D2.p, (float *)f->DY.p, (float *)f->loss.p, s),
          "mlp forward");
  HIP_TRY(ix,
          launch_mlp_wgrad(B, X, nullptr, (float *)f->H1.p, (float *)f->H2.p, (float *)f->D1.p, (float *)f->D2.p,
                           (float *)f->DY.p, grad, s),
          "mlp wgrad");
  float l = 0;
  HIP_TRY(ix, hipMemcpyAsync(&l, f->loss.p, 4, hipMemcpyDeviceToHost, s), "loss readback");
  HIP_TRY(ix, hipStreamSynchronize(s), "sync");
  if (loss) *loss = l / (float)B;
  return SNN_OK;
}

// ---------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------
extern "C" snn_status snn_filter_train(snn_index *ix, uint32_t nq, const uint64_t *indptr, uint64_t total,
                                       const uint32_t *coords, const float *vals, const snn_filter_params *pr,
                                       snn_filter_report *rep) {
  if (!ix || !pr || !indptr || nq == 0) return SNN_E_INVALID;
  if (pr->k == 0 || pr->k > kMaxK || pr->epochs == 0 || pr->batch == 0 || pr->batch > 65536 || !(pr->lr > 0) ||
      !(pr->holdout > 0 && pr->holdout < 1) || !(pr->target_fallback > 0 && pr->target_fallback < 1))
    return ix->fail(SNN_E_INVALID, "filter_train: bad parameters");
  LearnedFilter *f = filter_of(ix);
  hipStream_t s = ix->stream;
  snn_status st = ensure_table(ix, f, pr->feature_seed);
  if (st != SNN_OK) return st;
  snn_filter_report R{};
  hipEvent_t ea, eb;
  HIP_TRY(ix, hipEventCreate(&ea), "event");
  HIP_TRY(ix, hipEventCreate(&eb), "event");

  // 1. features of every training query
  HIP_TRY(ix, f->tX.ensure((size_t)nq * kFeat * 4, s), "train features");
  st = features(ix, f, nq, indptr, coords, vals, (float *)f->tX.p, s);
  if (st != SNN_OK) return st;

  // 2. labels ln(s_k) from the plain method, in chunks
  const uint32_t k = pr->k;
  // queries per labelling search: the tile candidates of a chunk (tiles x
  // min(k, tile) x 8 bytes per query) stay within about 2 GiB
  const uint64_t tile_docs = (uint64_t)kBlock * (uint64_t)std::max(16, ix->tune.R_batch);
  const uint64_t tiles = std::max<uint64_t>(1, (ix->next_fresh + tile_docs - 1) / tile_docs);
  const uint64_t per_query = tiles * std::min<uint64_t>(k, tile_docs) * 8;
  const uint32_t chunk = (uint32_t)std::max<uint64_t>(256, std::min<uint64_t>(16384, (2ull << 30) / per_query));
  DevBuf lab;
  HIP_TRY(ix, lab.ensure((size_t)chunk * k * 8 + (size_t)chunk * 4 + 256, s), "label buffers");
  HIP_TRY(ix, f->ty.ensure((size_t)nq * 4, s), "labels");
  uint32_t *lid = (uint32_t *)lab.p;
  float *lsc = (float *)(lid + (size_t)chunk * k);
  uint32_t *lcnt = (uint32_t *)(lsc + (size_t)chunk * k);
  HIP_TRY(ix, hipEventRecord(ea, s), "event");
  for (uint32_t q0 = 0; q0 < nq; q0 += chunk) {
    const uint32_t nc = std::min(chunk, nq - q0);
    st = ix->run_search(nc, indptr + q0, total, coords, vals, k, SNN_MODE_BATCHED, lid, lsc, lcnt, s, SearchOpts{});
    if (st != SNN_OK) return st;
    HIP_TRY(ix, launch_labels(nc, k, lsc, lcnt, (float *)f->ty.p + q0, s), "labels");
  }
  HIP_TRY(ix, hipEventRecord(eb, s), "event");
  std::vector<float> y(nq);
  HIP_TRY(ix, hipMemcpyAsync(y.data(), f->ty.p, (size_t)nq * 4, hipMemcpyDeviceToHost, s), "labels readback");
  HIP_TRY(ix, hipStreamSynchronize(s), "sync");
  (void)hipEventElapsedTime(&R.label_ms, ea, eb);
  lab.release();

  // 3. split labelled queries into train / holdout
  std::vector<uint32_t> labelled;
  for (uint32_t q = 0; q < nq; ++q)
    if (std::isfinite(y[q])) labelled.push_back(q);
  R.n_unlabelled = nq - (uint32_t)labelled.size();
  std::mt19937_64 rng(pr->seed);
  std::shuffle(labelled.begin(), labelled.end(), rng);
  const uint32_t nh = std::max<uint32_t>(1, (uint32_t)(labelled.size() * pr->holdout));
  if (labelled.size() < nh + 16) return ix->fail(SNN_E_INVALID, "filter_train: only %zu labelled queries", labelled.size());
  std::vector<uint32_t> hold(labelled.begin(), labelled.begin() + nh), train(labelled.begin() + nh, labelled.end());
  R.n_train = (uint32_t)train.size();
  R.n_holdout = nh;

  // 4. initialise: He-uniform weights, zero biases, b3 = mean label
  std::vector<float> P(kParams, 0.0f);
  auto init = [&](int off, int fan_out, int fan_in) {
    const double a = std::sqrt(6.0 / fan_in);
    std::uniform_real_distribution<double> U(-a, a);
    for (int i = 0; i < fan_out * fan_in; ++i) P[off + i] = (float)U(rng);
  };
  init(kOffW1, kHid, kFeat);
  init(kOffW2, kHid, kHid);
  init(kOffW3, 1, kHid);
  double my = 0;
  for (uint32_t q : train) my += y[q];
  P[kOffB3] = (float)(my / train.size());
  for (int i = 0; i < kHid; ++i) P[kOffW3 + i] *= 0.1f;
  st = load_params(ix, f, P.data());
  if (st != SNN_OK) return st;
  f->k = k;
  f->ready = true;

  // 5. minibatch Adam
  const uint32_t B = pr->batch;
  st = ensure_train_bufs(ix, f, B);
  if (st != SNN_OK) return st;
  HIP_TRY(ix, f->trow.ensure((size_t)train.size() * 4, s), "rows");
  HIP_TRY(ix, f->tyrow.ensure((size_t)train.size() * 4, s), "row labels");
  std::vector<float> yrow(train.size());
  HIP_TRY(ix, hipEventRecord(ea, s), "event");
  uint32_t steps = 0;
  for (uint32_t ep = 0; ep < pr->epochs; ++ep) {
    std::shuffle(train.begin(), train.end(), rng);
    for (size_t i = 0; i < train.size(); ++i) yrow[i] = y[train[i]];
    HIP_TRY(ix, hipStreamSynchronize(s), "sync");  // previous epoch's kernels read trow / tyrow
    HIP_TRY(ix, hipMemcpy(f->trow.p, train.data(), train.size() * 4, hipMemcpyHostToDevice), "rows copy");
    HIP_TRY(ix, hipMemcpy(f->tyrow.p, yrow.data(), yrow.size() * 4, hipMemcpyHostToDevice), "labels copy");
    for (size_t b0 = 0; b0 < train.size(); b0 += B) {
      const uint32_t nb = (uint32_t)std::min<size_t>(B, train.size() - b0);
      const uint32_t *rows = (const uint32_t *)f->trow.p + b0;
      HIP_TRY(ix,
              launch_mlp_fwd(nb, (float *)f->tX.p, rows, (uint16_t *)f->Pb.p, (float *)f->tmpy.p,
                             (float *)f->tyrow.p + b0, 1.0f / (float)nb, (float *)f->H1.p, (float *)f->H2.p,
                             (float *)f->D1.p, (float *)f->D2.p, (float *)f->DY.p, (float *)f->loss.p, s),
              "mlp forward");
      HIP_TRY(ix,
              launch_mlp_wgrad(nb, (float *)f->tX.p, rows, (float *)f->H1.p, (float *)f->H2.p, (float *)f->D1.p,
                               (float *)f->D2.p, (float *)f->DY.p, (float *)f->G.p, s),
              "mlp wgrad");
      ++f->adam_t;
      const float b1 = 0.9f, b2 = 0.999f;
      const float c1 = 1.0f - std::pow(b1, (float)f->adam_t), c2 = 1.0f - std::pow(b2, (float)f->adam_t);
      HIP_TRY(ix,
              launch_adam((float *)f->P.p, (uint16_t *)f->Pb.p, (float *)f->G.p, (float *)f->M.p, (float *)f->V.p,
                          pr->lr, b1, b2, 1e-8f, c1, c2, s),
              "adam");
      ++steps;
    }
  }
  HIP_TRY(ix, hipEventRecord(eb, s), "event");
  HIP_TRY(ix, hipStreamSynchronize(s), "sync");
  (void)hipEventElapsedTime(&R.train_ms, ea, eb);
  R.steps = steps;

  // 6. calibrate delta on the holdout; report errors
  HIP_TRY(ix, f->yhat.ensure((size_t)nq * 4, s), "yhat");
  HIP_TRY(ix,
          launch_mlp_fwd(nq, (float *)f->tX.p, nullptr, (uint16_t *)f->Pb.p, (float *)f->yhat.p, nullptr, 0.0f,
                         nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, s),
          "mlp forward");
  std::vector<float> yh(nq);
  HIP_TRY(ix, hipMemcpyAsync(yh.data(), f->yhat.p, (size_t)nq * 4, hipMemcpyDeviceToHost, s), "yhat readback");
  HIP_TRY(ix, hipStreamSynchronize(s), "sync");
  double se = 0;
  for (uint32_t q : train) se += (double)(yh[q] - y[q]) * (yh[q] - y[q]);
  R.train_mse = (float)(se / train.size());
  std::vector<float> res;
  se = 0;
  for (uint32_t q : hold) {
    res.push_back(yh[q] - y[q]);
    se += (double)(yh[q] - y[q]) * (yh[q] - y[q]);
  }
  R.holdout_mse = (float)(se / hold.size());
  std::sort(res.begin(), res.end());
  size_t qi = (size_t)std::ceil((1.0 - pr->target_fallback) * res.size());
  if (qi >= res.size()) qi = res.size() - 1;
  // fallback happens when tau = exp(yhat - delta) > s_k, i.e. yhat - y > delta
  f->delta = res[qi];
  size_t over = 0;
  for (float r : res) over += r > f->delta;
  R.delta = f->delta;
  R.holdout_fallback = (float)over / (float)res.size();
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  if (rep) *rep = R;
  return SNN_OK;
}

// ---------------------------------------------------------------------------
// filtered search with fallback
// ---------------------------------------------------------------------------
// k: the selection's k (k' when re-ranking, then rerank_k results are kept)
snn_status snn_index::search_learned(uint32_t nq, const uint64_t *d_ptr, uint64_t total, const uint32_t *d_c,
                                     const float *d_v, uint32_t k, uint32_t max_coords, uint32_t rerank_k,
                                     uint32_t hash_cap, uint32_t *d_ids, float *d_sc, uint32_t *d_cnt,
                                     hipStream_t s) {
  LearnedFilter *f = filter;
  if (!f || !f->ready) return fail(SNN_E_INVALID, "search: no trained filter (call snn_filter_train first)");
  HIP_TRY(this, f->X.ensure((size_t)nq * kFeat * 4, s), "features");
  HIP_TRY(this, f->yhat.ensure((size_t)nq * 4, s), "yhat");
  HIP_TRY(this, f->thr.ensure((size_t)nq * 4, s), "thr");
  HIP_TRY(this, f->keff.ensure((size_t)nq * 4, s), "keff");
  LearnedPass lp;
  lp.table = (const uint32_t *)f->table.p;
  lp.Pb = (const uint16_t *)f->Pb.p;
  lp.X = (float *)f->X.p;
  lp.yhat = (float *)f->yhat.p;
  lp.thr = (uint32_t *)f->thr.p;
  lp.keff = (uint32_t *)f->keff.p;
  lp.delta = f->delta;
  lp.keff_value = (uint32_t)std::min<size_t>(k, live);
  lp.dim = cfg.dim;
  SearchOpts o;
  o.learned = &lp;
  o.max_coords = max_coords;
  o.rerank_k = rerank_k;
  o.hash_cap = hash_cap;
  return run_search(nq, d_ptr, total, d_c, d_v, k, SNN_MODE_LEARNED, d_ids, d_sc, d_cnt, s, o);
}

void snn_filter_release(snn_index *ix) {
  if (ix->filter) {
    ix->filter->release();
    delete ix->filter;
    ix->filter = nullptr;
  }
}
