// Autotuner for the search schedule: times candidate tile sizes and launch
// shapes on a caller-supplied batch and keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "snn_host.h"

using namespace snn;

namespace {

struct Cand {
  int R;
  bool persistent;
  uint32_t grid;
  int qgroup;
};

}  // namespace

extern "C" snn_status snn_get_schedule(snn_index *ix, snn_schedule *out) {
  if (!ix || !out) return SNN_E_INVALID;
  out->R_plain = ix->tune.R_plain;
  out->R_batch = ix->tune.R_batch;
  out->grid = ix->tune.grid;
  out->persistent = ix->tune.persistent ? 1u : 0u;
  out->best_ms = ix->tune_best_ms;
  out->default_ms = ix->tune_default_ms;
  out->tried = ix->tune_tried;
  out->qgroup = (uint32_t)ix->tune.qgroup;
  return SNN_OK;
}

static bool valid_R(int R) { return R == 16 || R == 32 || R == 64; }

// the (R, qgroup) pairs the batched kernels are built for
static bool valid_batch(int R, uint32_t Q) {
  return (Q == 1 && valid_R(R)) || (Q == 2 && (R == 8 || R == 16)) || (Q == 3 && R == 16) || (Q == 4 && R == 8);
}

extern "C" snn_status snn_set_schedule(snn_index *ix, const snn_schedule *in) {
  if (!ix || !in) return SNN_E_INVALID;
  if (!valid_R(in->R_plain) || !valid_batch(in->R_batch, in->qgroup) || in->grid == 0 || in->grid > (1u << 20) ||
      (in->qgroup > 1 && ix->cfg.h != 1))
    return ix->fail(SNN_E_INVALID, "schedule: invalid (R_batch, qgroup) or grid (qgroup > 1 needs h = 1)");
  ix->tune.R_plain = in->R_plain;
  ix->tune.R_batch = in->R_batch;
  ix->tune.qgroup = (int)in->qgroup;
  ix->tune.grid = in->grid;
  ix->tune.persistent = in->persistent != 0;
  return SNN_OK;
}

// time one batched pass (eager launch, events around the whole pass), ms
static snn_status time_pass(snn_index *ix, uint32_t nq, const uint64_t *ptr, uint64_t total, const uint32_t *c,
                            const float *v, uint32_t k, uint32_t *ids, float *sc, uint32_t *cnt, hipStream_t s,
                            int reps, float &ms_out) {
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return ix->fail(SNN_E_DEVICE, "event");
  snn_status st = ix->run_search(nq, ptr, total, c, v, k, SNN_MODE_BATCHED, ids, sc, cnt, s, SearchOpts{});  // warm-up
  float best = 1e30f;
  for (int r = 0; st == SNN_OK && r < reps; ++r) {
    (void)hipEventRecord(a, s);
    st = ix->run_search(nq, ptr, total, c, v, k, SNN_MODE_BATCHED, ids, sc, cnt, s, SearchOpts{});
    (void)hipEventRecord(b, s);
    if (st != SNN_OK) break;
    if (hipEventSynchronize(b) != hipSuccess) {
      st = ix->fail(SNN_E_DEVICE, "autotune sync");
      break;
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    best = std::min(best, ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  ms_out = best;
  return st;
}

extern "C" snn_status snn_autotune(snn_index *ix, uint32_t nq, const uint64_t *indptr, uint64_t total,
                                   const uint32_t *coords, const float *vals, uint32_t k, snn_schedule *out) {
  if (!ix) return SNN_E_INVALID;
  if (nq == 0 || k == 0 || k > kMaxK || !indptr) return ix->fail(SNN_E_INVALID, "autotune: bad arguments");
  hipStream_t s = ix->stream;
  DevBuf outb;
  hipError_t e = outb.ensure((size_t)nq * k * 8 + (size_t)nq * 4 + 256, s);
  if (e != hipSuccess) return ix->hip_fail(e, "autotune buffers");
  uint32_t *ids = (uint32_t *)outb.p;
  float *sc = (float *)(ids + (size_t)nq * k);
  uint32_t *cnt = (uint32_t *)(sc + (size_t)nq * k);
  const Tune saved = ix->tune;
  const bool saved_graph = ix->use_graphs;
  const bool saved_prof = ix->prof_on;
  ix->use_graphs = false;
  ix->prof_on = false;
  std::vector<Cand> cands;
  for (int R : {16, 32, 64}) {
    for (uint32_t g : {1024u, 2048u, 4096u}) cands.push_back({R, true, g, 1});
    cands.push_back({R, false, 0u, 1});
  }
  if (ix->cfg.h == 1)
    for (auto rq : {std::make_pair(16, 2), std::make_pair(16, 3), std::make_pair(8, 4)}) {
      for (uint32_t g : {2048u, 4096u}) cands.push_back({rq.first, true, g, rq.second});
      cands.push_back({rq.first, false, 0u, rq.second});
    }
  float def_ms = 0, best_ms = 1e30f;
  Cand best = {saved.R_batch, saved.persistent, saved.grid, saved.qgroup};
  snn_status st = time_pass(ix, nq, indptr, total, coords, vals, k, ids, sc, cnt, s, 2, def_ms);
  uint32_t tried = 0;
  for (const Cand &c : cands) {
    if (st != SNN_OK) break;
    ix->tune.R_batch = c.R;
    ix->tune.qgroup = c.qgroup;
    ix->tune.persistent = c.persistent;
    ix->tune.grid = c.persistent ? c.grid : saved.grid;
    float ms = 0;
    st = time_pass(ix, nq, indptr, total, coords, vals, k, ids, sc, cnt, s, 2, ms);
    ++tried;
    if (st == SNN_OK && ms < best_ms) {
      best_ms = ms;
      best = {c.R, c.persistent, c.persistent ? c.grid : saved.grid, c.qgroup};
    }
  }
  // plain (one query at a time): the tile size sets how many workgroups one query fills
  float best_plain = 1e30f;
  int best_plain_R = saved.R_plain;
  const uint32_t nqp = std::min<uint32_t>(nq, 32);
  for (int R : {16, 32, 64}) {
    if (st != SNN_OK) break;
    ix->tune.R_plain = R;
    hipEvent_t a = nullptr, b = nullptr;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    st = ix->run_search(nqp, indptr, total, coords, vals, k, SNN_MODE_PLAIN, ids, sc, cnt, s, SearchOpts{});
    (void)hipEventRecord(a, s);
    if (st == SNN_OK) st = ix->run_search(nqp, indptr, total, coords, vals, k, SNN_MODE_PLAIN, ids, sc, cnt, s, SearchOpts{});
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    ++tried;
    if (st == SNN_OK && ms < best_plain) {
      best_plain = ms;
      best_plain_R = R;
    }
  }
  (void)hipStreamSynchronize(s);
  outb.release();
  ix->use_graphs = saved_graph;
  ix->prof_on = saved_prof;
  if (st != SNN_OK) {
    ix->tune = saved;
    return st;
  }
  ix->tune.R_batch = best.R;
  ix->tune.qgroup = best.qgroup;
  ix->tune.persistent = best.persistent;
  ix->tune.grid = best.grid;
  ix->tune.R_plain = best_plain_R;
  ix->tune_best_ms = best_ms;
  ix->tune_default_ms = def_ms;
  ix->tune_tried = tried;
  ix->graphs.clear();
  return snn_get_schedule(ix, out ? out : &ix->last_sched);
}
