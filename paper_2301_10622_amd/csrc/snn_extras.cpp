// Parts of snn_index that the learned filter and the autotuner fill in.
#include "snn_host.h"

void snn_index::tune_init() {
  tune = snn::Tune{};
}

void snn_index::release_extras() {
  graphs.clear();
  for (hipEvent_t e : prof_events) (void)hipEventDestroy(e);
  for (hipEvent_t e : prof_pool) (void)hipEventDestroy(e);
  prof_events.clear();
  prof_pool.clear();
}

snn_status snn_index::search_learned(uint32_t, const uint64_t *, uint64_t, const uint32_t *, const float *, uint32_t,
                                     uint32_t *, float *, uint32_t *, hipStream_t) {
  return fail(SNN_E_INVALID, "search: no trained filter (call snn_filter_train first)");
}
