// Parts of snn_index that the learned filter and the autotuner fill in.
#include "snn_host.h"

void snn_index::tune_init() {
  tune = snn::Tune{};
}

void snn_index::release_extras() {
  graphs.clear();
  snn_filter_release(this);
  for (hipEvent_t e : prof_events) (void)hipEventDestroy(e);
  for (hipEvent_t e : prof_pool) (void)hipEventDestroy(e);
  prof_events.clear();
  prof_pool.clear();
}

