// Learned scheduler (network inference and training). Placeholder hooks until
// the network kernels are in place.
#include "daic_internal.h"

namespace daic {
daic_status learned_prepare(daic_problem*, const daic_sched_model*, hipStream_t) {
  return fail(DAIC_E_UNSUPPORTED, "learned scheduler not available");
}
daic_status learned_scores(daic_problem*, const daic_sched_model*, hipStream_t, const float**) {
  return fail(DAIC_E_UNSUPPORTED, "learned scheduler not available");
}
void learned_after_round(daic_problem*, hipStream_t) {}
}  // namespace daic
