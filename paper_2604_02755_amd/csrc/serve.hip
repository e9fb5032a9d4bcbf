// Continuous-batching request loop (placeholder until the scheduler lands).
#include "runtime.hpp"

namespace nlth {
void Ctx::ensure_worker() {}
void Ctx::worker_loop() {}
}  // namespace nlth

using namespace nlth;

extern "C" {
int nlth_submit(nlth_ctx*, const nlth_mesh*, const nlth_problem*, nlth_result*, uint64_t*) { return NLTH_EINVAL; }
int nlth_poll(nlth_ctx*, uint64_t, int32_t*) { return NLTH_ENOTFOUND; }
int nlth_wait(nlth_ctx*, uint64_t, double) { return NLTH_ENOTFOUND; }
int nlth_cancel(nlth_ctx*, uint64_t) { return NLTH_ENOTFOUND; }
}
