// placeholder definitions (replaced by the adjoint and batching translation units)
#include "teno.h"
extern "C" {
teno_status teno_batch_create(const teno_grid *, int32_t, const teno_opts *, void *, teno_batch **) { return TENO_E_UNSUPPORTED; }
teno_status teno_batch_destroy(teno_batch *) { return TENO_E_UNSUPPORTED; }
size_t teno_batch_total_elems(const teno_batch *) { return 0; }
size_t teno_batch_offset(const teno_batch *, int32_t) { return 0; }
teno_status teno_batch_run(teno_batch *, void *, int32_t, int32_t) { return TENO_E_UNSUPPORTED; }
teno_status teno_batch_poll(teno_batch *) { return TENO_E_UNSUPPORTED; }
}
