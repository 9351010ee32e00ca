// placeholder translation unit, replaced by the batch engine
#include "s4_internal.h"
using namespace s4;
extern "C" {
int s4_index_build(const uint8_t *, const uint64_t *, uint64_t, void *, s4_index **) { return fail(S4_EINVAL, "index not built"); }
int s4_index_free(s4_index *) { return S4_OK; }
int s4_index_lengths(const s4_index *, uint64_t *) { return fail(S4_EINVAL, "index not built"); }
int s4_index_info(const s4_index *, uint64_t *, uint64_t *, uint64_t *, uint64_t *) { return fail(S4_EINVAL, "index not built"); }
int s4_index_list(const s4_index *, uint64_t, s4_list **) { return fail(S4_EINVAL, "index not built"); }
int s4_batch_plan(const s4_index *, const uint32_t *, const uint64_t *, uint64_t, void *, s4_batch **) { return fail(S4_EINVAL, "batch not built"); }
int s4_batch_free(s4_batch *) { return S4_OK; }
uint64_t s4_batch_results_bound(const s4_batch *) { return 0; }
int s4_batch_run(s4_batch *, uint64_t *, uint64_t *, uint32_t *, uint64_t, int, void *) { return fail(S4_EINVAL, "batch not built"); }
int s4_batch_query_ticks(const s4_batch *, uint64_t *, void *) { return fail(S4_EINVAL, "batch not built"); }
int s4_batch_autotune(s4_batch *, uint64_t *, uint64_t *, uint32_t *, uint64_t, int, void *, s4_tuning *, double *) { return fail(S4_EINVAL, "batch not built"); }
}
