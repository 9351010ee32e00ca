// placeholder translation unit, replaced by the server implementation
#include "s4_internal.h"
using namespace s4;
extern "C" {
int s4_server_create(const s4_index *, const s4_server_config *, s4_server **) { return fail(S4_EINVAL, "server not built"); }
int s4_server_submit(s4_server *, const uint32_t *, uint32_t, uint64_t *) { return fail(S4_EINVAL, "server not built"); }
int s4_server_poll(s4_server *, uint64_t *, uint64_t *, uint64_t *, uint32_t *, uint64_t, uint64_t *, uint32_t, uint32_t *) { return fail(S4_EINVAL, "server not built"); }
int s4_server_stats_get(const s4_server *, s4_server_stats *) { return fail(S4_EINVAL, "server not built"); }
int s4_server_destroy(s4_server *) { return S4_OK; }
}
