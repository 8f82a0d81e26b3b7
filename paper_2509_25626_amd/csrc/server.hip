// Continuous-batching render server (placeholder entry points; the batched
// implementation replaces these).
#include "runtime_internal.h"

using namespace cds;

extern "C" {

cds_status cds_server_create(cds_ctx*, const cds_server_opts*, cds_server** out) {
    if (out) *out = nullptr;
    return fail(CDS_ERR_INVALID_ARG, "server not available in this build");
}
cds_status cds_server_add_scene(cds_server*, const cds_scene*, int32_t*) {
    return fail(CDS_ERR_INVALID_ARG, "server not available in this build");
}
cds_status cds_server_submit(cds_server*, int32_t, const cds_camera*, float*, uint64_t*) {
    return fail(CDS_ERR_INVALID_ARG, "server not available in this build");
}
cds_status cds_server_poll(cds_server*, uint64_t, int32_t*, double*) {
    return fail(CDS_ERR_INVALID_ARG, "server not available in this build");
}
cds_status cds_server_drain(cds_server*) { return fail(CDS_ERR_INVALID_ARG, "server not available in this build"); }
cds_status cds_server_get_stats(cds_server*, cds_server_stats*) {
    return fail(CDS_ERR_INVALID_ARG, "server not available in this build");
}
void cds_server_destroy(cds_server*) {}

}  // extern "C"
