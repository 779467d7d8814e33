// server.cpp -- continuous-batching request loop (entry points; loop implementation follows).
#include "runtime.hpp"

extern "C" dpcs_status dpcs_server_create(dpcs_context ctx, size_t, int32_t, dpcs_server* out) {
    if (out) *out = nullptr;
    return dpcs::fail(ctx, DPCS_E_UNSUPPORTED, "server not available in this build");
}
extern "C" dpcs_status dpcs_server_submit(dpcs_server, const dpcs_request*) { return DPCS_E_UNSUPPORTED; }
extern "C" int32_t dpcs_server_poll(dpcs_server, uint64_t*, int32_t*, double*, int32_t) { return 0; }
extern "C" dpcs_status dpcs_server_stats(dpcs_server, int64_t*) { return DPCS_E_UNSUPPORTED; }
extern "C" dpcs_status dpcs_server_destroy(dpcs_server) { return DPCS_E_UNSUPPORTED; }
