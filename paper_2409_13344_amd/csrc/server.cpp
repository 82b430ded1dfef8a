// Continuous-batching request server (placeholder until the serving loop lands).
#include <hip/hip_runtime.h>

#include "appga.h"
#include "appga_impl.h"

using namespace appga;

extern "C" appga_status appga_server_start(appga_ctx *ctx, const appga_server_cfg *cfg,
                                           appga_server **out) {
    clear_error();
    (void)ctx;
    (void)cfg;
    (void)out;
    return fail(APPGA_E_INVALID_ARG, "serving is not available in this build");
}

extern "C" appga_status appga_submit(appga_server *srv, const appga_matrix *mat, const float *g,
                                     const float *gamma, const appga_params *params,
                                     uint64_t *ticket) {
    clear_error();
    (void)srv; (void)mat; (void)g; (void)gamma; (void)params; (void)ticket;
    return fail(APPGA_E_INVALID_ARG, "serving is not available in this build");
}

extern "C" appga_status appga_wait(appga_server *srv, uint64_t ticket, float *f_out,
                                   appga_stats *stats, int32_t timeout_ms) {
    clear_error();
    (void)srv; (void)ticket; (void)f_out; (void)stats; (void)timeout_ms;
    return fail(APPGA_E_INVALID_ARG, "serving is not available in this build");
}

extern "C" appga_status appga_server_stop(appga_server *srv) {
    clear_error();
    (void)srv;
    return fail(APPGA_E_INVALID_ARG, "serving is not available in this build");
}
