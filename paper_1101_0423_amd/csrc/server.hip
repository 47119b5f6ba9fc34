// server.hip -- request serving entry points (dwf_submit / dwf_poll).
#include "dwf_ctx.h"

using namespace dwf;

extern "C" {

int dwf_submit(dwf_ctx* c, const double* b, const dwf_solve_params* p, uint64_t* ticket) {
    (void)c; (void)b; (void)p; (void)ticket;
    return fail(DWF_EINVAL, "request server not available in this build");
}

int dwf_submit_mass(dwf_ctx* c, const double* b, double mq, const dwf_solve_params* p, uint64_t* ticket) {
    (void)c; (void)b; (void)mq; (void)p; (void)ticket;
    return fail(DWF_EINVAL, "request server not available in this build");
}

int dwf_poll(uint64_t ticket, double* x, dwf_solve_stats* st, int timeout_us) {
    (void)ticket; (void)x; (void)st; (void)timeout_us;
    return fail(DWF_ENOTFOUND, "unknown ticket");
}

int dwf_server_stats_get(dwf_server_stats* out, int reset) {
    (void)reset;
    if (!out) return fail(DWF_EINVAL, "NULL out");
    *out = dwf_server_stats{};
    return DWF_OK;
}

}  // extern "C"
