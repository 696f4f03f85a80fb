// Continuous-batching request server (pe_submit / pe_wait / pe_cancel).
#include "pe_runtime.h"

using namespace pe;

namespace pe {
void server_shutdown(pe_ctx) {}
}  // namespace pe

extern "C" {
pe_status pe_submit(pe_ctx, pe_scene, const pe_solve_desc*, pe_result*, pe_ticket*) {
    return set_error(PE_EUNSUPPORTED, "server not built");
}
pe_status pe_wait(pe_ctx, pe_ticket, int64_t) { return set_error(PE_EUNSUPPORTED, "server not built"); }
pe_status pe_cancel(pe_ctx, pe_ticket) { return set_error(PE_EUNSUPPORTED, "server not built"); }
pe_status pe_server_stats(pe_ctx, double*, int32_t) { return set_error(PE_EUNSUPPORTED, "server not built"); }
}
