// Continuous-batching request server (placeholder until the scheduler lands).
#include "runtime.h"

using namespace bfi;

extern "C" {

bfi_status bfi_server_create(bfi_context *, const bfi_server_config *, bfi_server **)
{
    return fail(BFI_EUNSUPPORTED, "server not built yet");
}
bfi_status bfi_server_submit(bfi_server *, const bfi_request *, uint64_t *)
{
    return fail(BFI_EUNSUPPORTED, "server not built yet");
}
bfi_status bfi_server_poll(bfi_server *, uint64_t, bfi_result *, int32_t *, double *)
{
    return fail(BFI_EUNSUPPORTED, "server not built yet");
}
bfi_status bfi_server_wait(bfi_server *, uint64_t, double, bfi_result *, int32_t *, double *)
{
    return fail(BFI_EUNSUPPORTED, "server not built yet");
}
bfi_status bfi_server_cancel(bfi_server *, uint64_t)
{
    return fail(BFI_EUNSUPPORTED, "server not built yet");
}
bfi_status bfi_server_stats_get(bfi_server *, bfi_server_stats *)
{
    return fail(BFI_EUNSUPPORTED, "server not built yet");
}
bfi_status bfi_server_destroy(bfi_server *) { return BFI_OK; }

}  // extern "C"
