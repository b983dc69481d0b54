// rfi_serve.cpp -- serving runtime of librfimad (continuous batching of
// per-stream blocks with device-resident carry state).
#include <hip/hip_runtime.h>

#include "rfi_runtime.hpp"

extern "C" {

int rfi_server_create(const rfi_server_config*, rfi_server** out)
{
    if (out) *out = nullptr;
    return RFI_ERR_UNSUPPORTED;
}
int rfi_server_add_stream(rfi_server*, uint32_t, int32_t, float, int32_t) { return RFI_ERR_UNSUPPORTED; }
int rfi_server_submit(rfi_server*, uint32_t, const void*, void*, int64_t, rfi_window_stats*, uint64_t*)
{
    return RFI_ERR_UNSUPPORTED;
}
int rfi_server_dispatch(rfi_server*) { return RFI_ERR_UNSUPPORTED; }
int rfi_server_poll(rfi_server*, uint64_t, int32_t*, int64_t*, int64_t*) { return RFI_ERR_UNSUPPORTED; }
int rfi_server_sync(rfi_server*) { return RFI_ERR_UNSUPPORTED; }
int rfi_server_flush(rfi_server*, uint32_t, void*, rfi_window_stats*, int64_t*) { return RFI_ERR_UNSUPPORTED; }
int rfi_server_snapshot(rfi_server*, uint32_t, int64_t*, int32_t*, void*) { return RFI_ERR_UNSUPPORTED; }
int rfi_server_restore(rfi_server*, uint32_t, int64_t, int32_t, const void*) { return RFI_ERR_UNSUPPORTED; }
int rfi_server_counters(const rfi_server*, uint64_t*, uint64_t*, uint64_t*, uint64_t*) { return RFI_ERR_UNSUPPORTED; }
int rfi_server_destroy(rfi_server*) { return RFI_OK; }

}  // extern "C"
