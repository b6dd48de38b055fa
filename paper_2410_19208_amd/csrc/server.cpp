// Placeholder request server (replaced by the continuous-batching server).
#include "psdproj.h"
extern "C" {
psdproj_status psdproj_server_create(size_t, int32_t, psdproj_server_t* out) { if (out) *out = nullptr; return PSDPROJ_E_INVALID; }
psdproj_status psdproj_submit(psdproj_server_t, const psdproj_desc*, const void*, int64_t, void*, int64_t, uint64_t*) { return PSDPROJ_E_INVALID; }
psdproj_status psdproj_poll(psdproj_server_t, uint64_t, psdproj_result*) { return PSDPROJ_E_INVALID; }
psdproj_status psdproj_wait(psdproj_server_t, uint64_t, psdproj_result*, double) { return PSDPROJ_E_INVALID; }
psdproj_status psdproj_server_times(psdproj_server_t, uint64_t, double*, double*, double*) { return PSDPROJ_E_INVALID; }
void psdproj_server_destroy(psdproj_server_t) {}
}
