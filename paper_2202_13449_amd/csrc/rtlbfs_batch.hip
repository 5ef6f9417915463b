// rtlbfs_batch.hip -- batched many-domain stepping (placeholder until the
// work-list kernel lands: every entry point reports RTLBFS_EUNSUPPORTED).
#include <hip/hip_runtime.h>

#include "../../include/rtlbfs.h"

extern "C" {
size_t rtlbfs_batch_workspace_bytes(int, const rtlbfs_mesh *, const rtlbfs_opts *) { return 0; }
int rtlbfs_batch_create(int, const rtlbfs_mesh *, const double *, const double *, double, const rtlbfs_bc *,
                        const rtlbfs_opts *, void *, void *, size_t, rtlbfs_batch_t *out) {
    if (out) *out = nullptr;
    return RTLBFS_EUNSUPPORTED;
}
int rtlbfs_batch_step(rtlbfs_batch_t, int64_t) { return RTLBFS_EUNSUPPORTED; }
int rtlbfs_batch_nusselt(rtlbfs_batch_t, int, rtlbfs_nu *) { return RTLBFS_EUNSUPPORTED; }
int rtlbfs_batch_residual(rtlbfs_batch_t, int, double *, double *) { return RTLBFS_EUNSUPPORTED; }
int rtlbfs_batch_get_field(rtlbfs_batch_t, int, int, double *, size_t) { return RTLBFS_EUNSUPPORTED; }
int rtlbfs_batch_get_info(rtlbfs_batch_t, int, rtlbfs_info *) { return RTLBFS_EUNSUPPORTED; }
int rtlbfs_batch_sync(rtlbfs_batch_t) { return RTLBFS_EUNSUPPORTED; }
int rtlbfs_batch_destroy(rtlbfs_batch_t) { return RTLBFS_OK; }
}
