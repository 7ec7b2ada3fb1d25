// pca.hip -- principal-component path construction (placeholder until the
// matrix-core kernel lands).
#include <hip/hip_runtime.h>

#include "qcpw_host.h"

namespace qcpw {

qcpw_status enqueue_pca(Context *ctx, const LaunchPlan &lp, hipStream_t stream, const LaunchDesc &ld,
                        const OptDev *d_opts)
{
    (void)ctx; (void)lp; (void)stream; (void)ld; (void)d_opts;
    return fail(QCPW_EINVAL, "PCA path construction is not available in this build");
}

}  // namespace qcpw
