// Instances of the fused per-path kernel: FP32-mixed, Brownian bridge,
// nested scrambling.
#include "paths_kernel.h"

namespace qcpw {

const void *paths_fn_f32_bb_owen(bool wide)
{
    return wide ? reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_BB, true, false, true>)
                : reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_BB, true, false, false>);
}

}  // namespace qcpw
