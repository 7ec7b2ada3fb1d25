// Instances of the fused per-path kernel: FP32-mixed, Brownian bridge,
// digital shift.
#include "paths_kernel.h"

namespace qcpw {

const void *paths_fn_f32_bb(bool wide)
{
    return wide ? reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_BB, false, false, true>)
                : reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_BB, false, false, false>);
}

}  // namespace qcpw
