// Instances of the fused per-path kernel: FP32-mixed, standard construction
// (and the basket).
#include "paths_kernel.h"

namespace qcpw {

const void *paths_fn_f32_std(bool owen, bool wide)
{
    if (owen)
        return wide ? reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_STANDARD, true, false, true>)
                    : reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_STANDARD, true, false, false>);
    return wide ? reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_STANDARD, false, false, true>)
                : reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_STANDARD, false, false, false>);
}

}  // namespace qcpw
