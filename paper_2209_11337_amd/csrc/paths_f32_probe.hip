// Instances of the fused per-path kernel that also record the Sobol
// coordinates they consume (FP32-mixed, wide register budget).
#include "paths_kernel.h"

namespace qcpw {

const void *paths_fn_f32_probe(int path, bool owen)
{
    if (path == QCPW_PATH_STANDARD)
        return owen ? reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_STANDARD, true, true, true>)
                    : reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_STANDARD, false, true, true>);
    return owen ? reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_BB, true, true, true>)
                : reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_BB, false, true, true>);
}

}  // namespace qcpw
