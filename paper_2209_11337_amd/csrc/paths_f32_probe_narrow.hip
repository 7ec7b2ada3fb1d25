// Coordinate-recording instances of the fused per-path kernel for bridge
// launches planned for the 80-VGPR budget (FP32-mixed): they walk the
// compile-time bridges where the plan assigns them.
#include "paths_kernel.h"

namespace qcpw {

const void *paths_fn_f32_probe_narrow(bool owen)
{
    return owen ? reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_BB, true, true, false>)
                : reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_BB, false, true, false>);
}

}  // namespace qcpw
