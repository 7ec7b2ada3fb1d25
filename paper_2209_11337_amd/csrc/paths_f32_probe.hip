// Instances of the fused per-path kernel that also record the Sobol
// coordinates they consume (FP32-mixed).  The bridge takes the register
// budget its launch plan was made for (the 80-VGPR instances walk the
// compile-time bridges, paths_f32_probe_narrow.hip); the standard
// construction plans alike for both and records with the wide budget.
#include "paths_kernel.h"

namespace qcpw {

const void *paths_fn_f32_probe(int path, bool owen, bool wide)
{
    if (path == QCPW_PATH_STANDARD)
        return owen ? reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_STANDARD, true, true, true>)
                    : reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_STANDARD, false, true, true>);
    if (!wide) return paths_fn_f32_probe_narrow(owen);
    return owen ? reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_BB, true, true, true>)
                : reinterpret_cast<const void *>(&paths_kernel<true, QCPW_PATH_BB, false, true, true>);
}

}  // namespace qcpw
