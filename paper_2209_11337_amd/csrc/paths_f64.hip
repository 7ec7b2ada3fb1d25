// Instances of the fused per-path kernel: plain FP64.
#include "paths_kernel.h"

namespace qcpw {

template <int PATHK>
static const void *f64_fn(bool owen, bool probe)
{
    if (probe)
        return owen ? reinterpret_cast<const void *>(&paths_kernel<false, PATHK, true, true, false>)
                    : reinterpret_cast<const void *>(&paths_kernel<false, PATHK, false, true, false>);
    return owen ? reinterpret_cast<const void *>(&paths_kernel<false, PATHK, true, false, false>)
                : reinterpret_cast<const void *>(&paths_kernel<false, PATHK, false, false, false>);
}

const void *paths_fn_f64(int path, bool owen, bool probe)
{
    return path == QCPW_PATH_STANDARD ? f64_fn<QCPW_PATH_STANDARD>(owen, probe) : f64_fn<QCPW_PATH_BB>(owen, probe);
}

}  // namespace qcpw
