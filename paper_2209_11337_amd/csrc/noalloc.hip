// noalloc.hip -- qmc_cpw_greeks_noalloc: the Greeks call for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// The launch workspace of the fused kernel (option table, unit prefix,
// work-queue heads, per-unit partials, per-replication means, and staged
// host outputs) lives in `scratch`, a fixed device array of
// QCPW_NOALLOC_BYTES that each device holds from the library's load until
// the process ends.  In host code the array's name is only a stand-in for
// it: its device address is looked up once per device with
// hipGetSymbolAddress and only that address is handed to copies and
// kernels.  The queue heads start at zero because they are part of the one
// host-to-device copy that sets up every launch; nothing else must start at
// zero.  Every call on a device shares its array: calls that overlap on one
// device (on different streams, or from several threads) race on it.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>

#include "qcpw_host.h"

namespace qcpw {

static __device__ __align__(256) unsigned char scratch[QCPW_NOALLOC_BYTES];

static std::mutex g_scratch_mu;
static void *g_scratch[64];   // device address of `scratch`, per device ordinal

// Device address of this device's scratch array (device current).
static qcpw_status scratch_address(int device, char **out)
{
    if (device < 0 || device >= 64) return fail(QCPW_EINVAL, "device ordinal out of range for the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(QCPW_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[device] = p;
    }
    *out = (char *)g_scratch[device];
    return QCPW_OK;
}

}  // namespace qcpw

using namespace qcpw;

extern "C" qcpw_status qmc_cpw_greeks_noalloc(const qcpw_option_spec *option_specs, int32_t n_opts, int32_t d,
                                              int64_t n_points, int32_t n_shifts, int32_t path_construction,
                                              double *out_greeks, double *out_stderr, const qcpw_run_config *cfg)
{
    set_error("");
    qcpw_run_config c;
    memset(&c, 0, sizeof c);
    c.device = -1;
    if (cfg) c = *cfg;
    if (!out_greeks || !out_stderr) return fail(QCPW_EINVAL, "output pointer is NULL");
    qcpw_status st = validate_call(option_specs, n_opts, d, n_points, n_shifts, path_construction, c.precision,
                                   c.pca_gemm, c.block_threads);
    if (st != QCPW_OK) return st;
    if (path_construction != QCPW_PATH_BB && path_construction != QCPW_PATH_STANDARD)
        return fail(QCPW_EINVAL, "the no-allocation call runs the BB and STANDARD constructions (the PCA factors "
                                 "are built on first use)");
    if (c.flags & ~QCPW_FLAG_OWEN) return fail(QCPW_EINVAL, "only QCPW_FLAG_OWEN is accepted");
    const bool owen = (c.flags & QCPW_FLAG_OWEN) != 0;
    Context *ctx = nullptr;
    st = get_context(c.device, &ctx);   // first call on a device: builds its tables (set-up)
    if (st != QCPW_OK) return st;
    char *ws = nullptr;
    st = scratch_address(ctx->tab.device, &ws);
    if (st != QCPW_OK) return st;
    std::lock_guard<std::mutex> lk(ctx->mu);
    LaunchPlan lp;
    // block_threads 0: the autotuner's earlier choice or a default, never its
    // probe launches
    st = plan_launch(ctx, option_specs, n_opts, d, n_points, n_shifts, path_construction, c.precision, c.pca_gemm,
                     c.block_threads ? c.block_threads : -1, lp, nullptr, owen);
    if (st != QCPW_OK) return st;
    const size_t n = (size_t)n_opts;
    const size_t out_bytes = n * 4 * sizeof(double);
    const size_t ps_bytes = n * (size_t)n_shifts * 4 * sizeof(double);
    const size_t out_al = (out_bytes + 255) / 256 * 256;
    const size_t need = (launch_workspace_bytes(lp) + 255) / 256 * 256;
    const bool dev_out = c.outputs_on_device != 0;
    const size_t total = need + (dev_out ? 0 : 3 * out_al + (c.out_per_shift ? ps_bytes : 0));
    if (total > (size_t)QCPW_NOALLOC_BYTES)
        return fail(QCPW_ENOMEM, "the launch needs " + std::to_string(total) + " bytes of scratch, more than the " +
                                     std::to_string((size_t)QCPW_NOALLOC_BYTES) +
                                     " the no-allocation call holds (fewer options, points or replications fit)");
    hipStream_t stream = (hipStream_t)c.stream;
    double *g = out_greeks, *e = out_stderr, *ps = c.out_per_shift, *sg = c.out_paper_sigma;
    if (!dev_out) {
        char *p = ws + need;
        g = (double *)p;
        e = (double *)(p + out_al);
        sg = c.out_paper_sigma ? (double *)(p + 2 * out_al) : nullptr;
        ps = c.out_per_shift ? (double *)(p + 3 * out_al) : nullptr;
    }
    st = enqueue_launch(ctx, lp, stream, g, e, ps, ws, need, nullptr, false, sg);
    if (st != QCPW_OK) return st;
    if (!dev_out) {
        QCPW_HIP(hipMemcpyAsync(out_greeks, g, out_bytes, hipMemcpyDeviceToHost, stream));
        QCPW_HIP(hipMemcpyAsync(out_stderr, e, out_bytes, hipMemcpyDeviceToHost, stream));
        if (c.out_per_shift)
            QCPW_HIP(hipMemcpyAsync(c.out_per_shift, ps, ps_bytes, hipMemcpyDeviceToHost, stream));
        if (c.out_paper_sigma)
            QCPW_HIP(hipMemcpyAsync(c.out_paper_sigma, sg, out_bytes, hipMemcpyDeviceToHost, stream));
        QCPW_HIP(hipStreamSynchronize(stream));
    }
    return QCPW_OK;
}
