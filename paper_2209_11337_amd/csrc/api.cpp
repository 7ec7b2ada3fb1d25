// api.cpp -- the C ABI: argument checks, per-device contexts with their
// resident tables, workspace management and the synchronous entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "qcpw_host.h"

namespace qcpw {

#include "ninv_table.inc"

// the option record's size and field offsets are ABI
static_assert(sizeof(qcpw_option_spec) == 80, "qcpw_option_spec is 80 bytes");
static_assert(sizeof(qcpw_run_config) == 48 && offsetof(qcpw_run_config, out_paper_sigma) == 40,
              "qcpw_run_config layout");
static_assert(offsetof(qcpw_option_spec, seed) == 48 && offsetof(qcpw_option_spec, n_points) == 56 &&
                  offsetof(qcpw_option_spec, rho) == 72,
              "qcpw_option_spec field offsets");

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

qcpw_status fail(qcpw_status code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

qcpw_status Workspace::ensure(size_t need, size_t cap)
{
    if (need <= bytes) return QCPW_OK;
    if (ptr) {
        QCPW_HIP(hipFree(ptr));
        ptr = nullptr;
        bytes = 0;
    }
    size_t want = std::max(need, std::min(need + need / 4, cap));
    hipError_t e = hipMalloc(&ptr, want);
    if (e != hipSuccess) {
        ptr = nullptr;
        return fail(QCPW_ENOMEM, "hipMalloc of " + std::to_string(want) + " workspace bytes failed");
    }
    bytes = want;
    return QCPW_OK;
}

static std::mutex g_ctx_mu;
static std::vector<std::unique_ptr<Context>> g_ctx;

static qcpw_status init_tables(Context *ctx, int device)
{
    DeviceTables &t = ctx->tab;
    t.device = device;
    hipDeviceProp_t prop;
    QCPW_HIP(hipGetDeviceProperties(&prop, device));
    t.n_cu = prop.multiProcessorCount;

    std::vector<uint32_t> dir, lane;
    build_direction_numbers(dir);
    build_lane_table(dir, lane);
    std::vector<PlanStep> all;
    std::vector<PlanStep64> all64;
    t.plan_off.assign(QCPW_MAX_N + 1, 0);
    t.depth.assign(QCPW_MAX_N + 1, 0);
    for (int n = 1; n <= QCPW_MAX_N; ++n) {
        std::vector<PlanStep> s;
        std::vector<PlanStep64> s64;
        int depth = build_bridge_plan(n, s, s64);
        if (depth < 0) return fail(QCPW_EDEVICE, "bridge plan disagrees with the compile-time bridges");
        if (depth > QCPW_STACK_MAX) return fail(QCPW_EDEVICE, "bridge plan deeper than the kernel's stack");
        t.max_stack = std::max(t.max_stack, depth);
        t.depth[n] = depth;
        t.plan_off[n] = (int32_t)all.size();
        all.insert(all.end(), s.begin(), s.end());
        all64.insert(all64.end(), s64.begin(), s64.end());
    }
    // split-bridge plans, each checked against the plan walker's: the FP64
    // factor its walk applies must equal the plan's bit for bit, or n keeps
    // the plan walker
    std::vector<uint32_t> sev((size_t)(QCPW_MAX_N + 1) * QCPW_SPLIT_EVENTS * QCPW_EV_WORDS, 0u);
    std::vector<uint16_t> sdim((size_t)(QCPW_MAX_N + 1) * QCPW_SPLIT_SLOTS, 0);
    t.split_slots.assign(QCPW_MAX_N + 1, 0);
    for (int n = QCPW_SUB_MIN_LEN; n <= QCPW_MAX_N; ++n) {
        std::vector<uint32_t> ev;
        std::vector<uint16_t> sd;
        const int slots = build_split_plan(n, ev, sd);
        if (slots <= 0 || slots > (n > QCPW_WIDE_MIN_N ? 8 : QCPW_UQ) * 64) continue;
        std::vector<double> A_split, A_plan;
        split_plan_factor(n, 1.0, ev, A_split);
        build_factor(QCPW_PATH_BB, n, 1.0, A_plan);
        if (memcmp(A_split.data(), A_plan.data(), A_plan.size() * sizeof(double)) != 0) continue;
        t.split_slots[n] = slots;
        std::copy(ev.begin(), ev.end(), sev.begin() + (size_t)n * QCPW_SPLIT_EVENTS * QCPW_EV_WORDS);
        std::copy(sd.begin(), sd.end(), sdim.begin() + (size_t)n * QCPW_SPLIT_SLOTS);
    }
    // every n from QCPW_SUB_MIN_LEN on has a split plan (the compile-time
    // bridges give its bits, and the 128-VGPR kernel instances walk their n
    // with it): a missing one is a defect of the plan builder
    for (int n = QCPW_SUB_MIN_LEN; n <= QCPW_MAX_N; ++n)
        if (t.split_slots[n] == 0)
            return fail(QCPW_EDEVICE, "no split-bridge plan for n = " + std::to_string(n));
    QCPW_HIP(hipMalloc(&t.split_ev, sev.size() * 4));
    QCPW_HIP(hipMalloc(&t.split_dim, sdim.size() * 2));
    QCPW_HIP(hipMemcpy(t.split_ev, sev.data(), sev.size() * 4, hipMemcpyHostToDevice));
    QCPW_HIP(hipMemcpy(t.split_dim, sdim.data(), sdim.size() * 2, hipMemcpyHostToDevice));
    QCPW_HIP(hipMalloc(&t.dir, dir.size() * 4));
    QCPW_HIP(hipMalloc(&t.lane, lane.size() * 4));
    QCPW_HIP(hipMalloc(&t.plan, all.size() * sizeof(PlanStep)));
    QCPW_HIP(hipMalloc(&t.plan64, all64.size() * sizeof(PlanStep64)));
    QCPW_HIP(hipMemcpy(t.dir, dir.data(), dir.size() * 4, hipMemcpyHostToDevice));
    QCPW_HIP(hipMemcpy(t.lane, lane.data(), lane.size() * 4, hipMemcpyHostToDevice));
    QCPW_HIP(hipMemcpy(t.plan, all.data(), all.size() * sizeof(PlanStep), hipMemcpyHostToDevice));
    QCPW_HIP(hipMemcpy(t.plan64, all64.data(), all64.size() * sizeof(PlanStep64), hipMemcpyHostToDevice));
    QCPW_HIP(hipMalloc(&t.ninv_tab, sizeof(QCPW_NINV_TAB)));
    QCPW_HIP(hipMemcpy(t.ninv_tab, QCPW_NINV_TAB, sizeof(QCPW_NINV_TAB), hipMemcpyHostToDevice));
    QCPW_HIP(hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking));
    QCPW_HIP(hipEventCreateWithFlags(&ctx->ws_done, hipEventDisableTiming));
    return QCPW_OK;
}

qcpw_status get_context(int device, Context **out)
{
    int cur = 0;
    if (device < 0) {
        QCPW_HIP(hipGetDevice(&cur));
        device = cur;
    }
    int count = 0;
    QCPW_HIP(hipGetDeviceCount(&count));
    if (device >= count) return fail(QCPW_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    if ((int)g_ctx.size() < count) g_ctx.resize(count);
    if (!g_ctx[device]) {
        std::unique_ptr<Context> c(new Context());
        QCPW_HIP(hipSetDevice(device));
        qcpw_status st = init_tables(c.get(), device);
        if (st != QCPW_OK) return st;
        g_ctx[device] = std::move(c);
    }
    QCPW_HIP(hipSetDevice(device));
    *out = g_ctx[device].get();
    return QCPW_OK;
}

// Unit-dt principal-component factor for n coordinates (the kernels scale
// the normals by sqrt(dt) instead), resident per n, in the layouts the PCA
// kernels read: FP32 k-major At[k][row] (NP x NP, zero padded, NP = n rounded
// up to 32), the same split as BF16 hi + lo in 16-wide k slabs
// [k/16][row][16], and n x n FP64 row-major.
qcpw_status get_pca(Context *ctx, int n, double dt, const Context::Pca **out, bool full)
{
    for (auto &p : ctx->pca)
        if (p.n == n && p.dt == dt && p.full == full) {
            *out = &p;
            return QCPW_OK;
        }
    // rows x n matrix the kernels multiply by the n sampled normals
    std::vector<double> A, a1;
    int rows = n;
    if (full) {
        std::vector<double> F;
        rows = n + 1;
        build_pca_factor(rows, dt, F);   // d x d, column 0 = conditioned component
        A.assign((size_t)rows * n, 0.0);
        a1.assign(rows, 0.0);
        for (int j = 0; j < rows; ++j) {
            a1[j] = F[(size_t)j * rows];
            for (int k = 0; k < n; ++k) A[(size_t)j * n + k] = F[(size_t)j * rows + k + 1];
        }
    } else {
        build_pca_factor(n, dt, A);
    }
    const int NP = (std::max(rows, 1) + 31) / 32 * 32;
    std::vector<float> At((size_t)NP * NP, 0.0f);
    std::vector<uint16_t> hi((size_t)NP * NP, 0), lo((size_t)NP * NP, 0);
    auto to_bf16 = [](float x) -> uint16_t {   // round to nearest even
        uint32_t u;
        memcpy(&u, &x, 4);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
    };
    auto from_bf16 = [](uint16_t h) -> float {
        uint32_t u = (uint32_t)h << 16;
        float x;
        memcpy(&x, &u, 4);
        return x;
    };
    for (int row = 0; row < rows; ++row)
        for (int k = 0; k < n; ++k) {
            const float a = (float)A[(size_t)row * n + k];
            At[(size_t)k * NP + row] = a;
            const uint16_t h = to_bf16(a);
            const size_t blk = ((size_t)(k / 16) * NP + row) * 16 + (k % 16);
            hi[blk] = h;
            lo[blk] = to_bf16(a - from_bf16(h));
        }
    Context::Pca p;
    p.n = n;
    p.dt = dt;
    p.np = NP;
    p.full = full;
    if (A.empty()) A.assign(1, 0.0);
    QCPW_HIP(hipMalloc(&p.At, At.size() * 4));
    QCPW_HIP(hipMalloc(&p.A64, A.size() * 8));
    if (full) {
        QCPW_HIP(hipMalloc(&p.a1, a1.size() * 8));
        QCPW_HIP(hipMemcpy(p.a1, a1.data(), a1.size() * 8, hipMemcpyHostToDevice));
    }
    QCPW_HIP(hipMalloc(&p.Ahi, hi.size() * 2));
    QCPW_HIP(hipMalloc(&p.Alo, lo.size() * 2));
    QCPW_HIP(hipMemcpy(p.At, At.data(), At.size() * 4, hipMemcpyHostToDevice));
    QCPW_HIP(hipMemcpy(p.A64, A.data(), A.size() * 8, hipMemcpyHostToDevice));
    QCPW_HIP(hipMemcpy(p.Ahi, hi.data(), hi.size() * 2, hipMemcpyHostToDevice));
    QCPW_HIP(hipMemcpy(p.Alo, lo.data(), lo.size() * 2, hipMemcpyHostToDevice));
    ctx->pca.push_back(p);
    *out = &ctx->pca.back();
    return QCPW_OK;
}

}  // namespace qcpw

using namespace qcpw;

extern "C" {

const char *qcpw_last_error(void) { return g_last_error.c_str(); }

const char *qcpw_version(void) { return "qmc-cpw-mi355x 0.1 (gfx950)"; }

}  // extern "C"

namespace qcpw {

static constexpr size_t kMaxGraphs = 16;

static void append(std::vector<unsigned char> &k, const void *p, size_t n)
{
    const unsigned char *b = (const unsigned char *)p;
    k.insert(k.end(), b, b + n);
}

static void free_graph(Context::Graph &g)
{
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    if (g.ws) (void)hipFree(g.ws);
    if (g.host) (void)hipHostFree(g.host);
    g = Context::Graph();
}

// QCPW_FLAG_GRAPH: replay the captured graph of an identical earlier call, or
// capture this call's device work (the set-up copy from a pinned buffer,
// per-path kernel, finalize) into a new graph with its own workspace.
static qcpw_status run_graph(Context *ctx, const qcpw_option_spec *specs, int32_t n_opts, int32_t d,
                             int64_t n_points, int32_t n_shifts, int32_t path, const qcpw_run_config &c,
                             double *g_out, double *e_out)
{
    std::vector<unsigned char> key;
    append(key, specs, sizeof(qcpw_option_spec) * (size_t)n_opts);
    const int64_t scal[] = {n_opts, d, n_points, n_shifts, path, c.precision, c.pca_gemm, c.block_threads, c.flags};
    append(key, scal, sizeof scal);
    const void *ptrs[] = {c.stream, g_out, e_out, c.out_per_shift, c.out_paper_sigma};
    append(key, ptrs, sizeof ptrs);
    hipStream_t stream = (hipStream_t)c.stream;
    for (auto &g : ctx->graphs)
        if (g.key == key) {
            g.last_use = ++ctx->graph_clock;
            QCPW_HIP(hipGraphLaunch(g.exec, stream));
            return QCPW_OK;
        }
    LaunchPlan lp;
    qcpw_status st = plan_launch(ctx, specs, n_opts, d, n_points, n_shifts, path, c.precision, c.pca_gemm,
                                 c.block_threads, lp, nullptr, (c.flags & QCPW_FLAG_OWEN) != 0);
    if (st != QCPW_OK) return st;
    if (ctx->graphs.size() >= kMaxGraphs) {   // evict the least recently used
        size_t lru = 0;
        for (size_t i = 1; i < ctx->graphs.size(); ++i)
            if (ctx->graphs[i].last_use < ctx->graphs[lru].last_use) lru = i;
        QCPW_HIP(hipDeviceSynchronize());
        free_graph(ctx->graphs[lru]);
        ctx->graphs.erase(ctx->graphs.begin() + (long)lru);
    }
    Context::Graph g;
    g.key = key;
    const size_t need = launch_workspace_bytes(lp);
    const size_t hbytes = launch_upload_bytes(lp);
    if (hipMalloc(&g.ws, need) != hipSuccess || hipHostMalloc(&g.host, hbytes, hipHostMallocDefault) != hipSuccess) {
        free_graph(g);
        return fail(QCPW_ENOMEM, "graph workspace allocation failed");
    }
    fill_launch_upload(lp, g.host);
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        free_graph(g);
        return fail(QCPW_EDEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    }
    st = enqueue_launch(ctx, lp, stream, g_out, e_out, c.out_per_shift, g.ws, need, g.host, false,
                        c.out_paper_sigma);
    e = hipStreamEndCapture(stream, &g.graph);
    if (st != QCPW_OK || e != hipSuccess) {
        free_graph(g);
        return st != QCPW_OK ? st : fail(QCPW_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        free_graph(g);
        return fail(QCPW_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    g.last_use = ++ctx->graph_clock;
    ctx->graphs.push_back(g);
    QCPW_HIP(hipGraphLaunch(ctx->graphs.back().exec, stream));
    return QCPW_OK;
}

}  // namespace qcpw

extern "C" {

qcpw_status qmc_cpw_greeks_ex(const qcpw_option_spec *option_specs, int32_t n_opts, int32_t d,
                              int64_t n_points, int32_t n_shifts, int32_t path_construction,
                              double *out_greeks, double *out_stderr, const qcpw_run_config *cfg)
{
    g_last_error.clear();
    qcpw_run_config c;
    memset(&c, 0, sizeof c);
    c.device = -1;
    if (cfg) c = *cfg;
    if (!out_greeks || !out_stderr) return fail(QCPW_EINVAL, "output pointer is NULL");
    qcpw_status st = validate_call(option_specs, n_opts, d, n_points, n_shifts, path_construction,
                                   c.precision, c.pca_gemm, c.block_threads);
    if (st != QCPW_OK) return st;
    if (c.flags & ~(QCPW_FLAG_GRAPH | QCPW_FLAG_OWEN)) return fail(QCPW_EINVAL, "unknown flags");
    const bool owen = (c.flags & QCPW_FLAG_OWEN) != 0;
    if ((c.flags & QCPW_FLAG_GRAPH) && !c.outputs_on_device)
        return fail(QCPW_EINVAL, "QCPW_FLAG_GRAPH needs outputs_on_device");
    Context *ctx = nullptr;
    st = get_context(c.device, &ctx);
    if (st != QCPW_OK) return st;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (c.flags & QCPW_FLAG_GRAPH) {
        return run_graph(ctx, option_specs, n_opts, d, n_points, n_shifts, path_construction, c, out_greeks,
                         out_stderr);
    }
    LaunchPlan lp;
    st = plan_launch(ctx, option_specs, n_opts, d, n_points, n_shifts, path_construction, c.precision,
                     c.pca_gemm, c.block_threads, lp, nullptr, owen);
    if (st != QCPW_OK) return st;
    const size_t n = (size_t)n_opts;
    const size_t out_bytes = n * 4 * sizeof(double);
    const size_t ps_bytes = n * (size_t)n_shifts * 4 * sizeof(double);
    const size_t need = launch_workspace_bytes(lp);
    const bool dev_out = c.outputs_on_device != 0;
    const size_t out_al = (out_bytes + 255) / 256 * 256;
    const size_t extra = dev_out ? 0 : 3 * out_al + (c.out_per_shift ? ps_bytes : 0) + 256;
    hipStream_t stream = (hipStream_t)c.stream;   // NULL is the default stream
    if (ctx->ws_pending) {
        // the workspace may still be in use by a launch on another stream
        if (need + extra > ctx->ws.bytes) QCPW_HIP(hipEventSynchronize(ctx->ws_done));
        else QCPW_HIP(hipStreamWaitEvent(stream, ctx->ws_done, 0));
    }
    st = ctx->ws.ensure(need + extra);
    if (st != QCPW_OK) return st;
    char *ws = (char *)ctx->ws.ptr;
    double *g = out_greeks, *e = out_stderr, *ps = c.out_per_shift, *sg = c.out_paper_sigma;
    if (!dev_out) {
        char *p = ws + need;
        g = (double *)p;
        e = (double *)(p + out_al);
        sg = c.out_paper_sigma ? (double *)(p + 2 * out_al) : nullptr;
        ps = c.out_per_shift ? (double *)(p + 3 * out_al) : nullptr;
    }
    st = enqueue_launch(ctx, lp, stream, g, e, ps, ws, need, nullptr, true, sg);
    if (st != QCPW_OK) return st;
    QCPW_HIP(hipEventRecord(ctx->ws_done, stream));
    ctx->ws_pending = true;
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

qcpw_status qcpw_kernel_timer(int32_t device, int32_t op, double *total_ms, int64_t *launches)
{
    g_last_error.clear();
    if (op != QCPW_TIMER_START && op != QCPW_TIMER_READ && op != QCPW_TIMER_STOP)
        return fail(QCPW_EINVAL, "op must be QCPW_TIMER_START, _READ or _STOP");
    Context *ctx = nullptr;
    qcpw_status st = get_context(device, &ctx);
    if (st != QCPW_OK) return st;
    std::lock_guard<std::mutex> lk(ctx->mu);
    Context::Timer &tm = ctx->timer;
    if (op == QCPW_TIMER_START) {
        tm.on = true;
        tm.used = 0;
        return QCPW_OK;
    }
    double total = 0.0;
    for (size_t i = 0; i + 1 < tm.used; i += 2) {
        QCPW_HIP(hipEventSynchronize(tm.ev[i + 1]));
        float ms = 0.0f;
        QCPW_HIP(hipEventElapsedTime(&ms, tm.ev[i], tm.ev[i + 1]));
        total += ms;
    }
    if (total_ms) *total_ms = total;
    if (launches) *launches = (int64_t)(tm.used / 2);
    if (op == QCPW_TIMER_STOP) tm.on = false;
    return QCPW_OK;
}

qcpw_status qmc_cpw_greeks(const qcpw_option_spec *option_specs, int32_t n_opts, int32_t d, int64_t n_points,
                           int32_t n_shifts, int32_t path_construction, double *out_greeks, double *out_stderr)
{
    return qmc_cpw_greeks_ex(option_specs, n_opts, d, n_points, n_shifts, path_construction, out_greeks,
                             out_stderr, nullptr);
}

static qcpw_status points(uint64_t seed, int32_t shift_index, int32_t n_dims, int64_t k0, int64_t count,
                          uint32_t *out, bool owen);

qcpw_status qcpw_sobol_points(uint64_t seed, int32_t shift_index, int32_t n_dims, int64_t k0, int64_t count,
                              uint32_t *out)
{
    return points(seed, shift_index, n_dims, k0, count, out, false);
}

qcpw_status qcpw_scrambled_points(uint64_t seed, int32_t shift_index, int32_t n_dims, int64_t k0, int64_t count,
                                  uint32_t *out)
{
    return points(seed, shift_index, n_dims, k0, count, out, true);
}

static qcpw_status points(uint64_t seed, int32_t shift_index, int32_t n_dims, int64_t k0, int64_t count,
                          uint32_t *out, bool owen)
{
    g_last_error.clear();
    if (!out) return fail(QCPW_EINVAL, "out is NULL");
    if (n_dims < 1 || n_dims > QCPW_TAB_DIMS) return fail(QCPW_EINVAL, "n_dims out of range");
    if (count < 1 || count > (int64_t(1) << 24)) return fail(QCPW_EINVAL, "count out of range");
    if (k0 < 0 || k0 + count > (int64_t(1) << 32)) return fail(QCPW_EINVAL, "points beyond 2^32");
    if (shift_index < 0 || shift_index > QCPW_MAX_SHIFTS) return fail(QCPW_EINVAL, "shift_index out of range");
    Context *ctx = nullptr;
    qcpw_status st = get_context(-1, &ctx);
    if (st != QCPW_OK) return st;
    std::lock_guard<std::mutex> lk(ctx->mu);
    const size_t bytes = (size_t)count * n_dims * 4;
    if (ctx->ws_pending) QCPW_HIP(hipEventSynchronize(ctx->ws_done));
    st = ctx->ws.ensure(bytes);
    if (st != QCPW_OK) return st;
    st = launch_sobol_points(ctx, seed, shift_index, n_dims, k0, count, (uint32_t *)ctx->ws.ptr, ctx->own_stream,
                             owen);
    if (st != QCPW_OK) return st;
    QCPW_HIP(hipMemcpyAsync(out, ctx->ws.ptr, bytes, hipMemcpyDeviceToHost, ctx->own_stream));
    QCPW_HIP(hipStreamSynchronize(ctx->own_stream));
    return QCPW_OK;
}

qcpw_status qcpw_path_coordinates(const qcpw_option_spec *spec, int32_t n_shifts, int32_t path_construction,
                                  int32_t precision, int32_t flags, uint32_t *out)
{
    g_last_error.clear();
    if (!out) return fail(QCPW_EINVAL, "out is NULL");
    qcpw_status st = validate_call(spec, 1, 0, 0, n_shifts, path_construction, precision, QCPW_GEMM_FP32, 0);
    if (st != QCPW_OK) return st;
    if (path_construction != QCPW_PATH_BB && path_construction != QCPW_PATH_STANDARD)
        return fail(QCPW_EINVAL, "coordinates are recorded by the per-path kernel (BB and STANDARD)");
    if (flags & ~QCPW_FLAG_OWEN) return fail(QCPW_EINVAL, "only QCPW_FLAG_OWEN is accepted");
    const bool owen = (flags & QCPW_FLAG_OWEN) != 0;
    const bool basket = spec->type == QCPW_BASKET_ASIAN_CALL || spec->type == QCPW_BASKET_ASIAN_PUT;
    const int64_t ndims = (int64_t)(spec->d - 1) + (basket ? (int64_t)spec->n_assets * spec->d : 0);
    if (ndims < 1) return fail(QCPW_EINVAL, "the option has no sampled coordinate (d = 1)");
    const int64_t N = spec->n_points;
    if ((int64_t)n_shifts * N * ndims * 4 > (int64_t(1) << 28))
        return fail(QCPW_EINVAL, "n_shifts * n_points * dimensions * 4 exceeds 2^28 bytes");
    Context *ctx = nullptr;
    st = get_context(-1, &ctx);
    if (st != QCPW_OK) return st;
    std::lock_guard<std::mutex> lk(ctx->mu);
    LaunchPlan lp;
    st = plan_launch(ctx, spec, 1, 0, 0, n_shifts, path_construction, precision, QCPW_GEMM_FP32, 256, lp, nullptr,
                     owen);
    if (st != QCPW_OK) return st;
    const OptDev &op = lp.opts[0];
    const size_t need = (launch_workspace_bytes(lp) + 255) / 256 * 256;
    const size_t pbytes = (size_t)lp.total_units * op.unit_pts * ndims * 4;
    if (ctx->ws_pending) QCPW_HIP(hipEventSynchronize(ctx->ws_done));
    st = ctx->ws.ensure(need + 1024 + pbytes);
    if (st != QCPW_OK) return st;
    char *ws = (char *)ctx->ws.ptr;
    double *g = (double *)(ws + need);
    lp.probe = (uint32_t *)(ws + need + 1024);
    st = enqueue_launch(ctx, lp, ctx->own_stream, g, g + 4, g + 8, ws, need);
    if (st != QCPW_OK) return st;
    std::vector<uint32_t> rec(pbytes / 4);
    QCPW_HIP(hipMemcpyAsync(rec.data(), lp.probe, pbytes, hipMemcpyDeviceToHost, ctx->own_stream));
    QCPW_HIP(hipStreamSynchronize(ctx->own_stream));
    // recorded as [unit][batch][dim][lane], unit = l * chunks + chunk, point
    // k = chunk * unit_pts + batch * 64 + lane
    for (int64_t l = 0; l < n_shifts; ++l)
        for (int64_t k = 0; k < N; ++k) {
            const int64_t pb = l * (int64_t)op.chunks * (op.unit_pts / 64) + k / 64;
            const uint32_t *src = rec.data() + (size_t)pb * ndims * 64 + (k & 63);
            uint32_t *dst = out + ((size_t)l * N + k) * ndims;
            for (int64_t j = 0; j < ndims; ++j) dst[j] = src[j * 64];
        }
    return QCPW_OK;
}

qcpw_status qcpw_path_factor(int32_t path_construction, int32_t d, double T, double *out)
{
    g_last_error.clear();
    if (!out) return fail(QCPW_EINVAL, "out is NULL");
    if (path_construction != QCPW_PATH_BB && path_construction != QCPW_PATH_PCA &&
        path_construction != QCPW_PATH_STANDARD && path_construction != QCPW_PATH_PCA_FULL)
        return fail(QCPW_EINVAL, "unknown path_construction");
    const int dmax = path_construction == QCPW_PATH_PCA        ? QCPW_MAX_D_PCA
                     : path_construction == QCPW_PATH_PCA_FULL ? QCPW_MAX_D_PCA_FULL
                                                               : QCPW_MAX_D;
    if (d < 1 || d > dmax) return fail(QCPW_EDIMS, "d out of range");
    if (!(T > 0) || !std::isfinite(T)) return fail(QCPW_EINVAL, "T must be finite and > 0");
    std::vector<double> A;
    if (path_construction == QCPW_PATH_PCA_FULL) build_pca_factor(d, T / d, A);
    else build_factor(path_construction, d - 1, T / d, A);
    if (path_construction == QCPW_PATH_BB) {
        // the split bridge's walk (FP32 kernel) must apply the same factor
        // as the plan walker's, bit for bit; NaNs report a mismatch
        std::vector<uint32_t> ev;
        std::vector<uint16_t> sd;
        if (build_split_plan(d - 1, ev, sd) > 0) {
            std::vector<double> As;
            split_plan_factor(d - 1, T / d, ev, As);
            if (memcmp(As.data(), A.data(), A.size() * sizeof(double)) != 0)
                std::fill(A.begin(), A.end(), std::nan(""));
        }
    }
    if (!A.empty()) memcpy(out, A.data(), A.size() * sizeof(double));
    return QCPW_OK;
}

}  // extern "C"
