// qcpw_host.h -- host-side declarations of the QMC-CPW library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qmc_cpw.h"
#include "qcpw_internal.h"

namespace qcpw {

// ---- tables.cpp -----------------------------------------------------------
void build_direction_numbers(std::vector<uint32_t> &dir);
void build_lane_table(const std::vector<uint32_t> &dir, std::vector<uint32_t> &lane);
int build_bridge_plan(int n, std::vector<PlanStep> &steps, std::vector<PlanStep64> &steps64);
int build_split_plan(int n, std::vector<uint32_t> &events, std::vector<uint16_t> &slot_dim);
void split_plan_factor(int n, double dt, const std::vector<uint32_t> &events, std::vector<double> &A);
void build_pca_factor(int n, double dt, std::vector<double> &A);
void build_factor(int path, int n, double dt, std::vector<double> &A);

// ---- errors ---------------------------------------------------------------
void set_error(const std::string &msg);
qcpw_status fail(qcpw_status code, const std::string &msg);
#define QCPW_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::qcpw::fail(QCPW_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---- device context (one per device, lives until process exit) -----------
struct DeviceTables {
    int device = -1;
    int n_cu = 0;
    uint32_t *dir = nullptr;     // [QCPW_TAB_DIMS][32]
    uint32_t *lane = nullptr;    // [QCPW_TAB_DIMS][64]
    PlanStep *plan = nullptr;    // all bridge plans, n = 1..QCPW_MAX_N
    PlanStep64 *plan64 = nullptr;
    float4 *ninv_tab = nullptr;  // FP32 inverse-normal cubic table (1024 cells)
    std::vector<int32_t> plan_off;   // [QCPW_MAX_N + 1]
    std::vector<int32_t> depth;      // [QCPW_MAX_N + 1] bridge stack depth per n
    int max_stack = 0;
    uint32_t *split_ev = nullptr;    // split-bridge events [QCPW_MAX_N + 1][QCPW_SPLIT_EVENTS][QCPW_EV_WORDS]
    uint16_t *split_dim = nullptr;   // slot dimensions [QCPW_MAX_N + 1][QCPW_SPLIT_SLOTS]
    std::vector<int32_t> split_slots;   // [QCPW_MAX_N + 1] slots used, 0: no split bridge for n
};

// Grow-only device workspace.
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
    // grow to at least need bytes (25 % spare, never beyond cap); keeps the
    // buffer when it is large enough
    qcpw_status ensure(size_t need, size_t cap = SIZE_MAX);
};

struct Context {
    std::mutex mu;               // serialises launches on this device
    DeviceTables tab;
    hipStream_t own_stream = nullptr;
    Workspace ws;                // per-launch device buffers
    hipEvent_t ws_done = nullptr;   // recorded after the last launch that used ws
    bool ws_pending = false;
    // PCA factors, keyed by (n, dt bits)
    // full = false: the n x n factor of the d - 1 coordinates after x_1;
    // full = true: the d x d factor of all d dates without its first column
    // (rows = dates, n = d - 1 columns), plus that first column a1 (FP64).
    struct Pca { int n; double dt; int np; bool full = false; float *At = nullptr; double *A64 = nullptr;
                 uint16_t *Ahi = nullptr, *Alo = nullptr; double *a1 = nullptr; };
    std::deque<Pca> pca;     // deque: pointers stay valid as factors are added
    std::map<int, int> tuned;   // autotuned workgroup size per (path, precision, n bucket)
    // captured launch graphs (QCPW_FLAG_GRAPH), keyed by the call's argument bytes
    struct Graph {
        std::vector<unsigned char> key;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        void *ws = nullptr;
        void *host = nullptr;    // pinned copies of the uploaded OptDev[] and unit prefix
        uint64_t last_use = 0;
    };
    std::vector<Graph> graphs;
    uint64_t graph_clock = 0;
    // qcpw_kernel_timer: event pairs around the main kernel of eager calls
    struct Timer { bool on = false; std::vector<hipEvent_t> ev; size_t used = 0; } timer;
};

qcpw_status get_context(int device, Context **out);
qcpw_status get_pca(Context *ctx, int n, double dt, const Context::Pca **out, bool full = false);

// ---- launches (kernels.hip) -------------------------------------------------
// One launch of the fused per-path kernel: the sorted options
// [opt0, opt0 + n_opts) and their work units [unit0, unit0 + units), with
// the kernel instance (register budget) and workgroup size chosen for them.
struct LaunchSeg {
    int32_t opt0 = 0, n_opts = 0;
    int64_t unit0 = 0, units = 0;
    int max_n = 0;                     // lane rows: the largest Sobol dimension count of a path
    int stack_depth = 0;               // deepest bridge stack among the options
    int block_threads = 0;
    bool wide = false;                 // FP32 kernel instance with 128 VGPRs and 8 slot registers
};
#define QCPW_MAX_SEGS 2

struct LaunchPlan {
    // host copies of what the kernels read
    std::vector<OptDev> opts;          // sorted by cost (descending)
    std::vector<int64_t> unit_prefix;  // [n_opts + 1]
    std::vector<int32_t> order;        // opts[i] is caller's option order[i]
    int max_n = 0;
    int path = 0;
    int precision = 0;
    int pca_gemm = 0;
    int n_shifts = 0;
    int block_threads = 0;             // the first launch's (256 for the matrix-core PCA kernels)
    int64_t total_units = 0;           // work units dealt by the queues
    int64_t member_units = 0;          // further units whose partials a group leader's units write
    int64_t full_blocks = 0;           // PCA_FULL in FP64: workgroups with a global scratch tile
    bool owen = false;                 // nested scrambling instead of the digital shift
    uint32_t *probe = nullptr;         // device buffer: run the coordinate-recording kernel instance
    std::vector<LaunchSeg> segs;       // fused per-path kernel launches, in order (bridge, standard)
    std::vector<const Context::Pca *> pca;   // per sorted option (PCA and PCA_FULL)
};

// Argument checks of a Greeks call (host only, no device needed).
qcpw_status validate_call(const qcpw_option_spec *specs, int32_t n_opts, int32_t d, int64_t n_points,
                          int32_t n_shifts, int32_t path, int32_t precision, int32_t pca_gemm,
                          int32_t block_threads);

// Builds the per-option constants and work units.  k_begin (optional, per
// caller option) starts an option's points at a multiple of QCPW_CHUNK
// instead of 0; n_points then counts the points from there.
// force_wide (fused kernel, FP32): -1 chooses the launches and their
// register budgets, 0 / 1 makes one launch of the 80- / 128-VGPR instances.
qcpw_status plan_launch(Context *ctx, const qcpw_option_spec *specs, int32_t n_opts, int32_t d,
                        int64_t n_points, int32_t n_shifts, int32_t path, int32_t precision,
                        int32_t pca_gemm, int32_t block_threads, LaunchPlan &lp,
                        const int64_t *k_begin = nullptr, bool owen = false, int force_wide = -1);

// Device bytes one launch needs in the workspace.
size_t launch_workspace_bytes(const LaunchPlan &lp);
// Host bytes a launch uploads to the start of its workspace (option table,
// unit prefix, zeroed work-queue heads), and the routine that writes them.
size_t launch_upload_bytes(const LaunchPlan &lp);
void fill_launch_upload(const LaunchPlan &lp, void *dst);

// Enqueues the whole hot path on `stream`: uploads, the per-path kernel, the
// finalize kernel; results go to dev_out_greeks / dev_out_stderr ([n][4],
// caller order) and optionally dev_out_per_shift ([n][L][4]) and
// dev_out_sigma ([n][4], the spread of the replications).
// h_upload: the launch_upload_bytes(lp) bytes to upload (default: written
// from lp into a host buffer here; graph capture passes a pinned copy that
// outlives the call).
qcpw_status enqueue_launch(Context *ctx, const LaunchPlan &lp, hipStream_t stream,
                           double *dev_out_greeks, double *dev_out_stderr,
                           double *dev_out_per_shift, void *ws, size_t ws_bytes,
                           const void *h_upload = nullptr, bool timed = false,
                           double *dev_out_sigma = nullptr);

qcpw_status launch_sobol_points(Context *ctx, uint64_t seed, int32_t shift_index, int32_t n_dims,
                                int64_t k0, int64_t count, uint32_t *dev_out, hipStream_t stream,
                                bool owen = false);

int autotune_block_threads(Context *ctx, const LaunchPlan &lp, const LaunchSeg &sg);
// The autotuner's choice if it has one for the launch's key, else a default;
// never launches or allocates.  plan_launch takes block_threads < 0 as this.
int known_block_threads(Context *ctx, const LaunchPlan &lp, const LaunchSeg &sg);
// Instances of the fused per-path kernel (paths_*.hip), as kernel pointers.
const void *paths_fn_f32_bb(bool wide);
const void *paths_fn_f32_bb_owen(bool wide);
const void *paths_fn_f32_std(bool owen, bool wide);
const void *paths_fn_f32_probe(int path, bool owen, bool wide);
const void *paths_fn_f32_probe_narrow(bool owen);
const void *paths_fn_f64(int path, bool owen, bool probe);
// Runs the autotuner for every lane-table bucket of (path, precision,
// scrambling) ahead of use; caller holds ctx->mu.
void pretune_block_threads(Context *ctx, int path, int precision, bool owen);

// Fails unless kernel `fn` has no static LDS (its dynamic LDS starts at 0).
qcpw_status check_lds_at_zero(const void *fn);

}  // namespace qcpw
