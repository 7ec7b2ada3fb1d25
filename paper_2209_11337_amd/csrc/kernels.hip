// kernels.hip -- launch planning for the fused per-path QMC-CPW kernel
// (paths_kernel.h), the per-replication finalize kernel, the Sobol probe
// kernel, the workgroup-size autotuner and the launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <set>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <numeric>

#include "qcpw_host.h"
#include "device_math.h"

namespace qcpw {

// One block per option: replication estimates C_l (chunk partials added in
// chunk order), then the mean over replications and its standard error.
// per_shift: [n_opts(caller order)][L][4].
// out_sigma (optional): the spread of the single replications about the mean.
__global__ __launch_bounds__(256) void finalize_kernel(const OptDev *opts, const double *partials,
                                                       double *per_shift, double *out_mean,
                                                       double *out_stderr, double *out_sigma)
{
    __shared__ double red_s[256], red_c[256];
    const OptDev &op = opts[blockIdx.x];
    const int L = op.n_shifts;
    const int t = threadIdx.x;
    double *Cl = per_shift + (size_t)op.out_index * L * 4;
    const double invN = 1.0 / (double)op.n_points;
    for (int l = t; l < L; l += blockDim.x) {
        for (int i = 0; i < 4; ++i) {
            double S = 0.0, C = 0.0;
            for (int64_t k = 0; k < op.chunks; ++k) {
                const double *p = partials + (op.unit0 + (int64_t)l * op.chunks + k) * 8;
                const double t2 = S + p[i];
                const double bp = t2 - S;
                C += (S - (t2 - bp)) + (p[i] - bp) + p[4 + i];
                S = t2;
            }
            Cl[l * 4 + i] = (S + C) * invN;
        }
    }
    __syncthreads();
    for (int i = 0; i < 4; ++i) {
        // mean: strided compensated sums, then a fixed pairwise tree
        double S = 0.0, C = 0.0;
        for (int l = t; l < L; l += blockDim.x) acc_add(S, C, Cl[l * 4 + i]);
        red_s[t] = S;
        red_c[t] = C;
        __syncthreads();
        for (int w = blockDim.x / 2; w >= 1; w >>= 1) {
            if (t < w) {
                const double a = red_s[t], b = red_s[t + w];
                const double s2 = a + b, bp = s2 - a;
                red_c[t] = red_c[t] + red_c[t + w] + ((a - (s2 - bp)) + (b - bp));
                red_s[t] = s2;
            }
            __syncthreads();
        }
        const double mean = (red_s[0] + red_c[0]) / (double)L;
        __syncthreads();
        double V = 0.0;
        for (int l = t; l < L; l += blockDim.x) {
            const double dv = Cl[l * 4 + i] - mean;
            V += dv * dv;
        }
        red_s[t] = V;
        __syncthreads();
        for (int w = blockDim.x / 2; w >= 1; w >>= 1) {
            if (t < w) red_s[t] += red_s[t + w];
            __syncthreads();
        }
        if (t == 0) {
            out_mean[op.out_index * 4 + i] = mean;
            out_stderr[op.out_index * 4 + i] =
                L >= 2 ? sqrt(red_s[0] / ((double)L * (double)(L - 1))) : NAN;
            if (out_sigma) out_sigma[op.out_index * 4 + i] = L >= 2 ? sqrt(red_s[0] / (double)L) : NAN;
        }
        __syncthreads();
    }
}

// Shifted Sobol integers through the same lane-table / uniform-part split
// the per-path kernel uses.  One wave per 64 consecutive points; out is
// [count][n_dims].  k0 need not be a multiple of 64: the wave's base is
// rounded down and lanes outside [k0, k0 + count) store nothing.
template <bool OWEN>
__global__ __launch_bounds__(64) void sobol_points_kernel(const uint32_t *dir, const uint32_t *lane_tab,
                                                          uint64_t seed, int shift, int n_dims, int64_t k0,
                                                          int64_t count, uint32_t *out)
{
    const int lane = threadIdx.x;
    const uint64_t base = ((uint64_t)k0 & ~63ull) + (uint64_t)blockIdx.x * 64;
    const uint64_t k = base + lane;
    const bool in = k >= (uint64_t)k0 && k < (uint64_t)(k0 + count);
    const uint64_t g = (base ^ (base >> 1)) >> 5;
    for (int j0 = 0; j0 < n_dims; j0 += 64) {
        // lane holds U for dimension j0 + lane
        const int jl = j0 + lane;
        uint32_t u = 0, key = 0;
        if (jl < n_dims) {
            key = jl == 0 ? 0u : digital_shift(seed, shift, jl);
            uint64_t gg = g;
            for (int b = 5; gg != 0; ++b, gg >>= 1)
                if (gg & 1) u ^= dir[(size_t)jl * 32 + b];
            if (!OWEN) u ^= key;
        }
        const int jmax = min(64, n_dims - j0);
        for (int jj = 0; jj < jmax; ++jj) {
            const int j = j0 + jj;
            uint32_t y = lane_tab[(size_t)j * 64 + lane] ^ rdlane(u, jj);
            if (OWEN && j > 0) y = owen_scramble(y, rdlane(key, jj));   // dimension 0 stays as it is
            if (in) out[(size_t)(k - (uint64_t)k0) * n_dims + j] = y;
        }
    }
}

// ------------------------------------------------------------------------
// launch planning (host)
// ------------------------------------------------------------------------
static inline bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

qcpw_status validate_call(const qcpw_option_spec *specs, int32_t n_opts, int32_t d, int64_t n_points,
                          int32_t n_shifts, int32_t path, int32_t precision, int32_t pca_gemm,
                          int32_t block_threads)
{
    if (!specs) return fail(QCPW_EINVAL, "option_specs is NULL");
    if (n_opts < 1) return fail(QCPW_EINVAL, "n_opts must be >= 1");
    if (n_shifts < 1 || n_shifts > QCPW_MAX_SHIFTS) return fail(QCPW_EINVAL, "n_shifts out of range");
    if (path != QCPW_PATH_BB && path != QCPW_PATH_PCA && path != QCPW_PATH_STANDARD &&
        path != QCPW_PATH_PCA_FULL)
        return fail(QCPW_EINVAL, "unknown path_construction");
    if (precision != QCPW_FP64 && precision != QCPW_FP32_MIXED) return fail(QCPW_EINVAL, "unknown precision");
    if (pca_gemm != QCPW_GEMM_FP32 && pca_gemm != QCPW_GEMM_BF16X3) return fail(QCPW_EINVAL, "unknown pca_gemm");
    if (!qcpw_block_threads_ok(block_threads))
        return fail(QCPW_EINVAL, "block_threads must be 0 or a multiple of 64 in [64, 1024]");
    if (d < 0 || n_points < 0) return fail(QCPW_EINVAL, "negative d or n_points");
    const int dmax = path == QCPW_PATH_PCA        ? QCPW_MAX_D_PCA
                     : path == QCPW_PATH_PCA_FULL ? QCPW_MAX_D_PCA_FULL
                                                  : QCPW_MAX_D;
    for (int i = 0; i < n_opts; ++i) {
        const qcpw_option_spec &sp = specs[i];
        const int di = d ? d : sp.d;
        const int64_t Ni = n_points ? n_points : sp.n_points;
        if (sp.type < QCPW_ARITH_ASIAN_CALL || sp.type > QCPW_BASKET_ASIAN_PUT)
            return fail(QCPW_EINVAL, "option " + std::to_string(i) + ": unknown type");
        if (sp.reserved != 0)
            return fail(QCPW_EINVAL, "option " + std::to_string(i) + ": reserved field must be 0");
        if (qcpw_is_basket(sp.type)) {
            if (path != QCPW_PATH_STANDARD)
                return fail(QCPW_EINVAL, "option " + std::to_string(i) + ": baskets use the standard construction");
            if (sp.n_assets < 1 || sp.n_assets > QCPW_MAX_ASSETS)
                return fail(QCPW_EINVAL, "option " + std::to_string(i) + ": n_assets must be in [1, " +
                                             std::to_string(QCPW_MAX_ASSETS) + "]");
            if (!(std::isfinite(sp.rho) && sp.rho > 0.0 && sp.rho <= 1.0))
                return fail(QCPW_EINVAL, "option " + std::to_string(i) + ": rho must be in (0, 1]");
            if (di >= 1 && (int64_t)(di - 1) + (int64_t)sp.n_assets * di > QCPW_MAX_BASKET_DIMS)
                return fail(QCPW_EDIMS, "option " + std::to_string(i) + ": (d - 1) + n_assets d exceeds " +
                                            std::to_string(QCPW_MAX_BASKET_DIMS));
        }
        if (path == QCPW_PATH_PCA_FULL && sp.type != QCPW_ARITH_ASIAN_CALL && sp.type != QCPW_BINARY_ASIAN_CALL &&
            sp.type != QCPW_LOOKBACK_FIXED_CALL)
            return fail(QCPW_EINVAL, "option " + std::to_string(i) +
                                         ": conditioning on the first principal component covers the "
                                         "arithmetic and binary Asian and the lookback calls");
        if (di < 1) return fail(QCPW_EINVAL, "option " + std::to_string(i) + ": d must be >= 1");
        if (di > dmax)
            return fail(QCPW_EDIMS, "option " + std::to_string(i) + ": d = " + std::to_string(di) +
                                        " exceeds " + std::to_string(dmax) + " for this path construction");
        if (Ni < 1 || Ni > (int64_t(1) << 32))
            return fail(QCPW_EINVAL, "option " + std::to_string(i) + ": n_points must be in [1, 2^32]");
        if (!finite_pos(sp.S0) || !finite_pos(sp.K) || !finite_pos(sp.sigma) || !finite_pos(sp.T) ||
            !std::isfinite(sp.r))
            return fail(QCPW_EINVAL, "option " + std::to_string(i) +
                                         ": S0, K, sigma, T must be finite and > 0, r finite");
    }
    return QCPW_OK;
}

// Compile-time bridges (FP32 kernel): on unless QCPW_FIXED_BRIDGES=0.
static bool fixed_bridges_on()
{
    static const bool on = [] {
        const char *e = getenv("QCPW_FIXED_BRIDGES");
        return !(e && e[0] == '0');
    }();
    return on;
}

// Split bridge (FP32 kernel, n >= QCPW_SUB_MIN_LEN): on unless
// QCPW_SPLIT_BRIDGE=0 (then the plan walker takes those options).  Both
// switches are diagnostics: with either one off, an option's bits may
// depend on which kernel instance its launch runs (the compile-time and
// split walks give the same bits, the plan walker does not).
static bool split_bridge_on()
{
    static const bool on = [] {
        const char *e = getenv("QCPW_SPLIT_BRIDGE");
        return !(e && e[0] == '0');
    }();
    return on;
}

static size_t paths_lds_bytes(const LaunchPlan &lp, const LaunchSeg &sg, int bd, int *stk_off = nullptr);

// How an option is walked by a launch of the given register budget
// (compile-time bridge in the 80-VGPR instances, split bridge, or the plan
// walker with its LDS stack), with the uniform slots it needs.
struct Walk {
    bool split;
    int slots, depth;
};
static Walk walk_of(Context *ctx, const LaunchPlan &lp, const OptDev &op, bool wide)
{
    const bool f32 = lp.precision == QCPW_FP32_MIXED;
    const bool fixed = f32 && !wide && fixed_bridges_on() && qcpw_has_fixed_bridge(op.n);
    Walk w;
    w.split = lp.path == QCPW_PATH_BB && f32 && !fixed && split_bridge_on() && ctx->tab.split_slots[op.n] > 0;
    w.slots = w.split ? ctx->tab.split_slots[op.n] : op.ndims;
    w.depth = (lp.path == QCPW_PATH_BB && op.n >= 1 && !fixed && !w.split) ? ctx->tab.depth[op.n] : 0;
    return w;
}

// The walks of a launch's options, and its lane rows, stack depth and units.
static void assign_walks(Context *ctx, LaunchPlan &lp, LaunchSeg &sg)
{
    sg.max_n = 0;
    sg.stack_depth = 0;
    for (int i = sg.opt0; i < sg.opt0 + sg.n_opts; ++i) {
        OptDev &op = lp.opts[i];
        const Walk w = walk_of(ctx, lp, op, sg.wide);
        op.split = w.split ? 1 : 0;
        op.n_slots = w.slots;
        sg.stack_depth = std::max(sg.stack_depth, w.depth);
        sg.max_n = std::max(sg.max_n, op.ndims);
    }
    sg.unit0 = lp.unit_prefix[sg.opt0];
    sg.units = lp.unit_prefix[sg.opt0 + sg.n_opts] - sg.unit0;
}

// Uniform-slot registers of the instances: the 80-VGPR ones hold QCPW_UQ.
static bool slots_fit_narrow(const LaunchPlan &lp, const LaunchSeg &sg)
{
    for (int i = sg.opt0; i < sg.opt0 + sg.n_opts; ++i)
        if (lp.opts[i].n_slots > QCPW_UQ * 64) return false;
    return true;
}

// The fused kernel's launches.  FP64: one.  FP32: the 80-VGPR instances
// (six waves per SIMD) as long as the lane rows fit the LDS of enough
// workgroups to use them; up to QCPW_WIDE_MIN_N rows that holds at 512
// threads, beyond it at 768 threads (two workgroups, 24 waves per CU) while
// two such workgroups fit.  Longer rows leave room for one workgroup, where
// the 128-VGPR instances (16 waves per CU, eight slot registers) are
// faster.  A launch that mixes both kinds of options is split in two: the
// options that lead the sorted order (those the 80-VGPR instances would walk
// with an LDS stack, then the longest) in a launch of the 128-VGPR
// instances, the others in a launch of the 80-VGPR ones -- when the latter
// hold at least a quarter of the work and the call is large enough that the
// first launch's last units cost little.  Each option's work units, hence
// its bits, do not depend on the launch that runs them.
static void plan_segments(Context *ctx, LaunchPlan &lp, int force_wide)
{
    const bool f32 = lp.precision == QCPW_FP32_MIXED;
    const int n = (int)lp.opts.size();
    LaunchSeg all;
    all.opt0 = 0;
    all.n_opts = n;
    all.wide = f32 && (force_wide >= 0 ? force_wide != 0 : lp.max_n > QCPW_WIDE_MIN_N);
    int split_at = n;   // first option of an 80-VGPR launch after the 128-VGPR one (n: none)
    if (f32 && force_wide < 0 && all.wide) {
        // longest suffix of the sorted options that two 768-thread workgroups
        // run from the LDS
        LaunchSeg t;
        t.wide = false;
        for (int s = n - 1; s >= 0; --s) {
            const Walk w = walk_of(ctx, lp, lp.opts[s], false);
            t.max_n = std::max(t.max_n, lp.opts[s].ndims);
            t.stack_depth = std::max(t.stack_depth, w.depth);
            if (w.slots > QCPW_UQ * 64 || 2 * ((paths_lds_bytes(lp, t, 768) + 2047) / 2048 * 2048) > 160 * 1024)
                break;
            split_at = s;
        }
        if (split_at == 0) {
            all.wide = false;
            split_at = n;
        } else if (split_at < n) {
            double work = 0.0, tail = 0.0;
            for (int i = 0; i < n; ++i) {
                const double w = (double)(lp.unit_prefix[i + 1] - lp.unit_prefix[i]) * std::max(lp.opts[i].ndims, 1);
                work += w;
                if (i >= split_at) tail += w;
            }
            if (!(tail >= 0.25 * work && lp.total_units >= 8192)) split_at = n;
        }
    }
    lp.segs.clear();
    all.n_opts = split_at;
    lp.segs.push_back(all);
    if (split_at < n) {
        LaunchSeg nar;
        nar.opt0 = split_at;
        nar.n_opts = n - split_at;
        nar.wide = false;
        lp.segs.push_back(nar);
    }
    for (LaunchSeg &sg : lp.segs) {
        assign_walks(ctx, lp, sg);
        // a forced 80-VGPR launch whose slots do not fit takes the 128-VGPR instances
        if (f32 && !sg.wide && !slots_fit_narrow(lp, sg)) {
            sg.wide = true;
            assign_walks(ctx, lp, sg);
        }
    }
}

qcpw_status plan_launch(Context *ctx, const qcpw_option_spec *specs, int32_t n_opts, int32_t d,
                        int64_t n_points, int32_t n_shifts, int32_t path, int32_t precision,
                        int32_t pca_gemm, int32_t block_threads, LaunchPlan &lp, const int64_t *k_begin,
                        bool owen, int force_wide)
{
    {
        qcpw_status st = validate_call(specs, n_opts, d, n_points, n_shifts, path, precision, pca_gemm,
                                       block_threads < 0 ? 0 : block_threads);
        if (st != QCPW_OK) return st;
    }
    lp = LaunchPlan();
    lp.owen = owen;
    lp.path = path;
    lp.precision = precision;
    lp.pca_gemm = pca_gemm;
    lp.n_shifts = n_shifts;
    std::vector<OptDev> opts(n_opts);
    std::vector<double> cost(n_opts);
    for (int i = 0; i < n_opts; ++i) {
        const qcpw_option_spec &sp = specs[i];
        const int di = d ? d : sp.d;
        const int64_t Ni = n_points ? n_points : sp.n_points;
        const int64_t kb = k_begin ? k_begin[i] : 0;
        if (kb < 0 || kb % QCPW_CHUNK != 0 || kb + Ni > (int64_t(1) << 32))
            return fail(QCPW_EINVAL, "option " + std::to_string(i) + ": bad point range");
        OptDev &op = opts[i];
        memset(&op, 0, sizeof op);
        op.type = sp.type;
        op.d = di;
        op.n = di - 1;
        op.path = path;
        op.n_points = Ni;
        op.k_begin = kb;
        op.seed = sp.seed;
        op.n_shifts = n_shifts;
        op.out_index = i;
        const bool pca_like = path == QCPW_PATH_PCA || path == QCPW_PATH_PCA_FULL;
        op.unit_pts = (int32_t)(pca_like ? QCPW_CHUNK : qcpw_unit_points(Ni));
        op.chunks = (int32_t)((Ni + op.unit_pts - 1) / op.unit_pts);
        op.plan_off = (path == QCPW_PATH_BB && op.n >= 1) ? ctx->tab.plan_off[op.n] : 0;
        const double LOG2E = 1.4426950408889634074;
        const double dt = sp.T / di, t1 = dt;
        const double omega = sp.r - 0.5 * sp.sigma * sp.sigma;
        op.zscale = sp.sigma * std::sqrt(dt) * LOG2E;
        op.ydrift_n = omega * op.n * dt * LOG2E;
        op.ydrift_1 = omega * dt * LOG2E;
        op.kappa = (sp.r + 0.5 * sp.sigma * sp.sigma) * dt * LOG2E;
        op.inv_sig_log2e = 1.0 / (sp.sigma * LOG2E);
        op.s1 = sp.sigma * std::sqrt(t1);
        op.inv_s1 = 1.0 / op.s1;
        op.sqrt_t1 = std::sqrt(t1);
        op.inv_sigma = 1.0 / sp.sigma;
        op.c0 = std::log(sp.K) - std::log(sp.S0) - omega * t1 +
                (qcpw_stat_of(sp.type) == QCPW_STAT_AVG ? std::log((double)di) : 0.0);
        op.h = std::exp(op.c0 - 0.5 * op.s1 * op.s1);
        op.S0 = sp.S0;
        op.K = sp.K;
        op.D = std::exp(-sp.r * sp.T);
        op.D1 = std::exp(sp.r * (t1 - sp.T));
        op.invd = 1.0 / di;
        op.inv_S0 = 1.0 / sp.S0;
        op.inv_S0sq = 1.0 / (sp.S0 * sp.S0);
        op.zs_t = (float)op.zscale;
        op.ydrift_n_f = (float)op.ydrift_n;
        op.ydrift_1_f = (float)op.ydrift_1;
        op.ndims = op.n;
        if (qcpw_is_basket(sp.type)) {
            // one-factor basket: x_1 drives sqrt(rho) of every asset's first step
            const int M = sp.n_assets;
            const double rho = sp.rho;
            op.n_assets = M;
            op.ndims = op.n + M * di;
            op.s1 = sp.sigma * std::sqrt(rho * t1);
            op.inv_s1 = 1.0 / op.s1;
            op.sqrt_t1 = std::sqrt(rho * t1);   // d s1 / d sigma
            op.c0 = std::log(sp.K) - std::log(sp.S0) - omega * t1 + std::log((double)M * di);
            op.h = std::exp(op.c0 - 0.5 * op.s1 * op.s1);
            op.D1 = std::exp(-sp.r * sp.T + omega * t1 + 0.5 * op.s1 * op.s1);
            op.vx_shift = -sp.sigma * (1.0 - rho) * t1;
            op.invd = 1.0 / ((double)M * di);
            op.b_common = std::sqrt(rho) * op.zscale;
            op.b_idio = std::sqrt(1.0 - rho) * op.zscale;
            op.b_common_f = (float)op.b_common;
            op.b_idio_f = (float)op.b_idio;
        }
        {
            const double sgn = qcpw_is_put(sp.type) ? -1.0 : 1.0;
            const double PHI_C = 0.398942280401432677939946;   // 1/sqrt(2 pi)
            op.sDK = sgn * op.D * op.K;
            op.sD1 = sgn * op.D1;
            op.h2 = 0.5 * op.h;
            op.gv = op.D * op.K * PHI_C * op.sqrt_t1;
            op.gg = op.D * op.K * PHI_C * op.inv_s1 * op.inv_S0sq;
            if (sp.type == QCPW_BINARY_ASIAN_CALL || sp.type == QCPW_BINARY_ASIAN_PUT) {
                op.gb = sgn * op.D * PHI_C;
                op.gd = op.gb * op.inv_s1 * op.inv_S0;
                op.gg = op.gb * op.inv_s1 * op.inv_S0sq;
            }
        }
        cost[i] = (double)std::max(op.ndims, 1) * (double)op.chunks;
        lp.max_n = std::max(lp.max_n, op.ndims);
    }
    // Matrix-core PCA (either conditioning): options whose paths are
    // identical -- same n, seed and point range, same z scale and drift,
    // same path statistic (they differ in strike or payoff) -- share one
    // product and one epilogue per tile; only the FP64 tail runs per option.
    // They are sorted next to each other and the first (leader) carries the
    // group.
    const bool grouping = (path == QCPW_PATH_PCA || path == QCPW_PATH_PCA_FULL) && precision == QCPW_FP32_MIXED;
    auto same_paths = [&](const OptDev &a, const OptDev &b) {
        return a.n == b.n && a.seed == b.seed && a.n_points == b.n_points && a.k_begin == b.k_begin &&
               a.zs_t == b.zs_t && a.ydrift_1_f == b.ydrift_1_f && qcpw_stat_of(a.type) == qcpw_stat_of(b.type);
    };
    // most expensive units first (longest-processing-time order); in FP32
    // bridge launches the options that the 80-VGPR instances would walk with
    // the plan walker (its LDS stack, 12 KiB per 768-thread workgroup at
    // n < 12) lead, so that a split call leaves them to the 128-VGPR launch
    // and its 80-VGPR launch needs no stack
    std::vector<char> stacked(n_opts, 0);
    if (path == QCPW_PATH_BB && precision == QCPW_FP32_MIXED)
        for (int i = 0; i < n_opts; ++i) stacked[i] = walk_of(ctx, lp, opts[i], false).depth > 0;
    std::vector<int32_t> order(n_opts);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const OptDev &x = opts[a], &y = opts[b];
        if (stacked[a] != stacked[b]) return stacked[a] > stacked[b];
        if (x.ndims != y.ndims || !grouping) return x.ndims > y.ndims;
        if (x.seed != y.seed) return x.seed < y.seed;
        if (x.n_points != y.n_points) return x.n_points < y.n_points;
        if (x.k_begin != y.k_begin) return x.k_begin < y.k_begin;
        if (x.zs_t != y.zs_t) return x.zs_t < y.zs_t;
        if (x.ydrift_1_f != y.ydrift_1_f) return x.ydrift_1_f < y.ydrift_1_f;
        return qcpw_stat_of(x.type) < qcpw_stat_of(y.type);
    });
    lp.opts.resize(n_opts);
    lp.unit_prefix.assign(n_opts + 1, 0);
    std::vector<int> members;
    int leader = -1;
    for (int i = 0; i < n_opts; ++i) {
        lp.opts[i] = opts[order[i]];
        OptDev &op = lp.opts[i];
        const int64_t units = (int64_t)op.chunks * n_shifts;
        if (grouping && leader >= 0 && lp.opts[leader].grp < QCPW_PCA_MAX_GROUP && same_paths(lp.opts[leader], op)) {
            op.grp = 0;   // a member: no units of its own to deal
            ++lp.opts[leader].grp;
            lp.unit_prefix[i + 1] = lp.unit_prefix[i];
            members.push_back(i);
            continue;
        }
        leader = i;
        op.grp = 1;
        op.unit0 = lp.unit_prefix[i];
        lp.unit_prefix[i + 1] = lp.unit_prefix[i] + units;
    }
    lp.order = order;
    lp.total_units = lp.unit_prefix[n_opts];
    // members' partials follow the dealt units
    for (int i : members) {
        lp.opts[i].unit0 = lp.total_units + lp.member_units;
        lp.member_units += (int64_t)lp.opts[i].chunks * n_shifts;
    }
    if (path == QCPW_PATH_BB || path == QCPW_PATH_STANDARD) {
        plan_segments(ctx, lp, force_wide);
        for (LaunchSeg &sg : lp.segs)
            sg.block_threads = block_threads > 0 ? block_threads
                               : block_threads < 0 ? known_block_threads(ctx, lp, sg)
                                                   : autotune_block_threads(ctx, lp, sg);
        lp.block_threads = lp.segs[0].block_threads;
    } else {
        lp.block_threads = block_threads > 0 ? block_threads : 256;
    }
    if (path == QCPW_PATH_PCA || path == QCPW_PATH_PCA_FULL) {
        const bool full = path == QCPW_PATH_PCA_FULL;
        lp.pca.resize(n_opts, nullptr);
        for (int i = 0; i < n_opts; ++i) {
            if (lp.opts[i].n == 0 && !full) continue;
            const Context::Pca *pc = nullptr;
            qcpw_status st = get_pca(ctx, lp.opts[i].n, 1.0, &pc, full);
            if (st != QCPW_OK) return st;
            lp.pca[i] = pc;
            lp.opts[i].pca_At = pc->At;
            lp.opts[i].pca_hi = pc->Ahi;
            lp.opts[i].pca_lo = pc->Alo;
            lp.opts[i].pca_A64 = pc->A64;
            lp.opts[i].pca_a1 = pc->a1;
            lp.opts[i].pca_np = pc->np;
        }
        // FP64 PCA_FULL keeps each tile's d x 64 products in a global scratch
        // tile per workgroup (they do not fit in LDS beside the FP64 normals)
        if (full && precision == QCPW_FP64)
            lp.full_blocks = std::min<int64_t>((int64_t)2 * std::max(ctx->tab.n_cu, 1), lp.total_units);
    }
    return QCPW_OK;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Workspace of one launch.  The option table, the unit prefix and the queue
// heads lead, so that one host-to-device copy of `upload` bytes (the heads
// as zeros) sets up a launch.
struct WsLayout {
    size_t opts, prefix, counter, upload, partials, per_shift, scratch, total;
};

static WsLayout ws_layout(const LaunchPlan &lp)
{
    WsLayout w;
    const size_t n = lp.opts.size();
    w.opts = 0;
    w.prefix = align_up(w.opts + n * sizeof(OptDev), 256);
    w.counter = align_up(w.prefix + (n + 1) * sizeof(int64_t), 256);
    w.upload = w.counter + QCPW_MAX_SEGS * QCPW_QUEUES * QCPW_QUEUE_STRIDE * sizeof(unsigned long long);
    w.partials = align_up(w.upload, 256);
    w.per_shift = align_up(w.partials + (size_t)(lp.total_units + lp.member_units) * 8 * sizeof(double), 256);
    w.scratch = align_up(w.per_shift + n * (size_t)lp.n_shifts * 4 * sizeof(double), 256);
    w.total = align_up(w.scratch + (size_t)lp.full_blocks * 64 * QCPW_MAX_D_PCA_FULL * sizeof(double), 256);
    return w;
}

size_t launch_upload_bytes(const LaunchPlan &lp) { return ws_layout(lp).upload; }

void fill_launch_upload(const LaunchPlan &lp, void *dst)
{
    const WsLayout w = ws_layout(lp);
    const size_t n = lp.opts.size();
    memset(dst, 0, w.upload);
    memcpy((char *)dst + w.opts, lp.opts.data(), n * sizeof(OptDev));
    memcpy((char *)dst + w.prefix, lp.unit_prefix.data(), (n + 1) * sizeof(int64_t));
}

size_t launch_workspace_bytes(const LaunchPlan &lp) { return ws_layout(lp).total; }

// LDS of the fused kernel at workgroup size bd.  FP32: the inverse-normal
// cells and the lane rows at fixed places (qcpw_row_word, with the copies of
// the gap's last rows when rows go beyond it), the bridge stacks
// after the last row, or in the gap below the upper cells when they fit
// there.  FP64: the rows from 0, then the stacks.  *stk_off (optional)
// receives the stacks' byte offset.
static size_t paths_lds_bytes(const LaunchPlan &lp, const LaunchSeg &sg, int bd, int *stk_off)
{
    const bool f32 = lp.precision == QCPW_FP32_MIXED;
    const size_t stack = lp.path == QCPW_PATH_BB ? (size_t)sg.stack_depth * bd * (f32 ? 4 : 8) : 0;
    if (!f32) {
        if (stk_off) *stk_off = sg.max_n * 256;
        return (size_t)sg.max_n * 256 + stack;
    }
    const bool in_gap = sg.max_n <= QCPW_LDS_GAP_ROWS;
    const size_t rows_end = in_gap ? QCPW_LDS_GAP_BEGIN + (size_t)sg.max_n * 256
                                   : (size_t)qcpw_row_word_hi(sg.max_n) * 4;
    const size_t s = (in_gap && rows_end + stack > QCPW_LDS_TAB_HI) ? QCPW_LDS_FIXED : rows_end;
    if (stk_off) *stk_off = (int)s;
    return std::max<size_t>(s + stack, QCPW_LDS_FIXED);
}

// ... against the CU's 160 KiB.
static bool paths_lds_fits(const LaunchPlan &lp, const LaunchSeg &sg, int bd)
{
    return paths_lds_bytes(lp, sg, bd) <= 160 * 1024;
}

// The FP32 kernels read the inverse-normal cells at absolute LDS addresses
// (cell address = bits of q), which holds only while the kernel has no
// static LDS, so that its dynamic LDS starts at address 0.  Checked once per
// kernel before its first launch.
qcpw_status check_lds_at_zero(const void *fn)
{
    static std::mutex mu;
    static std::set<const void *> ok;
    std::lock_guard<std::mutex> lk(mu);
    if (ok.count(fn)) return QCPW_OK;
    hipFuncAttributes at;
    QCPW_HIP(hipFuncGetAttributes(&at, fn));
    if (at.sharedSizeBytes != 0)
        return fail(QCPW_EDEVICE, "an FP32 kernel has static LDS; its inverse-normal cells must sit at address 0");
    ok.insert(fn);
    return QCPW_OK;
}

// The kernel instance of a launch: precision, construction, randomisation,
// coordinate recording and register budget (the one the plan was made for:
// compile-time bridges run only in the 80-VGPR instances).
static const void *select_paths_kernel(const LaunchPlan &lp, const LaunchSeg &sg)
{
    const bool f32 = lp.precision == QCPW_FP32_MIXED;
    if (!f32) return paths_fn_f64(lp.path, lp.owen, lp.probe != nullptr);
    if (lp.probe) return paths_fn_f32_probe(lp.path, lp.owen, sg.wide);
    if (lp.path == QCPW_PATH_STANDARD) return paths_fn_f32_std(lp.owen, sg.wide);
    return lp.owen ? paths_fn_f32_bb_owen(sg.wide) : paths_fn_f32_bb(sg.wide);
}

// Resident waves per CU of the fused kernel at workgroup size bd (0 if it
// cannot be resident): registers, LDS and the workgroup granularity decide.
static int resident_waves(const LaunchPlan &lp, const LaunchSeg &sg, int bd)
{
    if (!paths_lds_fits(lp, sg, bd)) return 0;
    const size_t lds = paths_lds_bytes(lp, sg, bd);
    const void *fn = select_paths_kernel(lp, sg);
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, bd, lds) != hipSuccess) return 0;
    return per_cu * bd / 64;
}

// Workgroup size of a fused-kernel launch, chosen by measurement among 256,
// 512, 768 and 1024 threads (whole multiples of the CU's four SIMDs, so that
// every SIMD holds the same number of waves).  The lane rows and
// inverse-normal cells are shared per workgroup and the bridge stack is per
// thread, so the best size depends on d and on the register budget.  Each
// size that can be resident is timed on a probe -- one arithmetic Asian
// option with the launch's largest d, 2^18 points x 64 replications (16384
// work units, a few per resident wave), on the launch's kernel instance --
// and the fastest is kept per (construction, precision, randomisation,
// register budget, lane-table size bucket).  QCPW_BLOCK_THREADS in the
// environment overrides the choice.  Results do not depend on it.
static int tune_key(const LaunchPlan &lp, const LaunchSeg &sg)
{
    return (((lp.path * 2 + lp.precision) * 2 + (lp.owen ? 1 : 0)) * 2 + (sg.wide ? 1 : 0)) * 64 + (sg.max_n + 31) / 32;
}

int autotune_block_threads(Context *ctx, const LaunchPlan &lp, const LaunchSeg &sg)
{
    if (lp.path == QCPW_PATH_PCA || lp.path == QCPW_PATH_PCA_FULL) return 256;
    if (const char *env = getenv("QCPW_BLOCK_THREADS")) {
        const int v = atoi(env);
        if (v != 0 && qcpw_block_threads_ok(v) && resident_waves(lp, sg, v) > 0) return v;
    }
    const int key = tune_key(lp, sg);
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) return it->second;
    qcpw_option_spec probe;
    memset(&probe, 0, sizeof probe);
    probe.type = QCPW_ARITH_ASIAN_CALL;
    probe.d = std::max(sg.max_n, 1) + 1;
    probe.S0 = 100.0; probe.K = 100.0; probe.r = 0.05; probe.sigma = 0.2; probe.T = 1.0;
    probe.seed = 0x51ab;
    probe.n_points = int64_t(1) << 18;
    const int n_probe_shifts = 64;
    const bool f32 = lp.precision == QCPW_FP32_MIXED;

    std::vector<LaunchPlan> plans;
    std::vector<int> cands;
    for (int bd : {256, 512, 768, 1024}) {
        LaunchPlan p;
        if (plan_launch(ctx, &probe, 1, 0, 0, n_probe_shifts, lp.path, lp.precision, lp.pca_gemm, bd, p, nullptr,
                        lp.owen, f32 ? (sg.wide ? 1 : 0) : -1) != QCPW_OK)
            continue;
        LaunchSeg &ps = p.segs[0];
        if (ps.wide != sg.wide) continue;
        ps.max_n = std::max(ps.max_n, sg.max_n);
        ps.stack_depth = std::max(ps.stack_depth, sg.stack_depth);
        p.max_n = ps.max_n;
        if (resident_waves(p, ps, bd) == 0) continue;
        cands.push_back(bd);
        plans.push_back(std::move(p));
    }
    (void)hipGetLastError();
    std::vector<size_t> pick;
    for (size_t i = 0; i < cands.size(); ++i) pick.push_back(i);

    int best = cands.empty() ? 256 : cands.back();
    float best_ms = 1e30f;
    void *ws = nullptr;
    double *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool ok = !pick.empty() && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
              hipMalloc(&out, 2 * 4 * sizeof(double) + n_probe_shifts * 4 * sizeof(double)) == hipSuccess;
    size_t ws_have = 0;
    for (size_t j = 0; ok && j < pick.size(); ++j) {
        const LaunchPlan &p = plans[pick[j]];
        const size_t need = launch_workspace_bytes(p);
        if (need > ws_have) {
            if (ws) (void)hipFree(ws);
            ws = nullptr;
            if (hipMalloc(&ws, need) != hipSuccess) { ok = false; break; }
            ws_have = need;
        }
        float ms = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            (void)hipEventRecord(e0, ctx->own_stream);
            if (enqueue_launch(ctx, p, ctx->own_stream, out, out + 4, out + 8, ws, ws_have) != QCPW_OK) {
                ms = 1e30f;
                break;
            }
            (void)hipEventRecord(e1, ctx->own_stream);
            (void)hipEventSynchronize(e1);
            float t = 0.0f;
            (void)hipEventElapsedTime(&t, e0, e1);
            if (rep > 0) ms = std::min(ms, t);   // first repetition warms up
        }
        if (ms < best_ms) { best_ms = ms; best = cands[pick[j]]; }
    }
    if (ws) (void)hipFree(ws);
    if (out) (void)hipFree(out);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipGetLastError();
    ctx->tuned[key] = best;
    return best;
}

// The workgroup size the autotuner has chosen for this launch's key, or --
// without running its probes, which allocate -- 768 threads for the 80-VGPR
// instances beyond QCPW_WIDE_MIN_N lane rows, else 512 (256 when those do
// not fit the LDS).
int known_block_threads(Context *ctx, const LaunchPlan &lp, const LaunchSeg &sg)
{
    if (lp.path == QCPW_PATH_PCA || lp.path == QCPW_PATH_PCA_FULL) return 256;
    auto it = ctx->tuned.find(tune_key(lp, sg));
    if (it != ctx->tuned.end()) return it->second;
    if (lp.precision == QCPW_FP32_MIXED && !sg.wide && sg.max_n > QCPW_WIDE_MIN_N && paths_lds_fits(lp, sg, 768))
        return 768;
    return paths_lds_fits(lp, sg, 512) ? 512 : 256;
}

// Tunes every lane-table size bucket of one (construction, precision,
// randomisation) ahead of use, for each register budget a launch of that
// size can take.
void pretune_block_threads(Context *ctx, int path, int precision, bool owen)
{
    const bool f32 = precision == QCPW_FP32_MIXED;
    for (int b = 0; 32 * b <= QCPW_MAX_N; ++b) {
        LaunchPlan lp;
        lp.path = path;
        lp.precision = precision;
        lp.owen = owen;
        LaunchSeg sg;
        sg.max_n = 32 * b;
        for (int wide = 0; wide < (f32 ? 2 : 1); ++wide) {
            sg.wide = wide != 0;
            if (f32 && sg.wide && sg.max_n <= QCPW_WIDE_MIN_N) continue;
            if (f32 && !sg.wide && sg.max_n > QCPW_WIDE_MIN_N && !paths_lds_fits(lp, sg, 768)) continue;
            (void)autotune_block_threads(ctx, lp, sg);
        }
    }
}

qcpw_status enqueue_pca(Context *ctx, const LaunchPlan &lp, hipStream_t stream, const LaunchDesc &ld,
                        const OptDev *d_opts);

qcpw_status enqueue_launch(Context *ctx, const LaunchPlan &lp, hipStream_t stream, double *dev_out_greeks,
                           double *dev_out_stderr, double *dev_out_per_shift, void *ws, size_t ws_bytes,
                           const void *h_upload, bool timed, double *dev_out_sigma)
{
    // qcpw_kernel_timer: a pair of events around the main kernel
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (timed && ctx->timer.on) {
        Context::Timer &tm = ctx->timer;
        while (tm.ev.size() < tm.used + 2) {
            hipEvent_t e = nullptr;
            QCPW_HIP(hipEventCreate(&e));
            tm.ev.push_back(e);
        }
        t0 = tm.ev[tm.used];
        t1 = tm.ev[tm.used + 1];
        tm.used += 2;
    }
    const WsLayout w = ws_layout(lp);
    if (ws_bytes < w.total) return fail(QCPW_ENOMEM, "workspace too small");
    char *base = (char *)ws;
    OptDev *d_opts = (OptDev *)(base + w.opts);
    int64_t *d_prefix = (int64_t *)(base + w.prefix);
    double *d_partials = (double *)(base + w.partials);
    double *d_per_shift = dev_out_per_shift ? dev_out_per_shift : (double *)(base + w.per_shift);
    unsigned long long *d_counter = (unsigned long long *)(base + w.counter);
    const size_t n = lp.opts.size();
    // options, unit prefix and zeroed queue heads in one copy
    std::vector<unsigned char> staged;
    if (!h_upload) {
        staged.resize(w.upload);
        fill_launch_upload(lp, staged.data());
        h_upload = staged.data();
    }
    QCPW_HIP(hipMemcpyAsync(base, h_upload, w.upload, hipMemcpyHostToDevice, stream));

    LaunchDesc ld;
    ld.opts = d_opts;
    ld.unit_prefix = d_prefix;
    ld.n_opts = (int32_t)n;
    ld.max_n = lp.max_n;
    ld.total_units = lp.total_units;
    ld.plan = ctx->tab.plan;
    ld.plan64 = ctx->tab.plan64;
    ld.dir = ctx->tab.dir;
    ld.lane = ctx->tab.lane;
    ld.partials = d_partials;
    ld.counter = d_counter;
    ld.scratch = (double *)(base + w.scratch);

    if (lp.path == QCPW_PATH_PCA || lp.path == QCPW_PATH_PCA_FULL) {
        if (t0) QCPW_HIP(hipEventRecord(t0, stream));
        qcpw_status st = enqueue_pca(ctx, lp, stream, ld, d_opts);
        if (st != QCPW_OK) return st;
        if (t1) QCPW_HIP(hipEventRecord(t1, stream));
    } else {
        // the launches (one, or the 128-VGPR one and then the 80-VGPR one):
        // each takes its options and units, with queue heads of its own
        if (lp.segs.empty() || lp.segs.size() > QCPW_MAX_SEGS) return fail(QCPW_EDEVICE, "launch without segments");
        for (size_t si = 0; si < lp.segs.size(); ++si) {
            const LaunchSeg &sg = lp.segs[si];
            if (sg.opt0 < 0 || sg.n_opts < 1 || (size_t)sg.opt0 + sg.n_opts > n || sg.units < 1 ||
                sg.unit0 != lp.unit_prefix[sg.opt0] || sg.unit0 + sg.units != lp.unit_prefix[sg.opt0 + sg.n_opts])
                return fail(QCPW_EDEVICE, "inconsistent launch segment");
            const int bd = sg.block_threads;
            if (!paths_lds_fits(lp, sg, bd)) return fail(QCPW_EDIMS, "LDS footprint exceeds 160 KiB");
            int a_stk_off = 0;
            const size_t lds = paths_lds_bytes(lp, sg, bd, &a_stk_off);
            const void *fn = select_paths_kernel(lp, sg);
            if (lp.precision == QCPW_FP32_MIXED) {
                qcpw_status st = check_lds_at_zero(fn);
                if (st != QCPW_OK) return st;
            }
            QCPW_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            int per_cu = 0;
            QCPW_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, bd, lds));
            if (per_cu < 1) return fail(QCPW_EDEVICE, "per-path kernel cannot be resident with this block size");
            int64_t grid = (int64_t)per_cu * ctx->tab.n_cu;
            grid = std::min<int64_t>(grid, sg.units);
            const OptDev *a_opts = ld.opts + sg.opt0;
            const int64_t *a_prefix = ld.unit_prefix + sg.opt0;
            const PlanStep *a_plan = ld.plan;
            const PlanStep64 *a_plan64 = ld.plan64;
            const uint32_t *a_sev = ctx->tab.split_ev;
            const uint16_t *a_sdim = ctx->tab.split_dim;
            const uint32_t *a_dir = ld.dir, *a_lane = ld.lane;
            const float4 *a_tab = ctx->tab.ninv_tab;
            double *a_part = ld.partials;
            unsigned long long *a_ctr = ld.counter + si * QCPW_QUEUES * QCPW_QUEUE_STRIDE;
            int a_nopts = sg.n_opts, a_maxn = sg.max_n, a_depth = sg.stack_depth;
            long long a_total = sg.units, a_base = sg.unit0;
            int a_fixed_arg = fixed_bridges_on() ? 1 : 0;
            uint32_t *a_probe = lp.probe;
            void *args[] = {&a_opts, &a_prefix, &a_plan, &a_plan64, &a_sev,  &a_sdim,      &a_dir,
                            &a_lane, &a_tab,    &a_part, &a_ctr,    &a_nopts, &a_maxn,     &a_depth,
                            &a_stk_off, &a_total, &a_base, &a_fixed_arg, &a_probe};
            if (t0 && si == 0) QCPW_HIP(hipEventRecord(t0, stream));
            QCPW_HIP(hipLaunchKernel(fn, dim3((unsigned)grid), dim3(bd), args, lds, stream));
        }
        if (t1) QCPW_HIP(hipEventRecord(t1, stream));
    }
    finalize_kernel<<<(unsigned)n, 256, 0, stream>>>(d_opts, d_partials, d_per_shift, dev_out_greeks, dev_out_stderr,
                                                     dev_out_sigma);
    QCPW_HIP(hipGetLastError());
    return QCPW_OK;
}

qcpw_status launch_sobol_points(Context *ctx, uint64_t seed, int32_t shift_index, int32_t n_dims, int64_t k0,
                                int64_t count, uint32_t *dev_out, hipStream_t stream, bool owen)
{
    const int64_t first = k0 & ~int64_t(63);
    const int64_t blocks = (k0 + count - first + 63) / 64;
    if (owen)
        sobol_points_kernel<true><<<(unsigned)blocks, 64, 0, stream>>>(ctx->tab.dir, ctx->tab.lane, seed,
                                                                       shift_index, n_dims, k0, count, dev_out);
    else
        sobol_points_kernel<false><<<(unsigned)blocks, 64, 0, stream>>>(ctx->tab.dir, ctx->tab.lane, seed,
                                                                        shift_index, n_dims, k0, count, dev_out);
    QCPW_HIP(hipGetLastError());
    return QCPW_OK;
}

}  // namespace qcpw
