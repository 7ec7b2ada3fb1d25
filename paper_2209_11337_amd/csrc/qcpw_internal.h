// qcpw_internal.h -- structures shared by the host library and the kernels.
//
// Device-resident tables (built once per device, kept for the process):
//   * dir[QCPW_TAB_DIMS][32]   Sobol direction numbers, dir[j][b] = g_{b+1} of
//                              dimension j as a 32-bit binary fraction.
//   * lane[QCPW_TAB_DIMS][64]  the low part of every point inside a wave:
//                              lane[j][t] = XOR of dir[j][b] over the set bits
//                              b of gray(t), t = 0..63.  Because point
//                              k = base + t with base a multiple of 64 has
//                              gray(k) = gray(base) XOR gray(t), the Sobol
//                              integer is lane[j][t] XOR (dir_j . gray(base)),
//                              and the second term is the same for the whole
//                              wave.
//   * bridge plans             one per n = d - 1 (see PlanStep).
// Per launch:
//   * OptDev[n_opts]           derived FP64 / FP32 constants of each option.
//   * unit prefix              work units (option, replication, chunk) of each
//                              option, options sorted by cost.
//   * partials[units][8]       per-chunk compensated sums (4 values + errors).
#pragma once
#include <stdint.h>

#define QCPW_TAB_DIMS 1024       // Sobol dimensions held on the device
#define QCPW_MAX_N 384           // conditioned coordinates in the fused kernel
#define QCPW_UQ 6                // QCPW_MAX_N / 64 registers of wave-uniform state
// LDS of the per-path kernel (all dynamic, so it starts at address 0):
// the lower-half inverse-normal cells at 0, the upper-half cells at
// QCPW_LDS_TAB_HI (the sign bit of the cell offset), the lane-table rows of
// dimensions 1..QCPW_LDS_GAP_ROWS between them and the rest after the upper
// cells; the bridge stacks follow the rows.  When rows go beyond the gap,
// the upper region starts with a second copy of the last QCPW_LDS_DUP_ROWS
// rows of the gap, so that a run of consecutive rows that crosses the gap
// (the split bridge reads a subtree's nodes of one level as such a run) can
// be read at one base and a fixed stride from the upper region.
#define QCPW_LDS_TAB_HI 0x8000
#define QCPW_LDS_GAP_BEGIN 0x1000
#define QCPW_LDS_FIXED (QCPW_LDS_TAB_HI + 0x1000)
#define QCPW_LDS_GAP_ROWS ((QCPW_LDS_TAB_HI - QCPW_LDS_GAP_BEGIN) / 256)
#define QCPW_LDS_DUP_ROWS 8

// 32-bit word offset of lane-table row r (dimension r + 1) in the upper
// region, r >= QCPW_LDS_GAP_ROWS - QCPW_LDS_DUP_ROWS
__host__ __device__ constexpr int qcpw_row_word_hi(int r)
{
    return QCPW_LDS_FIXED / 4 + 64 * (r - (QCPW_LDS_GAP_ROWS - QCPW_LDS_DUP_ROWS));
}
// 32-bit word offset in that LDS of lane-table row r (dimension r + 1)
__host__ __device__ constexpr int qcpw_row_word(int r)
{
    return r < QCPW_LDS_GAP_ROWS ? QCPW_LDS_GAP_BEGIN / 4 + 64 * r : qcpw_row_word_hi(r);
}
// ... and back: the row at a word offset of either region
__host__ __device__ constexpr int qcpw_word_row(uint32_t w)
{
    return w < QCPW_LDS_TAB_HI / 4 ? (int)(w - QCPW_LDS_GAP_BEGIN / 4) / 64
                                   : QCPW_LDS_GAP_ROWS - QCPW_LDS_DUP_ROWS + (int)(w - QCPW_LDS_FIXED / 4) / 64;
}

// Work queues of the fused kernel: one head per XCD, each on its own
// 256-byte line.  Queue q hands out units q, q + QCPW_QUEUES, ...
#define QCPW_QUEUES 8
#define QCPW_QUEUE_STRIDE 32     // u64 words between heads
#define QCPW_CHUNK 8192          // alignment of point ranges; points per PCA work unit

// Points per work unit of the fused kernel (one wave per unit): a function of
// the option's point count only, so an option's result does not depend on
// what else shares the launch or on the workgroup size.  256..4096 points,
// about N/256, a power of two (so it divides QCPW_CHUNK).
static inline int64_t qcpw_unit_points(int64_t n_points)
{
    int64_t c = 256;
    while (c < 4096 && c * 256 < n_points) c *= 2;
    return c;
}
// Workgroup sizes the fused kernel accepts: 0 (autotuned) or whole waves up
// to the kernel's launch bound.
static inline bool qcpw_block_threads_ok(int v) { return v == 0 || (v >= 64 && v <= 1024 && v % 64 == 0); }
#define QCPW_STACK_MAX 12        // bridge stack depth bound (ceil log2 QCPW_MAX_N + 2)
#define QCPW_PCA_NPAD 256        // padded factor size of the matrix-core PCA kernel
#define QCPW_PCA_MAX_GROUP 4     // options sharing one product and epilogue in the matrix-core PCA kernel
#define QCPW_FIXED_MAX_N 127     // largest n with a compile-time bridge

// n (= d - 1) that the FP32 kernel walks with a compile-time bridge; the
// host leaves such options out of the LDS stack size, so this is the one list.
__host__ __device__ constexpr bool qcpw_has_fixed_bridge(int n)
{
    return n == 15 || n == 31 || n == 63 || n == 127;
}

// Square root by Newton's method from above, usable in constant expressions
// (within one ulp).  The bridge weights of the run-time plans and of the
// compile-time bridges both come from this function, so they hold the same
// bits.
constexpr double qcpw_csqrt(double x)
{
    if (!(x > 0.0)) return 0.0;
    double r = x > 1.0 ? x : 1.0;
    for (int i = 0; i < 400; ++i) {
        const double nr = 0.5 * (r + x / r);
        if (!(nr < r)) break;
        r = nr;
    }
    return r;
}

// Sobol dimension of the midpoint of interval (lo, hi) in the bridge over
// grid points 0..n: intervals with hi - lo >= 2 taken breadth first from
// (0, n), left half before right half, get dimensions 2, 3, ... (dimension 1
// is the terminal point).  -1 if (lo, hi) is not such an interval.
constexpr int qcpw_bridge_dim(int n, int lo, int hi)
{
    int ql[2 * QCPW_FIXED_MAX_N + 4] = {}, qh[2 * QCPW_FIXED_MAX_N + 4] = {};
    if (n > QCPW_FIXED_MAX_N) return -1;
    int head = 0, tail = 0, next = 2;
    ql[tail] = 0;
    qh[tail] = n;
    ++tail;
    while (head < tail) {
        const int l = ql[head], r = qh[head];
        ++head;
        if (r - l < 2) continue;
        if (l == lo && r == hi) return next;
        ++next;
        const int m = (l + r) / 2;
        ql[tail] = l; qh[tail] = m; ++tail;
        ql[tail] = m; qh[tail] = r; ++tail;
    }
    return -1;
}

// Position of the midpoint of interval (lo, hi) in the order the kernels
// walk the bridge: depth first, a midpoint before its left half before its
// right half; the terminal point is step 0.  -1 if not such an interval.
constexpr int qcpw_bridge_step(int n, int lo, int hi)
{
    int sl[64] = {}, sh[64] = {};
    if (n > QCPW_FIXED_MAX_N) return -1;
    int top = 0, step = 1;
    sl[top] = 0;
    sh[top] = n;
    ++top;
    while (top > 0) {
        --top;
        const int l = sl[top], r = sh[top];
        if (r - l < 2) continue;
        if (l == lo && r == hi) return step;
        ++step;
        const int m = (l + r) / 2;
        sl[top] = m; sh[top] = r; ++top;   // right half, taken after the left half
        sl[top] = l; sh[top] = m; ++top;
    }
    return -1;
}

// Sobol dimension of the midpoint the kernels visit at step S (1 <= S < n)
// of the depth-first walk; -1 past the end.
constexpr int qcpw_bridge_dim_at_step(int n, int S)
{
    int sl[64] = {}, sh[64] = {};
    if (n > QCPW_FIXED_MAX_N) return -1;
    int top = 0, step = 1;
    sl[top] = 0;
    sh[top] = n;
    ++top;
    while (top > 0) {
        --top;
        const int l = sl[top], r = sh[top];
        if (r - l < 2) continue;
        if (step == S) return qcpw_bridge_dim(n, l, r);
        ++step;
        const int m = (l + r) / 2;
        sl[top] = m; sh[top] = r; ++top;
        sl[top] = l; sh[top] = m; ++top;
    }
    return -1;
}

// One step of a bridge plan, in the order the kernel walks the bridge: the
// intervals of the breadth-first bridge are visited depth first, so that only
// a short stack of right end points is live at any time.  Step 0 is the
// terminal point W~(n dt) (no push); step s >= 1 is the midpoint m of an
// interval (l, r): before it, `pops` times "L = R; R = stack.pop()"; then
// W_m = wl * L + wr * R + sd * z_{dim}; stack.push(R); R = W_m.
// A pop followed by the push of the value it returned leaves the stack as
// it was, so the kernel only writes when pops = 0 (slot = the stack depth
// before the step) and otherwise only reads: R = stack[slot] and, for
// pops >= 2, L = stack[slot + 1] (slot = depth - pops; depth after the
// step = slot + 1).
struct PlanStep {
    int32_t lds_off;   // qcpw_row_word(dim - 1): LDS word of the lane-table row of this step's dimension
    int32_t slot;      // stack slot written (pops = 0) or read (pops >= 1)
    int32_t pops;      // stack pops before the step
    int32_t dim;       // Sobol dimension of the step (1..n)
    float wl, wr, sd;  // (r-m)/(r-l), (m-l)/(r-l), sqrt((m-l)(r-m)/(r-l)) in units of sqrt(dt)
    float mf;          // float(m), m = grid index of the new point (1..n)
};
struct PlanStep64 {
    double wl, wr, sd, mf;
};

// ---- split bridge (FP32 kernel, any n >= QCPW_SUB_MIN_LEN) ---------------
// At level k of the bridge (k = 0 for the interval (0, n) itself) every
// interval has length floor(n / 2^k) or ceil(n / 2^k).  With k the smallest
// level whose lengths are at most QCPW_SUB_MAX_LEN, they lie in
// [QCPW_SUB_MIN_LEN, QCPW_SUB_MAX_LEN] (n >= QCPW_SUB_MIN_LEN), and each such
// interval is walked by a compile-time subtree of its length: its midpoints
// depth first with literal weights and pending right end points in
// registers.  Only the 2^k - 1 midpoints above level k ("top nodes") and
// every node's Sobol dimension come from the plan, as a list of events in
// depth-first order: the terminal point, then top midpoints and subtrees.
// The wave-uniform parts are laid out in "slots" (slot s in register s / 64,
// lane s % 64): the terminal and the top nodes first, then each subtree's
// nodes contiguous and inside one register, so that one row broadcast per
// node serves them.
#define QCPW_SUB_MIN_LEN 12
#define QCPW_SUB_MAX_LEN 24
#define QCPW_SPLIT_EVENTS 32     // 1 + (2^k - 1) + 2^k, k <= 4
#define QCPW_SPLIT_SLOTS 512     // 8 registers of 64 lanes
#define QCPW_EV_WORDS 16         // one 64-byte event, one scalar load
// Beyond 181 lane rows three 512-thread workgroups of the 80-VGPR kernel
// instances no longer fit the LDS of a CU: FP32 launches of more rows take
// those instances only at 768 threads while two such workgroups fit, and
// the 128-VGPR instances otherwise (the launch planner decides).
#define QCPW_WIDE_MIN_N 181

// The level k at which the split bridge of n starts its subtrees.
__host__ __device__ constexpr int qcpw_split_level(int n)
{
    int k = 0;
    while (((n + (1 << k) - 1) >> k) > QCPW_SUB_MAX_LEN) ++k;
    return k;
}

// Event header (word 0): kind, subtree length, slot register and lane.
enum { QCPW_EV_TERMINAL = 0, QCPW_EV_TOP = 1, QCPW_EV_SUB = 2 };
__host__ __device__ constexpr uint32_t qcpw_ev_header(int kind, int len, int reg, int lane)
{
    return (uint32_t)kind | ((uint32_t)len << 8) | ((uint32_t)reg << 16) | ((uint32_t)lane << 24);
}
// Event words: [0] header; [1] grid index m (terminal n, top midpoint m,
// subtree left end l); [2] float(m) bits; [3] float(2^23 + m) bits (an
// index carried in a float whose bits grow with it by one per step);
// terminal / top: [4] lane-table word of the node's dimension, [5] wl,
// [6] wr, [7] sd (units of sqrt(dt)); terminal: [8] the number of events;
// top: [8] l, [9] r (its interval); subtree: [4 + j], j = 0..4, the
// lane-table word of the first node of the subtree's level j.  The
// breadth-first numbering gives the nodes of one level of a subtree
// consecutive dimensions, left to right, so node i of level j reads the
// word [4 + j] + 64 i (qcpw_sub_pos gives (j, i) of a depth-first step).

// Level and left-to-right index, among the nodes of that level, of the
// depth-first step s of a subtree over (0, len).
struct QcpwSubPos {
    int level, index;
};
__host__ __device__ constexpr int qcpw_sub_left(int l, int r, int depth, int level, int lo)
{
    // nodes of the given level below (l, r) whose interval starts left of lo
    if (r - l < 2) return 0;
    if (depth == level) return l < lo ? 1 : 0;
    const int m = (l + r) / 2;
    return qcpw_sub_left(l, m, depth + 1, level, lo) + qcpw_sub_left(m, r, depth + 1, level, lo);
}
__host__ __device__ constexpr QcpwSubPos qcpw_sub_pos(int len, int s)
{
    int l = 0, r = len, step = 0, depth = 0;
    while (step != s) {
        const int m = (l + r) / 2;
        if (s <= step + (m - l - 1)) { step += 1; r = m; }   // in the left subtree (m - l - 1 nodes)
        else { step += m - l; l = m; }                      // skip the midpoint and its left subtree
        ++depth;
    }
    return QcpwSubPos{depth, qcpw_sub_left(0, len, 0, depth, l)};
}
#define QCPW_SUB_LEVELS 5        // levels of a subtree of length <= QCPW_SUB_MAX_LEN

// Depth-first position of the midpoint of (lo, hi) inside a subtree over
// (0, len) (root 0, left subtree before right subtree): the midpoint of an
// interval of length L is followed by the L - 2 midpoints below it.
__host__ __device__ constexpr int qcpw_sub_step(int len, int lo, int hi)
{
    int l = 0, r = len, step = 0;
    while (r - l >= 2) {
        const int m = (l + r) / 2;
        if (l == lo && r == hi) return step;
        if (hi <= m) { ++step; r = m; }
        else { step += m - l; l = m; }   // skip the midpoint and its left subtree's m - l - 1 nodes
    }
    return -1;
}

// Per-option constants (host-computed in FP64).
struct OptDev {
    int32_t type, d, n, path;     // n = d - 1
    int32_t plan_off;             // first PlanStep of this option's bridge plan
    int32_t chunks;               // work units per replication
    int32_t unit_pts;             // points per work unit
    int64_t n_points;             // points in this launch: k_begin .. k_begin + n_points - 1
    int64_t k_begin;              // first Sobol point (a multiple of QCPW_CHUNK)
    uint64_t seed;
    int64_t unit0;                // first work unit of this option
    int32_t n_shifts;
    int32_t out_index;            // row of this option in the caller's arrays
    // FP64 path constants (log2-space path Y_m = log2(S~(t_{m+1}) / S0))
    double zscale;                // sigma * sqrt(dt) * log2(e): z -> Y units
    double ydrift_n;              // omega * n * dt * log2(e): drift of Y_n
    double ydrift_1;              // omega * dt * log2(e): drift per step (standard)
    double kappa;                 // (r + sigma^2/2) dt log2(e): W - sigma tau = (Y - kappa m)/(sigma log2 e)
    double inv_sig_log2e;         // 1 / (sigma log2(e))
    double c0;                    // ln K - ln S0 - omega t1 (+ ln d for the arithmetic average)
    double h;                     // exp(c0 - s1^2/2)
    double inv_s1, s1, sqrt_t1, inv_sigma;
    double S0, K, D, D1, invd, inv_S0, inv_S0sq;
    float ydrift_n_f, ydrift_1_f;
    float zs_t;                   // zscale (FP32 table inverse normal)
    // principal-component factor of this option's n (unit dt), device layouts:
    const float *pca_At;          // [NP][NP] FP32, k-major: At[k][row]
    const uint16_t *pca_hi;       // [NP/16][NP][16] BF16 hi part, 16-wide k slabs
    const uint16_t *pca_lo;       // same, lo part
    const double *pca_A64;        // [n][n] FP64 row-major ([d][n] for PCA_FULL)
    const double *pca_a1;         // PCA_FULL: first column of the d x d unit-dt factor
    int32_t pca_np;               // rows / columns padded to a multiple of 32 (<= QCPW_PCA_NPAD)
    int32_t n_assets;             // basket: assets M (0 for the single-asset products)
    int32_t ndims;                // Sobol dimensions a path reads after x_1: n, or n + M d (basket)
    int32_t split;                // split bridge (FP32): 1 = walk the events of n, 0 = the plan
    int32_t n_slots;              // wave-uniform slots (split bridge) or ndims
    int32_t grp;                  // matrix-core PCA: options sharing this one's paths (leader), 0 (member)
    int32_t pad2_;
    // basket: scales of the common and idiosyncratic normals in Y units
    // (sqrt(rho), sqrt(1 - rho) times sigma sqrt(dt) log2 e), and the sigma
    // derivative of the drift factor exp(omega t1 + s1^2/2) per unit X
    double b_common, b_idio, vx_shift;
    float b_common_f, b_idio_f;
    // per-option factors of the FP64 tail (sgn = -1 for puts, phi_c =
    // 1/sqrt(2 pi)); averages, extremes: sDK = sgn D K, sD1 = sgn D1, h2 = h/2,
    // gv = D K phi_c sqrt_t1, gg = D K phi_c inv_s1 inv_S0sq; binary:
    // gb = sgn D phi_c, gd = gb inv_s1 inv_S0, gg = gb inv_s1 inv_S0sq
    double sDK, sD1, h2, gv, gg, gb, gd;
};

// Packed work description for one launch.
struct LaunchDesc {
    const OptDev *opts;           // [n_opts], sorted by cost
    const int64_t *unit_prefix;   // [n_opts + 1] exclusive prefix of units
    int32_t n_opts;
    int32_t max_n;                // largest n in the launch (LDS sizing)
    int64_t total_units;
    const PlanStep *plan;         // all plans
    const PlanStep64 *plan64;
    const uint32_t *dir;          // [QCPW_TAB_DIMS][32]
    const uint32_t *lane;         // [QCPW_TAB_DIMS][64]
    double *partials;             // [total_units][8]
    const uint32_t *split_ev;     // [QCPW_MAX_N + 1][QCPW_SPLIT_EVENTS][QCPW_EV_WORDS]
    const uint16_t *split_dim;    // [QCPW_MAX_N + 1][QCPW_SPLIT_SLOTS] Sobol dimension of each slot (0: none)
    double *scratch;              // FP64 PCA_FULL: [workgroup][date][64] products
    unsigned long long *counter;  // work-queue heads, QCPW_QUEUES of them, QCPW_QUEUE_STRIDE apart
};
