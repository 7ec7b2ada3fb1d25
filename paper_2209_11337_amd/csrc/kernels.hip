// kernels.hip -- the fused per-path QMC-CPW kernel for gfx950 (MI355X), the
// per-replication finalize kernel, and their launch planning.
//
// One persistent launch covers every option of a call.  Work units are
// (option, replication l, range of unit_pts consecutive Sobol points, a
// function of the option's point count alone); each wave pulls units from
// device counters and gives each lane one point per iteration, so for point
// k = base + lane (base a multiple of 64):
//
//   Sobol integer of dimension j (Sec. 2.2.2, XOR form of
//   eqn:GeneratorMatrixExpression, Gray-code order):
//       y_j = lane_table[j][lane]  XOR  U_j(base),
//   where U_j(base) = dir_j . gray(base) XOR s_{l,j} is the same for the
//   whole wave (the digital shift of Sec. 2.2.3 is folded in).  Stepping to
//   the next base changes U_j by two direction numbers only.  U is held in
//   registers, distributed over the lanes in the order the path consumes the
//   dimensions, and broadcast with v_readlane.
//
//   Inverse normal, path construction (Sec. 3.4.1 W~ = A z, Sec. 4.4 bridge
//   or Alg. 3 increments), exponentials and running sums (Sec. 4.1: nothing
//   about the path is stored) all stay in registers / LDS.  The path is
//   built directly in log2 space, Y_m = log2(S~(t_{m+1}) / S0), so each date
//   costs one exp2.
//
//   Per path, in FP64: breakpoint psi of the conditioned normal x_1
//   (Sec. 3.4.2), Phi tails, and price/delta/vega/gamma (Sec. 4.5), added
//   into compensated per-lane sums; a fixed wave butterfly reduces them to
//   one partial per unit.  The finalize kernel adds a replication's partials
//   in chunk order and forms mean and standard error over replications
//   (Sec. 5).
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

// ------------------------------------------------------------------------
// the fused per-path kernel
// ------------------------------------------------------------------------
struct UnitCtx {
    int64_t unit;
    int o;
    int shift;
    int64_t chunk;
};

// The wave-uniform part of the Sobol coordinates the lanes consume: for step
// s = lane + 64 q, U[q] = G_dim gray(base), folded with the digital shift
// (the lane table is folded too), or -- with nested scrambling -- raw, with
// the dimension's scrambling seed in Sd[q] (the lane table then raw too).
// PROBE instances also record every coordinate the walk consumes, at
// pr[(dim - 1) * 64 + lane] of the current 64-point batch, so that the
// integers of the per-path kernel itself can be checked bit for bit.
template <bool OWEN_, bool PROBE = false>
struct UParts {
    static constexpr bool OWEN = OWEN_;
    uint32_t U[QCPW_UQ];
    uint32_t Sd[OWEN ? QCPW_UQ : 1];
    uint32_t *pr;
    // randomised coordinate of step 64 q + k from the lane's table word
    __device__ __forceinline__ uint32_t bits(uint32_t lane_word, int q, int k) const
    {
        if constexpr (OWEN) return owen_scramble(lane_word ^ rdlane(U[q], k), rdlane(Sd[q], k));
        else return lane_word ^ rdlane(U[q], k);
    }
    __device__ __forceinline__ uint32_t rec(uint32_t y, int dim, int lane) const
    {
        if constexpr (PROBE) pr[(dim - 1) * 64 + lane] = y;
        return y;
    }
};

// LDS word of lane-table row r: around the inverse-normal cells in the FP32
// kernels (qcpw_row_word), contiguous from 0 in the FP64 kernels.
template <bool F32>
__device__ __forceinline__ int lane_row(int r)
{
    return F32 ? qcpw_row_word(r) : 64 * r;
}

template <bool F32, int MODE, class UP>
__device__ inline void run_bridge_wave(const LaunchDesc &ld, const OptDev &op, const uint32_t *lds_lane,
                                       typename Real<F32>::T *stk, int lane,
                                       const UP &U, PathSums<typename Real<F32>::T> &ps)
{
    using R = typename Real<F32>::T;
    const int n = op.n;
    const PlanStep *plan = ld.plan + op.plan_off;
    const PlanStep64 *plan64 = ld.plan64 + op.plan_off;
    R L = R(0), Rr;
    {   // terminal point
        const PlanStep st = plan[0];
        const uint32_t x = U.rec(U.bits(lds_lane[(F32 ? st.lds_off : (st.dim - 1) * 64) + lane], 0, 0), st.dim, lane);
        const R z = coord_tab<F32>(x, op);
        const R sd = F32 ? (R)st.sd * op.zs_t : (R)plan64[0].sd;
        const R drift = F32 ? (R)op.ydrift_n_f : (R)op.ydrift_n;
        Rr = fma(sd, z, drift);
        consume<R, MODE>(ps, Rr, F32 ? (R)st.mf : (R)plan64[0].mf);
    }
#pragma unroll
    for (int q = 0; q < QCPW_UQ; ++q) {
        const int s_lo = q == 0 ? 1 : 64 * q;
        const int s_hi = min(64 * (q + 1), n);
#pragma unroll 2
        for (int s = s_lo; s < s_hi; ++s) {
            const PlanStep st = plan[s];
            // stack: this lane's column, slot k at stk[64 k]
            R *slot = stk + st.slot * 64;
            if (st.pops == 0) {
                *slot = Rr;
            } else {
                const R r = slot[0];
                L = st.pops == 1 ? Rr : slot[64];
                Rr = r;
            }
            const uint32_t x =
                U.rec(U.bits(lds_lane[(F32 ? st.lds_off : (st.dim - 1) * 64) + lane], q, s - 64 * q), st.dim, lane);
            const R z = coord_tab<F32>(x, op);
            R Ym;
            R mf;
            if constexpr (F32) {
                Ym = fmaf(st.sd, __fmul_rn(z, op.zs_t), fmaf(st.wr, Rr, st.wl * L));
                mf = st.mf;
            } else {
                const PlanStep64 s64 = plan64[s];
                Ym = fma(s64.sd, z, fma(s64.wr, Rr, s64.wl * L));
                mf = s64.mf;
            }
            Rr = Ym;
            consume<R, MODE>(ps, Ym, mf);
        }
        if (s_hi >= n) break;
    }
}

// ---- compile-time bridges ------------------------------------------------
// For n = 15, 31, 63, 127 (d = 16, 32, 64, 128) the bridge is unrolled at
// compile time: the depth-first walk becomes template recursion over the
// intervals, the pending right end points live in registers (no LDS stack,
// no register shuffles), lane-table rows and U lanes are immediates, and the
// weights are literals.  The intervals, dimensions, step order, weights and
// formulas are those of the run-time plan (the host checks the plan against
// the same constexpr functions); price, delta and gamma come out bit-identical
// to the plan walker's, vega (from the FP32 sums of E Y and E m) within FP32
// rounding.  Removes about a quarter of the VALU work per date.
// The wave-uniform parts as the compile-time bridges read them.  Without
// scrambling they are copied once per 64 points into every row of 16 lanes
// (lane l of R[i] holds step 16 i + l mod 16), so that a DPP row broadcast
// (row_newbcast) hands step S's value to all lanes inside the very XOR that
// combines it with the lane word: no v_readlane per date.  With nested
// scrambling the distributed parts are read as in the plan walker.
template <class UP, int NSTEP, bool OWEN = UP::OWEN>
struct FixedU;

template <class UP, int NSTEP>
struct FixedU<UP, NSTEP, false> {
    static constexpr int NR = (NSTEP + 15) / 16;
    uint32_t R[NR];
    const UP &Up;
    __device__ __forceinline__ FixedU(const UP &U, int lane) : Up(U)
    {
#pragma unroll
        for (int i = 0; i < NR; ++i) R[i] = (uint32_t)__shfl((int)U.U[i / 4], 16 * (i % 4) + (lane & 15), 64);
    }
    template <int S>
    __device__ __forceinline__ uint32_t bits(uint32_t lane_word) const
    {
        return lane_word ^ (uint32_t)__builtin_amdgcn_update_dpp(0, (int)R[S / 16], 0x150 + S % 16, 0xF, 0xF, false);
    }
    __device__ __forceinline__ uint32_t rec(uint32_t y, int dim, int lane) const { return Up.rec(y, dim, lane); }
};

template <class UP, int NSTEP>
struct FixedU<UP, NSTEP, true> {
    const UP &U;
    __device__ __forceinline__ FixedU(const UP &u, int) : U(u) {}
    template <int S>
    __device__ __forceinline__ uint32_t bits(uint32_t lane_word) const
    {
        return U.bits(lane_word, S / 64, S % 64);
    }
    __device__ __forceinline__ uint32_t rec(uint32_t y, int dim, int lane) const { return U.rec(y, dim, lane); }
};

template <int MODE, class UP, int N, int LO, int HI>
__device__ __forceinline__ void fixed_interval(const uint32_t *row0, int lane, float zs,
                                               const FixedU<UP, N> &U, float WL, float WR,
                                               PathSums<float> &ps)
{
    if constexpr (HI - LO >= 2) {
        constexpr int M = (LO + HI) / 2;
        constexpr int DIM = qcpw_bridge_dim(N, LO, HI);
        constexpr int S = qcpw_bridge_step(N, LO, HI);
        static_assert(DIM >= 2 && S >= 1, "interval outside the bridge");
        constexpr float wl = (float)((double)(HI - M) / (double)(HI - LO));
        constexpr float wr = (float)((double)(M - LO) / (double)(HI - LO));
        constexpr float sd = (float)qcpw_csqrt((double)(M - LO) * (double)(HI - M) / (double)(HI - LO));
        const uint32_t x = U.rec(U.template bits<S>(row0[qcpw_row_word(DIM - 1)]), DIM, lane);
        const float z = ninv_table_f32(x);
        const float Ym = fmaf(sd, __fmul_rn(z, zs), fmaf(wr, WR, wl * WL));   // no contraction: as the plan walker
        consume<float, MODE>(ps, Ym, (float)M);
        fixed_interval<MODE, UP, N, LO, M>(row0, lane, zs, U, WL, Ym, ps);
        fixed_interval<MODE, UP, N, M, HI>(row0, lane, zs, U, Ym, WR, ps);
    }
}

template <int MODE, class UP, int N>
__device__ __forceinline__ void run_bridge_fixed(const OptDev &op, const uint32_t *lds_lane,
                                                 int lane, const UP &Ud, PathSums<float> &ps)
{
    const uint32_t *row0 = lds_lane + lane;
    const float zs = op.zs_t;
    constexpr float sd0 = (float)qcpw_csqrt((double)N);
    const FixedU<UP, N> U(Ud, lane);
    const float z = ninv_table_f32(U.rec(U.template bits<0>(row0[qcpw_row_word(0)]), 1, lane));   // terminal, dimension 1
    const float WR = fmaf(sd0 * zs, z, op.ydrift_n_f);
    consume<float, MODE>(ps, WR, (float)N);
    fixed_interval<MODE, UP, N, 0, N>(row0, lane, zs, U, 0.0f, WR, ps);
}

// true if op.n has a compile-time bridge (then the path is done)
template <int MODE, class UP>
__device__ inline bool bridge_fixed_any(const OptDev &op, const uint32_t *lds_lane, int lane,
                                        const UP &U, PathSums<float> &ps)
{
    if (!qcpw_has_fixed_bridge(op.n)) return false;
    switch (op.n) {
    case 15: run_bridge_fixed<MODE, UP, 15>(op, lds_lane, lane, U, ps); return true;
    case 31: run_bridge_fixed<MODE, UP, 31>(op, lds_lane, lane, U, ps); return true;
    case 63: run_bridge_fixed<MODE, UP, 63>(op, lds_lane, lane, U, ps); return true;
    case 127: run_bridge_fixed<MODE, UP, 127>(op, lds_lane, lane, U, ps); return true;
    default: return false;
    }
}

template <bool F32, int MODE, class UP>
__device__ inline void run_standard_wave(const OptDev &op, const uint32_t *lds_lane, int lane,
                                         const UP &U, PathSums<typename Real<F32>::T> &ps)
{
    using R = typename Real<F32>::T;
    const int n = op.n;
    const R drift = F32 ? (R)op.ydrift_1_f : (R)op.ydrift_1;
    const R zs = F32 ? (R)op.zs_t : R(1);   // the FP32 table gives a standard normal
    R Y = R(0);
#pragma unroll
    for (int q = 0; q < QCPW_UQ; ++q) {
        const int s_hi = min(64 * (q + 1), n);
        for (int s = 64 * q; s < s_hi; ++s) {
            const uint32_t y = U.rec(U.bits(lds_lane[lane_row<F32>(s) + lane], q, s - 64 * q), s + 1, lane);
            const R z = coord_tab<F32>(y, op);
            Y = Y + fma(zs, z, drift);
            consume<R, MODE>(ps, Y, (R)(s + 1));
        }
        if (s_hi >= n) break;
    }
}

// The uniform part of Sobol step s (dimension s + 1) for a step index known
// only at run time (wave-uniform): the register holding it is picked by a
// uniform branch.
template <class UP>
__device__ __forceinline__ uint32_t ubits_at(const UP &U, uint32_t lane_word, int s)
{
    const int k = s & 63;
    switch (s >> 6) {
    case 0: return U.bits(lane_word, 0, k);
    case 1: return U.bits(lane_word, 1, k);
    case 2: return U.bits(lane_word, 2, k);
    case 3: return U.bits(lane_word, 3, k);
    case 4: return U.bits(lane_word, 4, k);
    default: return U.bits(lane_word, QCPW_UQ - 1, k);
    }
}

// Basket of M assets (one-factor model), standard construction, in date
// order: the common part C_m = log2(e) (omega tau_m + sigma sqrt(rho) B~_0)
// (steps from dimensions 1..n) and asset i's idiosyncratic part
// I_i = log2(e) sigma sqrt(1 - rho) B_i(t_{m+1}) (dimensions n + 1 + i d + m)
// add to Y_{i,m} = C_m + I_i, and every (asset, date) pair feeds the
// average's sums, date 1 included (its idiosyncratic part is random).
template <bool F32, class UP>
__device__ inline void run_basket_wave(const OptDev &op, const uint32_t *lds_lane, int lane, const UP &U,
                                       PathSums<typename Real<F32>::T> &ps)
{
    using R = typename Real<F32>::T;
    const int n = op.n, d = op.d, M = op.n_assets;
    const R drift = F32 ? (R)op.ydrift_1_f : (R)op.ydrift_1;
    const R bc = F32 ? (R)op.b_common_f : (R)op.b_common;
    const R bi = F32 ? (R)op.b_idio_f : (R)op.b_idio;
    auto normal = [&](int s) -> R {
        const uint32_t y = U.rec(ubits_at(U, lds_lane[lane_row<F32>(s) + lane], s), s + 1, lane);
        if constexpr (F32) return ninv_table_f32(y);
        else return (R)ninv_f64(y);
    };
    R I[QCPW_MAX_ASSETS];
#pragma unroll
    for (int i = 0; i < QCPW_MAX_ASSETS; ++i) I[i] = R(0);
    ps.A1 = R(0);   // no date with a known value: every (asset, date) pair is summed below
    R Cm = R(0);
    for (int m = 0; m < d; ++m) {
        if (m >= 1) Cm = Cm + fma(bc, normal(m - 1), drift);
#pragma unroll
        for (int i = 0; i < QCPW_MAX_ASSETS; ++i) {
            if (i < M) {
                I[i] = fma(bi, normal(n + i * d + m), I[i]);
                consume<R, QCPW_STAT_AVG>(ps, Cm + I[i], (R)m);
            }
        }
    }
}

// One wave's 64 paths from the terminal point (bridge) or the first step
// (standard) to the last date, accumulated into ps.
template <bool F32, int PATHK, int MODE, class UP>
__device__ inline void walk_path(const LaunchDesc &ld, const OptDev &op, const uint32_t *lds_lane,
                                 typename Real<F32>::T *stk, int lane,
                                 const UP &U, PathSums<typename Real<F32>::T> &ps, int fixed_bridges)
{
    if constexpr (PATHK == QCPW_PATH_BB) {
        if constexpr (F32) {
            if (fixed_bridges && bridge_fixed_any<MODE>(op, lds_lane, lane, U, ps)) return;
        }
        run_bridge_wave<F32, MODE>(ld, op, lds_lane, stk, lane, U, ps);
    } else {
        if constexpr (MODE == QCPW_STAT_AVG) {
            if (op.n_assets > 0) {
                run_basket_wave<F32>(op, lds_lane, lane, U, ps);
                return;
            }
        }
        run_standard_wave<F32, MODE>(op, lds_lane, lane, U, ps);
    }
}

// U_j(base) (and its seed) for the dimensions this lane holds: steps s = lane + 64 q.
template <int PATHK>
__device__ inline int step_dim(const LaunchDesc &ld, const OptDev &op, int s)
{
    return (PATHK == QCPW_PATH_BB) ? ld.plan[op.plan_off + s].dim : s + 1;
}

template <int PATHK, class UP>
__device__ inline void init_uniform_part(const LaunchDesc &ld, const OptDev &op, int shift, int lane,
                                         uint64_t base, UP &U)
{
    const uint64_t g = (base ^ (base >> 1)) >> 5;   // gray(base) has no bits below 5
#pragma unroll
    for (int q = 0; q < QCPW_UQ; ++q) {
        const int s = lane + 64 * q;
        int dim;
        uint32_t u = 0, key = 0;
        if (s < op.ndims) {
            dim = step_dim<PATHK>(ld, op, s);
            key = digital_shift(op.seed, shift, dim);
            const uint32_t *v = ld.dir + (size_t)dim * 32;
            uint64_t gg = g;
            for (int b = 5; gg != 0; ++b, gg >>= 1)
                if (gg & 1) u ^= v[b];
        }
        if constexpr (UP::OWEN) {
            U.U[q] = u;
            U.Sd[q] = key;
        } else {
            U.U[q] = u ^ key;
        }
    }
}

// base -> base + 64: gray changes in bits 5 and 6 + ctz(base/64 + 1).
template <int PATHK, class UP>
__device__ inline void step_uniform_part(const LaunchDesc &ld, const OptDev &op, int lane, uint64_t base,
                                         UP &U)
{
    const int c = __builtin_ctzll((base >> 6) + 1);
#pragma unroll
    for (int q = 0; q < QCPW_UQ; ++q) {
        const int s = lane + 64 * q;
        if (s < op.ndims) {
            const uint32_t *v = ld.dir + (size_t)step_dim<PATHK>(ld, op, s) * 32;
            U.U[q] ^= v[5] ^ v[6 + c];
        }
    }
}

// Every wave pulls its own work units (option, replication, range of
// unit_pts consecutive points): no workgroup barrier after start-up, and the
// order of every sum depends on the unit alone.  The workgroup only shares
// the LDS tables (inverse-normal cells, lane rows of all dimensions the
// launch needs), loaded once.
// The FP32 kernel is bound by latency as much as by issue (every step waits
// on scalar plan loads and two dependent LDS reads), so it is held to 80
// VGPRs: six waves per SIMD instead of four (measured 1.3x faster); with
// 512-thread workgroups the LDS of three workgroups fits a CU at d = 64.
// PROBE instances (coordinate checks only) walk every option as an average
// and also store the coordinates each 64-point batch consumes at
// probe[((unit * unit_pts / 64 + batch) * ndims + dim - 1) * 64 + lane].
template <bool F32, int PATHK, bool OWEN, bool PROBE>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(F32 ? 6 : 1))) void paths_kernel(const OptDev *__restrict__ opts,
                                                     const int64_t *__restrict__ unit_prefix,
                                                     const PlanStep *__restrict__ plan_all,
                                                     const PlanStep64 *__restrict__ plan64_all,
                                                     const uint32_t *__restrict__ dir,
                                                     const uint32_t *__restrict__ lane_tab,
                                                     const float4 *__restrict__ ninv_tab,   // [2][256] cells
                                                     double *__restrict__ partials,
                                                     unsigned long long *__restrict__ counter,
                                                     int n_opts, int max_n, int stack_depth, int stk_off,
                                                     long long total_units, int fixed_bridges,
                                                     uint32_t *__restrict__ probe)
{
    LaunchDesc ld;
    ld.opts = opts;
    ld.unit_prefix = unit_prefix;
    ld.n_opts = n_opts;
    ld.max_n = max_n;
    ld.total_units = total_units;
    ld.plan = plan_all;
    ld.plan64 = plan64_all;
    ld.dir = dir;
    ld.lane = lane_tab;
    ld.partials = partials;
    ld.counter = counter;
    using R = typename Real<F32>::T;
    // all LDS is dynamic and starts at address 0, so a cell's address is its
    // byte offset: FP32 keeps the cells of both halves, lane rows
    // (qcpw_row_word) and stacks; FP64 the rows from 0 and the stacks
    extern __shared__ __align__(16) unsigned char smem[];
    const int bd = blockDim.x;
    uint32_t *lds_lane = (uint32_t *)smem;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // bridge stack: [wave][stack_depth][64]; this lane's column
    R *stk = (R *)(smem + stk_off) + (size_t)(tid >> 6) * stack_depth * 64 + lane;
    if (F32) {
        float4 *cells = (float4 *)smem;
        for (int i = tid; i < 2 * QCPW_NINV_TAB_CELLS; i += bd)
            cells[(i < QCPW_NINV_TAB_CELLS ? 0 : QCPW_LDS_TAB_HI / 16 - QCPW_NINV_TAB_CELLS) + i] = ninv_tab[i];
    }
    for (int i = tid; i < max_n * 64; i += bd) lds_lane[lane_row<F32>(i >> 6) + (i & 63)] = lane_tab[64 + i];
    __syncthreads();

    // Units are dealt out by QCPW_QUEUES counters, queue q holding units
    // q, q + QCPW_QUEUES, ...  All waves of the chip would otherwise take
    // turns on one atomic (served one after another in memory, of the order
    // of 10 ns each), which bounds launches of many cheap units.  Workgroups
    // go to the XCDs in turn, so a wave starts on the queue of its
    // workgroup's XCD and, once that queue is empty, helps the others in
    // order; it leaves after finding all of them empty.
    int o = 0;
    int q = blockIdx.x & (QCPW_QUEUES - 1);
    int empty = 0;
    for (;;) {
        unsigned long long u = 0;
        if (lane == 0) u = atomicAdd(counter + q * QCPW_QUEUE_STRIDE, 1ull);
        const long long j = ((long long)__builtin_amdgcn_readfirstlane((int)(u >> 32)) << 32) |
                            (unsigned)__builtin_amdgcn_readfirstlane((int)u);
        const long long unit = j * QCPW_QUEUES + q;
        if (unit >= total_units) {
            if (++empty == QCPW_QUEUES) break;
            q = (q + 1) & (QCPW_QUEUES - 1);
            continue;
        }

        // option of this unit (units are consumed in increasing order, so the
        // previous option is the usual answer)
        if (!(unit_prefix[o] <= unit && unit < unit_prefix[o + 1])) {
            int lo = 0, hi = n_opts - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (unit_prefix[mid] <= unit) lo = mid; else hi = mid - 1;
            }
            o = lo;
        }
        const OptDev &op = opts[o];
        const int64_t rem = unit - op.unit0;
        const int shift = (int)(rem / op.chunks);
        const int64_t chunk = rem - (int64_t)shift * op.chunks;

        double s[4] = {0.0, 0.0, 0.0, 0.0};
        double c[4] = {0.0, 0.0, 0.0, 0.0};
        const int64_t k_end = op.k_begin + op.n_points;
        const int64_t start = op.k_begin + chunk * op.unit_pts;
        const int64_t end = min(start + (int64_t)op.unit_pts, k_end);
        const int mode = qcpw_stat_of(op.type);
        UParts<OWEN, PROBE> U;
        init_uniform_part<PATHK>(ld, op, shift, lane, (uint64_t)start, U);
        for (int64_t base = start; base < end; base += 64) {
            const bool valid = base + lane < k_end;
            double F[4] = {0.0, 0.0, 0.0, 0.0};
            PathSums<R> ps;
            init_sums(ps);
            if constexpr (PROBE)
                U.pr = probe + ((unit * (op.unit_pts / 64) + (base - start) / 64) * op.ndims) * 64;
            if (op.ndims > 0) {
                switch (PROBE ? QCPW_STAT_AVG : mode) {
                case QCPW_STAT_MAX:
                    walk_path<F32, PATHK, QCPW_STAT_MAX>(ld, op, lds_lane, stk, lane, U, ps, fixed_bridges);
                    break;
                case QCPW_STAT_GEO:
                    walk_path<F32, PATHK, QCPW_STAT_GEO>(ld, op, lds_lane, stk, lane, U, ps, fixed_bridges);
                    break;
                case QCPW_STAT_MIN:
                    walk_path<F32, PATHK, QCPW_STAT_MIN>(ld, op, lds_lane, stk, lane, U, ps, fixed_bridges);
                    break;
                default:
                    walk_path<F32, PATHK, QCPW_STAT_AVG>(ld, op, lds_lane, stk, lane, U, ps, fixed_bridges);
                }
            }
            if (valid) {
                path_tail<R>(op, ps, mode, F);
#pragma unroll
                for (int i = 0; i < 4; ++i) acc_add(s[i], c[i], F[i]);
            }
            if (base + 64 < end) step_uniform_part<PATHK>(ld, op, lane, (uint64_t)base, U);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            wave_reduce(s[i], c[i]);
            if (lane == 0) {
                partials[unit * 8 + i] = s[i];
                partials[unit * 8 + 4 + i] = c[i];
            }
        }
    }
}


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
static size_t paths_lds_bytes(const LaunchPlan &lp, int bd, int *stk_off = nullptr);

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
        if (path == QCPW_PATH_PCA_FULL && sp.type != QCPW_ARITH_ASIAN_CALL && sp.type != QCPW_BINARY_ASIAN_CALL)
            return fail(QCPW_EINVAL, "option " + std::to_string(i) +
                                         ": conditioning on the first principal component covers "
                                         "arithmetic and binary Asian calls only");
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

qcpw_status plan_launch(Context *ctx, const qcpw_option_spec *specs, int32_t n_opts, int32_t d,
                        int64_t n_points, int32_t n_shifts, int32_t path, int32_t precision,
                        int32_t pca_gemm, int32_t block_threads, LaunchPlan &lp, const int64_t *k_begin,
                        bool owen)
{
    {
        qcpw_status st = validate_call(specs, n_opts, d, n_points, n_shifts, path, precision, pca_gemm,
                                       block_threads);
        if (st != QCPW_OK) return st;
    }
    if (owen && path != QCPW_PATH_BB && path != QCPW_PATH_STANDARD)
        return fail(QCPW_EINVAL, "nested scrambling is available with the BB and STANDARD constructions");

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
        cost[i] = (double)std::max(op.ndims, 1) * (double)op.chunks;
        lp.max_n = std::max(lp.max_n, op.ndims);
        // options walked by a compile-time bridge need no LDS stack
        const bool fixed = precision == QCPW_FP32_MIXED && fixed_bridges_on() && qcpw_has_fixed_bridge(op.n);
        if (path == QCPW_PATH_BB && op.n >= 1 && !fixed)
            lp.stack_depth = std::max(lp.stack_depth, ctx->tab.depth[op.n]);
    }
    // most expensive units first (longest-processing-time order)
    std::vector<int32_t> order(n_opts);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return opts[a].ndims > opts[b].ndims; });
    lp.opts.resize(n_opts);
    lp.unit_prefix.assign(n_opts + 1, 0);
    for (int i = 0; i < n_opts; ++i) {
        lp.opts[i] = opts[order[i]];
        lp.opts[i].unit0 = lp.unit_prefix[i];
        lp.unit_prefix[i + 1] = lp.unit_prefix[i] + (int64_t)lp.opts[i].chunks * n_shifts;
    }
    lp.order = order;
    lp.total_units = lp.unit_prefix[n_opts];
    lp.block_threads = block_threads ? block_threads : autotune_block_threads(ctx, lp);
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
    w.upload = w.counter + QCPW_QUEUES * QCPW_QUEUE_STRIDE * sizeof(unsigned long long);
    w.partials = align_up(w.upload, 256);
    w.per_shift = align_up(w.partials + (size_t)lp.total_units * 8 * sizeof(double), 256);
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
// cells and the lane rows at fixed places (qcpw_row_word), the bridge stacks
// after the last row, or in the gap below the upper cells when they fit
// there.  FP64: the rows from 0, then the stacks.  *stk_off (optional)
// receives the stacks' byte offset.
static size_t paths_lds_bytes(const LaunchPlan &lp, int bd, int *stk_off)
{
    const bool f32 = lp.precision == QCPW_FP32_MIXED;
    const size_t stack = lp.path == QCPW_PATH_BB ? (size_t)lp.stack_depth * bd * (f32 ? 4 : 8) : 0;
    if (!f32) {
        if (stk_off) *stk_off = lp.max_n * 256;
        return (size_t)lp.max_n * 256 + stack;
    }
    const bool in_gap = lp.max_n <= QCPW_LDS_GAP_ROWS;
    const size_t rows_end = in_gap ? QCPW_LDS_GAP_BEGIN + (size_t)lp.max_n * 256
                                   : QCPW_LDS_FIXED + (size_t)(lp.max_n - QCPW_LDS_GAP_ROWS) * 256;
    const size_t s = (in_gap && rows_end + stack > QCPW_LDS_TAB_HI) ? QCPW_LDS_FIXED : rows_end;
    if (stk_off) *stk_off = (int)s;
    return std::max<size_t>(s + stack, QCPW_LDS_FIXED);
}

// ... against the CU's 160 KiB.
static bool paths_lds_fits(const LaunchPlan &lp, int bd) { return paths_lds_bytes(lp, bd) <= 160 * 1024; }

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

template <bool F32, int PATHK, bool OWEN, bool PROBE>
static const void *paths_fn()
{
    return reinterpret_cast<const void *>(&paths_kernel<F32, PATHK, OWEN, PROBE>);
}

template <bool OWEN, bool PROBE>
static const void *select_paths_kernel_r(const LaunchPlan &lp)
{
    const bool f32 = lp.precision == QCPW_FP32_MIXED;
    if (lp.path == QCPW_PATH_STANDARD)
        return f32 ? paths_fn<true, QCPW_PATH_STANDARD, OWEN, PROBE>()
                   : paths_fn<false, QCPW_PATH_STANDARD, OWEN, PROBE>();
    return f32 ? paths_fn<true, QCPW_PATH_BB, OWEN, PROBE>() : paths_fn<false, QCPW_PATH_BB, OWEN, PROBE>();
}

static const void *select_paths_kernel(const LaunchPlan &lp)
{
    if (lp.probe) return lp.owen ? select_paths_kernel_r<true, true>(lp) : select_paths_kernel_r<false, true>(lp);
    return lp.owen ? select_paths_kernel_r<true, false>(lp) : select_paths_kernel_r<false, false>(lp);
}

// Resident waves per CU of the fused kernel at workgroup size bd (0 if it
// cannot be resident): registers, LDS and the workgroup granularity decide.
static int resident_waves(const LaunchPlan &lp, int bd)
{
    if (!paths_lds_fits(lp, bd)) return 0;
    const size_t lds = paths_lds_bytes(lp, bd);
    const void *fn = select_paths_kernel(lp);
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, bd, lds) != hipSuccess) return 0;
    return per_cu * bd / 64;
}

// Workgroup size of the fused kernel, chosen by measurement among 256, 512
// and 1024 threads (whole multiples of the CU's four SIMDs, so that every
// SIMD holds the same number of waves; sizes in between measured slower).
// The lane rows and inverse-normal cells are shared per workgroup and the
// bridge stack is per thread, so the best size depends on d.  Each size that
// can be resident is timed on a probe -- one arithmetic Asian option with the
// launch's largest d, 2^18 points x 64 replications (16384 work units, a few
// per resident wave) -- and the fastest is kept per (construction,
// precision, lane-table size bucket).  QCPW_BLOCK_THREADS in the environment
// overrides the choice.  Only the order of floating-point sums depends on it.
int autotune_block_threads(Context *ctx, const LaunchPlan &lp)
{
    if (lp.path == QCPW_PATH_PCA || lp.path == QCPW_PATH_PCA_FULL) return 256;
    if (const char *env = getenv("QCPW_BLOCK_THREADS")) {
        const int v = atoi(env);
        if (v != 0 && qcpw_block_threads_ok(v) && resident_waves(lp, v) > 0) return v;
    }
    const int key = ((lp.path * 2 + lp.precision) * 2 + (lp.owen ? 1 : 0)) * 64 + (lp.max_n + 31) / 32;
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) return it->second;
    qcpw_option_spec probe;
    memset(&probe, 0, sizeof probe);
    probe.type = QCPW_ARITH_ASIAN_CALL;
    probe.d = std::max(lp.max_n, 1) + 1;
    probe.S0 = 100.0; probe.K = 100.0; probe.r = 0.05; probe.sigma = 0.2; probe.T = 1.0;
    probe.seed = 0x51ab;
    probe.n_points = int64_t(1) << 18;
    const int n_probe_shifts = 64;

    std::vector<LaunchPlan> plans;
    std::vector<int> cands;
    for (int bd : {256, 512, 1024}) {
        LaunchPlan p;
        if (plan_launch(ctx, &probe, 1, 0, 0, n_probe_shifts, lp.path, lp.precision, lp.pca_gemm, bd, p, nullptr,
                        lp.owen) != QCPW_OK)
            continue;
        p.max_n = std::max(p.max_n, lp.max_n);
        p.stack_depth = std::max(p.stack_depth, lp.stack_depth);
        if (resident_waves(p, bd) == 0) continue;
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
        const int bd = lp.block_threads;
        if (!paths_lds_fits(lp, bd)) return fail(QCPW_EDIMS, "LDS footprint exceeds 160 KiB");
        int a_stk_off = 0;
        const size_t lds = paths_lds_bytes(lp, bd, &a_stk_off);
        const void *fn = select_paths_kernel(lp);
        if (lp.precision == QCPW_FP32_MIXED) {
            qcpw_status st = check_lds_at_zero(fn);
            if (st != QCPW_OK) return st;
        }
        QCPW_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        int per_cu = 0;
        QCPW_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, bd, lds));
        if (per_cu < 1) return fail(QCPW_EDEVICE, "per-path kernel cannot be resident with this block size");
        int64_t grid = (int64_t)per_cu * ctx->tab.n_cu;
        grid = std::min<int64_t>(grid, lp.total_units);
        const OptDev *a_opts = ld.opts;
        const int64_t *a_prefix = ld.unit_prefix;
        const PlanStep *a_plan = ld.plan;
        const PlanStep64 *a_plan64 = ld.plan64;
        const uint32_t *a_dir = ld.dir, *a_lane = ld.lane;
        const float4 *a_tab = ctx->tab.ninv_tab;
        double *a_part = ld.partials;
        unsigned long long *a_ctr = ld.counter;
        int a_nopts = ld.n_opts, a_maxn = ld.max_n, a_depth = lp.stack_depth;
        long long a_total = ld.total_units;
        int a_fixed_arg = fixed_bridges_on() ? 1 : 0;
        uint32_t *a_probe = lp.probe;
        void *args[] = {&a_opts, &a_prefix, &a_plan, &a_plan64, &a_dir, &a_lane, &a_tab, &a_part, &a_ctr,
                        &a_nopts, &a_maxn, &a_depth, &a_stk_off, &a_total, &a_fixed_arg, &a_probe};
        if (t0) QCPW_HIP(hipEventRecord(t0, stream));
        QCPW_HIP(hipLaunchKernel(fn, dim3((unsigned)grid), dim3(bd), args, lds, stream));
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
