// paths_kernel.h -- the fused per-path QMC-CPW kernel for gfx950 (MI355X).
//
// Included by the translation units that instantiate it (paths_*.hip), each
// a subset of the instances, so that they compile in parallel; the host code
// (kernels.hip) reaches the instances through the paths_fn_* functions.
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
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

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
template <bool OWEN_, bool PROBE_ = false, int NQ_ = QCPW_UQ>
struct UParts {
    static constexpr bool OWEN = OWEN_;
    static constexpr bool PROBE = PROBE_;
    static constexpr int NQ = NQ_;   // registers: 64 NQ slots
    uint32_t U[NQ];
    uint32_t Sd[OWEN ? NQ : 1];
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

// Sums of one subtree kept apart: sum E and sum E (m - l) with m - l a
// literal; folded into the path's sums (sum E m = l sum E + sum E (m - l))
// when the subtree ends.
struct SubSums {
    float A1, A2m;
};

template <int MODE, int M>
__device__ __forceinline__ void consume_sub(PathSums<float> &ps, SubSums &ss, float Y, uint32_t mb_bits_l)
{
    if constexpr (MODE == QCPW_STAT_AVG) {
        const float E = exp2_r(Y);
        ss.A1 += E;
        ps.A2y = fmaf(E, Y, ps.A2y);
        ss.A2m = fmaf(E, (float)M, ss.A2m);
    } else if constexpr (MODE == QCPW_STAT_GEO) {
        ps.A2y += Y;
    } else {
        consume<float, MODE>(ps, Y, __uint_as_float(mb_bits_l + (uint32_t)M));
    }
}

// ---- compile-time bridges ------------------------------------------------
// For n = 15, 31, 63, 127 (d = 16, 32, 64, 128) the bridge is unrolled at
// compile time: the depth-first walk becomes template recursion over the
// intervals, the pending right end points live in registers (no LDS stack,
// no register shuffles), lane-table rows and U lanes are immediates, and the
// weights are literals.  The intervals, dimensions, step order, weights and
// formulas are those of the run-time plan (the host checks the plan against
// the same constexpr functions), and the arithmetic average's sums are folded
// per subtree as in the split bridge: the results are bit-identical to the
// split bridge's for the same n, which the 128-VGPR instances use for these
// n instead (so an option gives the same bits whatever launch it is in).
// Removes about a quarter of the VALU work per date.
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

// The normals are formed QCPW_ZB steps at a time, ahead of the bridge
// arithmetic that consumes them (they do not depend on the path): the lane
// words and inverse-normal cells of a batch are all read before the first is
// used, so their LDS latencies overlap inside the wave.
#define QCPW_ZB 4

// Four normals of a batch.  Wide instances (128 VGPRs) keep the four cell
// reads in flight together; in the others the extra registers would push
// the wave-uniform state into scratch, so each read is waited for alone.
// CNT: the batch's normals that are used (the last batch of a walk may be
// partial; the others are neither read nor formed).
template <class UP, int CNT = 4>
__device__ __forceinline__ void ninv_batch(const uint32_t (&x)[4], float (&zb)[4])
{
    if constexpr (UP::NQ > QCPW_UQ && CNT == 4) {
        ninv_table_f32_x4(x, zb);
    } else {
#pragma unroll
        for (int i = 0; i < CNT; ++i) zb[i] = ninv_table_f32(x[i]);
    }
}

template <class UP, int N, int S0, int... I>
__device__ __forceinline__ void fixed_zbatch(const uint32_t *row0, int lane, const FixedU<UP, N> &U, float (&zb)[QCPW_ZB],
                                             std::integer_sequence<int, I...>)
{
    constexpr int dims[] = {qcpw_bridge_dim_at_step(N, S0 + I)...};
    uint32_t w[] = {(S0 + I < N ? row0[qcpw_row_word((dims[I] > 0 ? dims[I] : 1) - 1)] : 0u)...};
    uint32_t x[] = {U.template bits<S0 + I>(w[I])...};
    ((S0 + I < N ? (void)U.rec(x[I], dims[I], lane) : (void)0), ...);
    ninv_batch<UP, (N - S0 < QCPW_ZB ? N - S0 : QCPW_ZB)>(x, zb);
}

// LEVEL: depth of the interval (LO, HI); L0: left end of the subtree it
// lies in (-1 above the split bridge's subtree level).  The arithmetic
// average's sums of a subtree are kept apart and folded in when it ends, as
// the split bridge does, so that both walks of n give the same bits.
template <int MODE, class UP, int N, int LO, int HI, int LEVEL, int L0>
__device__ __forceinline__ void fixed_interval(const uint32_t *row0, int lane, float zs,
                                               const FixedU<UP, N> &U, float WL, float WR,
                                               PathSums<float> &ps, SubSums &ss, float (&zb)[QCPW_ZB])
{
    if constexpr (MODE == QCPW_STAT_AVG && L0 < 0 && LEVEL == qcpw_split_level(N)) {
        SubSums sub = {0.0f, 0.0f};
        fixed_interval<MODE, UP, N, LO, HI, LEVEL, LO>(row0, lane, zs, U, WL, WR, ps, sub, zb);
        ps.A1 += sub.A1;
        ps.A2m += fmaf((float)LO, sub.A1, sub.A2m);
    } else if constexpr (HI - LO >= 2) {
        constexpr int M = (LO + HI) / 2;
        constexpr int DIM = qcpw_bridge_dim(N, LO, HI);
        constexpr int S = qcpw_bridge_step(N, LO, HI);
        static_assert(DIM >= 2 && S >= 1, "interval outside the bridge");
        static_assert(qcpw_bridge_dim_at_step(N, S) == DIM, "step order");
        constexpr float wl = (float)((double)(HI - M) / (double)(HI - LO));
        constexpr float wr = (float)((double)(M - LO) / (double)(HI - LO));
        constexpr float sd = (float)qcpw_csqrt((double)(M - LO) * (double)(HI - M) / (double)(HI - LO));
        if constexpr ((S - 1) % QCPW_ZB == 0)
            fixed_zbatch<UP, N, S>(row0, lane, U, zb, std::make_integer_sequence<int, QCPW_ZB>());
        const float z = zb[(S - 1) % QCPW_ZB];
        const float Ym = fmaf(__fmul_rn(sd, zs), z, fmaf(wr, WR, wl * WL));   // as the split bridge
        if constexpr (L0 >= 0) consume_sub<MODE, M - L0>(ps, ss, Ym, 0u);
        else consume<float, MODE>(ps, Ym, (float)M);
        fixed_interval<MODE, UP, N, LO, M, LEVEL + 1, L0>(row0, lane, zs, U, WL, Ym, ps, ss, zb);
        fixed_interval<MODE, UP, N, M, HI, LEVEL + 1, L0>(row0, lane, zs, U, Ym, WR, ps, ss, zb);
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
    float zb[QCPW_ZB];
    SubSums ss = {0.0f, 0.0f};
    fixed_interval<MODE, UP, N, 0, N, 0, -1>(row0, lane, zs, U, 0.0f, WR, ps, ss, zb);
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

// ---- split bridge --------------------------------------------------------
// Any n >= QCPW_SUB_MIN_LEN (FP32): the top nodes of the bridge come from the
// plan's events, every interval at the split level is walked by a
// compile-time subtree of its length (see qcpw_internal.h).  Per subtree node
// the work is that of the compile-time bridges plus one address add for its
// lane-table row.

// Register `reg` (wave-uniform) of a slot array, by a tree of selects on the
// bits of reg: an indexed read of the array would make the compiler keep it
// in scratch memory.
template <int NQ>
__device__ __forceinline__ uint32_t pick_reg(const uint32_t (&V)[NQ], int reg)
{
    static_assert(NQ <= 8, "three select levels");
    auto at = [&](int q) { return q < NQ ? V[q] : V[0]; };
    const bool b0 = reg & 1, b1 = reg & 2, b2 = reg & 4;
    const uint32_t a0 = b0 ? at(1) : at(0), a1 = b0 ? at(3) : at(2);
    const uint32_t a2 = b0 ? at(5) : at(4), a3 = b0 ? at(7) : at(6);
    const uint32_t c0 = b1 ? a1 : a0, c1 = b1 ? a3 : a2;
    return b2 ? c1 : c0;
}

// Dimension of a lane-table word offset (probe instances only).
__device__ __forceinline__ int dim_of_row_word(uint32_t w) { return qcpw_word_row(w) + 1; }

// The wave-uniform parts of one subtree's nodes: slots base .. base + len - 2
// of register reg.  Without scrambling they are copied into every row of 16
// lanes (lane l of R[i] holds node 16 i + l % 16) for the row broadcast, as
// the compile-time bridges do; with nested scrambling the register and its
// seeds are read lane by lane.
template <class UP, bool OWEN = UP::OWEN>
struct SubU;

template <class UP>
struct SubU<UP, false> {
    uint32_t R0, R1;
    __device__ __forceinline__ SubU(const UP &U, int reg, int base, int lane)
    {
        // lane l reads lane base + 16 i + l % 16 (ds_bpermute takes the lane
        // from address bits 2..7: no wrap-around arithmetic needed)
        const int u = (int)pick_reg(U.U, reg);
        const int a = (lane & 15) * 4;
        R0 = (uint32_t)__builtin_amdgcn_ds_bpermute(a + base * 4, u);
        R1 = (uint32_t)__builtin_amdgcn_ds_bpermute(a + base * 4 + 64, u);
    }
    template <int S>
    __device__ __forceinline__ uint32_t bits(uint32_t lane_word) const
    {
        return lane_word ^ (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(S < 16 ? R0 : R1), 0x150 + S % 16, 0xF, 0xF,
                                                                 false);
    }
};

template <class UP>
struct SubU<UP, true> {
    uint32_t u, sd;
    int base;
    __device__ __forceinline__ SubU(const UP &U, int reg, int b, int) : u(pick_reg(U.U, reg)), sd(pick_reg(U.Sd, reg)), base(b) {}
    template <int S>
    __device__ __forceinline__ uint32_t bits(uint32_t lane_word) const
    {
        return owen_scramble(lane_word ^ rdlane(u, base + S), rdlane(sd, base + S));
    }
};

// Coordinate of a top node or the terminal point: their slots are the first
// 2^k <= 16, all in register 0, at the lane in the event header.
template <class UP>
__device__ __forceinline__ uint32_t top_bits(const UP &U, uint32_t h, uint32_t lane_word)
{
    const int k = h >> 24;
    if constexpr (UP::OWEN) return owen_scramble(lane_word ^ rdlane(U.U[0], k), rdlane(U.Sd[0], k));
    else return lane_word ^ rdlane(U.U[0], k);
}

// What a date adds to the path statistic, with its grid index given as
// float(m) bits (sums) and float(2^23 + m) bits (maximum / minimum: an index
// that orders like m and needs no conversion).
template <int MODE>
__device__ __forceinline__ void consume_ev(PathSums<float> &ps, float Y, uint32_t mf_bits, uint32_t mb_bits)
{
    if constexpr (MODE == QCPW_STAT_MAX || MODE == QCPW_STAT_MIN) consume<float, MODE>(ps, Y, __uint_as_float(mb_bits));
    else consume<float, MODE>(ps, Y, __uint_as_float(mf_bits));
}

// Number of levels of a subtree over (0, len).
__host__ __device__ constexpr int qcpw_sub_levels(int len)
{
    int lv = 0;
    for (int s = 0; s < len - 1; ++s)
        if (qcpw_sub_pos(len, s).level + 1 > lv) lv = qcpw_sub_pos(len, s).level + 1;
    return lv;
}

// This lane's LDS byte address in the first row of each level of a subtree
// (the event's word 4 + level): node i of a level reads 256 i bytes further,
// a compile-time offset.  In the 128-VGPR instances an empty asm keeps each
// base in a register for the whole subtree (the compiler would otherwise
// form it again per batch of nodes); the 80-VGPR instances leave that choice
// to the compiler (measured: pinned there, they were 1-2 % slower).
template <class UP, int LEN>
struct SubRows {
    static constexpr int LEVELS = qcpw_sub_levels(LEN);
    static constexpr bool PIN = UP::NQ > QCPW_UQ;
    const uint32_t *E, *row0;
    uint32_t b[PIN ? LEVELS : 1];
    __device__ __forceinline__ SubRows(const uint32_t *E_, const uint32_t *row0_, int lane) : E(E_), row0(row0_)
    {
        if constexpr (PIN) {
#pragma unroll
            for (int j = 0; j < LEVELS; ++j) {
                b[j] = (E[4 + j] + (uint32_t)lane) * 4u;
                asm("" : "+v"(b[j]));
            }
        }
    }
    template <int S>
    __device__ __forceinline__ uint32_t word() const
    {
        constexpr QcpwSubPos p = qcpw_sub_pos(LEN, S < LEN - 1 ? S : 0);   // past the subtree: a row that exists
        if constexpr (PIN) return *(const __attribute__((address_space(3))) uint32_t *)(b[p.level] + 256u * p.index);
        else return row0[E[4 + p.level] + 64 * p.index];
    }
    template <int S>
    __device__ __forceinline__ int dim() const   // probe instances only
    {
        constexpr QcpwSubPos p = qcpw_sub_pos(LEN, S < LEN - 1 ? S : 0);
        return qcpw_word_row(E[4 + p.level] + 64u * p.index) + 1;
    }
};

// Normals of subtree nodes S0 .. S0 + QCPW_ZB - 1 (those below LEN - 1).
template <class UP, int LEN, int S0, int... I>
__device__ __forceinline__ void sub_zbatch(const uint32_t *E, const SubRows<UP, LEN> &rows, int lane, const UP &U,
                                           const SubU<UP> &su, float (&zb)[QCPW_ZB], std::integer_sequence<int, I...>)
{
    uint32_t x[] = {su.template bits<S0 + I>(rows.template word<S0 + I>())...};
    if constexpr (UP::PROBE)
        ((S0 + I < LEN - 1 ? (void)U.rec(x[I], rows.template dim<S0 + I>(), lane) : (void)0), ...);
    ninv_batch<UP, (LEN - 1 - S0 < QCPW_ZB ? LEN - 1 - S0 : QCPW_ZB)>(x, zb);
}

template <int MODE, class UP, int LEN, int LO, int HI>
__device__ __forceinline__ void sub_interval(const uint32_t *E, const SubRows<UP, LEN> &rows, int lane, float zs,
                                             const UP &U, const SubU<UP> &su, float WL, float WR, SubSums &ss,
                                             PathSums<float> &ps, float (&zb)[QCPW_ZB])
{
    if constexpr (HI - LO >= 2) {
        constexpr int M = (LO + HI) / 2;
        constexpr int S = qcpw_sub_step(LEN, LO, HI);
        static_assert(S >= 0 && S < LEN - 1, "subtree step");
        constexpr float wl = (float)((double)(HI - M) / (double)(HI - LO));
        constexpr float wr = (float)((double)(M - LO) / (double)(HI - LO));
        constexpr float sd = (float)qcpw_csqrt((double)(M - LO) * (double)(HI - M) / (double)(HI - LO));
        if constexpr (S % QCPW_ZB == 0)
            sub_zbatch<UP, LEN, S>(E, rows, lane, U, su, zb, std::make_integer_sequence<int, QCPW_ZB>());
        const float z = zb[S % QCPW_ZB];
        // sd zs rounded first: the product depends on the interval length
        // alone, so the few distinct lengths of a subtree share it
        const float Ym = fmaf(__fmul_rn(sd, zs), z, fmaf(wr, WR, wl * WL));
        consume_sub<MODE, M>(ps, ss, Ym, E[3]);
        sub_interval<MODE, UP, LEN, LO, M>(E, rows, lane, zs, U, su, WL, Ym, ss, ps, zb);
        sub_interval<MODE, UP, LEN, M, HI>(E, rows, lane, zs, U, su, Ym, WR, ss, ps, zb);
    }
}

template <int MODE, class UP, int LEN>
__device__ __forceinline__ void run_subtree(const uint32_t *E, const uint32_t *row0, int lane, float zs, const UP &U,
                                            float L, float R, PathSums<float> &ps)
{
    const uint32_t h = E[0];
    const SubU<UP> su(U, (h >> 16) & 255, h >> 24, lane);
    SubSums ss = {0.0f, 0.0f};
    float zb[QCPW_ZB];
    const SubRows<UP, LEN> rows(E, row0, lane);
    sub_interval<MODE, UP, LEN, 0, LEN>(E, rows, lane, zs, U, su, L, R, ss, ps, zb);
    if constexpr (MODE == QCPW_STAT_AVG) {
        ps.A1 += ss.A1;
        ps.A2m += fmaf(__uint_as_float(E[2]), ss.A1, ss.A2m);
    }
}

template <int MODE, class UP>
__device__ inline void run_bridge_split(const LaunchDesc &ld, const OptDev &op, const uint32_t *lds_lane, int lane,
                                        const UP &U, PathSums<float> &ps)
{
    const uint32_t *ev = ld.split_ev + (size_t)op.n * (QCPW_SPLIT_EVENTS * QCPW_EV_WORDS);
    const uint32_t *row0 = lds_lane + lane;
    const float zs = op.zs_t;
    if constexpr (MODE == QCPW_STAT_MAX || MODE == QCPW_STAT_MIN) ps.bm = 8388608.0f;   // date 1 (m = 0), biased
    float L = 0.0f, R;
    const int n_ev = (int)ev[8];
    {   // terminal point
        uint32_t x = top_bits(U, ev[0], row0[ev[4]]);
        x = U.rec(x, 1, lane);
        const float z = ninv_table_f32(x);
        R = fmaf(__uint_as_float(ev[7]) * zs, z, op.ydrift_n_f);
        consume_ev<MODE>(ps, R, ev[2], ev[3]);
    }
    // pending right end points of the top nodes (at most 4 levels)
    float p0 = 0.0f, p1 = 0.0f, p2 = 0.0f, p3 = 0.0f;
    int sp = 0;
    for (int e = 1; e < n_ev; ++e) {
        const uint32_t *E = ev + e * QCPW_EV_WORDS;
        const uint32_t h = E[0];
        if ((h & 255) == QCPW_EV_TOP) {
            uint32_t x = top_bits(U, h, row0[E[4]]);
            if constexpr (UP::PROBE) x = U.rec(x, dim_of_row_word(E[4]), lane);
            const float z = ninv_table_f32(x);
            const float M = fmaf(__fmul_rn(__uint_as_float(E[7]), zs), z,
                                 fmaf(__uint_as_float(E[6]), R, __uint_as_float(E[5]) * L));
            consume_ev<MODE>(ps, M, E[2], E[3]);
            switch (sp) {
            case 0: p0 = R; break;
            case 1: p1 = R; break;
            case 2: p2 = R; break;
            default: p3 = R; break;
            }
            ++sp;
            R = M;
        } else {
            switch ((h >> 8) & 255) {
            case 12: run_subtree<MODE, UP, 12>(E, row0, lane, zs, U, L, R, ps); break;
            case 13: run_subtree<MODE, UP, 13>(E, row0, lane, zs, U, L, R, ps); break;
            case 14: run_subtree<MODE, UP, 14>(E, row0, lane, zs, U, L, R, ps); break;
            case 15: run_subtree<MODE, UP, 15>(E, row0, lane, zs, U, L, R, ps); break;
            case 16: run_subtree<MODE, UP, 16>(E, row0, lane, zs, U, L, R, ps); break;
            case 17: run_subtree<MODE, UP, 17>(E, row0, lane, zs, U, L, R, ps); break;
            case 18: run_subtree<MODE, UP, 18>(E, row0, lane, zs, U, L, R, ps); break;
            case 19: run_subtree<MODE, UP, 19>(E, row0, lane, zs, U, L, R, ps); break;
            case 20: run_subtree<MODE, UP, 20>(E, row0, lane, zs, U, L, R, ps); break;
            case 21: run_subtree<MODE, UP, 21>(E, row0, lane, zs, U, L, R, ps); break;
            case 22: run_subtree<MODE, UP, 22>(E, row0, lane, zs, U, L, R, ps); break;
            case 23: run_subtree<MODE, UP, 23>(E, row0, lane, zs, U, L, R, ps); break;
            default: run_subtree<MODE, UP, 24>(E, row0, lane, zs, U, L, R, ps); break;
            }
            // on to the pending right half: L = R, R = pop()
            L = R;
            if (sp > 0) {
                --sp;
                switch (sp) {
                case 0: R = p0; break;
                case 1: R = p1; break;
                case 2: R = p2; break;
                default: R = p3; break;
                }
            }
        }
    }
    if constexpr (MODE == QCPW_STAT_MAX || MODE == QCPW_STAT_MIN) ps.bm -= 8388608.0f;
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
template <bool F32, int PATHK, int MODE, bool FIXED, class UP>
__device__ inline void walk_path(const LaunchDesc &ld, const OptDev &op, const uint32_t *lds_lane,
                                 typename Real<F32>::T *stk, int lane,
                                 const UP &U, PathSums<typename Real<F32>::T> &ps, int fixed_bridges)
{
    if constexpr (PATHK == QCPW_PATH_BB) {
        if constexpr (F32) {
            if constexpr (FIXED)
                if (fixed_bridges && bridge_fixed_any<MODE>(op, lds_lane, lane, U, ps)) return;
            if (op.split) {
                run_bridge_split<MODE>(ld, op, lds_lane, lane, U, ps);
                return;
            }
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

// U_j(base) (and its seed) for the dimensions this lane holds: steps (or,
// for the split bridge, slots) s = lane + 64 q; 0 for a slot with none.
template <int PATHK>
__device__ inline int step_dim(const LaunchDesc &ld, const OptDev &op, int s)
{
    if (s >= op.n_slots) return 0;
    if (PATHK != QCPW_PATH_BB) return s + 1;
    return op.split ? (int)ld.split_dim[(size_t)op.n * QCPW_SPLIT_SLOTS + s] : ld.plan[op.plan_off + s].dim;
}

template <int PATHK, class UP>
__device__ inline void init_uniform_part(const LaunchDesc &ld, const OptDev &op, int shift, int lane,
                                         uint64_t base, UP &U)
{
    const uint64_t g = (base ^ (base >> 1)) >> 5;   // gray(base) has no bits below 5
#pragma unroll
    for (int q = 0; q < UP::NQ; ++q) {
        const int s = lane + 64 * q;
        int dim = step_dim<PATHK>(ld, op, s);
        uint32_t u = 0, key = 0;
        if (dim > 0) {
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
    for (int q = 0; q < UP::NQ; ++q) {
        const int dim = step_dim<PATHK>(ld, op, lane + 64 * q);
        if (dim > 0) {
            const uint32_t *v = ld.dir + (size_t)dim * 32;
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
// on two dependent LDS reads), so it is held to 80 VGPRs: six waves per
// SIMD instead of four (measured 1.3x faster); the LDS of three 512-thread
// workgroups fits a CU up to 181 lane rows, of two 768-thread ones up to 280.
// PROBE instances (coordinate checks only) walk every option as an average
// and also store the coordinates each 64-point batch consumes at
// probe[((unit * unit_pts / 64 + batch) * ndims + dim - 1) * 64 + lane].
// WIDE instances (FP32, launches whose lane rows leave room for one
// workgroup per CU, 4 waves per SIMD at 1024 threads anyway) may use 128
// VGPRs and hold 8 registers of wave-uniform slots, which the split bridge
// needs beyond n = 356; they walk n = 15, 31, 63, 127 with the split bridge
// too (the compile-time bridges would raise the register need of the whole
// kernel).  Coordinate-recording instances take the 128-VGPR budget either
// way (their code paths are those of the instance they record for; only the
// register allocation differs).
template <bool F32, int PATHK, bool OWEN, bool PROBE, bool WIDE>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(F32 ? ((WIDE || PROBE) ? 4 : 6) : 1))) void paths_kernel(
    const OptDev *__restrict__ opts, const int64_t *__restrict__ unit_prefix, const PlanStep *__restrict__ plan_all,
    const PlanStep64 *__restrict__ plan64_all, const uint32_t *__restrict__ split_ev,
    const uint16_t *__restrict__ split_dim, const uint32_t *__restrict__ dir, const uint32_t *__restrict__ lane_tab,
    const float4 *__restrict__ ninv_tab,   // [2][256] cells
    double *__restrict__ partials, unsigned long long *__restrict__ counter, int n_opts, int max_n, int stack_depth,
    int stk_off, long long total_units, long long unit_base, int fixed_bridges, uint32_t *__restrict__ probe)
{
    LaunchDesc ld;
    ld.split_ev = split_ev;
    ld.split_dim = split_dim;
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
    if (F32 && max_n > QCPW_LDS_GAP_ROWS) {
        // the upper region's copies of the gap's last rows
        constexpr int r0 = QCPW_LDS_GAP_ROWS - QCPW_LDS_DUP_ROWS;
        for (int i = tid; i < QCPW_LDS_DUP_ROWS * 64; i += bd)
            lds_lane[qcpw_row_word_hi(r0 + (i >> 6)) + (i & 63)] = lane_tab[64 + r0 * 64 + i];
    }
    __syncthreads();

    // Units are dealt out by QCPW_QUEUES counters, queue q holding units
    // q, q + QCPW_QUEUES, ...  All waves of the chip would otherwise take
    // turns on one atomic (served one after another in memory, of the order
    // of 10 ns each), which bounds launches of many cheap units.  Workgroups
    // go to the XCDs in turn, so a wave starts on the queue of its
    // workgroup's XCD and, once that queue is empty, helps the others in
    // order; it leaves after finding all of them empty.  A plain read of a
    // head first: a queue it shows drained (heads only grow) costs no atomic,
    // so the waves leaving at the end do not write to eight lines each.
    int o = 0;
    int q = blockIdx.x & (QCPW_QUEUES - 1);
    int empty = 0;
    for (;;) {
        unsigned long long *head = counter + q * QCPW_QUEUE_STRIDE;
        const unsigned long long v = *(volatile unsigned long long *)head;   // past the L1: the atomics' value
        long long j = ((long long)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32) |
                      (unsigned)__builtin_amdgcn_readfirstlane((int)v);
        if (j * QCPW_QUEUES + q < total_units) {
            unsigned long long u = 0;
            if (lane == 0) u = atomicAdd(head, 1ull);
            j = ((long long)__builtin_amdgcn_readfirstlane((int)(u >> 32)) << 32) |
                (unsigned)__builtin_amdgcn_readfirstlane((int)u);
        }
        if (j * QCPW_QUEUES + q >= total_units) {
            if (++empty == QCPW_QUEUES) break;
            q = (q + 1) & (QCPW_QUEUES - 1);
            continue;
        }
        // this launch's units follow unit_base in the option table's numbering
        const long long unit = unit_base + j * QCPW_QUEUES + q;

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

        // Per-lane FP64 sums of the unit's points (at most 64 per lane): plain
        // in the FP32-mixed kernels (their rounding stays below 64 ulps of
        // the summands' scale, far below the path's FP32 rounding),
        // compensated in the FP64 kernel; every sum across lanes, units and
        // replications is compensated in both.
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        double c[4] = {0.0, 0.0, 0.0, 0.0};
        const int64_t k_end = op.k_begin + op.n_points;
        const int64_t start = op.k_begin + chunk * op.unit_pts;
        const int64_t end = min(start + (int64_t)op.unit_pts, k_end);
        const int mode = qcpw_stat_of(op.type);
        UParts<OWEN, PROBE, WIDE ? 8 : QCPW_UQ> U;
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
                    walk_path<F32, PATHK, QCPW_STAT_MAX, !WIDE>(ld, op, lds_lane, stk, lane, U, ps, fixed_bridges);
                    break;
                case QCPW_STAT_GEO:
                    walk_path<F32, PATHK, QCPW_STAT_GEO, !WIDE>(ld, op, lds_lane, stk, lane, U, ps, fixed_bridges);
                    break;
                case QCPW_STAT_MIN:
                    walk_path<F32, PATHK, QCPW_STAT_MIN, !WIDE>(ld, op, lds_lane, stk, lane, U, ps, fixed_bridges);
                    break;
                default:
                    walk_path<F32, PATHK, QCPW_STAT_AVG, !WIDE>(ld, op, lds_lane, stk, lane, U, ps, fixed_bridges);
                }
            }
            if (valid) {
                path_tail<R>(op, ps, mode, F);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if constexpr (F32) s[i] += F[i];
                    else acc_add(s[i], c[i], F[i]);
                }
            }
            if (base + 64 < end) step_uniform_part<PATHK>(ld, op, lane, (uint64_t)base, U);
        }
        // the butterfly leaves the totals in every lane: lanes 0..7 store the
        // unit's 64-byte record with one coalesced store
        double rec = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            wave_reduce(s[i], c[i]);
            rec = lane == i ? s[i] : lane == 4 + i ? c[i] : rec;
        }
        // the partials' base passes through an empty asm so that its per-lane
        // address is formed here, not held (and spilled) across the unit loop
        double *pp = partials;
        asm volatile("" : "+s"(pp));
        if (lane < 8) pp[unit * 8 + lane] = rec;
    }
}


}  // namespace qcpw
