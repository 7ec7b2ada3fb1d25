// pca.hip -- principal-component path construction (Sec. 3.4.1: W~ = A z
// with A A^T = Sigma; here A holds the eigenvectors of Sigma scaled by the
// square roots of their eigenvalues, largest first).
//
// For a tile of 64 consecutive Sobol points the product W~ = A Z is a dense
// (n x n) by (n x 64) contraction, so it runs on the matrix cores.  A
// workgroup has one wave per 32 rows of the padded factor (at least two;
// eight for the full conditioning):
//
//   prologue   waves 1.. generate the tile's dimensions, an equal share each
//              (lane = point; Sobol via the lane table and a wave-uniform
//              part, digital shift, FP32 inverse normal, scaled to log2
//              units) and store Z^T in LDS, as FP32 or split into BF16
//              hi + lo, while wave 0 runs the previous tile's FP64 tails;
//   GEMM       wave w keeps rows 32 w .. 32 w + 31 of A in registers for the
//              whole work unit and multiplies them by both 32-point blocks:
//              FP32 v_mfma_f32_32x32x2f32, or three v_mfma_f32_32x32x16_bf16
//              per 16-wide k slab (hi*hi + hi*lo + lo*hi), accumulating in
//              FP32;
//   epilogue   Y_m = W'_m + drift m; E = exp2(Y) and the path sums (or the
//              running maximum) over the lane's rows; the two lane halves
//              and the waves of a point block are combined through LDS; the
//              FP64 tail (breakpoint, Phi tails, Greeks) runs on wave 0 and
//              feeds its compensated sums.
//
// The FP64 variant keeps Z^T in FP64 in LDS and forms A z with FP64 FMAs
// (A read as wave-uniform scalars), for exact parity with the oracle.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_math.h"
#include "qcpw_host.h"

namespace qcpw {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned short v8us __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

static constexpr int TP = 64;        // points per tile (one wave width)
static constexpr int PCA_WAVES = 4;     // waves per workgroup (FP64)
static constexpr int PCA_AS_WAVES = 8;  // waves per workgroup (matrix cores, one row block of A each)

__device__ inline unsigned short bf16_bits(float x)   // round to nearest even
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf16_value(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }

// unit of work -> (option index, replication, chunk)
__device__ inline void locate_unit(const int64_t *__restrict__ prefix, int n_opts, long long unit, int &o)
{
    if (!(prefix[o] <= unit && unit < prefix[o + 1])) {
        int lo = 0, hi = n_opts - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= unit) lo = mid; else hi = mid - 1;
        }
        o = lo;
    }
}

__device__ inline long long next_unit(unsigned long long *counter, long long *s_unit)
{
    if (threadIdx.x == 0) *s_unit = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    const long long v = *s_unit;
    const long long unit = ((long long)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32) |
                           (unsigned)__builtin_amdgcn_readfirstlane((int)v);
    __syncthreads();
    return unit;
}

// U_j(base) for dimension j (held by one lane), shift folded in.
__device__ inline uint32_t uniform_part(const uint32_t *__restrict__ dir, uint64_t seed, int shift, int j,
                                        uint64_t base, bool owen)
{
    // with nested scrambling the seed is applied after the XOR with the
    // lane word (owen_scramble), so the part stays raw
    uint32_t u = owen ? 0u : digital_shift(seed, shift, j);
    uint64_t g = (base ^ (base >> 1)) >> 5;
    const uint32_t *v = dir + (size_t)j * 32;
    for (int b = 5; g != 0; ++b, g >>= 1)
        if (g & 1) u ^= v[b];
    return u;
}

// Per-point sums of a path piece: the arithmetic average's sums, the running
// extreme of E with its Y and m (the maximum, or the minimum when `lo`, for
// the lookback put; compared on E, lowest m wins ties) and the sum of Y
// (geometric average).
template <typename R>
struct PcaSums {
    R A1, A2y, A2m;
    R bE, bY, bm;
    R sY;
};

template <typename R>
__device__ inline void sums_neutral(PcaSums<R> &ps, bool lo)
{
    ps.A1 = R(0); ps.A2y = R(0); ps.A2m = R(0);
    ps.bE = lo ? R(3.0e38) : R(0); ps.bY = R(0); ps.bm = R(1e30);
    ps.sY = R(0);
}

template <typename R>
__device__ inline bool sums_take(R E, R m, R bE, R bm, bool lo)
{
    return (lo ? E < bE : E > bE) || (E == bE && m < bm);
}

template <typename R>
__device__ inline void sums_merge(PcaSums<R> &a, const PcaSums<R> &b, bool lo)
{
    a.A1 += b.A1;
    a.A2y += b.A2y;
    a.A2m += b.A2m;
    a.sY += b.sY;
    const bool take = sums_take(b.bE, b.bm, a.bE, a.bm, lo);
    a.bE = take ? b.bE : a.bE;
    a.bY = take ? b.bY : a.bY;
    a.bm = take ? b.bm : a.bm;
}

template <typename R>
__device__ inline void sums_add_date(PcaSums<R> &ps, R Y, R mf, bool lo)
{
    const R E = exp2_r(Y);
    ps.A1 += E;
    ps.A2y = fma(E, Y, ps.A2y);
    ps.A2m = fma(E, mf, ps.A2m);
    ps.sY += Y;
    const bool take = sums_take(E, mf, ps.bE, ps.bm, lo);
    ps.bE = take ? E : ps.bE;
    ps.bY = take ? Y : ps.bY;
    ps.bm = take ? mf : ps.bm;
}

template <typename R>
__device__ inline PcaSums<R> shfl_xor_sums(const PcaSums<R> &p, int off)
{
    PcaSums<R> q;
    q.A1 = __shfl_xor(p.A1, off, 64);
    q.A2y = __shfl_xor(p.A2y, off, 64);
    q.A2m = __shfl_xor(p.A2m, off, 64);
    q.bE = __shfl_xor(p.bE, off, 64);
    q.bY = __shfl_xor(p.bY, off, 64);
    q.bm = __shfl_xor(p.bm, off, 64);
    q.sY = __shfl_xor(p.sY, off, 64);
    return q;
}

// Per-point combination of the wave partials in LDS, the date at tau = 0
// (E = 1, Y = 0) and the FP64 tail; wave 0, lane = point of the tile.
template <typename R>
__device__ inline void tile_tail(const OptDev &op, const PcaSums<R> *red, int lane, bool valid, int nwaves_pt,
                                 const int *waves_pt, double (&s)[4], double (&c)[4])
{
    PcaSums<R> ps;
    ps.A1 = R(1); ps.A2y = R(0); ps.A2m = R(0);   // date 1: E = 1, Y = 0, m = 0
    ps.bE = R(1); ps.bY = R(0); ps.bm = R(0);
    ps.sY = R(0);
    const bool lo = qcpw_stat_of(op.type) == QCPW_STAT_MIN;
    for (int i = 0; i < nwaves_pt; ++i) sums_merge(ps, red[waves_pt[i] * TP + lane], lo);
    if (valid) {
        const int mode = qcpw_stat_of(op.type);
        PathSums<R> t;
        t.A1 = ps.A1; t.A2y = mode == QCPW_STAT_GEO ? ps.sY : ps.A2y; t.A2m = ps.A2m;
        t.bY = ps.bY; t.bm = ps.bm;   // the tail forms E = 2^bY, the same value as bE
        double F[4];
        path_tail<R>(op, t, mode, F);
#pragma unroll
        for (int k = 0; k < 4; ++k) acc_add(s[k], c[k], F[k]);
    }
}

// ------------------------------------------------------------------------
// Conditioning on the first principal component of all d dates (PCA_FULL)
// ------------------------------------------------------------------------
// One point's FP64 tail, shared by PARTS (4 or 8) consecutive lanes; thread
// `part` takes the dates j = part (mod PARTS).  y(j)
// is date j's row of the factor (first column dropped) times the scaled
// normals, i.e. log2(e) sigma c_j, so that
//     ln S(t_j) = alpha_j + beta_j x,  alpha_j = ln S0 + omega t_j + sigma c_j,
//     beta_j = sigma sqrt(dt) a1_j
// in the conditioned component x.  The breakpoint psi solves
// (1/d) sum_j exp(alpha_j + beta_j psi) = K: Newton's method on the log of
// the sum, which is increasing and convex in x, started at the Jensen bound
// (to the right of the root), so the iterates decrease to the root.  Price,
// delta, vega and gamma then follow in closed form (arithmetic: the terms in
// d psi cancel at the root; binary: through d psi = -dF / F').
// P(lo < X < hi), X ~ N(0, 1), lo <= hi (hi may be +inf): from the upper
// tail when the interval lies right of 0, so far-out intervals keep their
// relative accuracy.
__device__ inline double norm_interval(double lo, double hi)
{
    if (lo >= 0.0) return 0.5 * erfc_f64<false>(lo * M_SQRT1_2) - (isinf(hi) ? 0.0 : 0.5 * erfc_f64<false>(hi * M_SQRT1_2));
    return (isinf(hi) ? 1.0 : 0.5 * erfc_f64<false>(-hi * M_SQRT1_2)) - 0.5 * erfc_f64<false>(-lo * M_SQRT1_2);
}

// Lookback (call on the discrete maximum) conditioned on the first principal
// component: ln S(t_j) = alpha_j + beta_j x are d increasing lines, their
// upper envelope M(x) is increasing, convex and piecewise linear, and the
// payoff is positive for x > psi = min_j (ln K - alpha_j) / beta_j.  The
// envelope is walked from psi (the line crossing ln K there, the steeper one
// on a tie) to +inf, each next line being the steeper one that overtakes the
// current one first; over a segment [a, b) of line j, with
// E_j = exp(alpha_j + beta_j^2 / 2) and dP = P(a - beta_j < X < b - beta_j),
//   G     += D [E_j dP - K P(a < X < b)],   delta += D E_j dP / S0,
//   vega  += D E_j [(c_j - sigma t_j) dP + a_j (beta_j dP + phi(a - beta_j) - phi(b - beta_j))],
// and gamma = D K phi(psi) / (S0^2 beta*) with beta* the slope on top at psi.
// The PARTS threads of a point scan their dates j = part (mod PARTS) and
// agree on each candidate through the same fixed butterfly.
template <int PARTS, typename YF>
__device__ inline void full_lookback_tail(const OptDev &op, YF y, int part, double F[4])
{
    constexpr double LN2 = 0.69314718055994530942;
    const int d = op.n + 1;
    const double sig = 1.0 / op.inv_sigma;
    const double sdt = op.zscale * LN2;     // sigma sqrt(dt)
    const double wdt = op.ydrift_1 * LN2;   // omega dt
    const double dt = op.sqrt_t1 * op.sqrt_t1;
    const double lnS0 = ln_f64<false>(op.S0), K = op.K, lnK = ln_f64<false>(op.K);
    const double *a1 = op.pca_a1;
    auto alpha = [&](int j) { return lnS0 + wdt * (j + 1) + LN2 * y(j); };
    auto beta = [&](int j) { return sdt * a1[j]; };
    // smallest x; equal x: steeper line; the same bits in all PARTS threads
    auto pick = [](double &x, int &j, double &b) {
#pragma unroll
        for (int m = 1; m < PARTS; m <<= 1) {
            const double xo = __shfl_xor(x, m, 64), bo = __shfl_xor(b, m, 64);
            const int jo = __shfl_xor(j, m, 64);
            if (xo < x || (xo == x && bo > b) || (xo == x && bo == b && jo < j)) {
                x = xo;
                b = bo;
                j = jo;
            }
        }
    };
    double psi = INFINITY, bs = 0.0;
    int js = d;
    for (int j = part; j < d; j += PARTS) {
        const double b = beta(j), xj = (lnK - alpha(j)) / b;
        if (xj < psi || (xj == psi && b > bs)) {
            psi = xj;
            bs = b;
            js = j;
        }
    }
    pick(psi, js, bs);
    const double bstar = bs;
    double G = 0.0, dl = 0.0, vg = 0.0;
    double x0 = psi;
    int j = js;
    for (int seg = 0; seg < d; ++seg) {
        const double aj = alpha(j), bj = bs;
        double x1 = INFINITY, bn = 0.0;
        int jn = d;
        for (int i = part; i < d; i += PARTS) {
            const double bi = beta(i);
            if (!(bi > bj)) continue;
            const double xi = (aj - alpha(i)) / (bi - bj);
            if (xi < x1 || (xi == x1 && bi > bn)) {
                x1 = xi;
                bn = bi;
                jn = i;
            }
        }
        pick(x1, jn, bn);
        if (x1 < x0) x1 = x0;   // a line crossing at x0 itself (rounding)
        const double E = exp_f64<false>(aj + 0.5 * bj * bj);
        const double dP = norm_interval(x0 - bj, x1 - bj);
        const double fa = 0.39894228040143267794 * exp_f64<false>(-0.5 * (x0 - bj) * (x0 - bj));
        const double fb = isinf(x1) ? 0.0 : 0.39894228040143267794 * exp_f64<false>(-0.5 * (x1 - bj) * (x1 - bj));
        const double das = LN2 * y(j) / sig - sig * dt * (j + 1);   // c_j - sigma t_j
        G += E * dP - K * norm_interval(x0, x1);
        dl += E * dP;
        vg += E * (das * dP + (bj / sig) * (bj * dP + fa - fb));
        if (jn >= d) break;
        j = jn;
        bs = bn;
        x0 = x1;
    }
    const double D = op.D, S0 = op.S0;
    F[0] = D * G;
    F[1] = D * dl / S0;
    F[2] = D * vg;
    F[3] = D * K * 0.39894228040143267794 * exp_f64<false>(-0.5 * psi * psi) / (S0 * S0 * bstar);
}

template <int PARTS, typename YF>
__device__ inline void full_point_tail(const OptDev &op, YF y, int part, double F[4])
{
    if (op.type == QCPW_LOOKBACK_FIXED_CALL) {
        full_lookback_tail<PARTS>(op, y, part, F);
        return;
    }
    constexpr double LN2 = 0.69314718055994530942;
    const int d = op.n + 1;
    const double sig = 1.0 / op.inv_sigma;
    const double sdt = op.zscale * LN2;     // sigma sqrt(dt)
    const double wdt = op.ydrift_1 * LN2;   // omega dt
    const double dt = op.sqrt_t1 * op.sqrt_t1;
    const double lnS0 = ln_f64<false>(op.S0), K = op.K;
    const double *a1 = op.pca_a1;
    auto quad_sum = [](double v) {          // the same bits in all PARTS threads of the point
#pragma unroll
        for (int m = 1; m < PARTS; m <<= 1) v += __shfl_xor(v, m, 64);
        return v;
    };
    double sa = 0.0, sb = 0.0;
    for (int j = part; j < d; j += PARTS) {
        sa += lnS0 + wdt * (j + 1) + LN2 * y(j);
        sb += sdt * a1[j];
    }
    sa = quad_sum(sa);
    sb = quad_sum(sb);
    const double x0 = (ln_f64<false>(K) - sa / d) / (sb / d);   // Jensen bound, right of the root
    const double lndk = ln_f64<false>(K * d);
    // Moments M_k = sum_j g_j beta_j^k of g_j = exp(alpha_j + beta_j x0), k = 0..KM:
    // S(x0 + delta) = sum_k M_k delta^k / k! is the Taylor series of the sum,
    // so Newton's method runs on it without further exponentials.
    constexpr int KM = 8;
    double Mk[KM + 1];
#pragma unroll
    for (int k = 0; k <= KM; ++k) Mk[k] = 0.0;
    double bmax = 0.0;
    // Two dates per step (the second weighted 0 past the last date): their
    // exponentials are independent dependency chains, which the two waves
    // per SIMD could not overlap otherwise.
    for (int j = part; j < d; j += 2 * PARTS) {
        const int jb = j + PARTS < d ? j + PARTS : j;
        const double wb = j + PARTS < d ? 1.0 : 0.0;
        const double be = sdt * a1[j], beb = sdt * a1[jb];
        double p = exp_f64<false>(lnS0 + wdt * (j + 1) + LN2 * y(j) + be * x0);
        double pb = wb * exp_f64<false>(lnS0 + wdt * (jb + 1) + LN2 * y(jb) + beb * x0);
#pragma unroll
        for (int k = 0; k <= KM; ++k) {
            Mk[k] += p + pb;
            p *= be;
            pb *= beb;
        }
        bmax = fmax(bmax, fmax(fabs(be), fabs(beb)));
    }
#pragma unroll
    for (int k = 0; k <= KM; ++k) Mk[k] = quad_sum(Mk[k]);
#pragma unroll
    for (int m = 1; m < PARTS; m <<= 1) bmax = fmax(bmax, __shfl_xor(bmax, m, 64));
    double delta = 0.0;
    for (int it = 0; it < 64; ++it) {
        double S = Mk[KM] / 40320.0, S1 = 0.0;   // 1/8!
        double fk = 40320.0;
#pragma unroll
        for (int k = KM - 1; k >= 0; --k) {      // S = sum M_k d^k/k!, S1 = sum M_{k+1} d^k/k!
            fk /= (k + 1);
            S1 = fma(S1, delta, Mk[k + 1] / fk);
            S = fma(S, delta, Mk[k] / fk);
        }
        const double dd = (ln_f64<false>(S) - lndk) * S / S1;
        delta -= dd;
        if (!(fabs(dd) > 1e-13 * (1.0 + fabs(x0 + delta)))) break;   // also ends on NaN
    }
    double x = x0 + delta;
    // The series' truncation error is below (bmax |delta|)^9 / 9! relative;
    // when that may exceed FP64 rounding, finish with Newton on the exact sum.
    if (!(bmax * fabs(delta) < 0.1)) {
        for (int it = 0; it < 64; ++it) {
            double S = 0.0, S1 = 0.0;
            for (int j = part; j < d; j += PARTS) {
                const double be = sdt * a1[j];
                const double g = exp_f64<false>(lnS0 + wdt * (j + 1) + LN2 * y(j) + be * x);
                S += g;
                S1 += be * g;
            }
            S = quad_sum(S);
            S1 = quad_sum(S1);
            const double dx = (ln_f64<false>(S) - lndk) * S / S1;
            x -= dx;
            if (!(fabs(dx) > 1e-12 * (1.0 + fabs(x)))) break;   // also ends on NaN
        }
    }
    const double psi = x;
    const double epsi = exp_f64<false>(-0.5 * psi * psi);
    const bool arith = op.type == QCPW_ARITH_ASIAN_CALL;
    double F1 = 0.0, F2 = 0.0, Fs = 0.0, sEP = 0.0, sV = 0.0, sAg = 0.0;
    // date j's terms (weight w: 1, or 0 for the padding date of the last step)
    auto terms = [&](int j, double w) {
        const double yj = y(j);
        const double al = lnS0 + wdt * (j + 1) + LN2 * yj, be = sdt * a1[j];
        const double a = be / sig;                                // first-column entry, W units
        const double das = LN2 * yj / sig - sig * dt * (j + 1);   // c_j - sigma t_j
        const double g = w * exp_f64<false>(al + be * psi);
        F1 += be * g;
        if (arith) {
            // EP = e^{alpha + beta^2/2} erfc(u)/2, u = (psi - beta)/sqrt 2; e^{alpha + beta^2/2 - u^2}
            // = g e^{-psi^2/2}, so EP = erfcx(u) g e^{-psi^2/2} / 2 for u >= 0 (no exponential)
            const double u = (psi - be) * M_SQRT1_2;
            const double t = 0.5 * erfcx_f64<false>(fabs(u)) * g * epsi;
            const double EP = u >= 0.0 ? t : w * exp_f64<false>(al + 0.5 * be * be) - t;
            sEP += EP;
            sV += EP * (das + be * a);
            sAg += a * g;
        } else {
            F2 += be * be * g;
            Fs += g * (das + psi * a);
        }
    };
    // two dates per step, as above
    for (int j = part; j < d; j += 2 * PARTS) {
        const bool two = j + PARTS < d;
        terms(j, 1.0);
        terms(two ? j + PARTS : j, two ? 1.0 : 0.0);
    }
    F1 = quad_sum(F1) / d;
    const double D = op.D, S0 = op.S0;
    const double phi0 = epsi * 0.39894228040143267794;
    if (arith) {
        sEP = quad_sum(sEP) / d;
        sV = quad_sum(sV) / d;
        sAg = quad_sum(sAg) / d;
        F[0] = D * (sEP - K * 0.5 * erfc_f64<false>(psi * M_SQRT1_2));
        F[1] = D * sEP / S0;
        F[2] = D * (sV + phi0 * sAg);
        F[3] = D * phi0 * K * K / (S0 * S0 * F1);
    } else {
        F2 = quad_sum(F2) / d;
        Fs = quad_sum(Fs) / d;
        const double psiS = -(K / S0) / F1;   // d psi / d S0
        F[0] = D * 0.5 * erfc_f64<false>(psi * M_SQRT1_2);
        F[1] = -D * phi0 * psiS;
        F[2] = D * phi0 * Fs / F1;
        F[3] = D * K * phi0 / (S0 * F1) * (-psi * psiS - 2.0 / S0 - F2 * psiS / F1);
    }
}

// The PARTS threads of point p = tid / PARTS run full_point_tail; the first
// writes F to Fb[p][4]; wave 0, lane p, hands each valid point's F[k] to
// acc(k, F[k]) (compensated sums in registers, or in LDS for the other
// options of a group).
template <int PARTS, typename YF, typename ACC>
__device__ inline void full_tile_tail(const OptDev &op, YF y_of, double *Fb, int tid, int lane, int wave,
                                      bool lane_valid_for_wave0, ACC acc)
{
    static_assert(PARTS == 4 || PARTS == 8, "threads per point");
    const int p = tid / PARTS, part = tid % PARTS;
    double F[4];
    if (p < TP) full_point_tail<PARTS>(op, [&](int j) { return y_of(p, j); }, part, F);
    if (part == 0 && p < TP) {
#pragma unroll
        for (int k = 0; k < 4; ++k) Fb[p * 4 + k] = F[k];
    }
    __syncthreads();
    if (wave == 0 && lane_valid_for_wave0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) acc(k, Fb[lane * 4 + k]);
    }
}

// ------------------------------------------------------------------------
// FP32-mixed: matrix-core GEMM
// ------------------------------------------------------------------------
// Eight waves, one 32-row block of A each (rows 32 w .. 32 w + 31 of the
// padded NP x NP factor), both 32-point blocks of the tile.  A is
// stationary: a wave loads its row block into registers once per work unit
// (128 VGPRs: FP32, or BF16 hi and lo) and every tile of the unit streams
// only Z^T through LDS, so A costs no bandwidth in the tile loop.
template <bool BF16X3, bool FULL>
__global__ __launch_bounds__(64 * PCA_AS_WAVES) __attribute__((amdgpu_waves_per_eu(2, 2))) void pca_f32_kernel(
    const OptDev *__restrict__ opts, const int64_t *__restrict__ unit_prefix, const uint32_t *__restrict__ dir,
    const uint32_t *__restrict__ lane_tab, const float4 *__restrict__ ninv_tab, double *__restrict__ partials,
    unsigned long long *__restrict__ counter, int n_opts, int np_max, long long total_units, int owen)
{
    // LDS (all dynamic, from address 0): the inverse-normal cells of both halves
    // at 0 and QCPW_LDS_TAB_HI, the wave partials between them, the Z^T tile
    // after: FP32 [TP][np+1], or BF16 hi and lo [TP][np+8] each
    extern __shared__ __align__(16) unsigned char smem[];   // no static LDS: smem is address 0
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // waves in the workgroup: 8 (PCA_FULL, and n > 224), else max(2, NP / 32) for
    // the launch's largest padded n: every wave then owns a row block of A
    // (the first also runs the tails), so a small n keeps as many waves per
    // CU on the matrix cores as a large one
    const int W = (int)(blockDim.x >> 6);
    const int lr = lane & 31, khalf = lane >> 5;
    const int zstride = BF16X3 ? np_max + 8 : np_max + 1;
    float *Zf = (float *)(smem + QCPW_LDS_FIXED);
    unsigned short *Zh = (unsigned short *)(smem + QCPW_LDS_FIXED);
    unsigned short *Zl = Zh + (size_t)TP * zstride;
    PcaSums<float> *red = (PcaSums<float> *)(smem + QCPW_LDS_GAP_BEGIN);   // [PCA_AS_WAVES][TP]
    long long *s_unit = (long long *)(smem + QCPW_LDS_GAP_BEGIN + PCA_AS_WAVES * TP * sizeof(PcaSums<float>));
    // compensated sums of the other members of a group (wave 0): [member - 1][8][TP]
    constexpr size_t MACC_OFF = QCPW_LDS_GAP_BEGIN + PCA_AS_WAVES * TP * sizeof(PcaSums<float>) + 64;
    double *macc = (double *)(smem + MACC_OFF);
    static_assert(MACC_OFF + (QCPW_PCA_MAX_GROUP - 1) * 8 * TP * sizeof(double) <= QCPW_LDS_TAB_HI, "gap");
    {
        float4 *cells = (float4 *)smem;
        for (int i = tid; i < 2 * QCPW_NINV_TAB_CELLS; i += blockDim.x)
            cells[(i < QCPW_NINV_TAB_CELLS ? 0 : QCPW_LDS_TAB_HI / 16 - QCPW_NINV_TAB_CELLS) + i] = ninv_tab[i];
        __syncthreads();
    }
    constexpr int KS = BF16X3 ? QCPW_PCA_NPAD / 16 : QCPW_PCA_NPAD / 2;           // k steps of the MFMA
    // this wave's row block: FP32 Ar[u] = A[row][2 u + khalf]; BF16: Ah/Al[u] = A[row][16 u + 8 khalf ..]
    float Ar[BF16X3 ? 1 : KS];
    v8us Ah[BF16X3 ? KS : 1], Al[BF16X3 ? KS : 1];
    const int row = 32 * wave + lr;
    int o = 0;
    for (;;) {
        const long long unit = next_unit(counter, s_unit);
        if (unit >= total_units) break;
        locate_unit(unit_prefix, n_opts, unit, o);
        const OptDev &op = opts[o];
        const int n = op.n, NP = op.pca_np;
        const int64_t rem = unit - op.unit0;
        const int shift = (int)(rem / op.chunks);
        const int64_t chunk = rem - (int64_t)shift * op.chunks;
        const int64_t k_end = op.k_begin + op.n_points;
        const int64_t t0 = op.k_begin + chunk * op.unit_pts;
        const int64_t t1 = min(t0 + (int64_t)op.unit_pts, k_end);
        const bool gemm_wave = wave < NP / 32;
        if (gemm_wave) {
#pragma unroll
            for (int u = 0; u < KS; ++u) {
                if (BF16X3) {
                    if (16 * u < NP) {
                        const size_t off = ((size_t)u * NP + row) * 16 + khalf * 8;
                        Ah[u] = *(const v8us *)&op.pca_hi[off];
                        Al[u] = *(const v8us *)&op.pca_lo[off];
                    }
                } else {
                    if (2 * u < NP) Ar[u] = op.pca_At[(size_t)(2 * u + khalf) * NP + row];
                }
            }
        }

        // padding columns of Z (k = n .. NP-1) must hold zeros (also after a
        // PCA_FULL epilogue has used the Z area for the products)
        auto zero_padding = [&] {
            for (int i = tid; i < TP * (NP - n); i += blockDim.x) {
                const int p = i / (NP - n), k = n + i % (NP - n);
                if (BF16X3) {
                    Zh[p * zstride + k] = 0;
                    Zl[p * zstride + k] = 0;
                } else {
                    Zf[p * zstride + k] = 0.0f;
                }
            }
        };
        zero_padding();
        // Waves 1..W-1 generate the normals (wave 0 meanwhile runs the previous
        // tile's FP64 tail): prologue wave pw = wave - 1 takes dimensions
        // 1 + PD pw .. PD (pw + 1), and its lane l holds the uniform part of 1 + PD pw + l.
        // (even with BF16 Z, so that pairs of columns share one 32-bit store);
        // PD <= 64 since W >= NP / 32 (checked at launch)
        const int PD0 = (n + W - 2) / (W - 1);
        const int PD = BF16X3 ? (PD0 + 1) & ~1 : PD0;
        const int pw = wave - 1;
        const int myj = 1 + PD * pw + lane;
        uint32_t U = 0;
        uint32_t Key = 0;   // nested scrambling: the dimension's seed
        if (wave > 0 && lane < PD && myj <= n) {
            U = uniform_part(dir, op.seed, shift, myj, (uint64_t)t0, owen != 0);
            if (owen) Key = digital_shift(op.seed, shift, myj);
        }
        const int jcount = wave > 0 ? max(0, min(PD, n - PD * pw)) : 0;
        double s[4] = {0.0, 0.0, 0.0, 0.0}, c[4] = {0.0, 0.0, 0.0, 0.0};
        // options sharing these paths (same product and epilogue, FP64 tail each)
        const int grp = op.grp;
        if (wave == 0)
            for (int i = 0; i < (grp - 1) * 8; ++i) macc[i * TP + lane] = 0.0;
        // ---- prologue: z' = Phi^{-1}(u) * sigma sqrt(dt) log2(e) for the 64 points of the
        // tile at `base` x this wave's dimensions, then the Gray-code step to the next tile
        const int jc = __builtin_amdgcn_readfirstlane(jcount);
        auto store_z = [&](int jj, float z) {
            const int k = PD * pw + jj;   // column of dimension j = k + 1
            if (BF16X3) {
                const unsigned short h = bf16_bits(z);
                Zh[lane * zstride + k] = h;
                Zl[lane * zstride + k] = bf16_bits(z - bf16_value(h));
            } else {
                Zf[lane * zstride + k] = z;
            }
        };
        // BF16 Z: columns k, k + 1 (k even) rounded to BF16 together, hi and lo
        // parts each stored as one 32-bit word
        auto store_pair = [&](int jj, float z0, float z1) {
            const int k = PD * pw + jj;
            const f32x2 v = {z0, z1};
            const uint32_t hb = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
            const f32x2 hv = {__uint_as_float(hb << 16), __uint_as_float(hb & 0xFFFF0000u)};
            const uint32_t lb = __builtin_bit_cast(uint32_t, __builtin_convertvector(v - hv, bf16x2));
            *(uint32_t *)&Zh[lane * zstride + k] = hb;
            *(uint32_t *)&Zl[lane * zstride + k] = lb;
        };
        auto prologue = [&](int64_t base) {
            // lane-table words eight at a time, all loads in flight before the first use
            for (int j0 = 0; j0 < jc; j0 += 8) {
                uint32_t w[8];
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    w[i] = j0 + i < jc ? lane_tab[(size_t)(1 + PD * pw + j0 + i) * 64 + lane] : 0u;
                // the group's eight cell reads go out before any store into Z, with
                // no branch between them, so their latencies overlap (past jc the
                // value is computed from a zero word and never stored)
                float z[8];
                if (owen) {
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        z[i] = ninv_table_f32(owen_scramble(w[i] ^ rdlane(U, j0 + i), rdlane(Key, j0 + i))) * op.zs_t;
                } else {
#pragma unroll
                    for (int i = 0; i < 8; ++i) z[i] = ninv_table_f32(w[i] ^ rdlane(U, j0 + i)) * op.zs_t;
                }
                if (j0 + 8 <= jc) {
#pragma unroll
                    for (int i = 0; i < 8; i += BF16X3 ? 2 : 1) {
                        if (BF16X3) store_pair(j0 + i, z[i], z[i + 1]);
                        else store_z(j0 + i, z[i]);
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < 8; i += BF16X3 ? 2 : 1) {
                        if (j0 + i >= jc) break;
                        if (BF16X3 && j0 + i + 1 < jc) store_pair(j0 + i, z[i], z[i + 1]);
                        else store_z(j0 + i, z[i]);
                    }
                }
            }
            if (base + TP < t1 && wave > 0 && lane < PD && myj <= n) {
                const uint32_t *v = dir + (size_t)myj * 32;
                U ^= v[5] ^ v[6 + __builtin_ctzll(((uint64_t)base >> 6) + 1)];
            }
        };
        prologue(t0);
        __syncthreads();

        for (int64_t base = t0; base < t1; base += TP) {
            // ---- GEMM on the matrix cores: rows of this wave x points 0..31 (acc0), 32..63 (acc1)
            v16f acc0 = (v16f){}, acc1 = (v16f){};
            if (gemm_wave) {
                // NP is a multiple of 32: one guard per 32 k, so that each group's LDS
                // reads can be scheduled ahead of its MFMAs
                constexpr int KG = BF16X3 ? 2 : 16;   // k steps per 32 k
#pragma unroll
                for (int g = 0; g < KS / KG; ++g) {
                    if (32 * g >= NP) continue;
#pragma unroll
                for (int u = g * KG; u < (g + 1) * KG; ++u) {
                    if (BF16X3) {
                        const int k = 16 * u + khalf * 8;
                        const v8bf bh0 = __builtin_bit_cast(v8bf, *(const v8us *)&Zh[lr * zstride + k]);
                        const v8bf bl0 = __builtin_bit_cast(v8bf, *(const v8us *)&Zl[lr * zstride + k]);
                        const v8bf bh1 = __builtin_bit_cast(v8bf, *(const v8us *)&Zh[(32 + lr) * zstride + k]);
                        const v8bf bl1 = __builtin_bit_cast(v8bf, *(const v8us *)&Zl[(32 + lr) * zstride + k]);
                        const v8bf h = __builtin_bit_cast(v8bf, Ah[u]), l = __builtin_bit_cast(v8bf, Al[u]);
                        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(l, bh0, acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(l, bh1, acc1, 0, 0, 0);
                        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h, bl0, acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h, bl1, acc1, 0, 0, 0);
                        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h, bh0, acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h, bh1, acc1, 0, 0, 0);
                    } else {
                        const int k = 2 * u + khalf;
                        acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(Ar[u], Zf[lr * zstride + k], acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(Ar[u], Zf[(32 + lr) * zstride + k], acc1, 0, 0, 0);
                    }
                }
                }
            }

            if constexpr (FULL) {
                // ---- epilogue: the d products of each point into LDS (over Z),
                // then the FP64 root-find and Greeks, eight threads per point
                const int cstride = NP + 1;
                float *Cb = Zf;
                __syncthreads();   // every wave is done reading Z
                if (gemm_wave) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int m = 32 * wave + (r >> 2) * 8 + khalf * 4 + (r & 3);
                        if (m <= n) {
                            Cb[lr * cstride + m] = acc0[r];
                            Cb[(32 + lr) * cstride + m] = acc1[r];
                        }
                    }
                }
                __syncthreads();
                auto y_of = [&](int p, int j) { return (double)Cb[p * cstride + j]; };
                full_tile_tail<PCA_AS_WAVES>(op, y_of, (double *)red, tid, lane, wave, base + lane < t1,
                                             [&](int k, double v) { acc_add(s[k], c[k], v); });
                // the group's other options: their own tails on the same products
                for (int mi = 1; mi < grp; ++mi) {
                    __syncthreads();   // wave 0 is done reading the previous tails' F
                    double *a = macc + (size_t)(mi - 1) * 8 * TP + lane;
                    full_tile_tail<PCA_AS_WAVES>(opts[o + mi], y_of, (double *)red, tid, lane, wave, base + lane < t1,
                                                 [&](int k, double v) {
                                                     double sk = a[k * TP], ck = a[(4 + k) * TP];
                                                     acc_add(sk, ck, v);
                                                     a[k * TP] = sk;
                                                     a[(4 + k) * TP] = ck;
                                                 });
                }
                __syncthreads();
                zero_padding();   // the prologue writes columns 0..n-1 only
                if (base + TP < t1) prologue(base + TP);
                __syncthreads();
                continue;
            }
            // ---- epilogue: exp2 and path sums over this lane's rows of its two points
            PcaSums<float> ps0, ps1;
            const bool lo = qcpw_stat_of(op.type) == QCPW_STAT_MIN;
            sums_neutral(ps0, lo);
            sums_neutral(ps1, lo);
            const float drift = op.ydrift_1_f;
            // each product needs one statistic: the average's sums (one exp2 and three
            // sums per date), the sum of Y, or the running extreme
            auto rows = [&](auto add) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int m = 32 * wave + (r >> 2) * 8 + khalf * 4 + (r & 3);
                    if (m < n) {
                        const float mf = (float)(m + 1);
                        add(ps0, fmaf(drift, mf, acc0[r]), mf);
                        add(ps1, fmaf(drift, mf, acc1[r]), mf);
                    }
                }
            };
            if (gemm_wave) {
                const int mode = qcpw_stat_of(op.type);
                if (mode == QCPW_STAT_AVG) {
                    rows([](PcaSums<float> &p, float Y, float mf) {
                        const float E = exp2_r(Y);
                        p.A1 += E;
                        p.A2y = fmaf(E, Y, p.A2y);
                        p.A2m = fmaf(E, mf, p.A2m);
                    });
                } else if (mode == QCPW_STAT_GEO) {
                    rows([](PcaSums<float> &p, float Y, float) { p.sY += Y; });
                } else {
                    rows([lo](PcaSums<float> &p, float Y, float mf) { sums_add_date<float>(p, Y, mf, lo); });
                }
            }
            // lane halves hold other rows of the same points; lane l keeps point l
            sums_merge(ps0, shfl_xor_sums(ps0, 32), lo);
            sums_merge(ps1, shfl_xor_sums(ps1, 32), lo);
            if (khalf) red[wave * TP + lane] = ps1;
            else red[wave * TP + lane] = ps0;
            __syncthreads();
            if (wave == 0) {   // this tile's tails, while the other waves fill Z with the next tile
                const int waves_pt[PCA_AS_WAVES] = {0, 1, 2, 3, 4, 5, 6, 7};
                tile_tail<float>(op, red, lane, base + lane < t1, W, waves_pt, s, c);
                for (int mi = 1; mi < grp; ++mi) {
                    double sm[4], cm[4];
                    double *acc = macc + (size_t)(mi - 1) * 8 * TP + lane;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        sm[i] = acc[i * TP];
                        cm[i] = acc[(4 + i) * TP];
                    }
                    tile_tail<float>(opts[o + mi], red, lane, base + lane < t1, W, waves_pt, sm, cm);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        acc[i * TP] = sm[i];
                        acc[(4 + i) * TP] = cm[i];
                    }
                }
            } else if (base + TP < t1) {
                prologue(base + TP);
            }
            __syncthreads();
        }
        if (wave == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                wave_reduce(s[i], c[i]);
                if (lane == 0) {
                    partials[unit * 8 + i] = s[i];
                    partials[unit * 8 + 4 + i] = c[i];
                }
            }
            // the members' partials at the same offset in their own units
            for (int mi = 1; mi < grp; ++mi) {
                const double *acc = macc + (size_t)(mi - 1) * 8 * TP + lane;
                const int64_t mu = opts[o + mi].unit0 + rem;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    double sm = acc[i * TP], cm = acc[(4 + i) * TP];
                    wave_reduce(sm, cm);
                    if (lane == 0) {
                        partials[mu * 8 + i] = sm;
                        partials[mu * 8 + 4 + i] = cm;
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------------
// FP64: the same tiles with Z^T in FP64 and FP64 FMAs
// ------------------------------------------------------------------------
template <bool FULL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void pca_f64_kernel(const OptDev *__restrict__ opts,
                                                      const int64_t *__restrict__ unit_prefix,
                                                      const uint32_t *__restrict__ dir,
                                                      const uint32_t *__restrict__ lane_tab,
                                                      double *__restrict__ partials,
                                                      unsigned long long *__restrict__ counter, int n_opts,
                                                      int n_max, long long total_units,
                                                      double *__restrict__ scratch, int owen)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ long long s_unit;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int zstride = n_max + 1;
    // PCA_FULL: this workgroup's [date][64] products (global, L2-resident)
    double *Cg = scratch + (size_t)blockIdx.x * QCPW_MAX_D_PCA_FULL * TP;
    double *Z = (double *)smem;                                              // [TP][n_max + 1]
    PcaSums<double> *red = (PcaSums<double> *)(smem + (size_t)TP * zstride * 8);   // [4][TP]

    int o = 0;
    for (;;) {
        const long long unit = next_unit(counter, &s_unit);
        if (unit >= total_units) break;
        locate_unit(unit_prefix, n_opts, unit, o);
        const OptDev &op = opts[o];
        const int n = op.n;
        const int64_t rem = unit - op.unit0;
        const int shift = (int)(rem / op.chunks);
        const int64_t chunk = rem - (int64_t)shift * op.chunks;
        const int64_t k_end = op.k_begin + op.n_points;
        const int64_t t0 = op.k_begin + chunk * op.unit_pts;
        const int64_t t1 = min(t0 + (int64_t)op.unit_pts, k_end);
        const int myj = 1 + 64 * wave + lane;
        uint32_t U = 0, Key = 0;
        if (myj <= n) {
            U = uniform_part(dir, op.seed, shift, myj, (uint64_t)t0, owen != 0);
            if (owen) Key = digital_shift(op.seed, shift, myj);
        }
        const int jcount = max(0, min(64, n - 64 * wave));
        double s[4] = {0.0, 0.0, 0.0, 0.0}, c[4] = {0.0, 0.0, 0.0, 0.0};

        for (int64_t base = t0; base < t1; base += TP) {
            for (int jj = 0; jj < jcount; ++jj) {
                const int j = 1 + 64 * wave + jj;
                uint32_t y = lane_tab[(size_t)j * 64 + lane] ^ rdlane(U, jj);
                if (owen) y = owen_scramble(y, rdlane(Key, jj));
                Z[lane * zstride + (j - 1)] = ninv_f64(y) * op.zscale;
            }
            if (base + TP < t1 && myj <= n) {
                const uint32_t *v = dir + (size_t)myj * 32;
                U ^= v[5] ^ v[6 + __builtin_ctzll(((uint64_t)base >> 6) + 1)];
            }
            __syncthreads();
            // rows m = wave, wave + 4, ...: W'_m = sum_i A[m][i] z'_i, four rows at a time
            PcaSums<double> ps;
            const bool lo = qcpw_stat_of(op.type) == QCPW_STAT_MIN;
            sums_neutral(ps, lo);
            const double drift = op.ydrift_1;
            const int rows = FULL ? n + 1 : n;
            for (int m0 = wave; m0 < rows; m0 += 16) {
                double acc[4] = {0.0, 0.0, 0.0, 0.0};
                const double *A0 = op.pca_A64 + (size_t)m0 * n;
                for (int i = 0; i < n; ++i) {
                    const double z = Z[lane * zstride + i];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (m0 + 4 * q < rows) acc[q] = fma(A0[(size_t)4 * q * n + i], z, acc[q]);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int m = m0 + 4 * q;
                    if (m < rows) {
                        if (FULL) {
                            Cg[(size_t)m * TP + lane] = acc[q];
                        } else {
                            const double mf = (double)(m + 1);
                            sums_add_date<double>(ps, fma(drift, mf, acc[q]), mf, lo);
                        }
                    }
                }
            }
            if constexpr (FULL) {
                __syncthreads();
                full_tile_tail<PCA_WAVES>(op, [&](int p, int j) { return Cg[(size_t)j * TP + p]; }, (double *)red, tid, lane,
                                          wave, base + lane < t1, [&](int k, double v) { acc_add(s[k], c[k], v); });
                __syncthreads();
                continue;
            }
            red[wave * TP + lane] = ps;
            __syncthreads();
            if (wave == 0) {
                const int waves_pt[4] = {0, 1, 2, 3};
                tile_tail<double>(op, red, lane, base + lane < t1, 4, waves_pt, s, c);
            }
            __syncthreads();
        }
        if (wave == 0) {
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
}

// ------------------------------------------------------------------------
// launch
// ------------------------------------------------------------------------
qcpw_status enqueue_pca(Context *ctx, const LaunchPlan &lp, hipStream_t stream, const LaunchDesc &ld,
                        const OptDev *d_opts)
{
    (void)d_opts;
    int np_max = 32, n_max = 1;
    for (const auto &op : lp.opts) {
        np_max = std::max(np_max, op.pca_np);
        n_max = std::max(n_max, op.n);
    }
    const void *fn;
    size_t lds;
    int extra;
    const bool full = lp.path == QCPW_PATH_PCA_FULL;
    if (lp.precision == QCPW_FP64) {
        fn = full ? reinterpret_cast<const void *>(&pca_f64_kernel<true>)
                  : reinterpret_cast<const void *>(&pca_f64_kernel<false>);
        lds = (size_t)TP * (n_max + 1) * 8 + (size_t)PCA_WAVES * TP * sizeof(PcaSums<double>);
        extra = n_max;
    } else {
        const bool bf = lp.pca_gemm == QCPW_GEMM_BF16X3;
        fn = bf ? (full ? reinterpret_cast<const void *>(&pca_f32_kernel<true, true>)
                        : reinterpret_cast<const void *>(&pca_f32_kernel<true, false>))
                : (full ? reinterpret_cast<const void *>(&pca_f32_kernel<false, true>)
                        : reinterpret_cast<const void *>(&pca_f32_kernel<false, false>));
        const size_t z = bf ? (size_t)2 * TP * (np_max + 8) * 2 : (size_t)TP * (np_max + 1) * 4;
        lds = QCPW_LDS_FIXED + z;   // cells, wave partials between them, then Z^T
        extra = np_max;
    }
    if (lds > 160 * 1024) return fail(QCPW_EDIMS, "PCA tile exceeds 160 KiB of LDS");
    if (lp.precision == QCPW_FP32_MIXED) {
        qcpw_status st = check_lds_at_zero(fn);
        if (st != QCPW_OK) return st;
    }
    QCPW_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    // matrix cores, first-date conditioning: one wave per 32 rows of the
    // launch's largest padded factor, at least two (the tails and a prologue
    // wave); PCA_FULL runs eight threads per point in its tail
    int waves = PCA_AS_WAVES;
    if (lp.precision == QCPW_FP32_MIXED && !full) {
        waves = std::min(PCA_AS_WAVES, std::max(2, np_max / 32));
        int n_top = 1;
        for (const auto &op : lp.opts) n_top = std::max(n_top, op.n);
        if ((n_top + waves - 2) / (waves - 1) > 64) return fail(QCPW_EDEVICE, "PCA prologue exceeds one wave per 64 dimensions");
    }
    const int bd = 64 * (lp.precision == QCPW_FP64 ? PCA_WAVES : waves);
    QCPW_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, bd, lds));
    if (per_cu < 1) return fail(QCPW_EDEVICE, "PCA kernel cannot be resident");
    int64_t grid = std::min<int64_t>((int64_t)per_cu * ctx->tab.n_cu, lp.total_units);
    if (full && lp.precision == QCPW_FP64) {
        if (lp.full_blocks < 1) return fail(QCPW_EDEVICE, "PCA_FULL scratch was not planned");
        grid = std::min<int64_t>(grid, lp.full_blocks);   // one scratch tile per workgroup
    }
    const OptDev *a_opts = ld.opts;
    const int64_t *a_prefix = ld.unit_prefix;
    const uint32_t *a_dir = ld.dir, *a_lane = ld.lane;
    double *a_part = ld.partials;
    unsigned long long *a_ctr = ld.counter;
    int a_nopts = ld.n_opts;
    long long a_total = ld.total_units;
    double *a_scratch = ld.scratch;
    const float4 *a_tab = ctx->tab.ninv_tab;
    int a_owen = lp.owen ? 1 : 0;
    void *args32[] = {&a_opts, &a_prefix, &a_dir, &a_lane, &a_tab, &a_part, &a_ctr, &a_nopts, &extra, &a_total, &a_owen};
    void *args64[] = {&a_opts, &a_prefix, &a_dir, &a_lane, &a_part, &a_ctr, &a_nopts, &extra, &a_total, &a_scratch,
                      &a_owen};
    QCPW_HIP(hipLaunchKernel(fn, dim3((unsigned)grid), dim3(bd), lp.precision == QCPW_FP64 ? args64 : args32, lds,
                             stream));
    return QCPW_OK;
}

}  // namespace qcpw
