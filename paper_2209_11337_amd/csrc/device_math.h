// device_math.h -- device helpers shared by the per-path and PCA kernels:
// digital shifts, the FP32 / FP64 inverse normal, path sums, the per-path
// FP64 tail (breakpoint, Phi tails, Greeks) and compensated reductions.
#pragma once
#include <hip/hip_runtime.h>

#include "qcpw_internal.h"
#include "../../include/qmc_cpw.h"

namespace qcpw {

#include "ninv_f32_coeffs.inc"
#include "ninv_table.inc"
#include "phi_f64_coeffs.inc"

// ------------------------------------------------------------------------
// device helpers
// ------------------------------------------------------------------------

// SplitMix64 (Steele, Lea, Flood 2014): output i of the generator seeded
// with `seed` is the variant-13 mixer applied to seed + (i + 1) * gamma.
__device__ __host__ inline uint64_t splitmix64_out(uint64_t seed, uint64_t i)
{
    uint64_t x = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    x ^= x >> 30;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__device__ inline uint32_t digital_shift(uint64_t seed, int l, int j)
{
    return (uint32_t)(splitmix64_out(seed, ((uint64_t)l << 16) | (uint64_t)j) >> 32);
}

template <int N>
__device__ inline float horner(const float (&c)[N], float v)
{
    float p = c[0];
#pragma unroll
    for (int i = 1; i < N; ++i) p = fmaf(p, v, c[i]);
    return p;
}

// Phi^{-1}((y + 1/2) 2^-32) * scale in FP32, with sa = scale * 2^-31
// (scale includes the sqrt(2) of Phi^{-1}(u) = sqrt(2) erfinv(2u - 1)).
// Folding y onto the lower half, m = min(y, ~y), gives q = (m + 1/2) 2^-32
// exactly from an integer.  The factor x = 2u - 1 = (y - 2^31 + 1/2) 2^-31
// is taken as (y - 2^31) 2^-31, signed so it carries the sign of the result;
// the dropped 2^-32 is below FP32 resolution of x except within 2^-31 of
// u = 1/2, where it moves z by less than 1e-9 absolute.  erfinv(x)/x is a
// polynomial in w = -ln(1 - x^2) = -ln(4 q (1 - q)) (two branches,
// coefficients in ninv_f32_coeffs.inc).
__device__ inline float ninv_scaled_f32(uint32_t y, float sa)
{
    const uint32_t m = y ^ (uint32_t)((int32_t)y >> 31);   // min(y, ~y)
    const float q = fmaf((float)m, 0x1p-32f, 0x1p-33f);
    const float xs = (float)(int32_t)(y ^ 0x80000000u) * sa;   // scale * (2u - 1)
    const float t = fmaf(-q, q, q);                         // q (1 - q) = (1 - x^2) / 4
    const float lg = __builtin_amdgcn_logf(t);              // log2 t
    constexpr float LN2 = 0.693147180559945309f;
    constexpr float LG_SPLIT = -(QCPW_NINV_WSPLIT / 0.693147180559945309f) - 2.0f;
    float p;
    if (lg > LG_SPLIT) {
        p = horner(QCPW_NINV_P, fmaf(lg, -LN2, -2.0f * LN2 - QCPW_NINV_C1));
    } else {
        const float w = fmaf(lg, -LN2, -2.0f * LN2);
        p = horner(QCPW_NINV_Q, __builtin_amdgcn_sqrtf(w) - QCPW_NINV_C2);
    }
    return p * xs;
}

// Nested (Owen) scrambling of one 32-bit coordinate in base 2 (Sec. 2.2.3):
// digit k (k = 1 most significant) is flipped by a function of digits
// 1..k-1 only.  On the bit-reversed value that is what a seeded addition
// (carries move up) and v ^= (v mod 2^24) * C with an even constant C (the
// product's bit i sees only bits below i) do; four such rounds follow the
// addition.  24-bit products (v_mul_u32_u24) run at the full VALU rate.
__device__ inline uint32_t owen_scramble(uint32_t y, uint32_t seed)
{
    uint32_t v = __builtin_bitreverse32(y) + seed;
    v ^= __umul24(v, 0xcca0d0u);
    v ^= __umul24(v, 0x6292a6u);
    v ^= __umul24(v, 0xb21bbau);
    v ^= __umul24(v, 0x70b6f2u);
    return __builtin_bitreverse32(v);
}

// Phi^{-1}((y + 1/2) 2^-32) in FP32 for the raw 32-bit Sobol coordinate y,
// from the cubic tables of ninv_table.inc held in LDS at address 0 (lower
// half) and QCPW_LDS_TAB_HI (upper half).  q = float(int32(y)) is y itself
// below 2^31 and -(2^32 - y) above; bits 16..31 of q masked with 0x8FF0 are
// the LDS address of the cell (sign: which half; low exponent and top
// mantissa bits: which cell), and the cubic is evaluated in |q| (a free
// source modifier).  Each half's table carries its own sign.
__device__ inline float ninv_table_f32(uint32_t y)
{
    static_assert(QCPW_NINV_CELL_BITS == 3 && QCPW_LDS_TAB_HI == 0x8000, "cell address = (bits >> 16) & 0x8FF0");
    const float q = (float)(int32_t)y;
    const uint32_t addr = (__float_as_uint(q) >> 16) & 0x8FF0u;
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    const f32x4 c = *(const __attribute__((address_space(3))) f32x4 *)addr;
    const float a = fabsf(q);
    return fmaf(fmaf(fmaf(c.x, a, c.y), a, c.z), a, c.w);
}

// Four of them with their cell reads in flight together: the compiler, short
// of registers, would otherwise reuse one register quadruple and wait for
// each read before issuing the next.  The four reads and their wait are one
// asm block (no output can be reused before its load has landed; the
// outputs are early-clobber, so no address is overwritten by a load).
__device__ inline void ninv_table_f32_x4(const uint32_t (&y)[4], float (&z)[4])
{
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    float q[4];
    uint32_t addr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        q[i] = (float)(int32_t)y[i];
        addr[i] = (__float_as_uint(q[i]) >> 16) & 0x8FF0u;
    }
    f32x4 c0, c1, c2, c3;
    asm volatile("ds_read_b128 %0, %4\n\t"
                 "ds_read_b128 %1, %5\n\t"
                 "ds_read_b128 %2, %6\n\t"
                 "ds_read_b128 %3, %7\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(c0), "=&v"(c1), "=&v"(c2), "=&v"(c3)
                 : "v"(addr[0]), "v"(addr[1]), "v"(addr[2]), "v"(addr[3]));
    const f32x4 c[4] = {c0, c1, c2, c3};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float a = fabsf(q[i]);
        z[i] = fmaf(fmaf(fmaf(c[i].x, a, c[i].y), a, c[i].z), a, c[i].w);
    }
}

__device__ inline float exp2_r(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ inline double exp2_r(double x) { return exp2(x); }

// Knuth two-sum: s + c accumulates x with the rounding error kept in c.
__device__ inline void acc_add(double &s, double &c, double x)
{
    const double t = s + x;
    const double bp = t - s;
    c += (s - (t - bp)) + (x - bp);
    s = t;
}

// Combine compensated pairs across the wave (xor butterfly, fixed order).
__device__ inline void wave_reduce(double &s, double &c)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double s2 = __shfl_xor(s, off, 64);
        const double c2 = __shfl_xor(c, off, 64);
        const double t = s + s2;
        const double bp = t - s;
        const double e = (s - (t - bp)) + (s2 - bp);
        s = t;
        c = (c + c2) + e;
    }
}

__device__ inline uint32_t rdlane(uint32_t v, int l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

template <typename R>
struct PathSums {
    R A1, A2y, A2m;   // sum E_m, sum E_m Y_m, sum E_m m   (averages)
    R bY, bm;         // running max (min) of Y_m and its m (lookback; E = 2^Y once, at the end)
};

// What a date adds to the path statistic: the arithmetic average's sums,
// the running maximum, or (geometric average) the sum of Y = log2 S~/S0.
enum { QCPW_STAT_AVG = 0, QCPW_STAT_MAX = 1, QCPW_STAT_GEO = 2, QCPW_STAT_MIN = 3 };

__host__ __device__ inline bool qcpw_is_put(int type)
{
    return (type >= QCPW_ARITH_ASIAN_PUT && type <= QCPW_GEOMETRIC_ASIAN_PUT) || type == QCPW_BASKET_ASIAN_PUT;
}

__host__ __device__ inline bool qcpw_is_basket(int type)
{
    return type == QCPW_BASKET_ASIAN_CALL || type == QCPW_BASKET_ASIAN_PUT;
}

__host__ __device__ inline int qcpw_stat_of(int type)
{
    return type == QCPW_LOOKBACK_FIXED_CALL ? QCPW_STAT_MAX
           : type == QCPW_LOOKBACK_FIXED_PUT ? QCPW_STAT_MIN
           : (type == QCPW_GEOMETRIC_ASIAN_CALL || type == QCPW_GEOMETRIC_ASIAN_PUT) ? QCPW_STAT_GEO
                                                                                   : QCPW_STAT_AVG;
}

template <typename R, int MODE>
__device__ inline void consume(PathSums<R> &ps, R Y, R mf)
{
    if (MODE == QCPW_STAT_MAX || MODE == QCPW_STAT_MIN) {
        // bitwise, not short-circuit: two compares and selects, no branch
        const bool better = MODE == QCPW_STAT_MAX ? Y > ps.bY : Y < ps.bY;
        const bool take = better | ((Y == ps.bY) & (mf < ps.bm));   // lowest index wins ties
        ps.bY = take ? Y : ps.bY;
        ps.bm = take ? mf : ps.bm;
    } else if (MODE == QCPW_STAT_GEO) {
        ps.A2y += Y;
    } else {
        const R E = exp2_r(Y);
        ps.A1 += E;
        ps.A2y = fma(E, Y, ps.A2y);
        ps.A2m = fma(E, mf, ps.A2m);
    }
}

// ---- compact FP64 elementary functions for the per-path tail -------------
// (few live registers, no special-case branches beyond what the path's
// values can reach: finite positive arguments for ln, non-positive for exp).
// Polynomial coefficients go through coef_after(): an empty asm that ties
// each coefficient to the previous Horner value, so the compiler materialises
// it (two scalar moves) just before its use instead of hoisting all of them
// into ~80 registers held across the point loop, which would halve the
// kernel's occupancy.  ORDERED = false drops the asm's volatile: the tie
// stays, but two independent evaluations may then interleave (with volatile
// their empty asms keep program order, which serialises the chains).
template <bool ORDERED = true>
__device__ inline double coef_after(double c, double dep)
{
    uint64_t b = __builtin_bit_cast(uint64_t, c);
    if constexpr (ORDERED) asm volatile("" : "+s"(b) : "v"(dep));
    else asm("" : "+s"(b) : "v"(dep));
    return __builtin_bit_cast(double, b);
}

// A pointer passed through an empty asm: loads through it cannot be hoisted
// out of the loop that calls the tail, so per-option fields are re-read
// (scalar loads, cache hits) instead of held in registers across the loop.
template <typename T>
__device__ inline const T *reread(const T *p)
{
    asm volatile("" : "+s"(p));
    return p;
}

// 1/d to ~1 ulp: hardware reciprocal refined by two Newton steps.
__device__ inline double recip_f64(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}

// ln x for finite x > 0: x = 2^e m, m in [sqrt(1/2), sqrt(2)),
// ln m = 2 atanh(s) = 2 (s + s^3/3 + ... + s^23/23), s = (m - 1)/(m + 1),
// |s| <= 0.1716; ln 2 split so that e ln2_hi is exact.
//
// SHORT = true (the kernels whose path statistic is an FP32 sum, itself
// rounded near 1e-7 relative): shorter expansions held to about 1e-12
// relative, here the series to s^13 (the first term left out, s^15/15, is
// at most 1.3e-12 of s).
template <bool ORDERED = true, bool SHORT = false>
__device__ inline double ln_f64(double x)
{
    int e;
    double m = frexp(x, &e);   // m in [1/2, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) * recip_f64(m + 1.0);
    const double z = s * s;
    constexpr int KTOP = SHORT ? 13 : 23;
    double p = coef_after<ORDERED>(1.0 / KTOP, z);
#pragma unroll
    for (int k = KTOP - 2; k >= 1; k -= 2) p = fma(p, z, coef_after<ORDERED>(1.0 / k, p));
    const double de = (double)e;
    return fma(de, 6.93147180369123816490e-01, fma(de, 1.90821492927058770002e-10, 2.0 * s * p));
}

// exp x for |x| < 700 (beyond, below about -745 it underflows to 0):
// x = k ln 2 + r, |r| <= ln2/2, e^r by its Taylor series to r^13, scaled by
// 2^k; SHORT: to r^10 (the remainder r^11/11! e^r <= 3.2e-13 relative).
template <bool ORDERED = true, bool SHORT = false>
__device__ inline double exp_f64(double x)
{
    const double k = rint(x * 1.44269504088896340736);
    double r = fma(-k, 6.93147180369123816490e-01, x);
    r = fma(-k, 1.90821492927058770002e-10, r);
    constexpr int JTOP = SHORT ? 10 : 13;
    double f = 1.0;
#pragma unroll
    for (int j = 2; j <= JTOP; ++j) f *= j;   // JTOP! (compile-time constant)
    double p = coef_after<ORDERED>(1.0 / f, r);
#pragma unroll
    for (int j = JTOP - 1; j >= 0; --j) {
        f /= (j + 1);                 // j! (compile-time constant after unrolling)
        p = fma(p, r, coef_after<ORDERED>(1.0 / f, p));
    }
    return ldexp(p, (int)k);
}

// erfcx(x) = exp(x^2) erfc(x) for x >= 0: t P(t), t = 3/(3 + x)
// (phi_f64_coeffs.inc: degree 21, 8.6e-16 relative; SHORT: degree 15,
// 1.5e-11 relative).
template <bool ORDERED = true, bool SHORT = false>
__device__ inline double erfcx_f64(double x)
{
    constexpr const double *P = SHORT ? QCPW_ERFCX_S : QCPW_ERFCX_P;
    constexpr int NP = SHORT ? (int)(sizeof(QCPW_ERFCX_S) / sizeof(double))
                             : (int)(sizeof(QCPW_ERFCX_P) / sizeof(double));
    const double t = QCPW_ERFCX_C * recip_f64(QCPW_ERFCX_C + x);
    double p = coef_after<ORDERED>(P[0], t);
#pragma unroll
    for (int i = 1; i < NP; ++i)
        p = fma(p, t, coef_after<ORDERED>(P[i], p));
    return t * p;
}

// erfc x for finite or infinite x: erfcx(|x|) e^{-x^2} with x^2 split into
// its rounded value and the rounding error (e^{-x^2} keeps its relative
// accuracy for large |x|), and 2 - that for x < 0.
template <bool ORDERED = true>
__device__ inline double erfc_f64(double x)
{
    const double a = fabs(x);
    const double a2 = a * a;
    if (!(a2 < 745.0)) return a2 == a2 ? (x < 0.0 ? 2.0 : 0.0) : x;   // underflow; NaN stays NaN
    const double e = exp_f64<ORDERED>(-a2) * (1.0 - fma(a, a, -a2));
    const double r = erfcx_f64<ORDERED>(a) * e;
    return x < 0.0 ? 2.0 - r : r;
}

// Phi^{-1}((y + 1/2) 2^-32) in FP64 for the raw 32-bit Sobol coordinate y.
// On the lower half (m = min(y, ~y), u = (m + 1/2) 2^-32 <= 1/2, z <= 0,
// so 1 - u is never formed) the FP32 estimate z0 (about 1e-6 relative) is
// refined by one Halley step on Phi(z) = u: with Phi(z) = e^{-z^2/2}
// erfcx(-z/sqrt 2)/2 and phi(z) = e^{-z^2/2}/sqrt(2 pi), the Newton
// correction is rho = (Phi(z0) - u)/phi(z0) = sqrt(2 pi) (erfcx(-z0/sqrt 2)/2
// - u e^{z0^2/2}) and, since Phi'' = -z phi, Halley's step is
// z0 - rho/(1 + z0 rho/2) = z0 - rho + z0 rho^2/2 + O(rho^3).  The error
// goes from about 1e-6 to below FP64 rounding (cubic convergence).
__device__ inline double ninv_f64(uint32_t y)
{
    const uint32_t m = (y >> 31) ? ~y : y;
    const double u = ((double)m + 0.5) * 0x1p-32;
    const double z0 = (double)ninv_scaled_f32(m, (float)(M_SQRT2 * 0x1p-31));   // <= 0
    const double ez = exp_f64(0.5 * z0 * z0);                                 // e^{+z0^2/2}
    const double ex = erfcx_f64(-z0 * M_SQRT1_2);
    const double rho = 2.50662827463100050242 * fma(0.5, ex, -u * ez);
    const double z = z0 - rho + 0.5 * z0 * rho * rho;
    return (y >> 31) ? -z : z;
}

// price, delta, vega, gamma of the smoothed payoff for one path (Sec. 4.5),
// from the path statistic X = S0 * Xs (Xs = A/d, the extreme E or the
// geometric mean, with A the sum of E = S~/S0) and its sigma derivative
// V_X = S0 * VXs.  All FP64.  The three Gaussian factors come from one
// exponential: with psi = (c0 - ln A)/s1 (Sec. 3.4.2), exp(-(psi - s1)^2/2)
// = exp(-psi^2/2) exp(c0 - s1^2/2) / A.  Calls pay for x_1 above psi and
// need 1 - Phi; puts pay below it and need Phi: both come from the smaller
// tail e = erfc(|a|)/2 = exp(-a^2) erfcx(|a|)/2, a = psi/sqrt 2, as e or
// 1 - e, so neither loses accuracy far from the money.  A put's price is
// the call's minus the forward of the payoff, so its Greeks are the call's
// with the X terms negated (binary: all negated).  For a basket (one-factor
// model) D1 = e^{-rT} e^{omega t1 + s1^2/2}, s1 = sigma sqrt(rho t1), and
// the vega gains vx_shift X from the sigma dependence of that factor.
// lnA = ln A (the path statistics that come as a power of two pass it in
// exactly; the others compute it).  SHORT: the shorter expansions of ln, exp
// and erfcx, for path statistics summed in FP32.
template <bool SHORT = false>
__device__ inline void path_greeks(const OptDev &op_in, double A, double lnA, double Xs, double VXs, double F[4])
{
    const OptDev &op = *reread(&op_in);
    const double psi = (op.c0 - lnA) * op.inv_s1;
    const double g0 = exp_f64<true, SHORT>(-0.5 * psi * psi);
    const double e0 = 0.5 * g0 * erfcx_f64<true, SHORT>(fabs(psi) * M_SQRT1_2);
    const bool put = qcpw_is_put(op.type);
    const double T0 = ((psi >= 0.0) != put) ? e0 : 1.0 - e0;    // call: 1 - Phi(psi); put: Phi(psi)
    // the per-option factors sDK, sD1, h2, gv, gg, gb, gd fold the products of
    // D, K, D1, h, S0, s1, sqrt(t1) and 1/sqrt(2 pi) (qcpw_internal.h)
    if (op.type == QCPW_BINARY_ASIAN_CALL || op.type == QCPW_BINARY_ASIAN_PUT) {
        const double Dphi = g0 * op.gb;                          // sgn D phi(psi)
        F[0] = op.D * T0;
        F[1] = g0 * op.gd;
        F[2] = Dphi * (VXs * recip_f64(Xs) * op.inv_s1 + psi * op.inv_sigma - op.sqrt_t1);
        F[3] = g0 * op.gg * (psi * op.inv_s1 - 1.0);
    } else {
        // the Gaussian factor at psi - s1 only where the payoff needs it
        const double psi1 = psi - op.s1;
        const double e1 = (g0 * op.h2) * recip_f64(A) * erfcx_f64<true, SHORT>(fabs(psi1) * M_SQRT1_2);
        const double T1 = ((psi1 >= 0.0) != put) ? e1 : 1.0 - e1;   // the same at psi - s1
        const double D1T1 = op.sD1 * T1;
        F[0] = fma(D1T1, op.S0 * Xs, -op.sDK * T0);
        F[1] = D1T1 * Xs;
        F[2] = fma(D1T1, op.S0 * fma(op.vx_shift, Xs, VXs), g0 * op.gv);
        F[3] = g0 * op.gg;
    }
}

template <typename R>
__device__ inline void path_tail(const OptDev &op_in, const PathSums<R> &ps, int mode, double F[4])
{
    constexpr bool SHORT = sizeof(R) == sizeof(float);   // the statistic is an FP32 sum
    const OptDev &op = *reread(&op_in);
    double A, lnA, Xs, VXs;
    if (mode == QCPW_STAT_MAX || mode == QCPW_STAT_MIN) {
        // A = 2^bY: ln A = bY ln 2 exactly (no logarithm of the rounded power)
        const double by = (double)ps.bY;
        A = exp_f64<true, SHORT>(by * 0.69314718055994530942);
        lnA = by * 0.69314718055994530942;
        Xs = A;
        VXs = A * (by - op.kappa * (double)ps.bm) * op.inv_sig_log2e;
    } else if (mode == QCPW_STAT_GEO) {
        // X/S0 = 2^{mean Y}; sum over dates of (W~ - sigma tau) = (sum Y - kappa sum m)/(sigma log2 e)
        const double sy = (double)ps.A2y;
        lnA = sy * op.invd * 0.69314718055994530942;
        A = exp_f64<true, SHORT>(lnA);
        Xs = A;
        VXs = A * (sy - op.kappa * 0.5 * (double)op.n * (double)(op.n + 1)) * op.invd * op.inv_sig_log2e;
    } else {
        A = (double)ps.A1;                      // ln d is folded into c0
        lnA = ln_f64<true, SHORT>(A);
        Xs = A * op.invd;
        VXs = ((double)ps.A2y - op.kappa * (double)ps.A2m) * op.invd * op.inv_sig_log2e;
    }
    path_greeks<SHORT>(op, A, lnA, Xs, VXs, F);
}

template <typename R>
__device__ inline void init_sums(PathSums<R> &ps)
{
    ps.A1 = R(1); ps.A2y = R(0); ps.A2m = R(0);   // date 1: S~ = S0, Y = 0
    ps.bY = R(0); ps.bm = R(0);
}

template <bool F32>
struct Real;
template <>
struct Real<true> { using T = float; };
template <>
struct Real<false> { using T = double; };

// Inverse normal of one Sobol coordinate y (raw 32 bits): FP32 from the LDS
// cubic tables as a standard normal (the caller applies the option's scale
// sigma sqrt(dt) log2(e)), FP64 already in Y units.
template <bool F32>
__device__ inline typename Real<F32>::T coord_tab(uint32_t y, const OptDev &op)
{
    if constexpr (F32) {
        return ninv_table_f32(y);
    } else {
        return ninv_f64(y) * op.zscale;
    }
}

}  // namespace qcpw
