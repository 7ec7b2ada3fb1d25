/*
 * oracle.c -- plain, slow FP64 CPU oracle for the QMC-CPW Greeks estimator
 * (Bilokon, Kucherenko, Williams, "Quasi-Monte Carlo methods for calculating
 * derivatives sensitivities on the GPU", arXiv 2209.11337).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code, header, table or constant generator with the HIP library: it builds
 * its own direction numbers from the raw Joe-Kuo (poly, m) data handed in by
 * its Python wrapper, its own digital shifts, its own inverse normal and its
 * own path factor, and it takes every step in the paper's order, one path
 * at a time, with no blocking or fusion.
 *
 * Conventions (readings of points the paper leaves open; each is listed in
 * the design notes):
 *   - d equally spaced monitoring dates t_j = j*T/d, j = 1..d; t_1 = T/d.
 *   - omega = r - sigma^2/2 (the drift in Sec. 3.4.1, eqn:Stilde1).
 *   - x_1 (the conditioned normal that drives W(t_1)) is integrated out in
 *     closed form and never drawn; Sobol dimension 0 is reserved for it.
 *     z_j (j = 1..n, n = d-1) comes from Sobol dimension j.
 *   - Brownian bridge: generic breadth-first bridge over the n grid points
 *     tau'_m = m*dt, m = 1..n, terminal point first (Sec. 4.4 generalised
 *     from 2^m steps to any n).
 *   - Lookback vega: the derivative of max_j S~(t_j) is the single term at
 *     the argmax; no 1/d factor (Sec. 4.5.3 printed formula carries a
 *     spurious 1/d, checked by finite differences).
 *   - Point k of the Sobol sequence is G * bits(gray(k)) (Gray-code order),
 *     points k = 0..N-1 including k = 0.
 *   - Uniform from a 32-bit integer y: u = (y + 1/2) * 2^-32.
 *   - Digital shift of replication l, dimension j: high 32 bits of output
 *     number (l * 2^16 + j) of SplitMix64 seeded with the option's seed.
 *   - Products beyond the paper's three (other payoffs under the same
 *     conditional template, Sec. 6.2): the geometric Asian call, and the puts
 *     of the arithmetic, binary, geometric Asian and of the fixed-strike
 *     lookback, the last on the discrete minimum.
 *   - ORC_BASKET / ORC_BASKET_PUT (products on several underlyings, Sec.
 *     6.2): M assets with the same S0 and sigma in a one-factor model,
 *     W_i = sqrt(rho) B_0 + sqrt(1 - rho) B_i, paid on the average over
 *     assets and dates; x_1 drives B_0(t_1); standard construction only, the
 *     common factor's z from dimensions 1..d-1, asset i's d increments from
 *     dimensions d + i d .. d + i d + d - 1.
 *   - ORC_PCA_FULL (the principal-component conditioning the paper names as
 *     the route to larger variance reduction, Sec. 7): W(t_1..t_d) = A z with
 *     A the d x d principal-component factor of the full covariance
 *     dt min(j, k); the first component z_1 (largest eigenvalue) is the
 *     conditioned variable, integrated out in closed form; z_2..z_d come from
 *     Sobol dimensions 1..d-1 (dimension 0 stays reserved).  Arithmetic and
 *     binary Asian calls, and the fixed-strike lookback call through the
 *     upper envelope of the log-prices' lines in the conditioned variable.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_BITS 32

enum { ORC_ARITH = 0, ORC_BINARY = 1, ORC_LOOKBACK = 2, ORC_GEOMETRIC = 3,
       ORC_ARITH_PUT = 4, ORC_BINARY_PUT = 5, ORC_LOOKBACK_PUT = 6, ORC_GEOMETRIC_PUT = 7,
       ORC_BASKET = 8, ORC_BASKET_PUT = 9 };
enum { ORC_BB = 0, ORC_PCA = 1, ORC_STANDARD = 2, ORC_PCA_FULL = 3 };
enum { ORC_RAND_SHIFT = 0, ORC_RAND_OWEN = 1 };

/* ------------------------------------------------------------------------
 * Sobol direction numbers (Sec. 2.2.2, eqn:SobolPrimitivePolynomial and
 * eqn:SobolRecurrenceRelation).
 *
 * poly[j]  : primitive polynomial x^q + c_1 x^{q-1} + ... + c_{q-1} x + 1 as
 *            a bit pattern (bit q leading term, bit 0 constant term);
 *            q = bit length - 1.  poly = 1 (q = 0) is dimension 0, whose
 *            generator matrix is the identity (van der Corput, Sec. 2.2.1).
 * minit    : [n_dims][minit_stride] initial m_1..m_q (odd, m_i < 2^i).
 * V        : [n_dims][32] output, V[j][b] = m_{b+1} * 2^(31-b), i.e. the
 *            direction number g_{b+1} = m_{b+1}/2^{b+1} as a 32-bit fraction.
 * ---------------------------------------------------------------------- */
int oracle_direction_numbers(int n_dims, const int64_t *poly,
                             const int64_t *minit, int minit_stride,
                             uint32_t *V)
{
    for (int j = 0; j < n_dims; ++j) {
        uint64_t p = (uint64_t)poly[j];
        int q = 0;
        while ((p >> (q + 1)) != 0) ++q;          /* degree */
        uint64_t m[ORC_MAX_BITS + 1];             /* m[1..32] */
        if (q == 0) {
            for (int i = 1; i <= ORC_MAX_BITS; ++i) m[i] = 1;
        } else {
            for (int i = 1; i <= q && i <= ORC_MAX_BITS; ++i) {
                m[i] = (uint64_t)minit[(size_t)j * minit_stride + (i - 1)];
                if ((m[i] & 1) == 0 || m[i] >= ((uint64_t)1 << i))
                    return -1;                    /* not a valid initial value */
            }
            /* m_i = 2 c_1 m_{i-1} ^ 4 c_2 m_{i-2} ^ ... ^ 2^{q-1} c_{q-1} m_{i-q+1}
             *       ^ 2^q m_{i-q} ^ m_{i-q}                                     */
            for (int i = q + 1; i <= ORC_MAX_BITS; ++i) {
                uint64_t v = ((uint64_t)1 << q) * m[i - q] ^ m[i - q];
                for (int k = 1; k <= q - 1; ++k) {
                    uint64_t c_k = (p >> (q - k)) & 1;
                    if (c_k) v ^= ((uint64_t)1 << k) * m[i - k];
                }
                m[i] = v;
            }
        }
        for (int b = 0; b < ORC_MAX_BITS; ++b)
            V[(size_t)j * 32 + b] = (uint32_t)(m[b + 1] << (31 - b));
    }
    return 0;
}

/* Point k, dimension j, of the unshifted sequence: the XOR of the direction
 * numbers selected by the binary digits of gray(k) = k ^ (k >> 1)
 * (eqn:GeneratorMatrixExpression and its XOR form). */
static uint32_t sobol_int(const uint32_t *Vj, uint64_t k)
{
    uint64_t g = k ^ (k >> 1);
    uint32_t y = 0;
    for (int b = 0; b < ORC_MAX_BITS; ++b)
        if ((g >> b) & 1) y ^= Vj[b];
    return y;
}

void oracle_sobol_points(const uint32_t *V, int n_dims, int64_t k0,
                         int64_t count, uint32_t *out /* [count][n_dims] */)
{
    for (int64_t i = 0; i < count; ++i)
        for (int j = 0; j < n_dims; ++j)
            out[i * n_dims + j] = sobol_int(V + (size_t)j * 32, (uint64_t)(k0 + i));
}

/* ------------------------------------------------------------------------
 * SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014): state advances by the golden-ratio gamma, each
 * output is the state passed through the variant-13 mixer.  Output number i
 * (0-based) of a generator seeded with s is mix(s + (i+1)*gamma).
 * ---------------------------------------------------------------------- */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Random digital shift of replication l in dimension j (Sec. 2.2.3: a
 * randomisation of the point set so that independent replications give an
 * error estimate). */
uint32_t oracle_shift(uint64_t seed, int l, int j)
{
    return (uint32_t)(oracle_splitmix64(seed, ((uint64_t)l << 16) + (uint64_t)j) >> 32);
}

/* ------------------------------------------------------------------------
 * Nested (Owen) scrambling of one coordinate in base 2 (Sec. 2.2.3): digit
 * k of the binary expansion (k = 1 the most significant) is flipped or not
 * by a random function of digits 1..k-1 only, so every subinterval of every
 * level is swapped independently.  On the bit-reversed value v (digit k ->
 * bit k-1) "flip bit i by a function of the bits below i" is what adding a
 * seed does (the carry) and what v ^= ((v mod 2^24) * C) does for an even
 * constant C (the product's bit i sees only bits below i); four such rounds
 * with fixed constants follow the seeded addition (the Laine-Karras style of
 * hash-based nested scrambling).  Each step is a bijection that maps a
 * uniform v to a uniform v, so each scrambled point is uniform for a random
 * seed, and scrambled nets stay nets.
 * ---------------------------------------------------------------------- */
static uint32_t reverse32(uint32_t x)
{
    uint32_t r = 0;
    for (int b = 0; b < 32; ++b) r |= ((x >> b) & 1u) << (31 - b);
    return r;
}

uint32_t oracle_owen(uint32_t y, uint32_t seed32)
{
    static const uint32_t C[4] = {0xcca0d0u, 0x6292a6u, 0xb21bbau, 0x70b6f2u};
    uint32_t v = reverse32(y) + seed32;
    for (int i = 0; i < 4; ++i) v ^= (v & 0xFFFFFFu) * C[i];
    return reverse32(v);
}

/* ------------------------------------------------------------------------
 * Inverse standard normal: Wichura, "Algorithm AS 241: The percentage
 * points of the normal distribution", Applied Statistics 37 (1988),
 * PPND16 (about 1e-16 relative accuracy).
 * ---------------------------------------------------------------------- */
double oracle_norm_inv(double p)
{
    double q = p - 0.5, r, x;
    if (fabs(q) <= 0.425) {
        r = 0.180625 - q * q;
        x = q * (((((((2.5090809287301226727e+3 * r + 3.3430575583588128105e+4) * r
                    + 6.7265770927008700853e+4) * r + 4.5921953931549871457e+4) * r
                    + 1.3731693765509461125e+4) * r + 1.9715909503065514427e+3) * r
                    + 1.3314166789178437745e+2) * r + 3.3871328727963666080e+0)
              / (((((((5.2264952788528545610e+3 * r + 2.8729085735721942674e+4) * r
                    + 3.9307895800092710610e+4) * r + 2.1213794301586595867e+4) * r
                    + 5.3941960214247511077e+3) * r + 6.8718700749205790830e+2) * r
                    + 4.2313330701600911252e+1) * r + 1.0);
        return x;
    }
    r = (q < 0.0) ? p : 1.0 - p;
    r = sqrt(-log(r));
    if (r <= 5.0) {
        r -= 1.6;
        x = (((((((7.74545014278341407640e-4 * r + 2.27238449892691845833e-2) * r
                 + 2.41780725177450611770e-1) * r + 1.27045825245236838258e+0) * r
                 + 3.64784832476320460504e+0) * r + 5.76949722146069140550e+0) * r
                 + 4.63033784615654529590e+0) * r + 1.42343711074968357734e+0)
            / (((((((1.05075007164441684324e-9 * r + 5.47593808499534494600e-4) * r
                 + 1.51986665636164571966e-2) * r + 1.48103976427480074590e-1) * r
                 + 6.89767334985100004550e-1) * r + 1.67638483018380384940e+0) * r
                 + 2.05319162663775882187e+0) * r + 1.0);
    } else {
        r -= 5.0;
        x = (((((((2.01033439929228813265e-7 * r + 2.71155556874348757815e-5) * r
                 + 1.24266094738807843860e-3) * r + 2.65321895265761230930e-2) * r
                 + 2.96560571828504891230e-1) * r + 1.78482653991729133580e+0) * r
                 + 5.46378491116411436990e+0) * r + 6.65790464350110377720e+0)
            / (((((((2.04426310338993978564e-15 * r + 1.42151175831644588870e-7) * r
                 + 1.84631831751005468180e-5) * r + 7.86869131145613259100e-4) * r
                 + 1.48753612908506148525e-2) * r + 1.36929880922735805310e-1) * r
                 + 5.99832206555887937690e-1) * r + 1.0);
    }
    return (q < 0.0) ? -x : x;
}

/* Standard normal cdf and density (library erfc/exp as primitives). */
double oracle_norm_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }
double oracle_norm_pdf(double x) { return exp(-0.5 * x * x) / sqrt(2.0 * M_PI); }

/* ------------------------------------------------------------------------
 * Path construction: W~ = A z  (Sec. 3.4.1, eqn:WboldTilde), the Brownian
 * motion W~(tau) = W(t_1 + tau) - W(t_1) at tau'_m = m*dt, m = 1..n.
 * W[0] = 0 is W~ at tau = 0 (date t_1).  W must hold n+1 values.
 * ---------------------------------------------------------------------- */

/* Standard construction (Alg. 3): left-to-right increments sqrt(dt)*z. */
static void build_standard(int n, double dt, const double *z, double *W)
{
    W[0] = 0.0;
    for (int m = 1; m <= n; ++m) W[m] = W[m - 1] + sqrt(dt) * z[m - 1];
}

/* Brownian bridge (Sec. 4.4): terminal value first from the first normal,
 * then the midpoint of every interval taken breadth first, each drawn from
 * its conditional law given the two ends.  z[0] -> W[n]; later normals go to
 * midpoints in queue order. */
static void build_bridge(int n, double dt, const double *z, double *W)
{
    W[0] = 0.0;
    if (n == 0) return;
    W[n] = sqrt(n * dt) * z[0];
    /* every split pushes two intervals: at most 2n - 1 entries ever queued */
    int *ql = (int *)malloc(sizeof(int) * (size_t)(2 * n + 1));
    int *qr = (int *)malloc(sizeof(int) * (size_t)(2 * n + 1));
    int head = 0, tail = 0, next = 1;
    ql[tail] = 0; qr[tail] = n; ++tail;
    while (head < tail) {
        int l = ql[head], r = qr[head]; ++head;
        if (r - l < 2) continue;
        int m = (l + r) / 2;
        double mean = ((double)(r - m) * W[l] + (double)(m - l) * W[r]) / (double)(r - l);
        double var = dt * (double)(m - l) * (double)(r - m) / (double)(r - l);
        W[m] = mean + sqrt(var) * z[next++];
        ql[tail] = l; qr[tail] = m; ++tail;
        ql[tail] = m; qr[tail] = r; ++tail;
    }
    free(ql); free(qr);
}

/* Principal-component factor of Sigma_{kl} = dt * min(k, l), k, l = 1..n
 * (Sec. 3.4.1 asks for any A with A A^T = Sigma; the principal components
 * are the choice that concentrates variance in the leading coordinates).
 * The eigenpairs of this matrix are known in closed form:
 *   lambda_i = dt / (4 sin^2((2i-1) pi / (2(2n+1)))),
 *   v_i(k)   = 2/sqrt(2n+1) * sin((2i-1) k pi / (2n+1)),
 * i = 1..n in decreasing lambda; every v_i(1) > 0 fixes the signs.
 * A_{k,i} = sqrt(lambda_i) v_i(k), row-major n x n.  The integer product
 * (2i-1)k is reduced modulo 2(2n+1) before scaling by pi so the sine's
 * argument stays below 2 pi and carries no large rounding error. */
void oracle_pca_factor(int n, double dt, double *A)
{
    long M = 2L * (2 * n + 1);
    for (int i = 1; i <= n; ++i) {
        double s = sin((2 * i - 1) * M_PI / (double)M);
        double sq_lam = sqrt(dt / (4.0 * s * s));
        for (int k = 1; k <= n; ++k) {
            long a = ((long)(2 * i - 1) * k) % M;
            double v = 2.0 / sqrt(2.0 * n + 1.0) * sin((double)a * M_PI / (double)(2 * n + 1));
            A[(size_t)(k - 1) * n + (i - 1)] = sq_lam * v;
        }
    }
}

/* Dense factor (principal components): W[1..n] = A z, A row-major n x n. */
static void build_dense(int n, const double *A, const double *z, double *W)
{
    W[0] = 0.0;
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += A[(size_t)k * n + i] * z[i];
        W[k + 1] = s;
    }
}

int oracle_build_path(int path, int n, double dt, const double *z,
                      const double *A, double *W)
{
    switch (path) {
    case ORC_BB: build_bridge(n, dt, z, W); return 0;
    case ORC_STANDARD: build_standard(n, dt, z, W); return 0;
    case ORC_PCA: if (!A) return -1; build_dense(n, A, z, W); return 0;
    default: return -1;
    }
}

/* ------------------------------------------------------------------------
 * Conditional payoff G and its pathwise derivatives for one path
 * (Sec. 3.4.2 and Sec. 4.5).  Given W~ at the d dates, returns
 * out = {price, delta, vega, gamma} of the smoothed payoff G(theta, z).
 * ---------------------------------------------------------------------- */
void oracle_path_greeks(int type, int d, double S0, double K, double r,
                        double sigma, double T, const double *W, double *out)
{
    double dt = T / d;
    double t1 = dt;
    double omega = r - 0.5 * sigma * sigma;
    double s1 = sigma * sqrt(t1);
    double D = exp(-r * T);
    double D1 = exp(r * (t1 - T));

    /* S~(t_j) = S0 exp(omega (t_j - t_1) + sigma W~(t_j - t_1))  (eqn:Stilde1) */
    double X = 0.0, VX = 0.0;
    if (type == ORC_LOOKBACK || type == ORC_LOOKBACK_PUT) {
        /* fixed-strike lookback: the call is on the discrete maximum, the put
         * on the discrete minimum; either extreme carries the common factor of x_1 */
        int jstar = 0;
        double best = 0.0;
        for (int m = 0; m < d; ++m) {
            double tau = m * dt;
            double St = S0 * exp(omega * tau + sigma * W[m]);
            int better = type == ORC_LOOKBACK ? St > best : St < best;
            if (m == 0 || better) { best = St; jstar = m; }   /* lowest index wins ties */
        }
        X = best;
        /* d S~extreme / d sigma = S~(t_j*) (W~ - sigma tau) at the arg-extreme */
        VX = best * (W[jstar] - sigma * jstar * dt);
    } else if (type == ORC_GEOMETRIC || type == ORC_GEOMETRIC_PUT) {
        /* geometric average: X = (prod_j S~(t_j))^{1/d} = S0 exp(mean_j (omega tau_j + sigma W~_j));
         * like the arithmetic average it carries the common factor of x_1, so
         * the same conditional payoff applies (Sec. 4.5 with another average) */
        double lsum = 0.0, vsum = 0.0;
        for (int m = 0; m < d; ++m) {
            double tau = m * dt;
            lsum += omega * tau + sigma * W[m];
            vsum += W[m] - sigma * tau;
        }
        X = S0 * exp(lsum / d);
        VX = X * vsum / d;
    } else {
        for (int m = 0; m < d; ++m) {
            double tau = m * dt;
            double St = S0 * exp(omega * tau + sigma * W[m]);
            X += St;
            VX += St * (W[m] - sigma * tau);
        }
        X /= d;
        VX /= d;
    }

    /* Breakpoint of the conditioned normal x_1: S(x_1) = X exp(omega t1 + s1 x1)
     * crosses K at psi (Sec. 3.4.2, psi_d). */
    double psi = (log(K) - log(X) - omega * t1) / s1;
    double Q0 = oracle_norm_cdf(-psi);          /* 1 - Phi(psi) */
    double Q1 = oracle_norm_cdf(s1 - psi);      /* 1 - Phi(psi - s1) */
    double phi0 = oracle_norm_pdf(psi);

    if (type == ORC_BINARY) {
        /* G = e^{-rT}[1 - Phi(psi)]  (eqn:GAnalyticalSolution, Sec. 4.5.1) */
        out[0] = D * Q0;
        out[1] = D * phi0 / (S0 * s1);
        out[2] = D * phi0 * (VX / (s1 * X) + psi / sigma - sqrt(t1));
        out[3] = D * phi0 / (S0 * S0 * s1) * (psi / s1 - 1.0);
    } else if (type == ORC_BINARY_PUT) {
        /* pays e^{-rT} when the average ends below K, i.e. x_1 < psi:
         * G = e^{-rT} Phi(psi); d psi/d S0 = -1/(S0 s1) */
        double P0 = oracle_norm_cdf(psi);
        out[0] = D * P0;
        out[1] = -D * phi0 / (S0 * s1);
        out[2] = -D * phi0 * (VX / (s1 * X) + psi / sigma - sqrt(t1));
        out[3] = -D * phi0 / (S0 * S0 * s1) * (psi / s1 - 1.0);
    } else if (type == ORC_ARITH_PUT || type == ORC_LOOKBACK_PUT || type == ORC_GEOMETRIC_PUT) {
        /* (K - X e^{omega t1 + s1 x1})^+ is positive for x1 < psi:
         * G = e^{-rT} K Phi(psi) - e^{r(t1-T)} X Phi(psi - s1); in the
         * derivatives the psi terms cancel at the breakpoint, as for the call */
        double P0 = oracle_norm_cdf(psi);
        double P1 = oracle_norm_cdf(psi - s1);
        out[0] = D * K * P0 - D1 * X * P1;
        out[1] = -D1 * (X / S0) * P1;
        out[2] = -D1 * P1 * VX + D * K * phi0 * sqrt(t1);
        out[3] = D * K * phi0 / (S0 * S0 * s1);
    } else {
        /* G = e^{r(t1-T)} X [1 - Phi(psi - s1)] - e^{-rT} K [1 - Phi(psi)]
         * (Sec. 4.5.2 arithmetic Asian, Sec. 4.5.3 lookback on the max; the
         * geometric average enters the same way) */
        out[0] = D1 * X * Q1 - D * K * Q0;
        out[1] = D1 * (X / S0) * Q1;
        out[2] = D1 * Q1 * VX + D * K * phi0 * sqrt(t1);
        out[3] = D * K * phi0 / (S0 * S0 * s1);
    }
}

/* ------------------------------------------------------------------------
 * Principal-component conditioning on the first component of the full
 * covariance (ORC_PCA_FULL).  With W(t_j) = a_j x + c_j, a_j = A_{j,1} > 0,
 * c_j = sum_{i>=2} A_{j,i} z_i, every log-price is affine in the
 * conditioned normal x:
 *     ln S(t_j) = alpha_j + beta_j x,  alpha_j = ln S0 + omega t_j + sigma c_j,
 *                                      beta_j = sigma a_j.
 * The average A(x) = (1/d) sum_j exp(alpha_j + beta_j x) is increasing and
 * convex in x, so A(x) = K has exactly one root psi; it is found by Newton's
 * method safeguarded by a bracket [lo, hi] (bisection whenever a Newton
 * step leaves it).  Then, with D = e^{-rT} and x ~ N(0, 1):
 *   arithmetic:  G = D [ (1/d) sum_j E_j Phi(beta_j - psi) - K Phi(-psi) ],
 *                E_j = exp(alpha_j + beta_j^2 / 2);
 *   binary:      G = D Phi(-psi).
 * The derivatives follow by the chain rule through alpha_j, beta_j and psi
 * (d alpha_j/d S0 = 1/S0, d alpha_j/d sigma = c_j - sigma t_j,
 * d beta_j/d sigma = a_j, d psi = -dF/F' with F(x) = A(x) - K); for the
 * arithmetic payoff the terms in d psi cancel at the root.
 * ---------------------------------------------------------------------- */
static double full_F(int d, const double *al, const double *be, double x, double K,
                     double *Fp)
{
    double s = 0.0, s1 = 0.0;
    for (int j = 0; j < d; ++j) {
        double g = exp(al[j] + be[j] * x);
        s += g;
        s1 += be[j] * g;
    }
    *Fp = s1 / d;
    return s / d - K;
}

double oracle_full_root(int d, const double *al, const double *be, double K)
{
    /* hi: by Jensen, A(x) >= exp(mean(alpha) + mean(beta) x), which equals K at
     * x = (ln K - mean alpha) / mean beta, so F(hi) >= 0 there */
    double ma = 0.0, mb = 0.0, Fp;
    for (int j = 0; j < d; ++j) { ma += al[j]; mb += be[j]; }
    ma /= d; mb /= d;
    double hi = (log(K) - ma) / mb;
    double lo = hi - 1.0;
    for (int i = 0; i < 200 && full_F(d, al, be, lo, K, &Fp) >= 0.0; ++i) lo -= (hi - lo);
    double x = hi;
    for (int it = 0; it < 200; ++it) {
        double F = full_F(d, al, be, x, K, &Fp);
        if (F == 0.0) return x;
        if (F > 0.0) hi = x; else lo = x;
        double xn = x - F / Fp;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);     /* safeguard */
        if (fabs(xn - x) <= 1e-15 * (1.0 + fabs(x)) || hi - lo <= 1e-15 * (1.0 + fabs(x))) return xn;
        x = xn;
    }
    return x;
}

/* ------------------------------------------------------------------------
 * Lookback (fixed-strike call on the discrete maximum) under the same
 * conditioning.  Every beta_j > 0, so M(x) = max_j (alpha_j + beta_j x), the
 * upper envelope of d increasing lines, is increasing, convex and piecewise
 * linear, and the payoff (e^{M(x)} - K)^+ is positive exactly for x > psi:
 *   psi = min_j (ln K - alpha_j) / beta_j
 * (M(x) <= ln K iff every line is, iff x <= each line's own crossing).
 * On [psi, inf) the envelope is a chain of segments [x_s, x_{s+1}) with one
 * line j_s on top; starting from the line that meets ln K at psi (the
 * steeper one on a tie), the next line is the steeper one that overtakes
 * the current line first.  Over a segment [a, b) of line j, with
 * E_j = exp(alpha_j + beta_j^2 / 2) and e^{alpha + beta x} phi(x) =
 * E phi(x - beta):
 *   int (e^{alpha_j + beta_j x} - K) phi = E_j dP_j - K (Phi(b) - Phi(a)),
 *        dP_j = Phi(b - beta_j) - Phi(a - beta_j)
 * (each difference of Phi taken as the probability of the interval, from
 * the upper tail right of 0);
 *   int e^{alpha_j + beta_j x} (alpha_j' + beta_j' x) phi
 *        = E_j [alpha_j' dP_j + beta_j' (beta_j dP_j + phi(a - beta_j) - phi(b - beta_j))].
 * The integrand is continuous across breakpoints and zero at psi, so the
 * derivatives of the price are the integrals of the payoff's derivatives:
 *   G     = D sum_s [E_j dP_j - K (Phi(b) - Phi(a))],
 *   delta = D sum_s E_j dP_j / S0                (d alpha_j / d S0 = 1/S0),
 *   vega  = D sum_s E_j [alpha_j' dP_j + a_j (beta_j dP_j + phi(a - beta_j) - phi(b - beta_j))],
 *           alpha_j' = c_j - sigma t_j, beta_j' = a_j,
 *   gamma = D K phi(psi) / (S0^2 beta*),  beta* the slope on top at psi
 *           (the only S0-dependence left in delta is the lower end psi,
 *           d psi / d S0 = -1 / (S0 beta*), and E* phi(psi - beta*) = K phi(psi)).
 * ---------------------------------------------------------------------- */
/* P(lo < X < hi) for X ~ N(0, 1), lo <= hi (hi may be +inf), from the
 * upper tail when the interval lies right of 0 so that it keeps its
 * relative accuracy far out. */
static double norm_interval(double lo, double hi)
{
    if (lo >= 0.0) return 0.5 * erfc(lo / sqrt(2.0)) - (isinf(hi) ? 0.0 : 0.5 * erfc(hi / sqrt(2.0)));
    return (isinf(hi) ? 1.0 : oracle_norm_cdf(hi)) - oracle_norm_cdf(lo);
}

static void full_lookback(int d, const double *al, const double *be, const double *a, const double *c,
                          double S0, double K, double sigma, double dt, double D, double *out)
{
    const double lnK = log(K);
    int j = 0;
    double psi = (lnK - al[0]) / be[0];
    for (int i = 1; i < d; ++i) {
        const double xi = (lnK - al[i]) / be[i];
        if (xi < psi || (xi == psi && be[i] > be[j])) { psi = xi; j = i; }
    }
    const double bstar = be[j];
    double G = 0.0, dl = 0.0, vg = 0.0;
    double x0 = psi;
    for (;;) {
        /* the steeper line that overtakes line j first, if any */
        int nx = -1;
        double x1 = INFINITY;
        for (int i = 0; i < d; ++i) {
            if (!(be[i] > be[j])) continue;
            const double xi = (al[j] - al[i]) / (be[i] - be[j]);
            if (xi < x1 || (xi == x1 && nx >= 0 && be[i] > be[nx])) { x1 = xi; nx = i; }
        }
        if (x1 < x0) x1 = x0;   /* rounding: a line crossing at x0 itself */
        const double E = exp(al[j] + 0.5 * be[j] * be[j]);
        const double fb = isinf(x1) ? 0.0 : oracle_norm_pdf(x1 - be[j]);
        const double fa = oracle_norm_pdf(x0 - be[j]);
        const double dP = norm_interval(x0 - be[j], x1 - be[j]);
        const double t = (j + 1) * dt;
        G += E * dP - K * norm_interval(x0, x1);
        dl += E * dP;
        vg += E * ((c[j] - sigma * t) * dP + a[j] * (be[j] * dP + fa - fb));
        if (nx < 0) break;
        j = nx;
        x0 = x1;
    }
    out[0] = D * G;
    out[1] = D * dl / S0;
    out[2] = D * vg;
    out[3] = D * K * oracle_norm_pdf(psi) / (S0 * S0 * bstar);
}

int oracle_path_greeks_full(int type, int d, double S0, double K, double r,
                            double sigma, double T, const double *a, const double *c,
                            double *out)
{
    if (type != ORC_ARITH && type != ORC_BINARY && type != ORC_LOOKBACK) return -1;
    double dt = T / d;
    double omega = r - 0.5 * sigma * sigma;
    double D = exp(-r * T);
    double *al = (double *)malloc(sizeof(double) * (size_t)d);
    double *be = (double *)malloc(sizeof(double) * (size_t)d);
    for (int j = 0; j < d; ++j) {
        double t = (j + 1) * dt;
        al[j] = log(S0) + omega * t + sigma * c[j];
        be[j] = sigma * a[j];
    }
    if (type == ORC_LOOKBACK) {
        full_lookback(d, al, be, a, c, S0, K, sigma, dt, D, out);
        free(al); free(be);
        return 0;
    }
    double psi = oracle_full_root(d, al, be, K);
    double phi0 = oracle_norm_pdf(psi);
    /* F'(psi), F''(psi), dF/dsigma at psi */
    double F1 = 0.0, F2 = 0.0, Fs = 0.0;
    double sEP = 0.0, sV = 0.0, sAg = 0.0;
    for (int j = 0; j < d; ++j) {
        double t = (j + 1) * dt;
        double g = exp(al[j] + be[j] * psi);
        double das = c[j] - sigma * t;                 /* d alpha_j / d sigma */
        F1 += be[j] * g;
        F2 += be[j] * be[j] * g;
        Fs += g * (das + psi * a[j]);
        double E = exp(al[j] + 0.5 * be[j] * be[j]);
        double P = oracle_norm_cdf(be[j] - psi);
        sEP += E * P;
        sV += E * P * (das + be[j] * a[j]);
        sAg += a[j] * g;
    }
    F1 /= d; F2 /= d; Fs /= d; sEP /= d; sV /= d; sAg /= d;
    if (type == ORC_ARITH) {
        out[0] = D * (sEP - K * oracle_norm_cdf(-psi));
        out[1] = D * sEP / S0;
        /* sum_j E_j phi(beta_j - psi) a_j = phi(psi) sum_j a_j exp(alpha_j + beta_j psi) */
        out[2] = D * (sV + phi0 * sAg);
        out[3] = D * phi0 * K * K / (S0 * S0 * F1);
    } else {
        double psiS = -(K / S0) / F1;                  /* d psi / d S0 */
        out[0] = D * oracle_norm_cdf(-psi);
        out[1] = -D * phi0 * psiS;
        out[2] = D * phi0 * Fs / F1;
        out[3] = D * K * phi0 / (S0 * F1) * (-psi * psiS - 2.0 / S0 - F2 * psiS / F1);
    }
    free(al); free(be);
    return 0;
}

/* ------------------------------------------------------------------------
 * Basket of M assets in a one-factor model (products on several
 * underlyings, Sec. 6.2): S_i(t) = S0 exp(omega t + sigma W_i(t)) with
 * W_i = sqrt(rho) B_0 + sqrt(1 - rho) B_i (independent Brownian motions; every
 * pair of assets has correlation rho), paid on X = (1/(M d)) sum_i sum_j
 * S_i(t_j).  Conditioning on x_1 = B_0(t_1)/sqrt(t_1) (Sec. 3.4.2): every
 * S_i(t_j) carries exp(sigma sqrt(rho) sqrt(t_1) x_1), so
 * X = Xt exp(omega t_1 + s1 x_1) with s1 = sigma sqrt(rho t_1) and
 *   Xt = (1/(M d)) sum S0 exp(omega tau_j + sigma (sqrt(rho) B~_0(tau_j)
 *        + sqrt(1 - rho) B_i(t_j))),   tau_j = t_j - t_1,
 * and the breakpoint psi = (ln K - ln Xt - omega t_1)/s1 is closed form.
 * With a = omega t_1, E[e^{a + s1 x}; x > psi] = e^{a + s1^2/2} Phi(s1 - psi),
 * so the call is e^{-rT} [Xt e^{a + s1^2/2} Phi(s1 - psi) - K Phi(-psi)];
 * a + s1^2/2 = r t_1 - (1 - rho) sigma^2 t_1 / 2 depends on sigma unless
 * rho = 1, which adds Xt d(a + s1^2/2)/d sigma to the pathwise sigma
 * derivative of Xt in the vega, and ds1/dsigma = sqrt(rho t_1).
 *
 * W0[m], m = 0..d-1 : B~_0(tau_m) (W0[0] = 0)
 * Bi[i*d + m]       : B_i(t_{m+1})
 * ---------------------------------------------------------------------- */
void oracle_basket_path_greeks(int type, int d, int M, double rho, double S0, double K, double r,
                               double sigma, double T, const double *W0, const double *Bi, double *out)
{
    double dt = T / d;
    double t1 = dt;
    double omega = r - 0.5 * sigma * sigma;
    double s1 = sigma * sqrt(rho * t1);
    double a = omega * t1;
    double D = exp(-r * T);
    double sr = sqrt(rho), sq = sqrt(1.0 - rho);
    double X = 0.0, VX = 0.0;
    for (int i = 0; i < M; ++i)
        for (int m = 0; m < d; ++m) {
            double tau = m * dt;
            double e = sr * W0[m] + sq * Bi[(size_t)i * d + m];
            double St = S0 * exp(omega * tau + sigma * e);
            X += St;
            VX += St * (e - sigma * tau);   /* d/dsigma of omega tau + sigma e */
        }
    X /= (double)M * d;
    VX /= (double)M * d;
    double Df = D * exp(a + 0.5 * s1 * s1);
    double dF = -sigma * (1.0 - rho) * t1;   /* d(a + s1^2/2)/d sigma */
    double psi = (log(K) - log(X) - a) / s1;
    double phi0 = oracle_norm_pdf(psi);
    double vs = VX + X * dF;
    if (type == ORC_BASKET) {
        double Q0 = oracle_norm_cdf(-psi), Q1 = oracle_norm_cdf(s1 - psi);
        out[0] = Df * X * Q1 - D * K * Q0;
        out[1] = Df * (X / S0) * Q1;
        out[2] = Df * Q1 * vs + D * K * phi0 * sqrt(rho * t1);
    } else {
        /* put: pays for x_1 < psi */
        double P0 = oracle_norm_cdf(psi), P1 = oracle_norm_cdf(psi - s1);
        out[0] = D * K * P0 - Df * X * P1;
        out[1] = -Df * (X / S0) * P1;
        out[2] = -Df * P1 * vs + D * K * phi0 * sqrt(rho * t1);
    }
    out[3] = D * K * phi0 / (S0 * S0 * s1);
}

/* Neumaier's compensated summation. */
typedef struct { double s, c; } orc_sum;
static void sum_add(orc_sum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double sum_val(const orc_sum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------------
 * One option, all replications (Sec. 5): for replication l the estimate
 * C_l = (1/N) sum_k F(theta, z_{l,k}) over the N shifted Sobol points;
 * C = (1/L) sum_l C_l; stderr = sqrt(sum_l (C_l - C)^2 / (L (L-1))).
 *
 * V        : [>= d][32] direction numbers
 * A        : n x n dense factor for ORC_PCA (row-major), else ignored
 * C_l      : [L][4] per-replication estimates (may be NULL)
 * mean     : [4], stderr: [4], abs_mean: [4] = (1/(N L)) sum |F| (the scale
 *            of the summands, used for scale-aware comparisons)
 * ---------------------------------------------------------------------- */
/* Replication l of one option: C_l[4] = (1/N) sum_k F(theta, z_{l,k}) over
 * points k = k0 .. k0 + N - 1, and abs_sum[4] += sum_k |F| (may be NULL). */
int oracle_replication(int type, int d, double S0, double K, double r, double sigma,
                       double T, uint64_t seed, int64_t k0, int64_t N, int l, int path,
                       int rand, const uint32_t *V, const double *A, double *C_l, double *abs_sum)
{
    if (d < 1 || N < 1 || k0 < 0) return -1;
    if (path == ORC_PCA_FULL && (!A || (type != ORC_ARITH && type != ORC_BINARY && type != ORC_LOOKBACK))) return -1;
    int n = d - 1;
    double dt = T / d;
    double *z = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *W = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *a1 = (double *)malloc(sizeof(double) * (size_t)d);
    if (path == ORC_PCA_FULL)   /* first column of the d x d factor */
        for (int j = 0; j < d; ++j) a1[j] = A[(size_t)j * d];
    orc_sum acc[4], ab[4];
    memset(acc, 0, sizeof acc);
    memset(ab, 0, sizeof ab);
    for (int64_t k = k0; k < k0 + N; ++k) {
        for (int j = 1; j <= n; ++j) {
            uint32_t y = sobol_int(V + (size_t)j * 32, (uint64_t)k);
            /* randomisation: digital shift (XOR) or nested scrambling, both
             * keyed by the same per-(replication, dimension) 32-bit value */
            y = rand == ORC_RAND_OWEN ? oracle_owen(y, oracle_shift(seed, l, j)) : (y ^ oracle_shift(seed, l, j));
            double u = ((double)y + 0.5) / 4294967296.0;
            z[j - 1] = oracle_norm_inv(u);
        }
        double F[4];
        if (path == ORC_PCA_FULL) {
            /* c_j = sum over components 2..d of A_{j,i} z_i */
            for (int j = 0; j < d; ++j) {
                double cj = 0.0;
                for (int i = 1; i < d; ++i) cj += A[(size_t)j * d + i] * z[i - 1];
                W[j] = cj;
            }
            oracle_path_greeks_full(type, d, S0, K, r, sigma, T, a1, W, F);
        } else {
            oracle_build_path(path, n, dt, z, A, W);
            oracle_path_greeks(type, d, S0, K, r, sigma, T, W, F);
        }
        for (int o = 0; o < 4; ++o) {
            sum_add(&acc[o], F[o]);
            sum_add(&ab[o], fabs(F[o]));
        }
    }
    for (int o = 0; o < 4; ++o) {
        C_l[o] = sum_val(&acc[o]) / (double)N;
        if (abs_sum) abs_sum[o] += sum_val(&ab[o]);
    }
    free(z); free(W); free(a1);
    return 0;
}

/* Replication l of a basket option (standard construction for every
 * Brownian motion): C_l[4] over points k0 .. k0 + N - 1, abs_sum[4] += sum |F|. */
int oracle_basket_replication(int type, int d, int M, double rho, double S0, double K, double r,
                              double sigma, double T, uint64_t seed, int64_t k0, int64_t N, int l,
                              int rand, const uint32_t *V, double *C_l, double *abs_sum)
{
    if (d < 1 || M < 1 || N < 1 || k0 < 0 || !(rho > 0.0 && rho <= 1.0)) return -1;
    if (type != ORC_BASKET && type != ORC_BASKET_PUT) return -1;
    int n = d - 1, dims = n + M * d;
    double dt = T / d, sdt = sqrt(dt);
    double *z = (double *)malloc(sizeof(double) * (size_t)(dims + 1));
    double *W0 = (double *)malloc(sizeof(double) * (size_t)d);
    double *Bi = (double *)malloc(sizeof(double) * (size_t)M * d);
    orc_sum acc[4], ab[4];
    memset(acc, 0, sizeof acc);
    memset(ab, 0, sizeof ab);
    for (int64_t k = k0; k < k0 + N; ++k) {
        for (int j = 1; j <= dims; ++j) {
            uint32_t y = sobol_int(V + (size_t)j * 32, (uint64_t)k);
            y = rand == ORC_RAND_OWEN ? oracle_owen(y, oracle_shift(seed, l, j)) : (y ^ oracle_shift(seed, l, j));
            z[j - 1] = oracle_norm_inv(((double)y + 0.5) / 4294967296.0);
        }
        /* common factor after x_1: B~_0(tau_m) = sqrt(dt) (z_1 + ... + z_m) */
        W0[0] = 0.0;
        for (int m = 1; m < d; ++m) W0[m] = W0[m - 1] + sdt * z[m - 1];
        /* asset i: B_i(t_{m+1}) = sqrt(dt) (sum of its first m + 1 increments) */
        for (int i = 0; i < M; ++i) {
            double b = 0.0;
            for (int m = 0; m < d; ++m) {
                b += sdt * z[n + i * d + m];
                Bi[(size_t)i * d + m] = b;
            }
        }
        double F[4];
        oracle_basket_path_greeks(type, d, M, rho, S0, K, r, sigma, T, W0, Bi, F);
        for (int o = 0; o < 4; ++o) {
            sum_add(&acc[o], F[o]);
            sum_add(&ab[o], fabs(F[o]));
        }
    }
    for (int o = 0; o < 4; ++o) {
        C_l[o] = sum_val(&acc[o]) / (double)N;
        if (abs_sum) abs_sum[o] += sum_val(&ab[o]);
    }
    free(z); free(W0); free(Bi);
    return 0;
}

/* All replications of a basket option: mean, stderr, abs_mean as oracle_option. */
int oracle_basket_option(int type, int d, int M, double rho, double S0, double K, double r,
                         double sigma, double T, uint64_t seed, int64_t N, int L, int rand,
                         const uint32_t *V, double *C_l, double *mean, double *stderr_, double *abs_mean)
{
    if (L < 1) return -1;
    double *Cl = (double *)malloc(sizeof(double) * (size_t)L * 4);
    double absum[4] = {0, 0, 0, 0};
    for (int l = 0; l < L; ++l)
        if (oracle_basket_replication(type, d, M, rho, S0, K, r, sigma, T, seed, 0, N, l, rand, V,
                                      Cl + 4 * l, absum) != 0) {
            free(Cl);
            return -1;
        }
    for (int o = 0; o < 4; ++o) {
        orc_sum s = {0, 0};
        for (int l = 0; l < L; ++l) sum_add(&s, Cl[l * 4 + o]);
        double C = sum_val(&s) / L;
        double ss = 0.0;
        for (int l = 0; l < L; ++l) ss += (Cl[l * 4 + o] - C) * (Cl[l * 4 + o] - C);
        mean[o] = C;
        stderr_[o] = (L >= 2) ? sqrt(ss / ((double)L * (L - 1))) : NAN;
        if (abs_mean) abs_mean[o] = absum[o] / ((double)N * L);
    }
    if (C_l) memcpy(C_l, Cl, sizeof(double) * (size_t)L * 4);
    free(Cl);
    return 0;
}

int oracle_option(int type, int d, double S0, double K, double r, double sigma,
                  double T, uint64_t seed, int64_t N, int L, int path, int rand,
                  const uint32_t *V, const double *A,
                  double *C_l, double *mean, double *stderr_, double *abs_mean)
{
    if (d < 1 || N < 1 || L < 1) return -1;
    double *Cl = (double *)malloc(sizeof(double) * (size_t)L * 4);
    double absum[4] = {0, 0, 0, 0};
    for (int l = 0; l < L; ++l)
        if (oracle_replication(type, d, S0, K, r, sigma, T, seed, 0, N, l, path, rand, V, A, Cl + 4 * l, absum) != 0) {
            free(Cl);
            return -1;
        }
    for (int o = 0; o < 4; ++o) {
        orc_sum s = {0, 0};
        for (int l = 0; l < L; ++l) sum_add(&s, Cl[l * 4 + o]);
        double C = sum_val(&s) / L;
        double ss = 0.0;
        for (int l = 0; l < L; ++l) ss += (Cl[l * 4 + o] - C) * (Cl[l * 4 + o] - C);
        mean[o] = C;
        stderr_[o] = (L >= 2) ? sqrt(ss / ((double)L * (L - 1))) : NAN;
        if (abs_mean) abs_mean[o] = absum[o] / ((double)N * L);
    }
    if (C_l) memcpy(C_l, Cl, sizeof(double) * (size_t)L * 4);
    free(Cl);
    return 0;
}

/* Many options, OpenMP over options (independent work).  Arrays are
 * structure-of-arrays of length n_opts; A_list[i] may be NULL unless
 * path == ORC_PCA.  Returns the number of threads used. */
int oracle_options(int n_opts, const int *type, const int *d, const double *S0,
                   const double *K, const double *r, const double *sigma,
                   const double *T, const uint64_t *seed, const int64_t *N,
                   int L, int path, int rand, const uint32_t *V, const double *const *A_list,
                   double *mean, double *stderr_, double *abs_mean, int n_threads)
{
    int used = 1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
    }
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int i = 0; i < n_opts; ++i) {
        oracle_option(type[i], d[i], S0[i], K[i], r[i], sigma[i], T[i], seed[i],
                      N[i], L, path, rand, V, A_list ? A_list[i] : NULL, NULL,
                      mean + 4 * i, stderr_ + 4 * i, abs_mean + 4 * i);
    }
    (void)n_threads;
    return used;
}
