/*
 * qmc_cpw.h -- C ABI of the MI355X QMC-CPW Greeks library.
 *
 * Method: Bilokon, Kucherenko, Williams, "Quasi-Monte Carlo methods for
 * calculating derivatives sensitivities on the GPU" (arXiv 2209.11337),
 * following Zhang and Wang's quasi-Monte Carlo conditional pathwise method.
 * For each option the library estimates price, delta, vega and gamma of the
 * smoothed payoff G(theta, z) = E[discounted payoff | z] (Sec. 3.4,
 * eqn:QmcCpwNewTargetDefinition), averaged over randomly shifted Sobol
 * points (Sec. 2.2.2-2.2.3) in L independent replications (Sec. 5).
 *
 * Path model (Sec. 3.4.1): d equally spaced monitoring dates t_j = j T / d,
 * S(t_j) = S~(t_j) exp(omega t_1 + sigma sqrt(t_1) x_1), omega = r - sigma^2/2,
 * where x_1 is integrated out in closed form and S~ is driven by
 * W~ = A z, z ~ N(0, I_{d-1}) with A A^T = Sigma (eqn:WboldTilde).
 *
 * Products (Sec. 4.5): arithmetic Asian call (average of S(t_1..t_d)),
 * binary Asian call (pays 1 if that average exceeds K) and fixed-strike
 * lookback call on the discrete maximum of S(t_1..t_d).
 *
 * All entry points are thread-safe with respect to each other unless stated
 * otherwise, return a qcpw_status (0 = success, < 0 = error) and never throw.
 * On an error nothing is written to the caller's outputs, and
 * qcpw_last_error() returns a message for the calling thread.
 */
#ifndef QMC_CPW_H
#define QMC_CPW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qcpw_status;
enum {
    QCPW_OK = 0,
    QCPW_EINVAL = -1,     /* an argument or option field is out of range      */
    QCPW_ENOMEM = -2,     /* device or host allocation failed                 */
    QCPW_EDEVICE = -3,    /* a HIP call failed (message names it)             */
    QCPW_EDIMS = -4,      /* d outside what the chosen construction supports  */
    QCPW_EBUSY = -5,      /* request still running (qcpw_poll)                */
    QCPW_ECANCELLED = -6, /* request was cancelled                            */
    QCPW_ENOTFOUND = -7   /* unknown request id                               */
};

/* Product (Sec. 4.5.1 binary Asian, 4.5.2 arithmetic Asian, 4.5.3 lookback).
 * Beyond the paper's three, more payoffs under the same conditional template
 * (the extension Sec. 6.2 describes):
 *  QCPW_GEOMETRIC_ASIAN_CALL  a call on the geometric average of S(t_j),
 *                             j = 1..d: the arithmetic call's formulas with X
 *                             the geometric mean; log X is normal, so its
 *                             expectation has a closed form to test against;
 *  *_PUT                      (K - X)^+ on the same average (binary: pays when
 *                             the average ends below K); the fixed-strike
 *                             lookback put is on the discrete minimum.  A put
 *                             pays for x_1 below the breakpoint.          */
enum { QCPW_ARITH_ASIAN_CALL = 0, QCPW_BINARY_ASIAN_CALL = 1, QCPW_LOOKBACK_FIXED_CALL = 2,
       QCPW_GEOMETRIC_ASIAN_CALL = 3, QCPW_ARITH_ASIAN_PUT = 4, QCPW_BINARY_ASIAN_PUT = 5,
       QCPW_LOOKBACK_FIXED_PUT = 6, QCPW_GEOMETRIC_ASIAN_PUT = 7,
       QCPW_BASKET_ASIAN_CALL = 8, QCPW_BASKET_ASIAN_PUT = 9 };
/* Basket (products on several underlyings, Sec. 6.2): n_assets assets with
 * the spec's S0 and sigma in a one-factor model, W_i = sqrt(rho) B_0 +
 * sqrt(1 - rho) B_i (every pair correlated by rho), paying on the average
 * of S_i(t_j) over assets and dates.  x_1 drives the common factor's first
 * step, so the breakpoint stays closed form with s1 = sigma sqrt(rho t_1).
 * delta and gamma are with respect to the common spot S0, vega to the
 * common sigma.  QCPW_PATH_STANDARD only; Sobol dimensions 1..d-1 drive the
 * common factor and d + i d .. d + i d + d - 1 asset i's increments, so
 * (d - 1) + n_assets d <= QCPW_MAX_BASKET_DIMS.                           */

/* Path construction.  The first three condition on the normal x_1 that
 * drives W(t_1) (Sec. 3.4.2) and build the d-1 remaining coordinates with a
 * factor A (Sec. 3.4.1 and Sec. 4.4):
 *  QCPW_PATH_BB       Brownian bridge: terminal value from the first normal,
 *                     then breadth-first midpoints, for any d (Sec. 4.4);
 *  QCPW_PATH_PCA      principal components of Sigma (largest first);
 *  QCPW_PATH_STANDARD left-to-right increments (Alg. 3).
 *  QCPW_PATH_PCA_FULL principal components of the covariance of all d dates
 *                     (W(t_j), j = 1..d); the first component (largest
 *                     eigenvalue) is the conditioned variable instead of x_1
 *                     -- the principal-component conditioning Sec. 7 names
 *                     for larger variance reduction.  Its breakpoint needs a
 *                     root-find (Newton, FP64; for the lookback the upper
 *                     envelope of the dates' log-price lines).  Arithmetic
 *                     and binary Asian and lookback calls; d <=
 *                     QCPW_MAX_D_PCA_FULL.                                  */
enum { QCPW_PATH_BB = 0, QCPW_PATH_PCA = 1, QCPW_PATH_STANDARD = 2, QCPW_PATH_PCA_FULL = 3 };

/* Arithmetic of the per-path work.  QCPW_FP64: everything in FP64.
 * QCPW_FP32_MIXED: inverse normal, path construction, exponentials and the
 * per-path sums in FP32; breakpoint, Phi tails, Greeks and every reduction
 * across paths in FP64. */
enum { QCPW_FP64 = 0, QCPW_FP32_MIXED = 1 };

/* Matrix-core arithmetic of the PCA product W~ = A z in QCPW_FP32_MIXED:
 * FP32 MFMA, or each FP32 operand split as hi + lo in BF16 with the three
 * products hi*hi + hi*lo + lo*hi accumulated in FP32.  Ignored otherwise. */
enum { QCPW_GEMM_FP32 = 0, QCPW_GEMM_BF16X3 = 1 };

/* One option.  Field order and sizes are part of the ABI (80 bytes). */
typedef struct {
    int32_t type;      /* QCPW_*_CALL, QCPW_*_PUT                              */
    int32_t d;         /* monitoring dates; used when the call's d == 0        */
    double S0;         /* spot S(0) > 0                                        */
    double K;          /* strike > 0                                           */
    double r;          /* risk-free rate (finite)                              */
    double sigma;      /* volatility > 0                                       */
    double T;          /* maturity > 0 (years)                                 */
    uint64_t seed;     /* seeds this option's digital shifts (so results do
                          not depend on which batch the option rides in)       */
    int64_t n_points;  /* Sobol points per replication; used when the call's
                          n_points == 0                                        */
    int32_t n_assets;  /* basket types: assets in the basket, 1..QCPW_MAX_ASSETS;
                          ignored by the other types                          */
    int32_t reserved;  /* must be 0                                            */
    double rho;        /* basket types: pairwise correlation, 0 < rho <= 1     */
} qcpw_option_spec;

/* Limits. */
#define QCPW_MAX_D 385          /* d - 1 <= 384 conditioned coordinates (BB, STANDARD) */
#define QCPW_MAX_D_PCA 257      /* PCA factor padded to at most 256 x 256            */
#define QCPW_MAX_D_PCA_FULL 256 /* full-covariance factor, d x d <= 256 x 256         */
#define QCPW_MAX_SHIFTS 65535   /* replications per option                           */
#define QCPW_MAX_ASSETS 8       /* assets in a basket                                */
#define QCPW_MAX_BASKET_DIMS 384 /* Sobol dimensions of a basket path                */

/*
 * qmc_cpw_greeks -- price, delta, vega, gamma of n_opts options.
 *
 * option_specs      host array [n_opts], read only, caller-owned.
 * n_opts            >= 1.
 * d                 monitoring dates for every option (1..QCPW_MAX_D, or up
 *                   to QCPW_MAX_D_PCA with PCA, QCPW_MAX_D_PCA_FULL with
 *                   PCA_FULL); 0 = use each spec's d.
 * n_points          Sobol points k = 0..n_points-1 per replication, in Gray
 *                   code order (1..2^32; powers of two recommended); 0 = use
 *                   each spec's n_points.
 * n_shifts          replications L (1..QCPW_MAX_SHIFTS); replication l uses
 *                   the digital shift s_{l,j} = high 32 bits of output
 *                   l*2^16 + j of SplitMix64 seeded with the option's seed.
 * path_construction QCPW_PATH_*.
 * out_greeks        host array [n_opts][4] = {price, delta, vega, gamma}:
 *                   C = (1/L) sum_l C_l, C_l = (1/n) sum_k F(theta, z_{l,k}).
 * out_stderr        host array [n_opts][4]: sqrt(sum_l (C_l - C)^2 / (L(L-1)));
 *                   NaN when L == 1, 0 when d == 1 (no sampled coordinate).
 *
 * Computes in QCPW_FP64 on the current HIP device and returns when the
 * results are on the host.  Errors: QCPW_EINVAL (bad pointer, count, enum
 * or non-finite/non-positive field), QCPW_EDIMS (d too large for the
 * construction), QCPW_ENOMEM, QCPW_EDEVICE.
 */
qcpw_status qmc_cpw_greeks(const qcpw_option_spec *option_specs, int32_t n_opts,
                           int32_t d, int64_t n_points, int32_t n_shifts,
                           int32_t path_construction,
                           double *out_greeks, double *out_stderr);

/* Run options for qmc_cpw_greeks_ex. */
typedef struct {
    int32_t precision;          /* QCPW_FP64 or QCPW_FP32_MIXED                    */
    int32_t pca_gemm;           /* QCPW_GEMM_FP32 or QCPW_GEMM_BF16X3              */
    int32_t device;             /* HIP device ordinal, -1 = current                */
    int32_t outputs_on_device;  /* 1: out_greeks/out_stderr/out_per_shift are device
                                   pointers, results written on `stream`, call
                                   returns without waiting for them                */
    void *stream;               /* hipStream_t to run on (NULL = the default stream) */
    double *out_per_shift;      /* optional [n_opts][L][4] per-replication C_l       */
    int32_t block_threads;      /* 0 = autotuned; else a multiple of 64 in [64, 1024]
                                   (workgroup size of the per-path kernel's launches;
                                   the PCA kernel always uses 256)                  */
    int32_t flags;              /* QCPW_FLAG_* bits                                  */
    double *out_paper_sigma;    /* optional [n_opts][4]: the spread of the single
                                   replications sqrt((1/L) sum_l (C - C_l)^2), the
                                   sigma Sec. 5 reports (= out_stderr sqrt(L - 1));
                                   host or device as out_greeks; NaN when L == 1  */
} qcpw_run_config;

/* Capture the device work of a call into a HIP graph the first time a given
 * argument set is seen and replay the graph for later calls with identical
 * arguments (same specs, sizes, enums, stream and output pointers).  Requires
 * outputs_on_device; the graph keeps its own device workspace (up to 16
 * graphs are cached per device, least recently used evicted). */
#define QCPW_FLAG_GRAPH 1

/* Randomise the Sobol points by nested (Owen) scrambling (Sec. 2.2.3)
 * instead of the random digital shift: digit k of each coordinate is
 * flipped by a random function of the digits above it, seeded per
 * (replication l, dimension j) by the same 32-bit value s_{l,j} that is the
 * digital shift otherwise (hash-based nested scrambling: a seeded addition
 * and four rounds v ^= (v mod 2^24) * C, C even, on the bit-reversed
 * value).  Every path construction; also accepted by
 * qcpw_server_create. */
#define QCPW_FLAG_OWEN 2

/*
 * qmc_cpw_greeks_ex -- as qmc_cpw_greeks with explicit precision, device,
 * stream and output placement.  cfg may be NULL (defaults of
 * qmc_cpw_greeks).  Options of different d, n_points and type share one
 * persistent launch -- or two, when the call mixes options whose Sobol
 * dimensions fill the LDS with others that run faster apart (an option's
 * results do not depend on which).  With outputs_on_device the caller keeps
 * the output buffers alive until the stream reaches them; the library's
 * temporary device buffers stay owned by the library and are reused by
 * later calls on the same device (calls on one device are serialised
 * internally).
 */
qcpw_status qmc_cpw_greeks_ex(const qcpw_option_spec *option_specs, int32_t n_opts,
                              int32_t d, int64_t n_points, int32_t n_shifts,
                              int32_t path_construction,
                              double *out_greeks, double *out_stderr,
                              const qcpw_run_config *cfg);

/*
 * qmc_cpw_greeks_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): qmc_cpw_greeks_ex with the launch workspace in a fixed device
 * array of QCPW_NOALLOC_BYTES per device, held from the library's load
 * until the process ends, instead of library-allocated buffers.  Same
 * arguments, results and errors as qmc_cpw_greeks_ex, except:
 *   - path_construction QCPW_PATH_BB or QCPW_PATH_STANDARD, flags 0 or
 *     QCPW_FLAG_OWEN (QCPW_EINVAL otherwise);
 *   - block_threads 0 takes the autotuner's earlier choice for each
 *     launch's shape if there is one, else 512 threads (768 for the
 *     launches that need them to fill a CU) -- its probe launches are
 *     never run here;
 *   - QCPW_ENOMEM, before any device work, when the launch needs more than
 *     QCPW_NOALLOC_BYTES: 64 bytes per work unit (units = sum over options
 *     of n_shifts * ceil(n_points / unit points), 256..4096 points per unit)
 *     plus about 400 bytes per option, and with host outputs their staging.
 * Nothing is allocated and nothing freed by the call; the first call of the
 * library on a device (any entry point) builds the device tables, so a
 * caller that must not allocate at all makes one call first.  Every call on
 * a device shares its array, which keeps the last call's contents: calls
 * that overlap on one device (different streams or threads) race on it.
 */
#define QCPW_NOALLOC_BYTES (64 << 20)
qcpw_status qmc_cpw_greeks_noalloc(const qcpw_option_spec *option_specs, int32_t n_opts,
                                   int32_t d, int64_t n_points, int32_t n_shifts,
                                   int32_t path_construction,
                                   double *out_greeks, double *out_stderr,
                                   const qcpw_run_config *cfg);

/*
 * qcpw_sobol_points -- the shifted Sobol integers the kernels consume, for
 * checking them bit for bit: out[k][j] = (G_j gray(k0 + k)) XOR s_{l,j},
 * k = 0..count-1, j = 0..n_dims-1 (dimension 0 unshifted), computed on the
 * device by a kernel of its own through the same lane-table / wave-uniform
 * split as the per-path kernel (qcpw_path_coordinates records what the
 * per-path kernel itself consumes).  out is a host array [count][n_dims]
 * (uint32).  n_dims <= 1024, count <= 2^24.
 */
qcpw_status qcpw_sobol_points(uint64_t seed, int32_t shift_index, int32_t n_dims,
                              int64_t k0, int64_t count, uint32_t *out);

/*
 * qcpw_scrambled_points -- as qcpw_sobol_points with nested scrambling
 * (QCPW_FLAG_OWEN) in place of the digital shift: out[k][j] =
 * owen(G_j gray(k0 + k), s_{l,j}) for j >= 1, dimension 0 unscrambled.
 */
qcpw_status qcpw_scrambled_points(uint64_t seed, int32_t shift_index, int32_t n_dims,
                                  int64_t k0, int64_t count, uint32_t *out);

/*
 * qcpw_path_coordinates -- the randomised Sobol integers (Sec. 2.2.2 XOR form
 * in Gray-code order, then the digital shift or, with QCPW_FLAG_OWEN in
 * flags, nested scrambling, Sec. 2.2.3) exactly as the fused per-path kernel
 * consumes them while it walks one option, recorded by an instance of that
 * kernel that also stores every coordinate it reads: out[l][k][j] for
 * replication l < n_shifts, point k < spec->n_points and dimension j + 1,
 * j < spec->d - 1 (plus n_assets * d for baskets).  spec: one option (its
 * d and n_points fields are used); path_construction QCPW_PATH_BB or
 * QCPW_PATH_STANDARD; precision as for _ex (the FP32 kernel walks
 * d = 16, 32, 64, 128 with its compile-time bridges).  out: host array,
 * caller-owned.  Errors: QCPW_EINVAL (as qmc_cpw_greeks, other
 * constructions or flags, d = 1, more than 2^28 bytes of output).
 */
qcpw_status qcpw_path_coordinates(const qcpw_option_spec *spec, int32_t n_shifts, int32_t path_construction,
                                  int32_t precision, int32_t flags, uint32_t *out);

/*
 * qcpw_path_factor -- the factor A (row-major (d-1) x (d-1), FP64) that the
 * library uses for path_construction with d dates and maturity T, for
 * inspection (A A^T = Sigma).  out must hold (d-1)^2 doubles; for
 * QCPW_PATH_PCA_FULL it is the d x d factor of the covariance of all d dates
 * (column 0 = the conditioned component) and out must hold d^2 doubles.
 */
qcpw_status qcpw_path_factor(int32_t path_construction, int32_t d, double T, double *out);

/*
 * qcpw_kernel_timer -- measurement of the main kernel (the fused per-path
 * kernel, or the PCA kernel) of each qmc_cpw_greeks / qmc_cpw_greeks_ex call
 * on `device` (-1 = current) that runs eagerly (not from a captured graph,
 * not from a server).  The library records a pair of HIP events on the
 * call's stream around that kernel alone (before its first and after its
 * last launch when the call takes two).
 *   op = QCPW_TIMER_START: forget earlier pairs and start recording;
 *   op = QCPW_TIMER_READ:  wait for the recorded events, write the summed
 *        kernel time in milliseconds to *total_ms and the number of timed
 *        launches to *launches (either pointer may be NULL); keep recording;
 *   op = QCPW_TIMER_STOP:  as READ, then stop recording.
 * Errors: QCPW_EINVAL for another op, QCPW_EDEVICE without a usable device.
 */
#define QCPW_TIMER_START 1
#define QCPW_TIMER_READ 2
#define QCPW_TIMER_STOP 3
qcpw_status qcpw_kernel_timer(int32_t device, int32_t op, double *total_ms, int64_t *launches);

/* Message describing the calling thread's last error ("" if none). */
const char *qcpw_last_error(void);

/* Library version string. */
const char *qcpw_version(void);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of Greek requests on one device.
 *
 * A server owns a worker thread, a device work queue and an HBM budget.
 * qcpw_submit admits a request (a small portfolio with a target standard
 * error): it is charged its device footprint against hbm_budget_bytes and
 * queued; the worker packs queued requests into launches as budget and
 * batch slots free up, so requests that arrive while others run join the
 * next launch.  A request starts at 2^14 points per option and doubles the
 * points (reusing all earlier points, since Sobol points extend) until
 * every option's delta, vega and gamma standard errors are at most
 * target_stderr * max(1, |value|), or 2^22 points are reached.
 * --------------------------------------------------------------------------- */
typedef struct qcpw_server qcpw_server;

/* cfg: precision / device / block_threads as for _ex (stream and output
 * fields ignored).  hbm_budget_bytes > 0 bounds the device memory of the
 * server's launch workspaces together (two launch slots, each at most half
 * of it; the resident tables are not counted).  With block_threads == 0 the
 * workgroup-size autotuner runs for every lane-table bucket here, so that no
 * request pays for its probe launches.  *out receives the server. */
qcpw_status qcpw_server_create(const qcpw_run_config *cfg, int64_t hbm_budget_bytes,
                               qcpw_server **out);

/* Copies the specs; 1 <= n_opts <= 4096; every spec's d field is used
 * (n_points is ignored: the target sets the count).  A request is admitted
 * into a launch when its smallest slice (8192 points of every option) fits
 * the memory left in that launch's slot; QCPW_ENOMEM if it cannot fit even
 * an empty slot.  *request_id receives the id. */
qcpw_status qcpw_submit(qcpw_server *srv, const qcpw_option_spec *specs, int32_t n_opts,
                        int32_t n_shifts, int32_t path_construction,
                        double target_stderr, uint64_t *request_id);

/* QCPW_EBUSY while the request runs; QCPW_OK once results are copied to
 * out_greeks/out_stderr ([n_opts][4] host arrays, may be NULL) and
 * *out_points_used (points per replication reached, may be NULL); the
 * request is then forgotten.  QCPW_ECANCELLED / QCPW_ENOTFOUND otherwise. */
qcpw_status qcpw_poll(qcpw_server *srv, uint64_t request_id, double *out_greeks,
                      double *out_stderr, int64_t *out_points_used);

/* Blocks until the request finishes (or is cancelled), then as qcpw_poll. */
qcpw_status qcpw_wait(qcpw_server *srv, uint64_t request_id, double *out_greeks,
                      double *out_stderr, int64_t *out_points_used);

/* Cancels a queued or running request; its result is dropped. */
qcpw_status qcpw_cancel(qcpw_server *srv, uint64_t request_id);

/* Counters since creation: [0] admitted, [1] completed, [2] cancelled,
 * [3] launches, [4] device bytes of the launches in flight, [5] their peak,
 * [6] queued now, [7] device bytes the launch workspaces hold now. */
qcpw_status qcpw_server_stats(qcpw_server *srv, int64_t out[8]);

/* Stops taking work at once, waits for the launches in flight (at most two,
 * each bounded in size), then cancels every queued or running request. */
qcpw_status qcpw_server_destroy(qcpw_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* QMC_CPW_H */
