/*
 * cefield.h -- C ABI of the MI355X (gfx950) circulant-embedding Gaussian field
 * generator.
 *
 * Method: Carron, Wolk & Szapudi (2014), "On fast generation of cosmological
 * random fields", arXiv:1406.6072.  A survey grid of N_i cells per axis is
 * embedded in a periodic grid of M_i = 2 N_i cells; the DFT of the two-point
 * function on that grid gives the circulant eigenvalues; seeded complex white
 * noise scaled by their square root and inverse-transformed gives two exact,
 * independent Gaussian realizations (real and imaginary parts) on the survey
 * cells; these are exponentiated (lognormal) and Poisson sampled, and the
 * binned power spectrum and its covariance are estimated from them.
 *
 * Conventions for every entry point:
 *  - All functions are C, never throw, and return a ce_status.  Argument
 *    errors are detected on the host before anything is enqueued.
 *  - Device pointers are plain HIP device addresses owned by the caller (for
 *    example PyTorch tensors); host pointers are marked "host".  Outputs are
 *    written, never accumulated into, unless stated.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is enqueued asynchronously on it; the caller synchronises.
 *  - A ce_ctx owns scratch memory.  Calls on one ctx must not overlap in time
 *    (use one ctx per stream / thread, or serialise).
 *  - Layouts are row-major with the last axis fastest.  A stack of `count`
 *    maps is count x N_0 x ... x N_{d-1}.  Realization r = 2j + s comes from
 *    pair j: s = 0 is the real part, s = 1 the imaginary part.
 *  - Supported: d = 2 or 3, every N_i even and >= 4, M_i = 2 N_i at most 4096
 *    (any factorisation: powers of two in radices up to 16, the primes up to 31
 *    in dedicated butterflies, larger primes in a generic prime stage), each
 *    embedding with fewer than 2^32 cells; in FP64, a first periodic side whose
 *    length has a prime factor above 31 is at most ~2400 (two of its lines,
 *    each with a second buffer for the ping-pong stages of such radices, must fit
 *    one workgroup's 160 KB of LDS).  Other sizes return CE_E_UNSUPPORTED.
 */
#ifndef CEFIELD_H
#define CEFIELD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CE_OK = 0,
  CE_E_INVALID = 1,      /* bad argument (null pointer, bad size, odd first realization, ...) */
  CE_E_NOT_PSD = 2,      /* embedding spectrum negative beyond round-off: the method does not apply */
  CE_E_OOM = 3,          /* device allocation failed or exceeds the ctx HBM budget */
  CE_E_UNSUPPORTED = 4,  /* geometry or option not implemented (see the limits above) */
  CE_E_DEVICE = 5,       /* HIP runtime error */
  CE_E_SAMPLER = 6       /* a device-side sampler/estimator condition was flagged (see ce_ctx_check) */
} ce_status;

typedef enum { CE_F32 = 0, CE_F64 = 1 } ce_precision;

typedef enum {
  CE_XI_TABLE = 0,   /* table on the lag octant, see ce_xi.table */
  CE_XI_EXP = 1,     /* p[0] exp(-r / p[1]) */
  CE_XI_POWEXP = 2   /* p[0] (1 + r/p[1])^(-p[2]) exp(-r/p[3]); p[3] <= 0 means no cut-off */
} ce_xi_kind;

/* Survey grid: ndim axes of n[i] cells of side h[i] (the grid of Sec. 2, x = h i, i = 0..N-1). */
typedef struct {
  int32_t ndim;
  int64_t n[3];
  double h[3];
} ce_geometry;

/* Transforms applied to xi when its lag table is built (flags, combinable; applied in this order).
 * CE_XI_CELL_AVERAGE: xi is the unfiltered isotropic two-point function omega of the density
 *   contrast and the table holds its average over pairs of cells, the square top-hat filtered
 *   function of App. A: the overlap integral eq. exactformula (Gauss-Legendre, ~1e-14 relative)
 *   for lags shorter than 15 max(h_0, h_1), the derivative expansion eq. CoolEq (second order,
 *   5-point differences in ln r of step 2e-3, written for rectangular cells) beyond.  2-D maps
 *   and the EXP / POWEXP kinds only (CE_E_UNSUPPORTED otherwise).
 * CE_XI_LOGNORMAL: the table holds ln(1 + value) (eq. Lncov): the Gaussian field is the
 *   log-density A, and rho = exp(A - sigma_A^2/2) has covariance `value` (sigma_A^2 is the
 *   plan's sigma2).  A value <= -1 has no logarithm: the plan is rejected (CE_E_NOT_PSD). */
typedef enum {
  CE_XI_CELL_AVERAGE = 1,
  CE_XI_LOGNORMAL = 2
} ce_xi_transform;

/* Two-point function xi of the Gaussian field; isotropic kinds take the distance r = |x|,
 * x = (l_0 h_0, ..., l_{d-1} h_{d-1}).
 * CE_XI_TABLE: host FP64 array of xi at lags (l_0 h_0, ..., l_{d-1} h_{d-1}) for
 * l_i in [0, N_i], row-major, shape (N_0+1) x ... ; it must describe a function that is
 * even in every axis.  The table is copied during ce_plan_embedding.
 * transform: 0 or a combination of ce_xi_transform flags. */
typedef struct {
  int32_t kind;
  double p[4];
  const double* table;
  int32_t transform;
} ce_xi;

typedef struct {
  double lambda_min;     /* smallest circulant eigenvalue before clamping (DFT of the lag table) */
  double lambda_max;     /* largest */
  double sigma2;         /* the lag table at 0 (xi(0) after its transforms): variance of each cell */
  int64_t n_negative;    /* eigenvalues below zero (full embedding grid, before clamping) */
  int64_t n_clamped;     /* eigenvalues set to zero (= n_negative when the plan is accepted) */
  size_t device_bytes;   /* device memory held by the plan */
} ce_plan_info;

typedef struct ce_ctx ce_ctx;
typedef struct ce_plan ce_plan;

/* Map kinds for ce_estimate_pk. */
typedef enum {
  CE_MAP_FIELD = 0,        /* real maps in the given precision; the spectrum of the map itself */
  CE_MAP_COUNTS_DELTAG = 1 /* int32 counts; the spectrum of delta_g = (N/f - N^)/N^ (Sec. 3.2) */
} ce_map_kind;

const char* ce_status_string(ce_status s);

/* Library version string (static storage). */
const char* ce_version(void);

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the scratch and
 * plan memory the ctx may hold (0 = no bound).  Errors: CE_E_INVALID, CE_E_DEVICE. */
ce_status ce_ctx_create(int device, size_t hbm_budget_bytes, ce_ctx** out);
void ce_ctx_destroy(ce_ctx* ctx);

/* Synchronise the ctx's last stream and report device-side flags: CE_E_SAMPLER if a Poisson
 * draw exceeded its step bound or a counts map had N_tot = 0 since the last check. */
ce_status ce_ctx_check(ce_ctx* ctx, void* stream);

/* Free the ctx's cached pipeline scratch (it is allocated again on the next call that needs
 * it).  Waits for the device first.  Errors: CE_E_INVALID, CE_E_DEVICE. */
ce_status ce_ctx_trim(ce_ctx* ctx);

/* Context options.
 * CE_OPT_UNPRUNED (default 0): when non-zero, ce_generate_fields computes every output of every
 * inverse pass on the full (2N)^d embedding and crops to the survey only when storing -- the
 * plain, unpruned form of the method, kept as a comparator.  Results are identical up to
 * rounding order.  Schedule options change only the launch shape: every output (fields, delta,
 * counts, N_tot, P(k), covariance) stays bitwise identical (the FP64 shell sums are grouped in
 * blocks of lines fixed by the grid, shells and precision, not by the schedule).
 * Errors: CE_E_INVALID. */
typedef enum {
  CE_OPT_UNPRUNED = 1,
  /* Schedule: maximum lines per workgroup (a power of two <= 64; 0 = automatic, the default)
   * for the noise pass, the inner-axis passes, the last inverse pass and the binning pass.
   * The library lowers a requested value to what the LDS and the 512-thread limit allow. */
  CE_OPT_LINES_NOISE = 2,
  CE_OPT_LINES_INNER = 3,
  CE_OPT_LINES_LAST = 4,
  CE_OPT_LINES_BINS = 5,
  /* Schedule: tile order of the noise pass: 0 (default) = the line groups of one pair run
   * together (their strided output segments merge in L2); 1 = the workgroups of one line group
   * for consecutive pairs run together (the sqrt(lambda) lines they read stay in L2). */
  CE_OPT_NOISE_ORDER = 6,
  /* Schedule: LDS bytes a binning-pass workgroup may use (16384 .. 163840; default 81920,
   * two workgroups per CU).  More LDS allows more lines per workgroup. */
  CE_OPT_BIN_LDS = 7,
  /* Schedule: with CE_OPT_NOISE_ORDER 0, the noise pass orders its workgroups in blocks of this
   * many pairs (1 .. 65536, default 1): inside a block the workgroups of one line group for the
   * block's pairs run together, so the sqrt(lambda) lines they read are fetched once per block. */
  CE_OPT_NOISE_BLOCK = 8,
  /* Schedule: ce_pipeline_run_batch runs its groups of different shapes concurrently on up to
   * this many internal streams (1 .. 16, default 4), each with its own scratch, forked from and
   * joined back into the call's stream. */
  CE_OPT_BATCH_LANES = 9,
  /* Schedule: pairs each noise-pass workgroup generates for its lines, one after another (1 .. 64;
   * 0 = automatic, the default: up to 8 while the pass keeps 4096 workgroups). The octant of
   * sqrt(lambda) is fetched from HBM once per that many pairs. */
  CE_OPT_NOISE_PAIRS = 10
} ce_option;
ce_status ce_ctx_set_option(ce_ctx* ctx, int32_t option, int64_t value);

/* Profiling: with enable != 0 every kernel the ctx launches is bracketed by HIP events on its
 * launch stream.  ce_ctx_profile_read synchronises on those events and reports, per kernel
 * name, the summed duration and the launch count since the previous read (which it resets).
 * names: host buffer of max * 32 bytes (NUL-terminated names); total_ms, launches: host arrays
 * of max; *n receives the number of entries written.  Errors: CE_E_INVALID, CE_E_DEVICE. */
ce_status ce_ctx_set_profiling(ce_ctx* ctx, int32_t enable);
ce_status ce_ctx_profile_read(ce_ctx* ctx, int32_t max, char* names, double* total_ms, int64_t* launches,
                              int32_t* n);

/* Embedding plan (Sec. 2, eqs. grid and Specd; condition).
 * Builds the lag table c(m) = xi(h lag(m)) on the (2N)^d periodic grid (lag index N stands for
 * -N, the minimum image), takes its FP64 DFT on the device (the circulant eigenvalues lambda,
 * P~ = h^d lambda), and checks lambda >= 0 (eq. condition).  If lambda_min < -neg_tol *
 * lambda_max the plan is rejected with CE_E_NOT_PSD and *out is left NULL; otherwise negative
 * values are clamped to 0.  neg_tol < 0 selects the default 1e-13.  The plan keeps
 * sqrt(lambda / M^d) on the eigenvalue octant in `precision` on the device; `info` (nullable)
 * is filled in both cases; a non-finite eigenvalue (a table value <= -1 under CE_XI_LOGNORMAL, an
 * infinite xi) is reported as lambda_min = -inf and rejects the plan.  Synchronous.  Errors: CE_E_INVALID, CE_E_UNSUPPORTED, CE_E_OOM,
 * CE_E_NOT_PSD, CE_E_DEVICE. */
ce_status ce_plan_embedding(ce_ctx* ctx, const ce_geometry* geom, const ce_xi* xi,
                            ce_precision precision, double neg_tol, ce_plan** out,
                            ce_plan_info* info);
/* k-space sampling comparator (Sec. 3.3, eq. Periodicboxmodes): a plan on a periodic box of
 * `box` cells per axis (square / cubic, box >= N_i, even, the cell side h equal on every axis)
 * whose survey is cells [0, N_i) of the box.  The mode variances follow the continuous Fourier
 * transform of the isotropic xi (after CE_XI_LOGNORMAL, if set): lambda(q) = P(|k_q|) / h^d with
 * P(k) = 2 pi int r J0(k r) xi(r) dr (2-D) or 4 pi int r^2 sinc(k r) xi(r) dr (3-D), k_q =
 * 2 pi q~ / (box h), evaluated on the device by Gauss-Legendre panels up to the radius where the
 * exponential cut-off of xi reaches e^-40; lambda(0) = 0 (the DC mode is zeroed).  Kinds
 * CE_XI_EXP and CE_XI_POWEXP with a cut-off (p[3] > 0); CE_XI_CELL_AVERAGE and tables are
 * CE_E_UNSUPPORTED.  The plan's sigma2 is the cell variance of the box field, sum(lambda) / box^d.
 * The plan runs through every generator and pipeline entry point like an embedding plan (which
 * is the case box = 2N with the discrete spectrum).  Synchronous.  Errors: CE_E_INVALID,
 * CE_E_UNSUPPORTED, CE_E_OOM, CE_E_NOT_PSD, CE_E_DEVICE. */
ce_status ce_plan_periodic(ce_ctx* ctx, const ce_geometry* geom, int64_t box, const ce_xi* xi,
                           ce_precision precision, double neg_tol, ce_plan** out, ce_plan_info* info);
void ce_plan_release(ce_plan* plan);

/* The lag octant a plan for (geom, xi) starts from: xi, transformed as xi->transform asks, at
 * lags l_i in [0, N_i] (row-major (N_0+1) x ... doubles, device buffer `out`, caller owns).
 * Asynchronous on `stream` (a CE_XI_TABLE is read before the call returns).
 * Errors: CE_E_INVALID, CE_E_UNSUPPORTED, CE_E_DEVICE. */
ce_status ce_xi_lag_octant(ce_ctx* ctx, const ce_geometry* geom, const ce_xi* xi, double* out,
                           void* stream);
ce_status ce_plan_get_info(const ce_plan* plan, ce_plan_info* info);

/* Copy the FP64 eigenvalue octant lambda(q), q_i in [0, M_i / 2] (before clamping), row-major
 * (M_0/2+1) x ..., into device buffer out (caller owns, prod (M_i/2+1) doubles; M_i = 2 N_i for
 * an embedding plan, the box side for a periodic plan). */
ce_status ce_plan_eigenvalues(const ce_plan* plan, double* out, void* stream);

/* Gaussian realizations (Sec. 2, eq. Papos2 and the discrete construction after eq. Specd).
 * For pair j the modes are X(q) = sqrt(M^d lambda(q)) (a + i b), a, b iid N(0,1) from
 * Philox4x32-10 (key = seed, counter (floor(l/2), j, request_id, 0), l the row-major embedding
 * cell index; words x0,x1 -> cell 2p, x2,x3 -> cell 2p+1; Box-Muller), Z = M^-d sum_q X(q)
 * exp(+2 pi i q.m/M) restricted to m_i in [0, N_i); realization 2j = Re Z, 2j+1 = Im Z.
 * Writes realizations first_realization .. +count-1 (first_realization even) to out_fields:
 * count x N^d elements of float (CE_F32 plan) or double (CE_F64 plan).
 * Errors: CE_E_INVALID, CE_E_OOM, CE_E_DEVICE. */
ce_status ce_generate_fields(ce_ctx* ctx, const ce_plan* plan, uint64_t seed, uint32_t request_id,
                             uint64_t first_realization, int64_t count, void* out_fields,
                             void* stream);

/* Lognormal density and Poisson counts (Sec. 3.1, step i and eq. sampling).
 * For each cell: delta = exp(g - sigma2/2) - 1 in the plan precision (sigma2 = xi(0));
 * mu = (nbar f) (1 + delta) in FP64 from delta as stored; count ~ Poisson(mu) by FP64 chunked
 * inversion (chunks of mean 64; chunk c of survey cell l in realization r uses the 52-bit
 * uniform from Philox4x32-10 with key = seed and counter (l, floor(r/2), request_id, 1 + c),
 * words x0,x1 for even r and x2,x3 for odd r).  fields: count x N^d (plan precision).
 * mask_f (nullable; f = 1 when NULL): N^d floats in [0, 1].  out_delta (nullable): like fields.
 * out_counts: count x N^d int32.  out_ntot (nullable): count int64 totals.
 * first_realization must equal the realization index of fields[0] (it selects the streams).
 * Errors: CE_E_INVALID, CE_E_DEVICE. */
ce_status ce_lognormal_poisson(ce_ctx* ctx, const ce_plan* plan, const void* fields, int64_t count,
                               double nbar, const float* mask_f, uint64_t seed,
                               uint32_t request_id, uint64_t first_realization, void* out_delta,
                               int32_t* out_counts, int64_t* out_ntot, void* stream);

/* Binned power spectrum (Sec. 3.2, eq. Def spec with the contrast of eq. Estim).
 * P_b = (h^d / N^d) (1/N_b) sum_{q in b} |F(q)|^2, F the DFT of the map (CE_MAP_FIELD) or of
 * delta_g = (N/f - N^)/N^ on f != 0 and 0 elsewhere, N^ = N_tot / sum f (CE_MAP_COUNTS_DELTAG;
 * ntot nullable -> computed; mask_f nullable -> f = 1).  Shells are linear in |k| on
 * (0, pi / max h_i]: mode q (signed frequencies q~_i) is in shell b when
 * b < nbins |k| / (pi / max h_i) <= b+1, |k|^2 = sum_i (2 pi q~_i / (N_i h_i))^2, decided exactly
 * in integers (square / cubic cells: b < nbins 2 sqrt(sum_i (q~_i / N_i)^2) <= b+1, with the least
 * common multiple of the N_i).  The sides N_i may differ (hyperrectangular surveys) and so may
 * the cell sides h_i, when their ratios are fractions of denominator <= 64 (an irrational ratio:
 * CE_E_UNSUPPORTED).  h^d is the cell volume prod_i h_i.  maps: count x N^d of float /
 * double (FIELD, per `precision`) or int32 (COUNTS).  out_pk: count x nbins doubles (device).
 * out_nmodes (nullable, device, nbins int64), out_kmean (nullable, device, nbins doubles: the
 * mean |k| = 2 pi |q~| / (N h) of each shell).  Bin sums are accumulated in FP64 in a fixed
 * order (bitwise reproducible).  Errors: CE_E_INVALID, CE_E_UNSUPPORTED, CE_E_DEVICE. */
ce_status ce_estimate_pk(ce_ctx* ctx, const ce_geometry* geom, ce_precision precision,
                         ce_map_kind kind, const void* maps, int64_t count, const int64_t* ntot,
                         const float* mask_f, int32_t nbins, double* out_pk, int64_t* out_nmodes,
                         double* out_kmean, void* stream);

/* ce_estimate_pk with user shells (the paper bins in ln l; or linear shells up to a kmax that
 * takes the corners): kedges is a host array of nbins + 1 strictly ascending |k| values >= 0
 * (units 1 / length, as h).  Mode q with t = nbins^2 L^2 (|k| h / pi)^2 (an exact integer, L the
 * least common multiple of the N_i) is in shell b when TH_b < t <= TH_{b+1}, TH_b =
 * nbins^2 L^2 (kedges[b] h / pi)^2 evaluated in FP64 in this order, rounded to the nearest
 * integer when within 1e-9 relative of one and down otherwise (so edges placed on modes by an
 * FP64 formula keep them in the lower shell, and linear edges on (0, pi/h] reproduce
 * ce_estimate_pk bitwise).  out_nmodes and out_kmean are those of these shells.  Errors: as
 * ce_estimate_pk; CE_E_INVALID for edges that are not finite, negative or ascending. */
ce_status ce_estimate_pk_edges(ce_ctx* ctx, const ce_geometry* geom, ce_precision precision,
                               ce_map_kind kind, const void* maps, int64_t count, const int64_t* ntot,
                               const float* mask_f, int32_t nbins, const double* kedges, double* out_pk,
                               int64_t* out_nmodes, double* out_kmean, void* stream);

/* Spectrum covariance across realizations (Sec. 3.2: covariance from many simulations; the
 * normalised matrix of eq. cuminfo).  pk: count x nbins doubles (device).  out_cov (nullable):
 * nbins^2, Cov_ab = 1/(count-1) sum_r (P_ra - mean_a)(P_rb - mean_b).  out_cnorm (nullable):
 * nbins^2, C_ab = (1/count) sum_r P_ra P_rb / (mean_a mean_b) - 1.  FP64, fixed order.
 * Errors: CE_E_INVALID (count < 2), CE_E_DEVICE. */
ce_status ce_pk_covariance(ce_ctx* ctx, const double* pk, int64_t count, int32_t nbins,
                           double* out_cov, double* out_cnorm, void* stream);

/* Largest number of shells of ce_cumulative_information. */
#define CE_INFO_MAX_BINS 2048

/* Cumulative information (Sec. 3.3, eq. cuminfo): out_info[b] = I(<= shell b) = the sum of the
 * elements of the inverse of the leading (b+1) x (b+1) block of the normalised spectrum
 * covariance C_ab = <P_a P_b> / (<P_a><P_b>) - 1 (the out_cnorm of ce_pk_covariance).  One
 * Cholesky factorisation of C in FP64 gives every prefix (the leading block of the factor is the
 * factor of the leading block).  cnorm: nbins x nbins doubles (device, row-major, symmetric; the
 * lower triangle is read); out_info: nbins doubles (device).  Entries from the first shell whose
 * block is not positive definite on are NaN (e.g. fewer realizations than shells).
 * 1 <= nbins <= CE_INFO_MAX_BINS.  Errors: CE_E_INVALID, CE_E_DEVICE. */
ce_status ce_cumulative_information(ce_ctx* ctx, const double* cnorm, int32_t nbins, double* out_info,
                                    void* stream);

/* Largest histogram length of ce_cic_histogram. */
#define CE_CIC_MAX_BINS 4096

/* Counts-in-cells histogram (Sec. 3.4): out_hist[r * nhist + N] = the number of cells i of map r
 * with f_i != 0 and count N, N = 0 .. nhist-1; counts outside that range are in no bin and fully
 * masked cells are ignored.  counts: count x cells int32 (device); mask_f (nullable: f = 1):
 * cells floats in [0, 1] (device); out_hist: count x nhist int64 (device), overwritten.  Exact in
 * integers.  1 <= nhist <= CE_CIC_MAX_BINS.  Errors: CE_E_INVALID, CE_E_DEVICE. */
ce_status ce_cic_histogram(ce_ctx* ctx, const int32_t* counts, int64_t cells, int64_t count,
                           const float* mask_f, int32_t nhist, int64_t* out_hist, void* stream);

/* Mean counts-in-cells histogram of the model (Sec. 3.4): out_pred[N] = <P^(N)> =
 * int dA G(A) sum_{f_i != 0} Pois(N; nbar f_i e^A), N = 0 .. nhist-1, G the normal law of the
 * log-density with mean -sigma2_A/2 and variance sigma2_A (a Poisson-lognormal mixture over the
 * cells' intensities).  The A integral is a Gauss-Legendre rule on mu +- 12 sigma (panels no
 * wider than sigma/2 and 1/sqrt(nhist), 8 nodes each); the pmf is formed in FP64 from logs.
 * mask_f (nullable: f = 1): cells floats in [0, 1] (device); out_pred: nhist doubles (device).
 * Waits for the host side of its tables before returning.  nbar > 0 and sigma2_A > 0 finite,
 * 1 <= nhist <= CE_CIC_MAX_BINS.  Errors: CE_E_INVALID, CE_E_DEVICE. */
ce_status ce_cic_predict(ce_ctx* ctx, const float* mask_f, int64_t cells, double nbar, double sigma2_A,
                         int32_t nhist, double* out_pred, void* stream);

/* A* map (Sec. 3.4, eq. As): in each cell with f_i != 0, the root A* of
 * e^{A*} N_bar_i sigma2_A + A* = sigma2_A (N_i - 1/2) with N_bar_i = nbar f_i, solved in FP64
 * (unique: the left side increases strictly with A*); cells with f_i = 0 hold 0.
 * subtract_mean != 0: A* minus its mean over the unmasked cells of the map, 0 on masked cells
 * (the map whose spectrum ce_estimate_pk estimates as CE_MAP_FIELD).  counts: count x cells
 * int32 (device); mask_f (nullable: f = 1): cells floats in [0, 1]; out_map: count x cells of
 * float (CE_F32) or double (CE_F64), rounded once from FP64; out_mean (nullable, device): count
 * doubles, the mean of A* over the unmasked cells of each map (0 when all are masked), summed
 * in a fixed order.  nbar > 0 and sigma2_A > 0 (the variance of the log-density, ln(1 +
 * sigma_delta^2)), both finite.  Errors: CE_E_INVALID, CE_E_DEVICE. */
ce_status ce_astar_map(ce_ctx* ctx, const int32_t* counts, int64_t cells, int64_t count,
                       const float* mask_f, double nbar, double sigma2_A, int32_t subtract_mean,
                       ce_precision precision, void* out_map, double* out_mean, void* stream);

/* The whole hot path fused: generate `count` realizations (as ce_generate_fields), lognormal +
 * Poisson counts (as ce_lognormal_poisson, f = 1, the same seed for fields and counts), the
 * counts spectrum (as ce_estimate_pk with CE_MAP_COUNTS_DELTAG) and, when out_cov or out_cnorm
 * is given and count >= 2, its covariance.  The noise is generated inside the first FFT pass,
 * the crop / lognormal / Poisson / first forward transform run in the epilogue of the last
 * inverse pass, and the shell sums in the epilogue of the last forward pass.  Every output
 * pointer except out_pk is nullable; results equal the unfused calls within the stated
 * tolerances (counts and N_tot exactly).  Errors: as the unfused calls. */
ce_status ce_pipeline_run(ce_ctx* ctx, const ce_plan* plan, uint64_t seed, uint32_t request_id,
                          uint64_t first_realization, int64_t count, double nbar, int32_t nbins,
                          void* out_fields, void* out_delta, int32_t* out_counts,
                          int64_t* out_ntot, double* out_pk, double* out_cov, double* out_cnorm,
                          void* stream);

/* ce_pipeline_run for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same computation and results, bit for
 * bit, as ce_pipeline_run with the same arguments, but every scratch buffer (the pass
 * intermediates, the shell records, the N_tot accumulators and the shell table, counted on the
 * device) is carved from one static device array of the library, 1 GiB per device (CE_NOALLOC_BYTES),
 * held by every device the library runs on until the process ends.  The call allocates nothing:
 * no hipMalloc, hipFree or allocating library routine (the twiddle tables of the plan's lengths
 * are built when the plan is created).  Realizations are processed in chunks of as many pairs as
 * the array holds; a geometry of which one pair does not fit (the noise-pass and inner-axis
 * intermediates of one pair plus its spectra above 1 GiB, e.g. 3-D sides above ~300) returns
 * CE_E_UNSUPPORTED before anything is enqueued.  Equal-width shells only (no user edges, no mask).
 * All calls on one device share the array and it keeps the last call's contents (everything that
 * must start at zero is cleared by a kernel in each call): calls that overlap in time on one
 * device race, whatever their ctx or stream, so serialise them.  Profiling events are not
 * recorded for this call.  Errors: as ce_pipeline_run; CE_E_UNSUPPORTED as above. */
#define CE_NOALLOC_BYTES ((size_t)1 << 30)
ce_status ce_pipeline_run_noalloc(ce_ctx* ctx, const ce_plan* plan, uint64_t seed, uint32_t request_id,
                                  uint64_t first_realization, int64_t count, double nbar, int32_t nbins,
                                  void* out_fields, void* out_delta, int32_t* out_counts, int64_t* out_ntot,
                                  double* out_pk, double* out_cov, double* out_cnorm, void* stream);

/* ce_pipeline_run with the user shells of ce_estimate_pk_edges (kedges: host, nbins + 1 strictly
 * ascending |k| values >= 0; the paper bins in ln l) and, when mask_f is not NULL, on a masked
 * survey as ce_pipeline_run_masked (the paper's setting: a masked field binned in ln l).
 * Everything else as ce_pipeline_run (ce_pipeline_run_masked with a mask); linear edges on
 * (0, pi/h] give those results bitwise.  Errors: as ce_pipeline_run; CE_E_INVALID for bad
 * edges. */
ce_status ce_pipeline_run_edges(ce_ctx* ctx, const ce_plan* plan, const float* mask_f, uint64_t seed,
                                uint32_t request_id, uint64_t first_realization, int64_t count, double nbar,
                                int32_t nbins,
                                const double* kedges, void* out_fields, void* out_delta, int32_t* out_counts,
                                int64_t* out_ntot, double* out_pk, double* out_cov, double* out_cnorm,
                                void* stream);

/* ce_pipeline_run on a masked survey (Sec. 3.1, eq. sampling; Sec. 3.2, eq. Estim): mask_f
 * (device, N^d floats in [0, 1], row-major, caller-owned) is the surface fraction f of each
 * survey cell.  Counts are drawn with rate nbar f rho; the spectra are those of
 * delta_g = (N/f - N^)/N^ on cells with f != 0 (0 elsewhere), N^ = N_tot / sum f, the contrast
 * ce_estimate_pk forms for counts with a mask.  The fused pass transforms N / (f nbar) - 1 on
 * f != 0 and the binning pass completes the contrast with the transform of the indicator f != 0
 * (computed once per call, held in context scratch: N^(d-1) x 2 (N_last/2 + 1) complex values), so
 * counts are stored only into out_counts when given; P(k) equals ce_estimate_pk's to rounding
 * (not bitwise).  mask_f = NULL is ce_pipeline_run.  Errors: as ce_pipeline_run. */
ce_status ce_pipeline_run_masked(ce_ctx* ctx, const ce_plan* plan, const float* mask_f, uint64_t seed,
                                 uint32_t request_id, uint64_t first_realization, int64_t count, double nbar,
                                 int32_t nbins, void* out_fields, void* out_delta, int32_t* out_counts,
                                 int64_t* out_ntot, double* out_pk, double* out_cov, double* out_cnorm, void* stream);

/* The mask-dependent part of ce_pipeline_run_masked computed once for repeated calls on one
 * survey (Sec. 3.1, eq. sampling; Sec. 3.2, eq. Estim): the sum of f and the transform of the
 * indicator f != 0 for plan's grid and precision, held in device memory the handle owns
 * (N^(d-1) x 2 (N_last/2 + 1) complex values plus 257 doubles, counted against ctx's budget).
 * mask_f (device, N^d floats, caller-owned) is read on `stream` by work enqueued there; the
 * handle records an event after that work, and every ce_pipeline_run_prepared call (on any
 * stream, with any ctx of the device) waits for it on its own stream before reading the handle,
 * so no synchronisation is needed between preparing and using it.  ce_mask_release frees the
 * handle (it waits for work that still reads it); release every handle before destroying the
 * ctx it was prepared with (the handle's memory is accounted to that ctx).  Errors:
 * CE_E_INVALID (null arguments, plan on another device), CE_E_OOM, CE_E_DEVICE. */
typedef struct ce_mask ce_mask;
ce_status ce_mask_prepare(ce_ctx* ctx, const ce_plan* plan, const float* mask_f, void* stream, ce_mask** out);
void ce_mask_release(ce_mask* mask);

/* ce_pipeline_run_edges on a masked survey with a prepared mask: mask_f must hold the values
 * the handle was prepared from (the fused pass reads the rates from it); kedges nullable
 * (equal-width shells).  Results equal ce_pipeline_run_edges with mask_f bit for bit.
 * Errors: as ce_pipeline_run_edges; CE_E_INVALID when the handle was prepared for another
 * grid, precision or device. */
ce_status ce_pipeline_run_prepared(ce_ctx* ctx, const ce_plan* plan, const float* mask_f, const ce_mask* mask,
                                   uint64_t seed, uint32_t request_id, uint64_t first_realization, int64_t count,
                                   double nbar, int32_t nbins, const double* kedges, void* out_fields,
                                   void* out_delta, int32_t* out_counts, int64_t* out_ntot, double* out_pk,
                                   double* out_cov, double* out_cnorm, void* stream);

/* Batched form of ce_pipeline_run: many requests, each with its own plan (geometry, xi,
 * precision), seed, request id, realizations, nbar and outputs.  Requests that share
 * (ndim, N, h, precision, nbins) form a group that runs each pass of the pipeline as one launch
 * over all the group's pairs, every pair reading its own sqrt(lambda) octant, Philox key and
 * counter words, sigma^2 and nbar from a descriptor table; so a batch of many small requests
 * costs a few launches per distinct shape instead of a few per request.  Every item's results
 * (fields, delta, counts, N_tot, P(k), covariance) equal, bit for bit, those of ce_pipeline_run
 * (ce_pipeline_run_edges for an item with kedges) called for that item alone with the same ctx
 * options.  All items must be valid for ce_pipeline_run (nothing is launched otherwise).
 * Errors: as ce_pipeline_run. */
typedef struct {
  const ce_plan* plan;
  uint64_t seed;
  uint32_t request_id;
  uint64_t first_realization;  /* even */
  int64_t count;
  double nbar;
  int32_t nbins;
  double* out_pk;       /* device, count x nbins */
  int32_t* out_counts;  /* device, nullable, count x N^d */
  int64_t* out_ntot;    /* device, nullable, count */
  double* out_cov;      /* device, nullable, nbins^2 (written when count >= 2) */
  double* out_cnorm;    /* device, nullable, nbins^2 (written when count >= 2) */
  const double* kedges; /* host, nullable: nbins + 1 shell edges in |k| as ce_pipeline_run_edges
                           (read during the call); items with different edges form different groups */
  void* out_fields;     /* device, nullable, count x N^d in the plan precision (Gaussian fields) */
  void* out_delta;      /* device, nullable, count x N^d in the plan precision (lognormal contrast) */
} ce_batch_item;
ce_status ce_pipeline_run_batch(ce_ctx* ctx, const ce_batch_item* items, int64_t n, void* stream);

/* Captured form of ce_pipeline_run (HIP graph).  Creation runs the pipeline once (sizing a
 * private scratch area owned by the graph, so nothing is allocated while replaying), then
 * captures it with the given output buffers.  Each ce_pipeline_graph_launch replays it on
 * `stream` and then advances the realizations by `count`: launch k (k = 0, 1, ...) produces
 * realizations first_realization + k*count .. + count - 1 into the same output buffers (read them
 * before the next launch).  count must be even.  The outputs and the plan must stay valid while
 * the graph exists; replays of one graph must not overlap.  Errors: as ce_pipeline_run,
 * CE_E_DEVICE if capture fails. */
typedef struct ce_graph ce_graph;
ce_status ce_pipeline_graph_create(ce_ctx* ctx, const ce_plan* plan, uint64_t seed, uint32_t request_id,
                                   uint64_t first_realization, int64_t count, double nbar, int32_t nbins,
                                   void* out_fields, void* out_delta, int32_t* out_counts, int64_t* out_ntot,
                                   double* out_pk, double* out_cov, double* out_cnorm, ce_graph** out);
ce_status ce_pipeline_graph_launch(ce_graph* graph, void* stream);
void ce_pipeline_graph_destroy(ce_graph* graph);

/* Request loop (continuous batching).  A server owns `slots` contexts with one stream each,
 * a plan context and an LRU cache of plans (sqrt(lambda) octants) keyed by (geometry, xi,
 * precision).  ce_server_submit queues a request and returns at once; a scheduler thread
 * admits the queue head (FIFO) as soon as a slot is free and its device footprint -- pipeline
 * scratch, plus the plan if it is not cached -- fits hbm_budget_bytes (evicting unused plans
 * first), together with up to max_group - 1 more queued requests of at most 256 MiB of scratch
 * each whose plans are cached and whose scratch still fits; a slot runs its group as one
 * ce_pipeline_run_batch call (one request: ce_pipeline_run), slots concurrently on their
 * streams.  Every request's results equal those of the same ce_pipeline_run issued alone (the
 * computation of a request does not depend on what else runs).  A failing request (for
 * example CE_E_NOT_PSD at plan time) fails alone; a device-side sampler flag (see
 * ce_ctx_check) fails the group it ran in.  The output buffers of a request must stay valid
 * until it is done.  Latency = completion observed by the scheduler minus the submit time
 * (host steady clock). */
typedef struct ce_server ce_server;
typedef struct {
  int32_t slots;            /* requests in flight at once (default 4, at most 32) */
  size_t hbm_budget_bytes;  /* bound on slot scratch + cached plans (0: 3/4 of the free device memory) */
  size_t plan_cache_bytes;  /* bound on cached plans (0: 32 GiB or a quarter of the budget if less) */
  int32_t max_group;        /* most requests admitted together (0: 256; 1: one request per launch) */
} ce_server_config;
typedef struct {
  ce_geometry geom;
  ce_xi xi;                 /* a table is copied at submit time */
  ce_precision precision;
  uint64_t seed;
  uint32_t request_id;
  int64_t realizations;     /* realizations 0 .. realizations-1 of this (seed, request_id) */
  double nbar;
  int32_t nbins;
  double* out_pk;           /* device, realizations x nbins */
  int32_t* out_counts;      /* device, nullable, realizations x N^d */
  int64_t* out_ntot;        /* device, nullable, realizations */
  double* out_cov;          /* device, nullable, nbins^2 (used when realizations >= 2) */
  const double* kedges;     /* host, nullable: nbins + 1 shell edges in |k| (copied at submit) */
  void* out_fields;         /* device, nullable, realizations x N^d in `precision` (Gaussian fields) */
  void* out_delta;          /* device, nullable, realizations x N^d in `precision` (lognormal contrast) */
} ce_request;
typedef struct {
  int64_t submitted, completed, failed, cache_hits, cache_misses, admission_stalls, queued;
  double p50_ms, p99_ms;    /* over completed requests */
  double elapsed_s;         /* since the server was created */
  size_t held_bytes;        /* slot scratch + cached plans accounted by the admission */
  int64_t launches;         /* slot launches (one per admitted group) */
  int64_t largest_group;    /* most requests admitted together */
} ce_server_stats;
ce_status ce_server_create(int device, const ce_server_config* cfg, ce_server** out);
ce_status ce_server_submit(ce_server* server, const ce_request* request, uint64_t* ticket);
/* ce_server_submit for n requests (host array) queued together, in order, under one lock, so
 * that the scheduler sees them at once (clients with many small requests: they are admitted in
 * groups).  tickets: host array of n.  All or nothing: CE_E_INVALID queues none. */
ce_status ce_server_submit_many(ce_server* server, const ce_request* requests, int64_t n, uint64_t* tickets);
/* Non-blocking.  *state: 0 queued, 1 running, 2 done, 3 failed, 4 cancelled; once a finished
 * state (>= 2) has been returned the ticket is forgotten. */
ce_status ce_server_poll(ce_server* server, uint64_t ticket, int32_t* state, ce_status* status,
                         double* latency_ms);
/* Non-blocking.  Returns in completion order up to `max` requests that reached a final state
 * (done, failed, cancelled) and were not yet returned by ce_server_poll or an earlier drain:
 * their tickets (required), states, statuses and latencies (nullable arrays of `max`), and
 * their number in *n.  Drained tickets are forgotten. */
ce_status ce_server_drain(ce_server* server, int32_t max, uint64_t* tickets, int32_t* states, ce_status* statuses,
                          double* latency_ms, int32_t* n);
/* Cancel a request that is still queued (CE_E_INVALID otherwise). */
ce_status ce_server_cancel(ce_server* server, uint64_t ticket);
ce_status ce_server_stats_read(ce_server* server, ce_server_stats* out);
/* Stops admitting, cancels queued requests, waits for running ones, frees everything. */
void ce_server_destroy(ce_server* server);

/* Launch schedule of the pipeline passes for one shape (ndim, sides, precision): lines per workgroup
 * of the noise pass (even, 2..32), the inner-axis passes (3-D), the last inverse pass and the
 * binning pass (powers of two up to 64; 0 = automatic), the noise pass's tile order (0/1), pair
 * blocks (1..65536) and pairs per workgroup (1..64), and the binning pass's LDS budget
 * (16384..163840 bytes).  Every schedule
 * gives bitwise identical results (fields, delta, counts, N_tot, P(k), covariance); the radix
 * plans of the line FFTs are fixed per length, since another order would change the rounding. */
typedef struct {
  int32_t lines_noise, lines_inner, lines_last, lines_bins;
  int32_t noise_order, noise_block;
  int32_t noise_pairs;  /* pairs each noise-pass workgroup generates for its lines (1..64; 0 = automatic) */
  int32_t reserved;     /* padding: ignored on input, 0 on output */
  int64_t bin_lds;
  double ms, default_ms;  /* ce_autotune: median step time of the chosen and of the default schedule */
} ce_schedule;

/* Autotuner: times ce_pipeline_run steps of `count` realizations of plan (counts, N_tot, P(k) in
 * nbins shells and the covariance, into private buffers, seed 1) under candidate schedules --
 * coordinate descent from the context's options over each knob, two sweeps, the median of `reps`
 * HIP-event timed steps per candidate, a candidate kept when 1% faster -- and installs the fastest
 * for the plan's shape in ctx; every later call on that shape (pipelines, fields, spectra, the
 * batch groups) uses it.  out (nullable) receives it with both timings.  Synchronous; allocates
 * its buffers.  Errors: as ce_pipeline_run, CE_E_INVALID for reps outside 1..100. */
ce_status ce_autotune(ce_ctx* ctx, const ce_plan* plan, int64_t count, double nbar, int32_t nbins, int32_t reps,
                      ce_schedule* out);
/* Install (schedule non-NULL) or remove (NULL) the schedule of a shape; read it back.  Errors:
 * CE_E_INVALID (bad values; ce_schedule_get: no schedule for the shape), CE_E_UNSUPPORTED. */
ce_status ce_schedule_set(ce_ctx* ctx, const ce_geometry* geom, ce_precision precision, const ce_schedule* schedule);
ce_status ce_schedule_get(ce_ctx* ctx, const ce_geometry* geom, ce_precision precision, ce_schedule* out);
/* Persist the context's tuned schedules as JSON ({"format": "cefield-schedules", "version": 1,
 * "arch": ..., "entries": [{"ndim", "n": [3], "precision": "f32"|"f64", "lines": [4], "noise_order",
 * "noise_block", "noise_pairs", "bin_lds"}]}) and load such a file into a context (entries added or replaced; a
 * malformed file or an invalid entry loads nothing).  path: host string.  Errors: CE_E_INVALID. */
ce_status ce_schedule_save(ce_ctx* ctx, const char* path);
ce_status ce_schedule_load(ce_ctx* ctx, const char* path);

/* Shell table of a grid on the host: N_b and mean |k| per shell (same rule as ce_estimate_pk:
 * any even sides, cell sides in ratios of small integers).  nmodes, kmean: host arrays of nbins.
 * Errors: CE_E_INVALID, CE_E_UNSUPPORTED (an irrational cell-side ratio). */
ce_status ce_shell_table(const ce_geometry* geom, int32_t nbins, int64_t* nmodes, double* kmean);

/* FFT factorisation chosen for a line length (host; for inspection).  Writes up to 16 radices
 * into radices (host) and their number into *nstages.  CE_E_UNSUPPORTED if L is not covered. */
ce_status ce_fft_factors(int32_t length, int32_t* radices, int32_t* nstages);

/* Debug / test: Philox4x32-10 words for counters (ctr[0] + i, ctr[1], ctr[2], ctr[3]),
 * i in [0, n_calls), key = seed; out_words: device, 4 n_calls uint32 (x0..x3 per call). */
ce_status ce_debug_philox(uint64_t seed, const uint32_t ctr[4], int64_t n_calls,
                          uint32_t* out_words, void* stream);

/* Debug / test: the complex normals eps(q) of one pair (before scaling), M^d complex values
 * (interleaved re, im) in the plan precision, row-major over the embedding grid. */
ce_status ce_debug_noise(const ce_plan* plan, uint64_t seed, uint32_t request_id, uint64_t pair,
                         void* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CEFIELD_H */
