// Internal interface between the host API (ce_api.cpp) and the device code
// (ce_kernels.hip).  Plain structs passed by value as kernel arguments.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace ce {

constexpr int kMaxStages = 16;
constexpr int kEPT = 16;        // FFT elements held per thread
constexpr int kMaxWG = 512;
constexpr size_t kMaxLdsBytes = 160 * 1024;  // LDS of one gfx950 CU, the most one workgroup can use

// One FFT line length: radices of the mixed-radix Stockham stages and the
// device table of forward roots tw[k] = exp(-2 pi i k / L) in the pass precision.
struct FftDesc {
  int32_t L = 0;
  int32_t nst = 0;
  int32_t rad[kMaxStages] = {};
  // per stage s: the span Ns (product of the radices before it), the multiplier of the exact
  // quotient j / Ns = umulhi(j, nsm) for j < 4096 (nsm = ceil(2^32 / Ns); unused when Ns = 1), and
  // the offset of the stage's twiddles in stw (complex elements; stages with Ns > 1)
  int32_t ns[kMaxStages] = {};
  uint32_t nsm[kMaxStages] = {};
  int32_t soff[kMaxStages] = {};
  const void* tw = nullptr;    // roots exp(-2 pi i k / L), k < L
  const void* stw = nullptr;   // per-stage twiddles exp(-2 pi i r k / (Ns R)), see ce_device.hpp
};

// A batch of line transforms.  Lines are (a, b), a in [0, A), b in [0, B); line
// element i of the input is at in + item*in_item + (a*L + i)*B + b, of the output at
// out + item*out_item + (a*K + i)*B + b.  R consecutive flattened line ids a*B + b
// form one workgroup; nlanes threads serve one line.
struct LineGeom {
  int64_t A = 0, B = 0;
  int64_t in_item = 0, out_item = 0;
  int64_t nitems = 0;
  int64_t groups_per_item = 0;
  int32_t L = 0, K = 0;
  int32_t R = 0, nlanes = 0;
  int32_t lpitch = 0;          // LDS elements per line buffer
  int32_t nbuf = 1;            // LDS buffers per line: 1 (in place) or 2 (ping-pong: a prime above 31)
  int32_t item_minor = 0;      // tile order: 0 = item-major (groups of one item adjacent), 1 = group-major
  int32_t item_block = 1;      // item-major order over blocks of this many items (group-major inside a block)
  // noise pass: each workgroup takes pairs_wg consecutive items (nitems counts such tiles of items;
  // items_total is the number of items)
  int32_t pairs_wg = 1;
  int64_t items_total = 0;
  // noise pass: line groups taken in the order 0, G-1, 1, G-2, ... (G groups per item), so the
  // groups whose lines mirror each other (b and M - b read one sqrt(lambda) line) run together
  int32_t mirror_order = 0;
  int32_t threads = 0;         // workgroup size when above R nlanes (the fused epilogue spreads its cells)
};

// Noise prologue of the first inverse pass (lines along axis 0 of the embedding).
// Per-pair parameters when one launch covers pairs of several requests that share a
// shape (batched pipeline): each pair brings its own plan, Philox key and counter words,
// lognormal variance, density and counts destination.
struct PairDesc {
  const void* sq = nullptr;    // sqrt(lambda / M^d) octant of the request's plan (pass precision)
  int32_t* counts = nullptr;   // nullable: counts of the pair's real part; imaginary part at + ncells
  void* fields = nullptr;      // nullable: field of the pair's real part (pass precision); imaginary at + ncells
  void* delta = nullptr;       // nullable: lognormal contrast, laid out as fields
  uint32_t k0 = 0, k1 = 0, rid = 0, pair = 0;
  double s2half = 0, nbar = 0;
  int32_t nreal = 2;           // realizations of the pair that were requested (1: real part only)
  int32_t pad = 0;
};

// Destination of one realization slot (2 per pair) of a batched P(k) reduction.
struct SlotOut {
  double* pk = nullptr;        // nullable: slot not requested
  int64_t* ntot = nullptr;     // nullable
};

// One request of a batched covariance: R spectra of nb shells at pk.
struct CovItem {
  const double* pk = nullptr;
  int64_t R = 0;
  double* cov = nullptr;
  double* cnorm = nullptr;
};

struct NoiseArgs {
  uint32_t k0 = 0, k1 = 0, rid = 0;
  uint64_t first_pair = 0;
  const unsigned long long* pair_base = nullptr;  // nullable: device offset added to first_pair (graph replays)
  int32_t ndim = 0;
  int32_t M[3] = {1, 1, 1};
  int32_t O[3] = {1, 1, 1};    // octant sides N_i + 1
  const void* sq = nullptr;    // sqrt(lambda / M^d) on the octant, axis 0 fastest (pass precision)
  const PairDesc* desc = nullptr;  // nullable: per-pair parameters (override k0, k1, rid, pairs, sq)
};

// Epilogue of the last inverse pass (rows along the last axis).
struct RowEpi {
  int32_t mode = 0;            // 0: complex store, 1: fields, 2: fused lognormal/Poisson/forward
  int64_t ncells = 0;          // survey cells per realization
  int64_t rows_per_m0 = 1;     // input rows per axis-0 index (3-D: the axis-1 extent of the input)
  int32_t keep0 = 0, keep1 = 1;  // survey extents of axes 0 and 1 (3-D); rows outside are dropped
  int32_t keep_last = 0;       // survey extent of the last axis
  int64_t count = 0;           // realizations covered by this call
  int64_t real_off = 0;        // local realization index of item 0's real part
  void* fields = nullptr;      // nullable (pass precision)
  void* delta = nullptr;       // nullable (pass precision)
  int32_t* counts = nullptr;   // nullable
  const float* mask = nullptr; // nullable: surface fraction f per survey cell (rate nbar f rho)
  unsigned long long* ntot = nullptr;  // per local realization (zeroed by the host)
  uint32_t* flags = nullptr;
  const double* inv = nullptr;  // RN(1/k), k = 0..4096, for the Poisson recursion
  double s2half = 0, nbar = 0;
  uint32_t k0 = 0, k1 = 0, rid = 0;
  uint64_t first_pair = 0;
  const unsigned long long* pair_base = nullptr;  // nullable, as in NoiseArgs
  const PairDesc* desc = nullptr;  // nullable: per-pair parameters (batched pipeline, mode 2)
  FftDesc fwd;                 // forward FFT of the packed counts row (length K)
  void* H = nullptr;           // separated spectra rows: W = 2 (K/2 + 1) complex per row (null: counts only)
  int64_t H_item = 0;
  // with a mask and H: the row transformed is N / (f nest) - 1 on f != 0 (0 elsewhere), nest =
  // 1 / inv_nest the expected intensity; the binning pass completes the contrast with the
  // window transform (BinArgs.win)
  double inv_nest = 1;
};

// Prologue of the standalone spectrum's first pass (rows of two real maps packed).
struct PairLoad {
  int32_t kind = 0;            // 0: real maps in pass precision, 1: int32 counts -> contrast, 2: mask indicator
  const void* maps = nullptr;
  int64_t count = 0;           // maps in the stack
  int64_t ncells = 0;
  const int64_t* ntot = nullptr;   // counts kind
  const float* mask = nullptr;     // counts kind, nullable
  const double* fsum = nullptr;    // device: sum of the mask (null: ncells)
  void* H = nullptr;
  int64_t H_item = 0;
};

// Binning epilogue of the last forward pass (lines along axis 0 of the spectra).
struct BinArgs {
  int32_t ndim = 0, N = 0, nb = 0, W = 0;   // N: side of axis 0 (the line length); W = 2 (N_last/2 + 1)
  int32_t N1 = 1;                           // 3-D: side of axis 1
  // shell rule: mode q~ is in shell s - 1 for the smallest s with s^2 LL >= T0 q~_0^2 + T1 q~_1^2
  // + Tl q~_last^2 (LL = lcm(sides)^2, T_i = 4 nb^2 lcm^2 / N_i^2; cubic: LL = N^2, T = 4 nb^2)
  int64_t T0 = 0, T1 = 0, Tl = 0, LL = 1;
  // nullable: user shell edges as integer thresholds of t (nb + 1, device): shell b holds
  // TH_b < t <= TH_{b+1} instead of the linear rule
  const int64_t* th = nullptr;
  int32_t G = 1;               // lines per partial record (a divisor of the lines per workgroup)
  double* partials = nullptr;  // [item][block of G lines][2][nb]
  // Masked 2-D fused pipeline (nullable win): the lines hold the transform A of N / (f nest) - 1
  // on f != 0; the contrast's transform is D = r A + (r - 1) Wm with r = nest sum(f) / N_tot of
  // the line's realization and Wm the transform of the indicator f != 0, stored N x W complex in
  // the pass precision, [q0][column] like the spectra (the first K/2 + 1 columns are used).
  const void* win = nullptr;
  const unsigned long long* ntot = nullptr;  // per local realization (2 item + s)
  const double* fsum = nullptr;              // device: sum of the mask
  double nest = 1;
};

// Plan-time DCT-I of the lag octant along one axis (FP64).
struct DctArgs {
  const double* in = nullptr;
  double* out = nullptr;
  int32_t M = 0;               // even-extension length along the axis
};

// ---- launchers (ce_kernels.hip) -------------------------------------------
hipError_t launch_lag_octant(int ndim, const int32_t* O, const double* h, int kind, const double* p,
                             double* out, hipStream_t s);
hipError_t launch_dct_axis(const LineGeom& g, const FftDesc& f, const DctArgs& a, hipStream_t s);
hipError_t launch_lambda_stats(const double* lam, int ndim, const int32_t* O, int64_t n, double* stats,
                               unsigned long long* nneg, hipStream_t s);
hipError_t launch_sqrt_table(const double* lam, int ndim, const int32_t* O, double inv_cells, int prec, void* out,
                             hipStream_t s);
hipError_t launch_noise_pass(int prec, const LineGeom& g, const FftDesc& f, const NoiseArgs& n, void* out,
                             hipStream_t s);
hipError_t launch_line_pass(int prec, int dir, const LineGeom& g, const FftDesc& f, const void* in, void* out,
                            hipStream_t s);
hipError_t launch_row_inverse(int prec, const LineGeom& g, const FftDesc& f, const RowEpi& e, const void* in,
                              hipStream_t s);
hipError_t launch_pair_forward(int prec, const LineGeom& g, const FftDesc& f, const PairLoad& p, hipStream_t s);
hipError_t launch_bin_pass(int prec, const LineGeom& g, const FftDesc& f, const BinArgs& b, const void* in,
                           hipStream_t s);
size_t bin_pass_lds(const LineGeom& g, int N, int nb, int G, size_t elem);  // bytes of LDS per workgroup
hipError_t launch_bin_reduce(double* partials, int64_t nitems, int64_t groups, int nb, int64_t count,
                             const int64_t* nmodes, double norm, int scale_kind, const unsigned long long* ntot_u,
                             const SlotOut* slots, double ncells, double* pk, uint32_t* flags, hipStream_t s);
hipError_t launch_lognormal_poisson(int prec, const void* fields, int64_t count, int64_t ncells, double s2half,
                                    double nbar, const float* mask, uint32_t k0, uint32_t k1, uint32_t rid,
                                    uint64_t first_real, void* delta, int32_t* counts, unsigned long long* ntot,
                                    const double* inv, uint32_t* flags, hipStream_t s);
hipError_t launch_count_totals(const int32_t* counts, int64_t count, int64_t ncells, unsigned long long* ntot,
                               hipStream_t s);
hipError_t launch_copy_ntot(const unsigned long long* src, int64_t* dst, int64_t n, hipStream_t s);
hipError_t launch_covariance(const double* pk, int64_t count, int nb, double* cov, double* cnorm, hipStream_t s);
hipError_t launch_covariance_batch(const CovItem* items, int64_t nitems, int nb, hipStream_t s);
hipError_t launch_debug_philox(uint32_t k0, uint32_t k1, const uint32_t* ctr, int64_t n, uint32_t* out,
                               hipStream_t s);
hipError_t launch_debug_noise(int prec, const NoiseArgs& n, uint64_t pair, int64_t cells, void* out, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s);
// N_b of the linear shells on the device (n: three sides, 1 for missing axes; T: the shell weights)
hipError_t launch_shell_counts(const int32_t* n, const int64_t* T, int64_t LL, int nb, int64_t* counts,
                               hipStream_t s);
hipError_t launch_mask_sum(const float* mask, int64_t n, double* out, hipStream_t s);  // out: 257 doubles
hipError_t launch_window_columns(int prec, const void* in, void* out, int64_t N0, int64_t C, hipStream_t s);
// transformed lag tables (ce_xi.hip).  Quadrature of one axis of a quadrant of the cell-overlap
// integral: nodes u in (0, 1) and weights a = (Gauss-Legendre weight x du/dt) (1 - u).
constexpr int kCellQuadNodes = 48;
struct CellQuad {
  double u[kCellQuadNodes];
  double a[kCellQuadNodes];
};
hipError_t launch_lag_cell_average(const int32_t* O, const double* h, int kind, const double* p, const CellQuad& q,
                                   double near_cells, double log_step, double* out, hipStream_t s);
hipError_t launch_log1p(double* p, int64_t n, hipStream_t s);
// Gauss-Legendre rule on a unit panel: nodes x in (0, 1), weights w summing to 1.
constexpr int kHankelNodes = 8;
struct HankelRule {
  double x[kHankelNodes];
  double w[kHankelNodes];
};
// lambda on the box octant (half + 1)^ndim: P(sqrt(s) kscale) inv_hd via the distinct values svals
// (nvals of them; sidx maps s to its index), pvals receives P per distinct value.
hipError_t launch_box_spectrum(int ndim, int32_t half, const int64_t* svals, int64_t nvals, const int32_t* sidx,
                               double kscale, double inv_hd, int kind, const double* p, int lognormal, double scale,
                               double R, const HankelRule& g, double* pvals, double* lam, hipStream_t s);
// counts-in-cells (ce_cic.hip)
hipError_t launch_cic_histogram(const int32_t* counts, const float* mask, int64_t cells, int64_t count, int nhist,
                                unsigned long long* hist, hipStream_t s);
int64_t astar_partials(int64_t cells, int64_t count);  // doubles of partial sums for the mean
hipError_t launch_cumulative_information(const double* C, int nb, double* work, double* out, hipStream_t s);
int64_t cic_predict_blocks(int64_t cells, int nq);  // workgroups per quadrature node of launch_cic_predict
hipError_t launch_cic_predict(const float* mask, int64_t cells, double nbar, const double* nodes,
                              const double* weights, int nq, const double* lgam, int nhist, double* partials,
                              double* out, hipStream_t s);
hipError_t launch_astar(int prec, const int32_t* counts, const float* mask, int64_t cells, int64_t count,
                        double nbar, double s2, bool subtract, void* out, double* partials, double* mean,
                        hipStream_t s);
hipError_t launch_advance(unsigned long long* p, unsigned long long by, hipStream_t s);

}  // namespace ce
