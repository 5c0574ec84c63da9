// gfx950 kernels of the circulant-embedding generator.
//
// Every multi-dimensional FFT is a sequence of line passes.  A pass loads R
// lines into LDS (coalesced: rows are contiguous, strided lines are read R
// consecutive lines at a time), runs the in-place Stockham stages, and writes
// only the outputs that are kept.  The inverse transform of the embedding is
// pruned per axis to the survey half (Sec. 2: only the restriction to the
// survey is used); the first pass synthesises the noise in its prologue and
// the last pass crops / exponentiates / samples in its epilogue.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <stdint.h>

#include "ce_device.hpp"
#include "ce_internal.hpp"

namespace ce {

// ---------------------------------------------------------------------------
// helpers

struct PassPos {
  int64_t item, grp, line0;
  int nl;
};

__device__ __forceinline__ PassPos pass_pos(const LineGeom& g) {
  const int64_t t = xcd_tile((int64_t)blockIdx.x, (int64_t)gridDim.x);
  PassPos p;
  if (g.item_minor) {
    p.grp = t / g.nitems;
    p.item = t - p.grp * g.nitems;
  } else if (g.item_block > 1) {
    // blocks of item_block items: within a block, the items of one line group are adjacent
    const int64_t per = g.groups_per_item * g.item_block;
    const int64_t blk = t / per, rem = t - blk * per;
    const int64_t i0 = blk * g.item_block;
    const int64_t left = g.nitems - i0;
    const int64_t kb = left < g.item_block ? left : g.item_block;
    p.grp = rem / kb;
    p.item = i0 + (rem - p.grp * kb);
  } else {
    p.item = t / g.groups_per_item;
    p.grp = t - p.item * g.groups_per_item;
  }
  if (g.mirror_order) p.grp = (p.grp & 1) ? g.groups_per_item - 1 - (p.grp >> 1) : (p.grp >> 1);
  p.line0 = p.grp * g.R;
  const int64_t nlines = g.A * g.B;
  const int64_t left = nlines - p.line0;
  p.nl = (int)(left < g.R ? left : g.R);
  return p;
}

// Line line0 + r of a group as (a, b), b = its index mod B: the group's first line is divided once
// (uniform over the workgroup; no per-lane 64-bit division) and each line steps from it.
__device__ __forceinline__ void split_line(int64_t line0, int r, int64_t B, int64_t& a, int64_t& b) {
  a = line0 / B;
  b = line0 - a * B + r;
  while (b >= B) {
    b -= B;
    ++a;
  }
}

template <typename T>
__device__ __forceinline__ cpx<T>* lds_lines() {
  extern __shared__ __align__(16) unsigned char ce_smem[];
  return reinterpret_cast<cpx<T>*>(ce_smem);
}

// Part of the lines of one group held in registers: elements k0 .. k0 + kPre - 1 of the
// thread (row lines: element lane + k nlanes; strided lines: c0 + k (blockDim / R)); at
// most kEPT per thread in all.  kPre keeps the array at 32 registers, which the compiler
// keeps in VGPRs (a larger private array would go to scratch memory).
template <typename T>
struct LinePrefetch {
  static constexpr int kPre = sizeof(T) == 4 ? kEPT : kEPT / 2;
  T x[kPre], y[kPre];  // separate scalar arrays: a struct array of doubles stays in scratch
};

template <typename T>
__device__ __forceinline__ void fetch_lines(LinePrefetch<T>& pf, const cpx<T>* __restrict__ in, const LineGeom& g,
                                            int64_t item, int64_t line0, int nl, int k0) {
  constexpr int P = LinePrefetch<T>::kPre;
  const cpx<T>* base = in + item * g.in_item;
  const int L = g.L;
  const int tid = threadIdx.x;
  if (g.B == 1) {
    const int r = tid / g.nlanes, lane = tid - r * g.nlanes;
    if (r < nl) {
      const cpx<T>* src = base + (line0 + r) * (int64_t)L;
#pragma unroll
      for (int k = 0; k < P; ++k) {
        const int i = lane + (k0 + k) * g.nlanes;
        if (i < L) {
          const cpx<T> v = src[i];
          pf.x[k] = v.x;
          pf.y[k] = v.y;
        }
      }
    }
  } else {
    const int R = g.R;
    const int r = tid % R, c0 = tid / R, step = (int)blockDim.x / R;
    if (r < nl) {
      int64_t a, b;
      split_line(line0, r, g.B, a, b);
      const cpx<T>* src = base + a * (int64_t)L * g.B + b;
#pragma unroll
      for (int k = 0; k < P; ++k) {
        const int i = c0 + (k0 + k) * step;
        if (i < L) {
          const cpx<T> v = src[(int64_t)i * g.B];
          pf.x[k] = v.x;
          pf.y[k] = v.y;
        }
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ void put_lines(cpx<T>* lds, const LinePrefetch<T>& pf, const LineGeom& g, int nl,
                                          int k0) {
  constexpr int P = LinePrefetch<T>::kPre;
  const int L = g.L;
  const int tid = threadIdx.x;
  if (g.B == 1) {
    const int r = tid / g.nlanes, lane = tid - r * g.nlanes;
    if (r < nl) {
      cpx<T>* dst = lds + r * g.lpitch;
#pragma unroll
      for (int k = 0; k < P; ++k) {
        const int i = lane + (k0 + k) * g.nlanes;
        if (i < L) dst[pidx(i)] = {pf.x[k], pf.y[k]};
      }
    }
  } else {
    const int R = g.R;
    const int r = tid % R, c0 = tid / R, step = (int)blockDim.x / R;
    if (r < nl) {
      cpx<T>* dst = lds + r * g.lpitch;
#pragma unroll
      for (int k = 0; k < P; ++k) {
        const int i = c0 + (k0 + k) * step;
        if (i < L) dst[pidx(i)] = {pf.x[k], pf.y[k]};
      }
    }
  }
}

// Load nl lines of length L (complex) into LDS: every element of the thread is requested
// before the first one is stored, so up to kEPT loads per thread are in flight.
template <typename T>
__device__ __forceinline__ void load_lines(cpx<T>* lds, const cpx<T>* __restrict__ in, const LineGeom& g,
                                           const PassPos& pp) {
  LinePrefetch<T> pf;
#pragma unroll
  for (int k0 = 0; k0 < kEPT; k0 += LinePrefetch<T>::kPre) {
    fetch_lines(pf, in, g, pp.item, pp.line0, pp.nl, k0);
    put_lines(lds, pf, g, pp.nl, k0);
  }
}

// Store the first K elements of each LDS line.
template <typename T>
__device__ __forceinline__ void store_lines(const cpx<T>* lds, cpx<T>* __restrict__ out, const LineGeom& g,
                                            const PassPos& pp) {
  cpx<T>* base = out + pp.item * g.out_item;
  const int K = g.K;
  const int tid = threadIdx.x, nthr = blockDim.x;
  if (g.B == 1) {
    const int r = tid / g.nlanes, lane = tid - r * g.nlanes;
    if (r < pp.nl) {
      cpx<T>* dst = base + (pp.line0 + r) * (int64_t)K;
      const cpx<T>* src = lds + r * g.lpitch;
      for (int i = lane; i < K; i += g.nlanes) dst[i] = src[pidx(i)];
    }
  } else {
    const int R = g.R;
    const int r = tid % R, c0 = tid / R, step = nthr / R;
    if (r < pp.nl) {
      int64_t a, b;
      split_line(pp.line0, r, g.B, a, b);
      cpx<T>* dst = base + a * (int64_t)K * g.B + b;
      const cpx<T>* src = lds + r * g.lpitch;
      for (int i = c0; i < K; i += step) dst[(int64_t)i * g.B] = src[pidx(i)];
    }
  }
}

__device__ __forceinline__ int mirror(int q, int M) { return q <= M - q ? q : M - q; }

// LDS buffers of line r: a (always), b (ping-pong kernels only, after all a buffers).
template <typename T>
__device__ __forceinline__ cpx<T>* buf_a(cpx<T>* lds, const LineGeom& g, int r) { return lds + r * g.lpitch; }
template <typename T>
__device__ __forceinline__ cpx<T>* buf_b(cpx<T>* lds, const LineGeom& g, int r) {
  return lds + (g.R + r) * g.lpitch;
}
// Base of the buffer set that holds the result after an FFT of f.  MIX: 0 power-of-two
// lengths (compile-time stages, in place), 1 lengths whose factors are 2, 3, 4, 5, 7, 8 (in
// place), 2 the same with primes 11..31 (in place), 3 lengths with a prime factor above 31
// (ping-pong: the result is in buffer b after an odd number of stages).
template <typename T, int MIX>
__device__ __forceinline__ cpx<T>* result_base(cpx<T>* lds, const LineGeom& g, const FftDesc& f) {
  return (MIX == 3 && (f.nst & 1)) ? lds + g.R * g.lpitch : lds;
}

// ---------------------------------------------------------------------------
// Poisson sampling by FP64 chunked inversion (no contraction: every step is a
// separately rounded IEEE operation, so an FP64 reference reproduces it).

constexpr int kMaxPoissonSteps = 4096;
constexpr double kChunkMean = 64.0;
constexpr double kMaxMu = 6.7108864e7;  // 2^20 chunks

// RN(1/k): entries k <= kInvLds come from a copy of the host table RN(1/k) that the kernel
// keeps in LDS (inv_lds); beyond it (never reached with chunk means of 64) the correctly
// rounded quotient, which equals the table entry.
constexpr int kInvLds = 256;
__device__ __forceinline__ double inv_k(const double* inv_lds, int k) {
  return k <= kInvLds ? inv_lds[k] : 1.0 / (double)k;
}

__device__ __forceinline__ int poisson_chunk(double u, double m, const double* inv_lds, uint32_t* flags) {
  // every step separately rounded: no contraction of the products into the sums
#pragma clang fp contract(off)
  double p = exp(-m);
  double F = p;
  int k = 0;
  while (u > F && p > 0.0) {
    ++k;
    if (k > kMaxPoissonSteps) {
      atomicOr(flags, 1u);
      break;
    }
    p = (p * m) * inv_k(inv_lds, k);
    F = F + p;
  }
  return k;
}

__device__ __forceinline__ int chunk_count(double mu) {
  return mu > 0.0 ? (int)ceil(mu * (1.0 / kChunkMean)) : 0;
}

__device__ __forceinline__ double chunk_mean(double mu, int c, int K) {
#pragma clang fp contract(off)
  return c == K - 1 ? mu - kChunkMean * (double)(K - 1) : kChunkMean;
}

// Counts of the two realizations of a pair at one cell; counter (cell, pair, rid, 1 + chunk).
constexpr int kStraight = 4;  // steps of the inversion taken without branches (1/j folds to RN(1/j))
__device__ __forceinline__ void poisson_pair(double mua, double mub, bool has_b, uint32_t cell, uint32_t pair,
                                             uint32_t rid, uint32_t k0, uint32_t k1, const double* inv_lds,
                                             uint32_t* flags, int& na, int& nb) {
#pragma clang fp contract(off)
  na = 0;
  nb = 0;
  if (!(mua <= kMaxMu) || (has_b && !(mub <= kMaxMu))) {
    atomicOr(flags, 2u);
    na = -1;
    nb = -1;
    return;
  }
  const int Ka = chunk_count(mua);
  const int Kb = has_b ? chunk_count(mub) : 0;
  const int Kmax = Ka > Kb ? Ka : Kb;
  for (int c = 0; c < Kmax; ++c) {
    const Words4 w = philox4x32_10(cell, pair, rid, 1u + (uint32_t)c, k0, k1);
    // the two inversions run in one loop, so a wave iterates max(steps a, steps b) times
    // rather than their sum; each realization's sequence of operations is that of
    // poisson_chunk
    const bool da = c < Ka, db = c < Kb;
    const double ua = unit52(w.x0, w.x1), ub = unit52(w.x2, w.x3);
    const double ma = da ? chunk_mean(mua, c, Ka) : 0.0;
    const double mb = db ? chunk_mean(mub, c, Kb) : 0.0;
    double pa = exp(-ma), pb = exp(-mb);
    double Fa = pa, Fb = pb;
    int ka = 0, kb = 0;
    bool ra = da && ua > Fa && pa > 0.0;
    bool rb = db && ub > Fb && pb > 0.0;
    // the first kStraight steps run for every lane without branches (a lane that has
    // stopped keeps its values), which is where nearly all draws at small means end;
    // only lanes still going enter the loop.  The values each lane keeps are those of
    // the step-by-step recursion.
#pragma unroll
    for (int j = 1; j <= kStraight; ++j) {
      const double qa = (pa * ma) * (1.0 / (double)j), qb = (pb * mb) * (1.0 / (double)j);
      const double Ga = Fa + qa, Gb = Fb + qb;
      if (ra) {
        ka = j;
        pa = qa;
        Fa = Ga;
        ra = ua > Ga && qa > 0.0;
      }
      if (rb) {
        kb = j;
        pb = qb;
        Fb = Gb;
        rb = ub > Gb && qb > 0.0;
      }
    }
    while (ra || rb) {
      if (ra) {
        ++ka;
        if (ka > kMaxPoissonSteps) {
          atomicOr(flags, 1u);
          ra = false;
        } else {
          pa = (pa * ma) * inv_k(inv_lds, ka);
          Fa = Fa + pa;
          ra = ua > Fa && pa > 0.0;
        }
      }
      if (rb) {
        ++kb;
        if (kb > kMaxPoissonSteps) {
          atomicOr(flags, 1u);
          rb = false;
        } else {
          pb = (pb * mb) * inv_k(inv_lds, kb);
          Fb = Fb + pb;
          rb = ub > Fb && pb > 0.0;
        }
      }
    }
    na += ka;
    nb += kb;
  }
}

template <typename T>
__device__ __forceinline__ T lognormal_delta(T g, T s2half);
template <>
__device__ __forceinline__ float lognormal_delta<float>(float g, float s2half) {
  return __expf(g - s2half) - 1.0f;
}
template <>
__device__ __forceinline__ double lognormal_delta<double>(double g, double s2half) {
  return exp(g - s2half) - 1.0;
}

// mu = (nbar f) (1 + delta) from delta as stored
__device__ __forceinline__ double intensity(double nbar, double f, double delta) {
#pragma clang fp contract(off)
  return (nbar * f) * (1.0 + delta);
}

// ---------------------------------------------------------------------------
// Plan kernels (FP64)

__global__ void k_lag_octant(int ndim, int32_t O0, int32_t O1, int32_t O2, double h0, double h1, double h2,
                             int kind, double p0, double p1, double p2, double p3, double* __restrict__ out) {
  const int64_t n = (int64_t)O0 * O1 * O2;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l2 = idx % O2, t = idx / O2;
    const int64_t l1 = t % O1, l0 = t / O1;
    const double x0 = h0 * (double)l0, x1 = h1 * (double)l1, x2 = h2 * (double)l2;
    double rr = x0 * x0;
    if (ndim > 1) rr += x1 * x1;
    if (ndim > 2) rr += x2 * x2;
    const double r = sqrt(rr);
    double v;
    if (kind == 1) {
      v = p0 * exp(-r / p1);
    } else {
      v = p0 * pow(1.0 + r / p1, -p2);
      if (p3 > 0) v *= exp(-r / p3);
    }
    out[idx] = v;
  }
}

// DCT-I along one axis of the lag octant via a length-M complex FFT of the even
// extension e(m) = c(min(m, M - m)); keeps Re of outputs q in [0, M/2].
template <int MIX>
__global__ void __launch_bounds__(512) k_dct_axis(LineGeom g, FftDesc f, DctArgs d) {
  cpx<double>* lds = lds_lines<double>();
  const PassPos pp = pass_pos(g);
  const int Od = d.M / 2 + 1;
  const int tid = threadIdx.x, nthr = blockDim.x;
  {
    const int R = g.R;
    const int r = tid % R, c0 = tid / R, step = nthr / R;
    if (r < pp.nl) {
      int64_t a, b;
      split_line(pp.line0, r, g.B, a, b);
      const double* src = d.in + a * (int64_t)Od * g.B + b;
      cpx<double>* dst = lds + r * g.lpitch;
      for (int i = c0; i < d.M; i += step) dst[pidx(i)] = {src[(int64_t)mirror(i, d.M) * g.B], 0.0};
    }
  }
  __syncthreads();
  const int r = tid / g.nlanes, lane = tid - r * g.nlanes;
  const bool active = r < pp.nl;
  line_fft<double, -1, MIX>(buf_a(lds, g, r), buf_b(lds, g, r), f, lane, g.nlanes, active, d.M);
  const cpx<double>* res = result_base<double, MIX>(lds, g, f);
  {
    const int R = g.R;
    const int rr = tid % R, c0 = tid / R, step = nthr / R;
    if (rr < pp.nl) {
      int64_t a, b;
      split_line(pp.line0, rr, g.B, a, b);
      double* dst = d.out + a * (int64_t)Od * g.B + b;
      const cpx<double>* src = res + rr * g.lpitch;
      for (int i = c0; i < Od; i += step) dst[(int64_t)i * g.B] = src[pidx(i)].x;
    }
  }
}

// min / max of the eigenvalue octant per block; negatives counted with their
// multiplicity on the full grid (2 per axis unless q_i is 0 or N_i).
__global__ void k_lambda_stats(const double* __restrict__ lam, int ndim, int32_t O0, int32_t O1, int32_t O2,
                               int64_t n, double* __restrict__ stats, unsigned long long* __restrict__ nneg) {
  __shared__ double smin[256], smax[256];
  __shared__ unsigned long long sneg;
  if (threadIdx.x == 0) sneg = 0;
  __syncthreads();
  double mn = INFINITY, mx = -INFINITY;
  unsigned long long neg = 0;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const double v = lam[idx];
    if (!isfinite(v)) {  // a NaN or infinite eigenvalue: report the bounds as -inf / +inf
      mn = -INFINITY;
      mx = INFINITY;
    }
    mn = fmin(mn, v);
    mx = fmax(mx, v);
    if (v < 0) {
      const int64_t l2 = idx % O2, t = idx / O2;
      const int64_t l1 = t % O1, l0 = t / O1;
      unsigned long long m = (l0 == 0 || l0 == O0 - 1) ? 1 : 2;
      if (ndim > 1) m *= (l1 == 0 || l1 == O1 - 1) ? 1 : 2;
      if (ndim > 2) m *= (l2 == 0 || l2 == O2 - 1) ? 1 : 2;
      neg += m;
    }
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  if (neg) atomicAdd(&sneg, neg);
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stats[2 * blockIdx.x] = smin[0];
    stats[2 * blockIdx.x + 1] = smax[0];
    if (sneg) atomicAdd(nneg, sneg);
  }
}

// sqrt(max(lambda, 0) / M^d), stored with axis 0 fastest: out[(o1 O2 + o2) O0 + o0] (the noise
// pass reads one embedding line -- fixed (o1, o2), all o0 -- contiguously).
template <typename T>
__global__ void k_sqrt_table(const double* __restrict__ lam, int32_t O0, int32_t O1, int32_t O2, double inv_cells,
                             T* __restrict__ out) {
  const int64_t n = (int64_t)O0 * O1 * O2;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o0 = i % O0, rest = i / O0;  // rest = o1 O2 + o2
    const double v = lam[o0 * ((int64_t)O1 * O2) + rest];
    out[i] = (T)sqrt((v > 0.0 ? v : 0.0) * inv_cells);
  }
}

// ---------------------------------------------------------------------------
// First inverse pass: noise synthesised in the prologue (Sec. 2, eq. Papos2),
// lines along axis 0 of the embedding; cells 2p and 2p+1 share one Philox call
// and lie on adjacent lines.

// Offset of embedding line b (the flattened axes 1..d-1) in the sqrt(lambda) octant (axis 0 fastest).
__device__ __forceinline__ uint32_t sq_line_offset(const NoiseArgs& n, uint32_t b) {
  if (n.ndim == 2) return (uint32_t)mirror((int)b, n.M[1]) * (uint32_t)n.O[0];
  const uint32_t q1 = b / (uint32_t)n.M[2], q2 = b - q1 * (uint32_t)n.M[2];
  return ((uint32_t)mirror((int)q1, n.M[1]) * (uint32_t)n.O[2] + (uint32_t)mirror((int)q2, n.M[2])) *
         (uint32_t)n.O[0];
}

template <typename T, int MIX>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2))) k_noise_pass(LineGeom g, FftDesc f, NoiseArgs n, cpx<T>* __restrict__ out) {
  cpx<T>* lds = lds_lines<T>();
  const PassPos pp0 = pass_pos(g);
  const int L = g.L;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int H = g.R / 2;  // line pairs
  const int rp = tid % H, c0 = tid / H, step = nthr / H;
  const bool has_lines = 2 * rp < pp0.nl;
  // even line id b = flattened index over axes 1..d-1; cells 2p, 2p+1 = (i, b), (i, b+1)
  const uint32_t b = (uint32_t)(pp0.line0 + 2 * rp);
  const uint32_t half_b = (uint32_t)(g.B >> 1);
  const uint32_t off0 = sq_line_offset(n, b), off1 = sq_line_offset(n, b + 1);
  // The workgroup generates pairs_wg pairs of the same lines one after another: the octant
  // values it reads for the first pair are still in the caches for the next ones, so the octant
  // comes from HBM once per pairs_wg pairs instead of once per pair.  The prime-butterfly
  // variants take one pair (their register footprint leaves no room for the loop).
  const int npw = MIX >= 2 ? 1 : g.pairs_wg;
  for (int ip = 0; ip < npw; ++ip) {
    PassPos pp = pp0;
    pp.item = pp0.item * npw + ip;
    if (pp.item >= g.items_total) break;  // uniform over the workgroup
    const PairDesc* pd = n.desc ? n.desc + pp.item : nullptr;
    const T* __restrict__ sq = static_cast<const T*>(pd ? pd->sq : n.sq);
    const uint32_t pair =
        pd ? pd->pair : (uint32_t)(n.first_pair + (n.pair_base ? *n.pair_base : 0ull) + pp.item);
    const uint32_t rid = pd ? pd->rid : n.rid, k0 = pd ? pd->k0 : n.k0, k1 = pd ? pd->k1 : n.k1;
    if (ip > 0) __syncthreads();  // the previous pair's lines have been stored
    if (has_lines) {
      cpx<T>* d0 = lds + (2 * rp) * g.lpitch;
      cpx<T>* d1 = d0 + g.lpitch;
      for (int i = c0; i < L; i += step) {
        // both octant values are loaded before the generator runs (and before any LDS
        // store, which the compiler could not move them across), so their latency is hidden
        const uint32_t o0 = (uint32_t)mirror(i, n.M[0]);
        const T s0 = sq[off0 + o0], s1 = sq[off1 + o0];
        const uint32_t p = (uint32_t)i * half_b + (b >> 1);
        const Words4 w = philox4x32_10(p, pair, rid, 0u, k0, k1);
        const cpx<T> e0 = normal_pair<T>(w.x0, w.x1);
        const cpx<T> e1 = normal_pair<T>(w.x2, w.x3);
        d0[pidx(i)] = c_scale(e0, s0);
        d1[pidx(i)] = c_scale(e1, s1);
      }
    }
    __syncthreads();
    // the thread index is made opaque per pair so that the FFT's per-lane twiddles are not
    // hoisted out of the pair loop (they would stay live across it and spill)
    int tv = tid;
    asm volatile("" : "+v"(tv));
    const int r = tv / g.nlanes, lane = tv - r * g.nlanes;
    line_fft<T, +1, MIX>(buf_a(lds, g, r), buf_b(lds, g, r), f, lane, g.nlanes, r < pp.nl, g.K);
    store_lines(result_base<T, MIX>(lds, g, f), out, g, pp);
  }
}

// Generic complex line pass (inner axes of 3-D transforms), pruned to K outputs.
// In place is allowed: a group reads all its lines before writing them.
template <typename T, int S, int MIX>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2))) k_line_pass(LineGeom g, FftDesc f, const cpx<T>* in, cpx<T>* out) {
  cpx<T>* lds = lds_lines<T>();
  const PassPos pp = pass_pos(g);
  load_lines(lds, in, g, pp);
  __syncthreads();
  const int r = threadIdx.x / g.nlanes, lane = threadIdx.x - r * g.nlanes;
  line_fft<T, S, MIX>(buf_a(lds, g, r), buf_b(lds, g, r), f, lane, g.nlanes, r < pp.nl, g.K);
  store_lines(result_base<T, MIX>(lds, g, f), out, g, pp);
}

// ---------------------------------------------------------------------------
// Forward transform of a packed pair row (a + i b) followed by the Hermitian
// separation F_a(k) = (G(k) + conj G(-k))/2, F_b(k) = (G(k) - conj G(-k))/(2i)
// for k in [0, K/2]; row written as [F_a(0..K/2) | F_b(0..K/2)].
template <typename T, int MIX>
__device__ __forceinline__ void forward_separate(cpx<T>* line, cpx<T>* other, const FftDesc& fwd, int lane,
                                                 int nlanes, bool active, cpx<T>* __restrict__ Hrow) {
  line = line_fft<T, -1, MIX>(line, other, fwd, lane, nlanes, active, fwd.L);
  if (active) {
    const int K = fwd.L, Kh = K / 2 + 1;
    for (int c = lane; c < 2 * Kh; c += nlanes) {
      const int s = c >= Kh, k = c - s * Kh;
      const cpx<T> gk = line[pidx(k)];
      const cpx<T> gm = line[pidx(k ? K - k : 0)];
      cpx<T> v;
      if (!s) {
        v = {(gk.x + gm.x) * T(0.5), (gk.y - gm.y) * T(0.5)};
      } else {
        // (gk - conj gm) / (2 i)
        v = {(gk.y + gm.y) * T(0.5), -(gk.x - gm.x) * T(0.5)};
      }
      Hrow[c] = v;
    }
  }
}

// Last inverse pass: rows along the last axis, pruned to the survey, with the
// crop epilogue (Sec. 2) and optionally the lognormal / Poisson step (Sec. 3.1)
// and the first forward transform of the counts (Sec. 3.2).
template <typename T, int MIX>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2))) k_row_inverse(LineGeom g, FftDesc f, RowEpi e, const cpx<T>* in) {
  cpx<T>* lds = lds_lines<T>();
  __shared__ unsigned long long tot[2];
  __shared__ double inv_s[kInvLds + 1];
  const PassPos pp = pass_pos(g);
  if (threadIdx.x < 2) tot[threadIdx.x] = 0;
  if (e.mode == 2)
    for (int i = threadIdx.x; i <= kInvLds; i += blockDim.x) inv_s[i] = e.inv[i];
  load_lines(lds, in, g, pp);
  __syncthreads();
  const int r = threadIdx.x / g.nlanes, lane = threadIdx.x - r * g.nlanes;
  const bool active = r < pp.nl;
  cpx<T>* line = line_fft<T, +1, MIX>(buf_a(lds, g, r), buf_b(lds, g, r), f, lane, g.nlanes, active, g.K);
  cpx<T>* other = (line == buf_a(lds, g, r)) ? buf_b(lds, g, r) : buf_a(lds, g, r);

  const int K = g.K;
  const int64_t row = pp.line0 + r;
  const int64_t ra = e.real_off + 2 * pp.item;  // local realization of the real part
  const PairDesc* pd = e.desc ? e.desc + pp.item : nullptr;
  const bool has_b = pd ? pd->nreal > 1 : ra + 1 < e.count;
  if (e.mode == 1) {
    // rows outside the survey exist only in the unpruned form
    const int64_t m0 = row / e.rows_per_m0, m1 = row - m0 * e.rows_per_m0;
    if (active && m0 < e.keep0 && m1 < e.keep1) {
      const int64_t crow = m0 * e.keep1 + m1;
      T* fa = static_cast<T*>(e.fields) + ra * e.ncells + crow * e.keep_last;
      T* fb = fa + e.ncells;
      for (int i = lane; i < e.keep_last; i += g.nlanes) {
        const cpx<T> z = line[pidx(i)];
        fa[i] = z.x;
        if (has_b) fb[i] = z.y;
      }
    }
    return;
  }
  // fused epilogue: the cells of the group's rows spread over every thread of the workgroup
  // (more threads per row than line lanes when rows are short)
  unsigned long long sa = 0, sb = 0;
  {
    const uint32_t pair =
        pd ? pd->pair : (uint32_t)(e.first_pair + (e.pair_base ? *e.pair_base : 0ull) + pp.item);
    const uint32_t rid = pd ? pd->rid : e.rid, k0 = pd ? pd->k0 : e.k0, k1 = pd ? pd->k1 : e.k1;
    const T s2h = (T)(pd ? pd->s2half : e.s2half);
    const double nbar = pd ? pd->nbar : e.nbar;
    T* fbase = pd ? static_cast<T*>(pd->fields) : (e.fields ? static_cast<T*>(e.fields) + ra * e.ncells : nullptr);
    T* dbase = pd ? static_cast<T*>(pd->delta) : (e.delta ? static_cast<T*>(e.delta) + ra * e.ncells : nullptr);
    int32_t* cbase = pd ? pd->counts : (e.counts ? e.counts + ra * e.ncells : nullptr);
    cpx<T>* set = line - r * g.lpitch;  // row 0 of the buffer set that holds the result
    // tpr threads per row (the line lanes when the workgroup has no more threads than them)
    const int tpr = (int)blockDim.x / g.R;
    const int rr = (int)threadIdx.x / tpr, i0 = (int)threadIdx.x - rr * tpr;
    const int64_t rowc = pp.line0 + rr;
    cpx<T>* lr = set + rr * g.lpitch;
    T* fa = fbase && rr < pp.nl ? fbase + rowc * K : nullptr;
    T* da = dbase && rr < pp.nl ? dbase + rowc * K : nullptr;
    int32_t* ca = cbase && rr < pp.nl ? cbase + rowc * K : nullptr;
    const float* fr = e.mask && rr < pp.nl ? e.mask + rowc * K : nullptr;
    for (int i = i0; rr < pp.nl && i < K; i += tpr) {
      const cpx<T> z = lr[pidx(i)];
      const T dla = lognormal_delta<T>(z.x, s2h);
      const T dlb = lognormal_delta<T>(z.y, s2h);
      const double f = fr ? (double)fr[i] : 1.0;
      const double mua = intensity(nbar, f, (double)dla);
      const double mub = intensity(nbar, f, (double)dlb);
      int na, nb;
      poisson_pair(mua, mub, has_b, (uint32_t)(rowc * K + i), pair, rid, k0, k1, inv_s, e.flags, na, nb);
      if (fa) {
        fa[i] = z.x;
        if (has_b) fa[i + e.ncells] = z.y;
      }
      if (da) {
        da[i] = dla;
        if (has_b) da[i + e.ncells] = dlb;
      }
      if (ca) {
        ca[i] = na;
        if (has_b) ca[i + e.ncells] = nb;
      }
      sa += (unsigned long long)na;
      sb += (unsigned long long)nb;
      if (fr) {
        // masked: N / (f nest) - 1 on f != 0, 0 elsewhere (the binning pass adds the window term)
        T va = T(0), vb = T(0);
        const T ft = (T)f;
        if (ft != T(0)) {
          const T q = (sizeof(T) == 4 ? (T)__builtin_amdgcn_rcpf((float)ft) : T(1) / ft) * (T)e.inv_nest;
          va = (T)na * q - T(1);
          if (has_b) vb = (T)nb * q - T(1);
        }
        lr[pidx(i)] = {va, vb};
      } else {
        lr[pidx(i)] = {(T)na, (T)nb};
      }
    }
  }
  if (sa) atomicAdd(&tot[0], sa);
  if (sb) atomicAdd(&tot[1], sb);
  __syncthreads();
  if (threadIdx.x == 0 && tot[0]) atomicAdd(&e.ntot[ra], tot[0]);
  if (threadIdx.x == 1 && tot[1] && has_b) atomicAdd(&e.ntot[ra + 1], tot[1]);
  if (!e.H) return;  // counts only (masked survey: the spectrum is taken from the stored counts)
  cpx<T>* Hrow = static_cast<cpx<T>*>(e.H) + pp.item * e.H_item + row * (int64_t)(2 * (K / 2 + 1));
  forward_separate<T, MIX>(line, other, e.fwd, lane, g.nlanes, active, Hrow);
}

// Standalone spectrum, first pass: rows of two maps packed as a + i b (the
// contrast delta_g for counts, Sec. 3.2 eq. Estim), forward transform, separation.
template <typename T, int MIX>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2))) k_pair_forward(LineGeom g, FftDesc f, PairLoad p) {
  cpx<T>* lds = lds_lines<T>();
  const PassPos pp = pass_pos(g);
  const int K = f.L;
  const int r = threadIdx.x / g.nlanes, lane = threadIdx.x - r * g.nlanes;
  const bool active = r < pp.nl;
  cpx<T>* line = buf_a(lds, g, r);
  const int64_t row = pp.line0 + r;
  const int64_t ma = 2 * pp.item;
  const bool has_b = ma + 1 < p.count;
  if (active) {
    if (p.kind == 0) {
      // eight elements of the thread requested before any is stored
      const T* a = static_cast<const T*>(p.maps) + ma * p.ncells + row * K;
      for (int i0 = lane; i0 < K; i0 += 8 * g.nlanes) {
        T va[8], vb[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int i = i0 + k * g.nlanes;
          va[k] = i < K ? a[i] : T(0);
          vb[k] = i < K && has_b ? a[i + p.ncells] : T(0);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int i = i0 + k * g.nlanes;
          if (i < K) line[pidx(i)] = {va[k], vb[k]};
        }
      }
    } else if (p.kind == 2) {
      const float* m = p.mask + row * K;
      for (int i = lane; i < K; i += g.nlanes) line[pidx(i)] = {m[i] != 0.0f ? T(1) : T(0), T(0)};
    } else {
      // delta_g = N / (f N^) - 1 on f != 0, 0 elsewhere, with 1 / N^ = fsum / N_tot formed once;
      // the per-cell reciprocal of f is the pass precision's (FP32: the hardware reciprocal)
      const int32_t* a = static_cast<const int32_t*>(p.maps) + ma * p.ncells + row * K;
      const double fsum = p.fsum ? *p.fsum : (double)p.ncells;
      const T ia = (T)(fsum / (double)p.ntot[ma]);
      const T ib = has_b ? (T)(fsum / (double)p.ntot[ma + 1]) : T(0);
      const float* mrow = p.mask ? p.mask + row * K : nullptr;
      for (int i0 = lane; i0 < K; i0 += 8 * g.nlanes) {
        // eight elements of the thread requested before any is used
        int32_t ca[8], cb[8];
        float fm[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int i = i0 + k * g.nlanes;
          ca[k] = i < K ? a[i] : 0;
          cb[k] = i < K && has_b ? a[i + p.ncells] : 0;
          fm[k] = i < K && mrow ? mrow[i] : 1.0f;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int i = i0 + k * g.nlanes;
          if (i >= K) continue;
          const T f = (T)fm[k];
          T va = T(0), vb = T(0);
          if (f != T(0)) {
            const T r = sizeof(T) == 4 ? (T)__builtin_amdgcn_rcpf((float)f) : T(1) / f;
            va = (T)ca[k] * r * ia - T(1);
            if (has_b) vb = (T)cb[k] * r * ib - T(1);
          }
          line[pidx(i)] = {va, vb};
        }
      }
    }
  }
  __syncthreads();
  cpx<T>* Hrow = static_cast<cpx<T>*>(p.H) + pp.item * p.H_item + row * (int64_t)(2 * (K / 2 + 1));
  forward_separate<T, MIX>(line, buf_b(lds, g, r), f, lane, g.nlanes, active, Hrow);
}

// ---------------------------------------------------------------------------
// Last forward pass with the shell sums of eq. Def spec.  Line b of the
// separated spectra holds (k_1 [3-D], s, k_last) with k_last in [0, N/2]; after
// the transform along axis 0, mode a = |k_0| in [0, N/2] of a line has the power
// v(a) = |F(a)|^2 + |F(N-a)|^2 (one term at a = 0, N/2) times the line weight
// (2 unless k_last is 0 or N/2: the half-space stands for both signs).  The
// shell integer t(a) = T0 a^2 + p (p the line's fixed part) grows with a, so the
// modes of shell b on a line are one contiguous range of a, found from the shell
// edges by an integer square root.  Each line's powers are first stored in its own
// LDS slots (slot a <- v(a); lane-local, slot a and N - a are read only by the lane
// of a), then one lane per shell adds the shell's range in increasing a; the lines
// of a group are combined per (realization, shell) in line order.  Every sum has a
// fixed order, so results are bitwise reproducible and independent of the number
// of items in a launch.

// Edge e_b of shell b (b in [0, nb]): shell b holds the modes with e_b < t <= e_{b+1};
// linear shells e_b = b^2 LL, user shells the thresholds th[b].
template <int TAB>
__device__ __forceinline__ int64_t shell_edge(const BinArgs& bn, int b) {
  return TAB ? bn.th[b] : (int64_t)b * b * bn.LL;
}

// Number of a in [0, amax] with T a^2 <= y (y may be negative): the count of modes of a line
// with t <= p + y.  FP32 square-root estimate, corrected exactly in integers (T a^2 < 2^63 for
// a <= amax + 1, the shell-rule range).
__device__ __forceinline__ int modes_upto(int64_t y, int64_t T, int amax) {
  if (y < 0) return 0;
  int a = (int)sqrtf((float)y / (float)T);
  a = a > amax + 1 ? amax + 1 : a;
  while (a > 0 && T * (int64_t)a * a > y) --a;
  while (a <= amax && T * (int64_t)(a + 1) * (a + 1) <= y) ++a;
  return a > amax ? amax + 1 : a + 1;
}

// Per-line partial sums of the shells (acc of line r: nb doubles at accr(r)), lines r < nl of
// the group that starts at line0; then, for every block of bn.G consecutive lines, the block's
// per-shell totals (lines in order, from zero) into the record rec[j][2][nb] of block j of the
// group.  The records depend only on the block, not on the lines per workgroup (a multiple of G),
// so the spectra are bitwise independent of the launch shape.
template <typename T, int WIN, int TAB>
__device__ __forceinline__ void bin_group(cpx<T>* res, const LineGeom& g, const BinArgs& bn, int64_t item,
                                          int64_t line0, int nl, double* acc_area, double* rec) {
  const int r = threadIdx.x / g.nlanes, lane = threadIdx.x - r * g.nlanes;
  const bool active = r < nl;
  // N, Nh: axis 0 (the line); Kh = N_last / 2 + 1 columns per realization of a pair
  const int N = bn.N, Nh = N / 2, nb = bn.nb, W = bn.W, Kh = W / 2, Nlh = Kh - 1;
  // shell sums of line r: in its own slots Nh + 1 .. N - 1 (free once the powers are formed)
  // when they hold nb values, else in the separate area
  const bool in_line = nb <= N - Nh - 1;
  auto accr = [&](int rr) -> double* {
    return in_line ? nullptr : acc_area + (int64_t)rr * nb;
  };
  cpx<T>* line = res + r * g.lpitch;
  int64_t p2 = 0;
  double wgt = 1.0;
  // line ln = line0 + r is (k1, kl) with kl = ln mod W: the group's first line is split once
  // (uniform over the workgroup) and each line steps from it
  const int64_t q0 = line0 / W;
  const int kl0 = (int)(line0 - q0 * W);
  if (active) {
    const int64_t ln = line0 + r;
    int kl = kl0 + r, k1 = (int)q0;
    while (kl >= W) {
      kl -= W;
      ++k1;
    }
    const int s = kl >= Kh;
    const int kz = kl - s * Kh;
    p2 = bn.Tl * kz * kz;  // the line's fixed part of t
    if (bn.ndim == 3) {
      if (k1 > bn.N1 / 2) k1 -= bn.N1;
      p2 += bn.T1 * k1 * k1;
    }
    // line weight (exact factor 1 or 2)
    wgt = (kz != 0 && kz != Nlh) ? 2.0 : 1.0;
    // masked pipeline (WIN): the line holds the transform A of N / (f nest) - 1; the
    // contrast's is D = rr A + rm Wm with rr = nest sum(f) / N_tot of the line's realization,
    // rm = rr - 1 and Wm the transform of the indicator f != 0, column-major ([column][q0] in
    // 2-D, [q1][column][q0] in 3-D: the line's window values are contiguous in q0)
    T rr = T(1), rm = T(0);
    const cpx<T>* wcol = nullptr;
    if (WIN) {
      const double nt = (double)bn.ntot[2 * item + s];
      const double rd = nt > 0.0 ? bn.nest * *bn.fsum / nt : 0.0;
      rr = (T)rd;
      rm = (T)(rd - 1.0);
      wcol = static_cast<const cpx<T>*>(bn.win) + ((ln - kl) + kz) * (int64_t)N;
    }
    // power of each mode pair in the pass precision (explicit fused multiply-adds: the same
    // rounding in every instantiation), stored as a double in slot a
    for (int a = lane; a <= Nh; a += g.nlanes) {
      cpx<T> v = line[pidx(a)];
      if (WIN) {
        const cpx<T> w = wcol[a];
        v = {rr * v.x + rm * w.x, rr * v.y + rm * w.y};
      }
      T pw = fma(v.x, v.x, v.y * v.y);
      if (a != 0 && a != Nh) {
        cpx<T> u = line[pidx(N - a)];
        if (WIN) {
          const cpx<T> w = wcol[N - a];
          u = {rr * u.x + rm * w.x, rr * u.y + rm * w.y};
        }
        pw += fma(u.x, u.x, u.y * u.y);
      }
      *reinterpret_cast<double*>(&line[pidx(a)]) = (double)pw;
    }
  }
  __syncthreads();
  if (active) {
    // shell b holds a in [lo, hi): e_b < T0 a^2 + p2 <= e_{b+1}
    double* ar = accr(r);
    for (int b = lane; b < nb; b += g.nlanes) {
      const int lo = modes_upto(shell_edge<TAB>(bn, b) - p2, bn.T0, Nh);
      const int hi = modes_upto(shell_edge<TAB>(bn, b + 1) - p2, bn.T0, Nh);
      double sum = 0.0;
      for (int a = lo; a < hi; ++a) sum += *reinterpret_cast<const double*>(&line[pidx(a)]);
      if (ar)
        ar[b] = wgt * sum;
      else
        *reinterpret_cast<double*>(&line[pidx(Nh + 1 + b)]) = wgt * sum;
    }
  }
  __syncthreads();
  const int G = bn.G;
  const int nrec = (nl + G - 1) / G;
  for (int t = threadIdx.x; t < nrec * 2 * nb; t += blockDim.x) {
    const int j = t / (2 * nb), sb = t - j * 2 * nb;
    const int s = sb / nb, b = sb - s * nb;
    double sum = 0.0;
    const int l1 = min(nl, (j + 1) * G);
    int kl = kl0 + j * G;
    while (kl >= W) kl -= W;
    for (int lr = j * G; lr < l1; ++lr) {
      if ((kl >= Kh) == s) {
        const double* ar = accr(lr);
        sum += ar ? ar[b] : *reinterpret_cast<const double*>(&res[lr * g.lpitch + pidx(Nh + 1 + b)]);
      }
      if (++kl == W) kl = 0;
    }
    rec[t] = sum;
  }
}

template <typename T, int MIX, int WIN, int TAB>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2))) k_bin_pass(LineGeom g, FftDesc f, BinArgs bn, const cpx<T>* in) {
  cpx<T>* lds = lds_lines<T>();
  const PassPos pp = pass_pos(g);
  const int nrec_wg = g.R / bn.G;                                            // records per workgroup
  double* rec = reinterpret_cast<double*>(lds + g.nbuf * g.R * g.lpitch);  // [R/G][2][nb]
  double* acc = rec + nrec_wg * 2 * bn.nb;                                  // [R][nb] when not in the lines
  load_lines(lds, in, g, pp);
  __syncthreads();
  const int r = threadIdx.x / g.nlanes, lane = threadIdx.x - r * g.nlanes;
  line_fft<T, -1, MIX>(buf_a(lds, g, r), buf_b(lds, g, r), f, lane, g.nlanes, r < pp.nl, f.L);
  bin_group<T, WIN, TAB>(result_base<T, MIX>(lds, g, f), g, bn, pp.item, pp.line0, pp.nl, acc, rec);
  __syncthreads();
  // the records of this group's blocks: block (line0 / G + j) of the item
  const int nrec = (pp.nl + bn.G - 1) / bn.G;
  const int64_t nblocks = (g.A * g.B + bn.G - 1) / bn.G;
  double* dst = bn.partials + (pp.item * nblocks + pp.line0 / bn.G) * 2 * bn.nb;
  for (int t = threadIdx.x; t < nrec * 2 * bn.nb; t += blockDim.x) dst[t] = rec[t];
}

// Many line groups per item: the partials of each run of kGroupChunk groups are summed in
// group order and the sum replaces the run's first entry (in place: a thread reads and
// writes only its own run); k_bin_reduce then adds the runs in order.
constexpr int kGroupChunk = 64;
__global__ void k_bin_chunk_sum(double* __restrict__ partials, int64_t nitems, int64_t groups, int nb) {
  const int64_t nchunks = (groups + kGroupChunk - 1) / kGroupChunk;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= nitems * nchunks * 2 * nb) return;
  const int64_t sb = idx % (2 * nb), t = idx / (2 * nb);
  const int64_t c = t % nchunks, item = t / nchunks;
  const int64_t g0 = c * kGroupChunk, g1 = g0 + kGroupChunk < groups ? g0 + kGroupChunk : groups;
  double* p = partials + (item * groups + g0) * 2 * nb + sb;
  const int64_t stride = 2 * (int64_t)nb;
  double acc = 0.0;
#pragma unroll 8
  for (int64_t g = 0; g < g1 - g0; ++g) acc += p[g * stride];
  p[0] = acc;
}

// pk[r][b] = norm * scale_r * sum_groups partial / N_b (groups taken gstep apart)
__global__ void k_bin_reduce(const double* __restrict__ partials, int64_t nitems, int64_t groups, int64_t gstep,
                             int nb, int64_t count, const int64_t* __restrict__ nmodes, double norm, int scale_kind,
                             const unsigned long long* __restrict__ ntot, const SlotOut* __restrict__ slots,
                             double ncells, double* __restrict__ pk, uint32_t* flags) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= nitems * 2 * nb) return;
  const int b = (int)(idx % nb);
  const int64_t rs = idx / nb;  // 2 * item + s
  if (rs >= count) return;
  double* dst = pk + rs * nb;
  if (slots) {  // batched pipeline: per-slot destinations, unrequested slots skipped
    dst = slots[rs].pk;
    if (!dst) return;
    if (b == 0 && slots[rs].ntot) *slots[rs].ntot = (int64_t)ntot[rs];
  }
  const int64_t item = rs / 2, s = rs - 2 * item;
  // unrolled so that several loads are in flight; the sum stays in group order
  const double* src = partials + (item * groups * 2 + s) * nb + b;
  const int64_t stride = 2 * (int64_t)nb * gstep;
  double acc = 0.0;
#pragma unroll 8
  for (int64_t gidx = 0; gidx < (groups + gstep - 1) / gstep; ++gidx) acc += src[gidx * stride];
  double scale = 1.0;
  if (scale_kind == 1) {
    const double nt = (double)ntot[rs];
    if (nt == 0.0) atomicOr(flags, 4u);
    const double nhat = nt / ncells;
    scale = 1.0 / (nhat * nhat);
  } else if (scale_kind == 2 && ntot[rs] == 0) {  // contrast formed in the binning pass
    atomicOr(flags, 4u);
  }
  dst[b] = norm * scale * acc / (double)nmodes[b];
}

__device__ __forceinline__ void covariance_entry(const double* __restrict__ pk, int64_t R, int nb, int64_t idx,
                                                 double* __restrict__ cov, double* __restrict__ cnorm) {
  const int a = (int)(idx / nb), b = (int)(idx % nb);
  double ma = 0.0, mb = 0.0;
#pragma unroll 8
  for (int64_t r = 0; r < R; ++r) {
    ma += pk[r * nb + a];
    mb += pk[r * nb + b];
  }
  ma /= (double)R;
  mb /= (double)R;
  double c = 0.0, s2 = 0.0;
#pragma unroll 8
  for (int64_t r = 0; r < R; ++r) {
    const double pa = pk[r * nb + a], pb = pk[r * nb + b];
    c += (pa - ma) * (pb - mb);
    s2 += pa * pb;
  }
  if (cov) cov[idx] = c / (double)(R - 1);
  if (cnorm) cnorm[idx] = (s2 / (double)R) / (ma * mb) - 1.0;
}

__global__ void k_covariance(const double* __restrict__ pk, int64_t R, int nb, double* __restrict__ cov,
                             double* __restrict__ cnorm) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx < (int64_t)nb * nb) covariance_entry(pk, R, nb, idx, cov, cnorm);
}

// one request per blockIdx.y
__global__ void k_covariance_batch(const CovItem* __restrict__ items, int nb) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const CovItem it = items[blockIdx.y];
  if (idx < (int64_t)nb * nb) covariance_entry(it.pk, it.R, nb, idx, it.cov, it.cnorm);
}

// ---------------------------------------------------------------------------
// Standalone lognormal + Poisson (one thread per realization and cell).
template <typename T>
__global__ void k_lognormal_poisson(const T* __restrict__ fields, int64_t count, int64_t ncells, double s2half,
                                    double nbar, const float* __restrict__ mask, uint32_t k0, uint32_t k1,
                                    uint32_t rid, uint64_t first_real, T* __restrict__ delta,
                                    int32_t* __restrict__ counts, unsigned long long* __restrict__ ntot,
                                    const double* __restrict__ inv, uint32_t* flags) {
  __shared__ unsigned long long acc;
  __shared__ double inv_s[kInvLds + 1];
  const int64_t blocks_per_map = (ncells + blockDim.x - 1) / blockDim.x;
  const int64_t k = blockIdx.x / blocks_per_map;
  const int64_t cell = (blockIdx.x - k * blocks_per_map) * blockDim.x + threadIdx.x;
  if (threadIdx.x == 0) acc = 0;
  for (int i = threadIdx.x; i <= kInvLds; i += blockDim.x) inv_s[i] = inv[i];
  __syncthreads();
  if (k < count && cell < ncells) {
    const uint64_t rr = first_real + (uint64_t)k;
    const T g = fields[k * ncells + cell];
    const T d = lognormal_delta<T>(g, (T)s2half);
    const double f = mask ? (double)mask[cell] : 1.0;
    const double mu = intensity(nbar, f, (double)d);
    int n = 0;
    if (!(mu <= kMaxMu)) {
      atomicOr(flags, 2u);
      n = -1;
    } else {
      const int K = chunk_count(mu);
      for (int c = 0; c < K; ++c) {
        const Words4 w = philox4x32_10((uint32_t)cell, (uint32_t)(rr >> 1), rid, 1u + (uint32_t)c, k0, k1);
        const double u = (rr & 1) ? unit52(w.x2, w.x3) : unit52(w.x0, w.x1);
        n += poisson_chunk(u, chunk_mean(mu, c, K), inv_s, flags);
      }
    }
    if (delta) delta[k * ncells + cell] = d;
    counts[k * ncells + cell] = n;
    if (n > 0) atomicAdd(&acc, (unsigned long long)n);
  }
  __syncthreads();
  if (threadIdx.x == 0 && acc && ntot) atomicAdd(&ntot[k], acc);
}

__global__ void k_count_totals(const int32_t* __restrict__ counts, int64_t count, int64_t ncells,
                               unsigned long long* __restrict__ ntot) {
  __shared__ unsigned long long acc;
  const int64_t blocks_per_map = (ncells + blockDim.x - 1) / blockDim.x;
  const int64_t k = blockIdx.x / blocks_per_map;
  const int64_t cell = (blockIdx.x - k * blocks_per_map) * blockDim.x + threadIdx.x;
  if (threadIdx.x == 0) acc = 0;
  __syncthreads();
  if (k < count && cell < ncells) {
    const int32_t v = counts[k * ncells + cell];
    if (v > 0) atomicAdd(&acc, (unsigned long long)v);
  }
  __syncthreads();
  if (threadIdx.x == 0 && acc) atomicAdd(&ntot[k], acc);
}

__global__ void k_copy_ntot(const unsigned long long* __restrict__ src, int64_t* __restrict__ dst, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (int64_t)src[i];
}

__global__ void k_advance(unsigned long long* p, unsigned long long by) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p += by;
}

// sum of the mask in FP64, in a fixed order: workgroup b's thread t adds cells b 256 + t,
// b 256 + t + 65536, ..., a tree gives the workgroup's partial, then one workgroup adds the 256
// partials by a tree
constexpr int kMaskSumBlocks = 256;
__global__ void __launch_bounds__(256) k_mask_sum(const float* __restrict__ mask, int64_t n,
                                                  double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * kMaskSumBlocks) s += (double)mask[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_mask_sum_final(double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[256];
  red[threadIdx.x] = part[threadIdx.x];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// N_b of the linear shells of a grid (the binning pass's integer rule: mode q~ is in shell s - 1 for
// the smallest s >= 0 with s^2 LL >= sum_i T_i q~_i^2) by visiting every mode; integer atomics, so
// the counts are exact in any order.  counts (nb) must start at zero.
__global__ void k_shell_counts(int32_t n0, int32_t n1, int32_t n2, int64_t T0, int64_t T1, int64_t T2, int64_t LL,
                               int nb, unsigned long long* __restrict__ counts) {
  const int64_t total = (int64_t)n0 * n1 * n2;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i2 = idx % n2, rest = idx / n2;
    const int64_t i1 = rest % n1, i0 = rest / n1;
    const int64_t q0 = i0 <= n0 / 2 ? i0 : i0 - n0, q1 = i1 <= n1 / 2 ? i1 : i1 - n1,
                  q2 = i2 <= n2 / 2 ? i2 : i2 - n2;
    const int64_t t = T0 * q0 * q0 + T1 * q1 * q1 + T2 * q2 * q2;
    int64_t s = (int64_t)sqrt((double)t / (double)LL);
    while (s > 0 && (s - 1) * (s - 1) * LL >= t) --s;
    while (s * s * LL < t) ++s;
    if (s >= 1 && s <= nb) atomicAdd(&counts[s - 1], 1ull);
  }
}

hipError_t launch_shell_counts(const int32_t* n, const int64_t* T, int64_t LL, int nb, int64_t* counts,
                               hipStream_t s) {
  const int64_t total = (int64_t)n[0] * n[1] * n[2];
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_shell_counts, dim3(blocks), dim3(256), 0, s, n[0], n[1], n[2], T[0], T[1], T[2], LL, nb,
                     reinterpret_cast<unsigned long long*>(counts));
  return hipGetLastError();
}

__global__ void k_zero_u64(unsigned long long* p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_debug_philox(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                               int64_t n, uint32_t* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Words4 w = philox4x32_10(c0 + (uint32_t)i, c1, c2, c3, k0, k1);
  out[4 * i + 0] = w.x0;
  out[4 * i + 1] = w.x1;
  out[4 * i + 2] = w.x2;
  out[4 * i + 3] = w.x3;
}

template <typename T>
__global__ void k_debug_noise(NoiseArgs n, uint32_t pair, int64_t cells, cpx<T>* __restrict__ out) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (2 * p >= cells) return;
  const Words4 w = philox4x32_10((uint32_t)p, pair, n.rid, 0u, n.k0, n.k1);
  out[2 * p] = normal_pair<T>(w.x0, w.x1);
  out[2 * p + 1] = normal_pair<T>(w.x2, w.x3);
}

// ---------------------------------------------------------------------------
// launchers

// Workgroups may use more than 64 KB of the 160 KB LDS of a gfx950 CU once the
// kernel's dynamic-LDS limit is raised.
#define CE_LAUNCH(kernel, grid, block, lds, stream, ...)                                                     \
  do {                                                                                                     \
    if ((lds) > 65536)                                                                                     \
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&kernel),                                    \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)(lds));                   \
    hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);                                      \
  } while (0)

static size_t lines_lds_bytes(const LineGeom& g, size_t elem) { return (size_t)g.nbuf * g.R * g.lpitch * elem; }

static dim3 pass_grid(const LineGeom& g) { return dim3((unsigned)(g.nitems * g.groups_per_item)); }
static dim3 pass_block(const LineGeom& g) {
  const int t = std::max(g.R * g.nlanes, g.threads);
  return dim3((unsigned)((t + 63) / 64 * 64));
}

hipError_t launch_lag_octant(int ndim, const int32_t* O, const double* h, int kind, const double* p, double* out,
                             hipStream_t s) {
  const int64_t n = (int64_t)O[0] * O[1] * O[2];
  const int blocks = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
  hipLaunchKernelGGL(k_lag_octant, dim3(blocks), dim3(256), 0, s, ndim, O[0], O[1], O[2], h[0], h[1], h[2], kind,
                     p[0], p[1], p[2], p[3], out);
  return hipGetLastError();
}

// two LDS buffers per line exactly for the ping-pong variant (primes above 31)
static bool nbuf_ok(const LineGeom& g, int mix) { return (mix == 3) == (g.nbuf == 2); }

// kernel variant of a transform (the MIX template argument)
static int fft_variant(const FftDesc& f) {
  int v = 0;
  for (int i = 0; i < f.nst; ++i) {
    const int r = f.rad[i];
    if (r & (r - 1)) v = std::max(v, r <= 7 ? 1 : r <= 31 ? 2 : 3);
  }
  return v;
}

template <int V>
struct Variant {
  static constexpr int value = V;
};
// calls fn(Variant<v>{}) for the run-time variant v
template <typename F>
static void with_variant(int v, F&& fn) {
  if (v == 3)
    fn(Variant<3>{});
  else if (v == 2)
    fn(Variant<2>{});
  else if (v == 1)
    fn(Variant<1>{});
  else
    fn(Variant<0>{});
}

hipError_t launch_dct_axis(const LineGeom& g, const FftDesc& f, const DctArgs& a, hipStream_t s) {
  const size_t lds = lines_lds_bytes(g, sizeof(cpx<double>));
  const int mix = fft_variant(f);
  if (!nbuf_ok(g, mix)) return hipErrorInvalidValue;
  with_variant(mix, [&](auto v) { CE_LAUNCH((k_dct_axis<decltype(v)::value>), pass_grid(g), pass_block(g), lds, s, g, f, a); });
  return hipGetLastError();
}

hipError_t launch_lambda_stats(const double* lam, int ndim, const int32_t* O, int64_t n, double* stats,
                               unsigned long long* nneg, hipStream_t s) {
  hipLaunchKernelGGL(k_lambda_stats, dim3(256), dim3(256), 0, s, lam, ndim, O[0], O[1], O[2], n, stats, nneg);
  return hipGetLastError();
}

hipError_t launch_sqrt_table(const double* lam, int ndim, const int32_t* O, double inv_cells, int prec, void* out,
                             hipStream_t s) {
  (void)ndim;
  const int64_t n = (int64_t)O[0] * O[1] * O[2];
  const int blocks = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
  if (prec == 0)
    hipLaunchKernelGGL(k_sqrt_table<float>, dim3(blocks), dim3(256), 0, s, lam, O[0], O[1], O[2], inv_cells,
                       static_cast<float*>(out));
  else
    hipLaunchKernelGGL(k_sqrt_table<double>, dim3(blocks), dim3(256), 0, s, lam, O[0], O[1], O[2], inv_cells,
                       static_cast<double*>(out));
  return hipGetLastError();
}

hipError_t launch_noise_pass(int prec, const LineGeom& g0, const FftDesc& f, const NoiseArgs& n, void* out,
                             hipStream_t s) {
  const int mix = fft_variant(f);
  if (!nbuf_ok(g0, mix) || g0.R < 2 || (g0.R & 1) || (g0.B & 1) || g0.pairs_wg < 1 ||
      g0.nitems * g0.pairs_wg < g0.items_total)
    return hipErrorInvalidValue;
  LineGeom g = g0;
  if (mix >= 2 && g.pairs_wg > 1) {  // those variants generate one pair per workgroup
    g.pairs_wg = 1;
    g.nitems = g.items_total;
  }
  with_variant(mix, [&](auto v) {
    constexpr int V = decltype(v)::value;
    if (prec == 0)
      CE_LAUNCH((k_noise_pass<float, V>), pass_grid(g), pass_block(g), lines_lds_bytes(g, sizeof(cpx<float>)), s, g,
                f, n, static_cast<cpx<float>*>(out));
    else
      CE_LAUNCH((k_noise_pass<double, V>), pass_grid(g), pass_block(g), lines_lds_bytes(g, sizeof(cpx<double>)), s,
                g, f, n, static_cast<cpx<double>*>(out));
  });
  return hipGetLastError();
}

template <typename T>
static void line_pass_t(int dir, int mix, const LineGeom& g, const FftDesc& f, const void* in, void* out,
                        hipStream_t s) {
  const size_t lds = lines_lds_bytes(g, sizeof(cpx<T>));
  const cpx<T>* i = static_cast<const cpx<T>*>(in);
  cpx<T>* o = static_cast<cpx<T>*>(out);
  with_variant(mix, [&](auto v) {
    constexpr int V = decltype(v)::value;
    if (dir > 0)
      CE_LAUNCH((k_line_pass<T, 1, V>), pass_grid(g), pass_block(g), lds, s, g, f, i, o);
    else
      CE_LAUNCH((k_line_pass<T, -1, V>), pass_grid(g), pass_block(g), lds, s, g, f, i, o);
  });
}

hipError_t launch_line_pass(int prec, int dir, const LineGeom& g, const FftDesc& f, const void* in, void* out,
                            hipStream_t s) {
  const int mix = fft_variant(f);
  if (!nbuf_ok(g, mix)) return hipErrorInvalidValue;
  if (prec == 0)
    line_pass_t<float>(dir, mix, g, f, in, out, s);
  else
    line_pass_t<double>(dir, mix, g, f, in, out, s);
  return hipGetLastError();
}

template <typename T>
static void row_inverse_t(int mix, const LineGeom& g, const FftDesc& f, const RowEpi& e, const void* in,
                          hipStream_t s) {
  const size_t lds = lines_lds_bytes(g, sizeof(cpx<T>));
  const cpx<T>* i = static_cast<const cpx<T>*>(in);
  with_variant(mix, [&](auto v) {
    CE_LAUNCH((k_row_inverse<T, decltype(v)::value>), pass_grid(g), pass_block(g), lds, s, g, f, e, i);
  });
}

hipError_t launch_row_inverse(int prec, const LineGeom& g, const FftDesc& f, const RowEpi& e, const void* in,
                              hipStream_t s) {
  const int mix = std::max(fft_variant(f), e.mode == 2 ? fft_variant(e.fwd) : 0);
  if (!nbuf_ok(g, mix)) return hipErrorInvalidValue;
  if (prec == 0)
    row_inverse_t<float>(mix, g, f, e, in, s);
  else
    row_inverse_t<double>(mix, g, f, e, in, s);
  return hipGetLastError();
}

template <typename T>
static void pair_forward_t(int mix, const LineGeom& g, const FftDesc& f, const PairLoad& p, hipStream_t s) {
  const size_t lds = lines_lds_bytes(g, sizeof(cpx<T>));
  with_variant(mix, [&](auto v) {
    CE_LAUNCH((k_pair_forward<T, decltype(v)::value>), pass_grid(g), pass_block(g), lds, s, g, f, p);
  });
}

hipError_t launch_pair_forward(int prec, const LineGeom& g, const FftDesc& f, const PairLoad& p, hipStream_t s) {
  const int mix = fft_variant(f);
  if (!nbuf_ok(g, mix)) return hipErrorInvalidValue;
  if (prec == 0)
    pair_forward_t<float>(mix, g, f, p, s);
  else
    pair_forward_t<double>(mix, g, f, p, s);
  return hipGetLastError();
}

template <typename T>
static void bin_pass_t(int mix, const LineGeom& g, const FftDesc& f, const BinArgs& b, const void* in,
                       hipStream_t s) {
  const size_t lds = bin_pass_lds(g, b.N, b.nb, b.G, sizeof(cpx<T>));
  const cpx<T>* i = static_cast<const cpx<T>*>(in);
  with_variant(mix, [&](auto v) {
    if (b.win && b.th)
      CE_LAUNCH((k_bin_pass<T, decltype(v)::value, 1, 1>), pass_grid(g), pass_block(g), lds, s, g, f, b, i);
    else if (b.win)
      CE_LAUNCH((k_bin_pass<T, decltype(v)::value, 1, 0>), pass_grid(g), pass_block(g), lds, s, g, f, b, i);
    else if (b.th)
      CE_LAUNCH((k_bin_pass<T, decltype(v)::value, 0, 1>), pass_grid(g), pass_block(g), lds, s, g, f, b, i);
    else
      CE_LAUNCH((k_bin_pass<T, decltype(v)::value, 0, 0>), pass_grid(g), pass_block(g), lds, s, g, f, b, i);
  });
}

// LDS of a binning-pass workgroup of R lines: the line buffers, the records of its blocks of G
// lines ([R/G][2][nb]) and, when a line's free slots (N/2 - 1 of them) cannot hold its nb shell
// sums, a separate [R][nb] area.
size_t bin_pass_lds(const LineGeom& g, int N, int nb, int G, size_t elem) {
  const bool in_line = nb <= N - N / 2 - 1;
  return lines_lds_bytes(g, elem) + (size_t)(g.R / G) * 2 * nb * sizeof(double) +
         (in_line ? 0 : (size_t)g.R * nb * sizeof(double));
}

hipError_t launch_bin_pass(int prec, const LineGeom& g, const FftDesc& f, const BinArgs& b, const void* in,
                           hipStream_t s) {
  if (b.G < 1 || g.R % b.G || bin_pass_lds(g, b.N, b.nb, b.G, prec ? sizeof(cpx<double>) : sizeof(cpx<float>)) >
                                   kMaxLdsBytes)
    return hipErrorInvalidValue;
  const int mix = fft_variant(f);
  if (!nbuf_ok(g, mix)) return hipErrorInvalidValue;
  if (prec == 0)
    bin_pass_t<float>(mix, g, f, b, in, s);
  else
    bin_pass_t<double>(mix, g, f, b, in, s);
  return hipGetLastError();
}

hipError_t launch_bin_reduce(double* partials, int64_t nitems, int64_t groups, int nb, int64_t count,
                             const int64_t* nmodes, double norm, int scale_kind, const unsigned long long* ntot_u,
                             const SlotOut* slots, double ncells, double* pk, uint32_t* flags, hipStream_t s) {
  int64_t gstep = 1;
  if (groups > kGroupChunk) {
    const int64_t m = nitems * ((groups + kGroupChunk - 1) / kGroupChunk) * 2 * nb;
    hipLaunchKernelGGL(k_bin_chunk_sum, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, partials, nitems, groups,
                       nb);
    gstep = kGroupChunk;
  }
  const int64_t n = nitems * 2 * nb;
  hipLaunchKernelGGL(k_bin_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, partials, nitems, groups,
                     gstep, nb, count, nmodes, norm, scale_kind, ntot_u, slots, ncells, pk, flags);
  return hipGetLastError();
}

hipError_t launch_lognormal_poisson(int prec, const void* fields, int64_t count, int64_t ncells, double s2half,
                                    double nbar, const float* mask, uint32_t k0, uint32_t k1, uint32_t rid,
                                    uint64_t first_real, void* delta, int32_t* counts, unsigned long long* ntot,
                                    const double* inv, uint32_t* flags, hipStream_t s) {
  const int64_t bpm = (ncells + 255) / 256;
  const dim3 grid((unsigned)(bpm * count));
  if (prec == 0)
    hipLaunchKernelGGL(k_lognormal_poisson<float>, grid, dim3(256), 0, s, static_cast<const float*>(fields), count,
                       ncells, s2half, nbar, mask, k0, k1, rid, first_real, static_cast<float*>(delta), counts, ntot,
                       inv, flags);
  else
    hipLaunchKernelGGL(k_lognormal_poisson<double>, grid, dim3(256), 0, s, static_cast<const double*>(fields),
                       count, ncells, s2half, nbar, mask, k0, k1, rid, first_real, static_cast<double*>(delta),
                       counts, ntot, inv, flags);
  return hipGetLastError();
}

hipError_t launch_count_totals(const int32_t* counts, int64_t count, int64_t ncells, unsigned long long* ntot,
                               hipStream_t s) {
  const int64_t bpm = (ncells + 255) / 256;
  hipLaunchKernelGGL(k_count_totals, dim3((unsigned)(bpm * count)), dim3(256), 0, s, counts, count, ncells, ntot);
  return hipGetLastError();
}

hipError_t launch_copy_ntot(const unsigned long long* src, int64_t* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_ntot, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_covariance(const double* pk, int64_t count, int nb, double* cov, double* cnorm, hipStream_t s) {
  const int64_t n = (int64_t)nb * nb;
  hipLaunchKernelGGL(k_covariance, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pk, count, nb, cov, cnorm);
  return hipGetLastError();
}

hipError_t launch_covariance_batch(const CovItem* items, int64_t nitems, int nb, hipStream_t s) {
  const int64_t n = (int64_t)nb * nb;
  for (int64_t i = 0; i < nitems; i += 65535) {
    const unsigned ny = (unsigned)std::min<int64_t>(65535, nitems - i);
    hipLaunchKernelGGL(k_covariance_batch, dim3((unsigned)((n + 255) / 256), ny), dim3(256), 0, s, items + i, nb);
  }
  return hipGetLastError();
}

hipError_t launch_debug_philox(uint32_t k0, uint32_t k1, const uint32_t* ctr, int64_t n, uint32_t* out,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_debug_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, k0, k1, ctr[0], ctr[1],
                     ctr[2], ctr[3], n, out);
  return hipGetLastError();
}

hipError_t launch_debug_noise(int prec, const NoiseArgs& n, uint64_t pair, int64_t cells, void* out, hipStream_t s) {
  const int64_t np = cells / 2;
  const dim3 grid((unsigned)((np + 255) / 256));
  if (prec == 0)
    hipLaunchKernelGGL(k_debug_noise<float>, grid, dim3(256), 0, s, n, (uint32_t)pair, cells,
                       static_cast<cpx<float>*>(out));
  else
    hipLaunchKernelGGL(k_debug_noise<double>, grid, dim3(256), 0, s, n, (uint32_t)pair, cells,
                       static_cast<cpx<double>*>(out));
  return hipGetLastError();
}

hipError_t launch_advance(unsigned long long* p, unsigned long long by, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, p, by);
  return hipGetLastError();
}

// Window transform to column-major: out[c][a] = in[a][c] for the first Kh columns of every
// W-wide block (the columns the binning pass reads), so that the pass reads it along a.
template <typename T>
__global__ void k_window_columns(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out, int64_t N0, int64_t C) {
  __shared__ cpx<T> tile[32][33];
  const int64_t a0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int64_t a = a0 + k, c = c0 + threadIdx.x;
    if (a < N0 && c < C) tile[k][threadIdx.x] = in[a * C + c];
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int64_t c = c0 + k, a = a0 + threadIdx.x;
    if (a < N0 && c < C) out[c * N0 + a] = tile[threadIdx.x][k];
  }
}

hipError_t launch_window_columns(int prec, const void* in, void* out, int64_t N0, int64_t C, hipStream_t s) {
  const dim3 grid((unsigned)((C + 31) / 32), (unsigned)((N0 + 31) / 32)), block(32, 8);
  if (prec == 0)
    hipLaunchKernelGGL(k_window_columns<float>, grid, block, 0, s, static_cast<const cpx<float>*>(in),
                       static_cast<cpx<float>*>(out), N0, C);
  else
    hipLaunchKernelGGL(k_window_columns<double>, grid, block, 0, s, static_cast<const cpx<double>*>(in),
                       static_cast<cpx<double>*>(out), N0, C);
  return hipGetLastError();
}

hipError_t launch_mask_sum(const float* mask, int64_t n, double* out, hipStream_t s) {
  // out[0] receives the sum; out[1 .. 256] hold the workgroup partials
  hipLaunchKernelGGL(k_mask_sum, dim3(kMaskSumBlocks), dim3(256), 0, s, mask, n, out + 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mask_sum_final, dim3(1), dim3(256), 0, s, out + 1, out);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace ce
