// Statistics beyond the spectrum.  Counts-in-cells statistics of Poisson maps (Sec. 3.4): the
// histogram of the counts over unmasked cells and its Poisson-lognormal prediction, and the A*
// map, the per-cell root of eq. As, whose spectrum is estimated like that of the galaxy
// contrast.  The cumulative information
// of the spectrum covariance (eq. cuminfo).
//
// Both read the counts once (int32) and the survey mask (float, optional).  The histogram
// is exact in integers (LDS counters in several copies, flushed with 64-bit atomics); the
// A* map is solved in FP64 in registers and its per-map mean is reduced in a fixed order,
// so every output is bitwise reproducible for a given launch shape.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ce_internal.hpp"

namespace ce {

namespace {

constexpr int kCicThreads = 256;
constexpr int kGridY = 65535;  // realizations per launch (grid y)

// Workgroups per map: enough to fill the chip for one map, about 8 cells per thread.
int64_t blocks_per_map(int64_t cells) {
  int64_t b = (cells + kCicThreads * 8 - 1) / (kCicThreads * 8);
  return b < 1 ? 1 : (b > 2048 ? 2048 : b);
}

// LDS counters: the workgroup holds ncopy copies of the histogram and thread t counts into
// copy t % ncopy, so lanes of a wave that see the same count (most of them, at low
// intensity) hit different words; the copies are an odd number of words apart, so equal
// counts also fall in different banks.  ncopy is the largest power of two <= 64 whose copies
// fit kHistLds.
constexpr int kHistLds = 48 * 1024;

__host__ __device__ inline int hist_stride(int nhist) { return nhist | 1; }
__host__ __device__ inline int hist_copies(int nhist) {
  int c = 64;
  while (c > 1 && (size_t)c * hist_stride(nhist) * 4 > (size_t)kHistLds) c >>= 1;
  return c;
}

__device__ __forceinline__ void hist_count(uint32_t* mine, int32_t n, bool keep, int nhist) {
  if (keep && (uint32_t)n < (uint32_t)nhist) atomicAdd(&mine[n], 1u);
}

// VEC: counts and mask read four cells at a time (cells % 4 == 0, 16-byte aligned maps).
template <bool VEC>
__global__ void __launch_bounds__(kCicThreads) k_cic_histogram(const int32_t* __restrict__ counts,
                                                               const float* __restrict__ mask, int64_t cells,
                                                               int nhist, unsigned long long* __restrict__ hist) {
  extern __shared__ uint32_t bins[];
  const int ncopy = hist_copies(nhist), stride_b = hist_stride(nhist);
  const int total = ncopy * stride_b;
  const int r = blockIdx.y;
  for (int i = threadIdx.x; i < total; i += kCicThreads) bins[i] = 0;
  __syncthreads();
  uint32_t* mine = bins + (threadIdx.x & (ncopy - 1)) * stride_b;
  const int32_t* c = counts + (int64_t)r * cells;
  const int64_t stride = (int64_t)gridDim.x * kCicThreads;
  if (VEC) {
    const int64_t q = cells >> 2;
    const int4* c4 = reinterpret_cast<const int4*>(c);
    const float4* m4 = reinterpret_cast<const float4*>(mask);
    for (int64_t i = blockIdx.x * (int64_t)kCicThreads + threadIdx.x; i < q; i += stride) {
      const int4 n = c4[i];
      const float4 f = mask ? m4[i] : make_float4(1.0f, 1.0f, 1.0f, 1.0f);
      hist_count(mine, n.x, f.x != 0.0f, nhist);
      hist_count(mine, n.y, f.y != 0.0f, nhist);
      hist_count(mine, n.z, f.z != 0.0f, nhist);
      hist_count(mine, n.w, f.w != 0.0f, nhist);
    }
  } else {
    for (int64_t i = blockIdx.x * (int64_t)kCicThreads + threadIdx.x; i < cells; i += stride)
      hist_count(mine, c[i], mask == nullptr || mask[i] != 0.0f, nhist);
  }
  __syncthreads();
  unsigned long long* h = hist + (int64_t)r * nhist;
  for (int i = threadIdx.x; i < nhist; i += kCicThreads) {
    uint32_t t = 0;
    for (int k = 0; k < ncopy; ++k) t += bins[k * stride_b + i];
    if (t) atomicAdd(&h[i], (unsigned long long)t);
  }
}

__global__ void k_zero_i64(unsigned long long* p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Root of g(A) = c e^A + A - d = 0 (eq. As with c = N_bar f sigma_A^2, d = sigma_A^2 (N - 1/2)).
// With A = d - w the equation becomes w e^w = c e^d, so w is the principal Lambert function
// of x = c e^d.  An FP32 estimate of w comes from Newton's method on w + ln w = y, y = ln x
// (concave and increasing in w, so the iterates stay positive), started at x / (1 + x) for
// y <= 1 and at the asymptotic y - ln y + ln y / y above, with hardware log / exp.  The root
// is then refined in FP64 by Halley's method on g itself (g' = c e^A + 1, g'' = c e^A), whose
// error contracts as e -> K e^3 with |K| <= 1/4, until a step falls below 2^-20 max(1, |A|).
// For large d the FP32 estimate of A = d - w loses digits to cancellation, so it is first
// replaced by two steps of A = ln(d - A) - ln c, a contraction by 1 / (d - A) there.
// lnb = ln(N_bar sigma_A^2) in FP64; the FP32 estimate takes ln c = lnb + ln f.
__device__ __forceinline__ double astar_solve(int32_t n, float f, double lnb, double c, double s2) {
  const double d = s2 * ((double)n - 0.5);
  // (a denormal f is scaled by 2^64 first: the hardware log may flush denormals to zero)
  const float lf = f < 0x1p-126f ? __logf(f * 0x1p64f) - 44.3614196f : __logf(f);
  const float y = (float)lnb + lf + (float)d;
  float w;
  if (y < -20.0f) {
    w = __expf(y);  // W(x) = x (1 - x + ...) with x below 2e-9
  } else {
    if (y <= 1.0f) {
      const float x = __expf(y);
      w = x * __builtin_amdgcn_rcpf(1.0f + x);
    } else {
      const float ly = __logf(y);
      w = y - ly + ly * __builtin_amdgcn_rcpf(y);
    }
    // the starting error is below 0.3 and contracts as e -> e^2 / 4 (or faster): three steps
    // reach FP32 rounding
#pragma unroll
    for (int it = 0; it < 3; ++it) w = w * (1.0f + y - __logf(w)) * __builtin_amdgcn_rcpf(1.0f + w);
  }
  double a = d - (double)w;
  if (d > 256.0 && w > 0.0f) {
    const double lc = log(c);
    a = log(d - a) - lc;
    a = log(d - a) - lc;
  }
  for (int it = 0; it < 12; ++it) {
    const double e = c * exp(a);
    const double g = e + a - d;
    const double g1 = e + 1.0;
    const double step = 2.0 * g * g1 / (2.0 * g1 * g1 - g * e);
    a -= step;
    if (fabs(step) <= 0x1p-20 * fmax(1.0, fabs(a))) break;
  }
  return a;
}

// MODE 0: write A* (0 on masked cells).  MODE 1: write A* - off (0 on masked cells) and the
// per-workgroup sums of A* and of the number of unmasked cells into
// partials[(r * gridDim.x + block) * 2 + {0, 1}].  The map minus its mean is then written by
// k_astar_shift from the stored values (one solve per cell); off, an estimate of the mean (the
// prior mean of the log-density), keeps the stored values centred so an FP32 map loses no digits.
template <typename T, int MODE>
__global__ void __launch_bounds__(kCicThreads) k_astar(const int32_t* __restrict__ counts,
                                                       const float* __restrict__ mask, int64_t cells,
                                                       double nbar, double lnb, double s2, double off,
                                                       T* __restrict__ out, double* __restrict__ partials) {
  const int r = blockIdx.y;
  const int32_t* c = counts + (int64_t)r * cells;
  double acc = 0.0, nk = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kCicThreads;
  for (int64_t i = blockIdx.x * (int64_t)kCicThreads + threadIdx.x; i < cells; i += stride) {
    const float f = mask ? mask[i] : 1.0f;
    double a = 0.0;
    if (f != 0.0f) {
      a = astar_solve(c[i], f, lnb, (nbar * (double)f) * s2, s2);
      acc += a;
      nk += 1.0;
      a -= off;
    }
    out[(int64_t)r * cells + i] = (T)a;
  }
  if (MODE == 1) {
    __shared__ double sa[kCicThreads], sn[kCicThreads];
    sa[threadIdx.x] = acc;
    sn[threadIdx.x] = nk;
    __syncthreads();
    for (int h = kCicThreads / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) {
        sa[threadIdx.x] += sa[threadIdx.x + h];
        sn[threadIdx.x] += sn[threadIdx.x + h];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      double* p = partials + ((int64_t)r * gridDim.x + blockIdx.x) * 2;
      p[0] = sa[0];
      p[1] = sn[0];
    }
  }
}

// A* - mean[r] on unmasked cells from the stored A* - off (masked cells stay 0).
template <typename T>
__global__ void __launch_bounds__(kCicThreads) k_astar_shift(const float* __restrict__ mask, int64_t cells,
                                                             double off, const double* __restrict__ mean,
                                                             T* __restrict__ out) {
  const int r = blockIdx.y;
  const double d = mean[r] - off;
  T* o = out + (int64_t)r * cells;
  const int64_t stride = (int64_t)gridDim.x * kCicThreads;
  for (int64_t i = blockIdx.x * (int64_t)kCicThreads + threadIdx.x; i < cells; i += stride)
    if (mask == nullptr || mask[i] != 0.0f) o[i] = (T)((double)o[i] - d);
}

// The same shift four cells at a time with 16-byte accesses (cells a multiple of 4, aligned
// buffers): the pass is bound by HBM and the wide accesses halve its instruction count.
template <typename T>
__device__ __forceinline__ T shifted(T v, float m, double d) {
  return m != 0.0f ? (T)((double)v - d) : v;
}
__device__ __forceinline__ void shift4(float* o, float4 m, double d) {
  float4 x = *reinterpret_cast<float4*>(o);
  x = make_float4(shifted(x.x, m.x, d), shifted(x.y, m.y, d), shifted(x.z, m.z, d), shifted(x.w, m.w, d));
  *reinterpret_cast<float4*>(o) = x;
}
__device__ __forceinline__ void shift4(double* o, float4 m, double d) {
  double2 x = reinterpret_cast<double2*>(o)[0], y = reinterpret_cast<double2*>(o)[1];
  x = make_double2(shifted(x.x, m.x, d), shifted(x.y, m.y, d));
  y = make_double2(shifted(y.x, m.z, d), shifted(y.y, m.w, d));
  reinterpret_cast<double2*>(o)[0] = x;
  reinterpret_cast<double2*>(o)[1] = y;
}
template <typename T>
__global__ void __launch_bounds__(kCicThreads) k_astar_shift4(const float* __restrict__ mask, int64_t cells,
                                                              double off, const double* __restrict__ mean,
                                                              T* __restrict__ out) {
  const int r = blockIdx.y;
  const double d = mean[r] - off;
  T* o = out + (int64_t)r * cells;
  const int64_t n4 = cells / 4;
  const int64_t stride = (int64_t)gridDim.x * kCicThreads;
  for (int64_t i = blockIdx.x * (int64_t)kCicThreads + threadIdx.x; i < n4; i += stride) {
    const float4 m = mask ? reinterpret_cast<const float4*>(mask)[i] : make_float4(1.0f, 1.0f, 1.0f, 1.0f);
    shift4(o + 4 * i, m, d);
  }
}

// mean[r] = (sum of A*) / (unmasked cells) from the partials of one map, in a fixed order;
// 0 when every cell is masked.
__global__ void __launch_bounds__(kCicThreads) k_astar_mean(const double* __restrict__ partials, int64_t blocks,
                                                            double* __restrict__ mean) {
  const int r = blockIdx.x;
  __shared__ double sa[kCicThreads], sn[kCicThreads];
  double a = 0.0, n = 0.0;
  for (int64_t b = threadIdx.x; b < blocks; b += kCicThreads) {
    a += partials[((int64_t)r * blocks + b) * 2];
    n += partials[((int64_t)r * blocks + b) * 2 + 1];
  }
  sa[threadIdx.x] = a;
  sn[threadIdx.x] = n;
  __syncthreads();
  for (int h = kCicThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sa[threadIdx.x] += sa[threadIdx.x + h];
      sn[threadIdx.x] += sn[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) mean[r] = sn[0] > 0.0 ? sa[0] / sn[0] : 0.0;
}

template <typename T, int MODE>
hipError_t astar_launch(const int32_t* counts, const float* mask, int64_t cells, int64_t count, double nbar,
                        double s2, double off, T* out, double* partials, hipStream_t s) {
  const int64_t bx = blocks_per_map(cells);
  for (int64_t r0 = 0; r0 < count; r0 += kGridY) {
    const int64_t nr = count - r0 < kGridY ? count - r0 : kGridY;
    hipLaunchKernelGGL((k_astar<T, MODE>), dim3((unsigned)bx, (unsigned)nr), dim3(kCicThreads), 0, s,
                       counts + r0 * cells, mask, cells, nbar, log(nbar * s2), s2, off, out + r0 * cells,
                       MODE == 1 ? partials + r0 * bx * 2 : nullptr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t astar_all(const int32_t* counts, const float* mask, int64_t cells, int64_t count, double nbar,
                     double s2, bool subtract, T* out, double* partials, double* mean, hipStream_t s) {
  if (!mean) return astar_launch<T, 0>(counts, mask, cells, count, nbar, s2, 0.0, out, nullptr, s);
  const double off = subtract ? -0.5 * s2 : 0.0;
  hipError_t e = astar_launch<T, 1>(counts, mask, cells, count, nbar, s2, off, out, partials, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_astar_mean, dim3((unsigned)count), dim3(kCicThreads), 0, s, partials, blocks_per_map(cells),
                     mean);
  e = hipGetLastError();
  if (e != hipSuccess || !subtract) return e;
  const bool wide = cells % 4 == 0 && reinterpret_cast<uintptr_t>(out) % (4 * sizeof(T)) == 0 &&
                    reinterpret_cast<uintptr_t>(mask) % 16 == 0;
  const int64_t bx = blocks_per_map(wide ? cells / 4 : cells);
  for (int64_t r0 = 0; r0 < count; r0 += kGridY) {
    const int64_t nr = count - r0 < kGridY ? count - r0 : kGridY;
    if (wide)
      hipLaunchKernelGGL((k_astar_shift4<T>), dim3((unsigned)bx, (unsigned)nr), dim3(kCicThreads), 0, s, mask,
                         cells, off, mean + r0, out + r0 * cells);
    else
      hipLaunchKernelGGL((k_astar_shift<T>), dim3((unsigned)bx, (unsigned)nr), dim3(kCicThreads), 0, s, mask,
                         cells, off, mean + r0, out + r0 * cells);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Mean histogram under the model (Sec. 3.4): <P^(N)> = int dA G(A) sum_{f_i != 0} Pois(N; nbar
// f_i e^A), G the normal law N(-s2/2, s2) of the log-density.  The A integral is a fixed rule
// (nodes a_q, weights w_q summing to 1 over the law) applied by the host; this kernel forms, for
// each node q, per-workgroup sums over its cells of the Poisson pmf with lam = nbar f e^{a_q},
// CH values of N at a time in registers: the first of a chunk from logs,
// exp(N ln(lam) - lam - lgamma(N + 1)) (exp(-lam) for the first chunk), the others by
// p_{N+1} = p_N lam / (N + 1).  Each is reduced over the workgroup in a fixed order into
// partials[(q * gridDim.x + block) * nhist + N].  lgam holds lgamma(N + 1) for N < nhist, then
// 1 / N for N = 1 .. nhist (at lgam[nhist + N - 1]).
template <int CH>
__global__ void __launch_bounds__(kCicThreads) k_cic_predict(const float* __restrict__ mask, int64_t cells,
                                                            double nbar, const double* __restrict__ nodes,
                                                            const double* __restrict__ lgam, int nhist,
                                                            double* __restrict__ partials) {
  constexpr int kPredChunk = CH;
  __shared__ double red[kCicThreads / 64][kPredChunk];
  const int q = blockIdx.y;
  const double ea = exp(nodes[q]);
  const int64_t stride = (int64_t)gridDim.x * kCicThreads;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c0 = 0; c0 < nhist; c0 += kPredChunk) {
    double acc[kPredChunk], acc2[kPredChunk];
#pragma unroll
    for (int j = 0; j < kPredChunk; ++j) acc[j] = acc2[j] = 0.0;
    // two cells per step (independent recursions side by side); a masked cell (f = 0) or a
    // missing second cell contributes exactly 0 through its own accumulators
    for (int64_t i = blockIdx.x * (int64_t)kCicThreads + threadIdx.x; i < cells; i += 2 * stride) {
      const int64_t i2 = i + stride;
      const float f = mask ? mask[i] : 1.0f;
      const float f2 = i2 < cells ? (mask ? mask[i2] : 1.0f) : 0.0f;
      const double lam = nbar * (double)f * ea, lam2 = nbar * (double)f2 * ea;
      double p = 0.0, p2 = 0.0;
      if (f != 0.0f) p = c0 == 0 ? exp(-lam) : exp((double)c0 * log(lam) - lam - lgam[c0]);
      if (f2 != 0.0f) p2 = c0 == 0 ? exp(-lam2) : exp((double)c0 * log(lam2) - lam2 - lgam[c0]);
      acc[0] += p;
      acc2[0] += p2;
#pragma unroll
      for (int j = 1; j < kPredChunk; ++j) {
        const int N = c0 + j;
        if (N < nhist) {
          const double r = lgam[nhist + N - 1];
          p *= lam * r;
          p2 *= lam2 * r;
          acc[j] += p;
          acc2[j] += p2;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kPredChunk; ++j) acc[j] += acc2[j];
    // fixed-order reduction: within each wave by halving, then the waves in order
#pragma unroll
    for (int j = 0; j < kPredChunk; ++j) {
      double v = acc[j];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0) red[wave][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < kPredChunk && c0 + (int)threadIdx.x < nhist) {
      double t = 0.0;
      for (int w = 0; w < kCicThreads / 64; ++w) t += red[w][threadIdx.x];
      partials[((int64_t)q * gridDim.x + blockIdx.x) * nhist + c0 + threadIdx.x] = t;
    }
    __syncthreads();
  }
}

// out[N] = sum_q w_q sum_b partials[q][b][N]: one workgroup per N, each thread a fixed strided
// set of nodes (blocks summed in order), then a tree over the workgroup.
__global__ void __launch_bounds__(kCicThreads) k_cic_predict_sum(const double* __restrict__ partials, int nq,
                                                                int64_t blocks, const double* __restrict__ weights,
                                                                int nhist, double* __restrict__ out) {
  __shared__ double red[kCicThreads];
  const int N = blockIdx.x;
  double acc = 0.0;
  for (int q = threadIdx.x; q < nq; q += kCicThreads) {
    double s = 0.0;
    for (int64_t b = 0; b < blocks; ++b) s += partials[((int64_t)q * blocks + b) * nhist + N];
    acc += weights[q] * s;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kCicThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[N] = red[0];
}

// Cumulative information (eq. cuminfo): I(<= b) = 1^T C_b^-1 1 for the leading b x b blocks C_b of
// the normalised spectrum covariance.  With the Cholesky factor C = L L^T, the leading block of L
// is the factor of C_b, so I(<= b) = sum_{i <= b} z_i^2 with z = L^-1 1 (forward substitution):
// one factorisation gives every prefix.  One workgroup; L overwrites the lower triangle of a copy
// of C in `work` (nb x nb); z and the right-hand side live in LDS.  A pivot that is not positive
// (C_b not positive definite) makes I NaN from that shell on.
constexpr int kInfoThreads = 1024;

__global__ void __launch_bounds__(kInfoThreads) k_cumulative_information(const double* __restrict__ C, int nb,
                                                                        double* __restrict__ work,
                                                                        double* __restrict__ out) {
  extern __shared__ double sh[];  // rhs[nb], z[nb]
  double* rhs = sh;
  double* z = sh + nb;
  __shared__ int nok;
  const int tid = threadIdx.x;
  for (int64_t i = tid; i < (int64_t)nb * nb; i += kInfoThreads) work[i] = C[i];
  for (int i = tid; i < nb; i += kInfoThreads) rhs[i] = 1.0;
  if (tid == 0) nok = nb;
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (tid == 0) {
      const double d = work[(int64_t)j * nb + j];
      if (d > 0.0)
        work[(int64_t)j * nb + j] = sqrt(d);
      else
        nok = j;
    }
    __syncthreads();
    if (nok == j) break;
    const double ljj = work[(int64_t)j * nb + j];
    for (int i = j + 1 + tid; i < nb; i += kInfoThreads) work[(int64_t)i * nb + j] /= ljj;
    __syncthreads();
    const int m = nb - j - 1;
    for (int64_t t = tid; t < (int64_t)m * m; t += kInfoThreads) {
      const int ii = (int)(t / m), kk = (int)(t - (int64_t)ii * m);
      if (kk <= ii) {
        const int i = j + 1 + ii, k = j + 1 + kk;
        work[(int64_t)i * nb + k] -= work[(int64_t)i * nb + j] * work[(int64_t)k * nb + j];
      }
    }
    __syncthreads();
  }
  const int np = nok;
  for (int j = 0; j < np; ++j) {
    if (tid == 0) z[j] = rhs[j] / work[(int64_t)j * nb + j];
    __syncthreads();
    for (int i = j + 1 + tid; i < np; i += kInfoThreads) rhs[i] -= work[(int64_t)i * nb + j] * z[j];
    __syncthreads();
  }
  if (tid == 0) {
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) {
      if (b < np) acc += z[b] * z[b];
      out[b] = b < np ? acc : NAN;
    }
  }
}

}  // namespace

int64_t astar_partials(int64_t cells, int64_t count) { return blocks_per_map(cells) * count * 2; }

// workgroups per quadrature node: about 64 cells per thread, and a few thousand workgroups in all
int64_t cic_predict_blocks(int64_t cells, int nq) {
  int64_t b = (cells + kCicThreads * 64 - 1) / (kCicThreads * 64);
  const int64_t cap = 4096 / (nq > 0 ? nq : 1);
  if (b > cap) b = cap;
  return b < 1 ? 1 : b;
}

hipError_t launch_cic_predict(const float* mask, int64_t cells, double nbar, const double* nodes,
                              const double* weights, int nq, const double* lgam, int nhist, double* partials,
                              double* out, hipStream_t s) {
  const int64_t bx = cic_predict_blocks(cells, nq);
  // 24 values of N per pass and two cells per step: wide enough for two independent FP64
  // recursions per thread, narrow enough to keep several waves per SIMD to hide their latency
  // (on a 2^20-cell mask with 42 bins, about half the time of 16 values and one cell)
  hipLaunchKernelGGL(k_cic_predict<24>, dim3((unsigned)bx, (unsigned)nq), dim3(kCicThreads), 0, s, mask, cells,
                     nbar, nodes, lgam, nhist, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cic_predict_sum, dim3((unsigned)nhist), dim3(kCicThreads), 0, s, partials, nq, bx, weights,
                     nhist, out);
  return hipGetLastError();
}

hipError_t launch_cumulative_information(const double* C, int nb, double* work, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_cumulative_information, dim3(1), dim3(kInfoThreads), sizeof(double) * 2 * (size_t)nb, s, C,
                     nb, work, out);
  return hipGetLastError();
}

hipError_t launch_cic_histogram(const int32_t* counts, const float* mask, int64_t cells, int64_t count, int nhist,
                                unsigned long long* hist, hipStream_t s) {
  const int64_t n = count * nhist;
  hipLaunchKernelGGL(k_zero_i64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, hist, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = sizeof(uint32_t) * (size_t)hist_copies(nhist) * (size_t)hist_stride(nhist);
  const bool vec = (cells & 3) == 0 && (reinterpret_cast<uintptr_t>(counts) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(mask) & 15) == 0;
  const int64_t bx = blocks_per_map(vec ? cells / 4 : cells);
  for (int64_t r0 = 0; r0 < count; r0 += kGridY) {
    const int64_t nr = count - r0 < kGridY ? count - r0 : kGridY;
    if (vec)
      hipLaunchKernelGGL(k_cic_histogram<true>, dim3((unsigned)bx, (unsigned)nr), dim3(kCicThreads), lds, s,
                         counts + r0 * cells, mask, cells, nhist, hist + r0 * nhist);
    else
      hipLaunchKernelGGL(k_cic_histogram<false>, dim3((unsigned)bx, (unsigned)nr), dim3(kCicThreads), lds, s,
                         counts + r0 * cells, mask, cells, nhist, hist + r0 * nhist);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_astar(int prec, const int32_t* counts, const float* mask, int64_t cells, int64_t count,
                        double nbar, double s2, bool subtract, void* out, double* partials, double* mean,
                        hipStream_t s) {
  if (prec) return astar_all<double>(counts, mask, cells, count, nbar, s2, subtract, static_cast<double*>(out),
                                     partials, mean, s);
  return astar_all<float>(counts, mask, cells, count, nbar, s2, subtract, static_cast<float*>(out), partials,
                          mean, s);
}

}  // namespace ce
