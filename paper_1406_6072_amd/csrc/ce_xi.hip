// Lag tables of transformed two-point functions (FP64, plan time):
//  * the cell average of an isotropic omega over pairs of cells of a 2-D map, i.e. the square
//    top-hat filtered two-point function of App. A: the overlap integral eq. exactformula
//    for lags shorter than 15 cell sides, the derivative expansion eq. CoolEq beyond;
//  * the lognormal target ln(1 + value) (eq. Lncov), applied in place to a finished table;
//  * the spectrum of the k-space comparator: the continuous Fourier transform of an isotropic
//    xi on the modes of a periodic box (eq. Periodicboxmodes).
//
// The overlap integral is split into the four quadrants of [-1, 1]^2 (the weights
// (1 - |e_0|)(1 - |e_1|) have a kink at e_i = 0) and each axis of a quadrant is mapped with
// u = (1 - cos(pi t)) / 2, which clusters Gauss-Legendre nodes at both ends of [0, 1]: lags
// are whole cells, so the kink of the distance |theta + (h_0 e_0, h_1 e_1)| (where it
// vanishes) always sits on a quadrant corner.  48 nodes per axis give ~1e-14 relative
// accuracy for the supported kinds.  One workgroup sums one lag in a fixed order.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ce_internal.hpp"

namespace ce {

namespace {

constexpr int kQThreads = 256;

// isotropic omega(r): kind 1 = p0 exp(-r/p1); kind 2 = p0 (1 + r/p1)^-p2 exp(-r/p3) (p3 <= 0:
// no cut-off)
__device__ __forceinline__ double omega_iso(int kind, double p0, double p1, double p2, double p3, double r) {
  if (kind == 1) return p0 * exp(-r / p1);
  double v = p0 * pow(1.0 + r / p1, -p2);
  if (p3 > 0) v *= exp(-r / p3);
  return v;
}

// |theta|^2 < rn^2 with each product rounded (no contraction), as the host decides it
__device__ __forceinline__ bool lag_is_near(double t0, double t1, double rn2) {
#pragma clang fp contract(off)
  return t0 * t0 + t1 * t1 < rn2;
}

__global__ void __launch_bounds__(kQThreads) k_lag_near(int32_t O0, int32_t O1, double h0, double h1, double rn2,
                                                         int kind, double p0, double p1, double p2, double p3,
                                                         CellQuad q, double* __restrict__ out) {
  const int l0 = blockIdx.x, l1 = blockIdx.y;
  if (l0 >= O0 || l1 >= O1) return;
  const double t0 = h0 * (double)l0, t1 = h1 * (double)l1;
  if (!lag_is_near(t0, t1, rn2)) return;
  constexpr int n = kCellQuadNodes;
  double acc = 0.0;
  for (int k = threadIdx.x; k < 4 * n * n; k += kQThreads) {
    const int quad = k / (n * n), rem = k - quad * n * n;
    const int i = rem / n, j = rem - i * n;
    const double s0 = (quad & 1) ? -1.0 : 1.0, s1 = (quad & 2) ? -1.0 : 1.0;
    const double x = t0 + s0 * h0 * q.u[i], y = t1 + s1 * h1 * q.u[j];
    acc += q.a[i] * q.a[j] * omega_iso(kind, p0, p1, p2, p3, sqrt(x * x + y * y));
  }
  __shared__ double red[kQThreads];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kQThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(int64_t)l0 * O1 + l1] = red[0];
}

// eq. CoolEq for cells of sides (h0, h1): omega + (1 / (12 theta^2)) [ (sum h_i^2 theta_i^2 /
// theta^2)(D2 - 2 D1) + D1 sum h_i^2 ], D1 and D2 the first two derivatives of omega in ln theta
// from 5-point central differences of step `step`.
__global__ void k_lag_far(int32_t O0, int32_t O1, double h0, double h1, double rn2, int kind, double p0, double p1,
                          double p2, double p3, double step, double* __restrict__ out) {
  const int64_t nl = (int64_t)O0 * O1;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < nl;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l0 = idx / O1, l1 = idx - l0 * O1;
    const double t0 = h0 * (double)l0, t1 = h1 * (double)l1;
    if (lag_is_near(t0, t1, rn2)) continue;
    const double t2 = t0 * t0 + t1 * t1;
    const double lt = log(sqrt(t2));
    const double fm2 = omega_iso(kind, p0, p1, p2, p3, exp(lt - 2.0 * step));
    const double fm1 = omega_iso(kind, p0, p1, p2, p3, exp(lt - step));
    const double f0 = omega_iso(kind, p0, p1, p2, p3, exp(lt));
    const double fp1 = omega_iso(kind, p0, p1, p2, p3, exp(lt + step));
    const double fp2 = omega_iso(kind, p0, p1, p2, p3, exp(lt + 2.0 * step));
    const double d1 = (fm2 - 8.0 * fm1 + 8.0 * fp1 - fp2) / (12.0 * step);
    const double d2 = (-fm2 + 16.0 * fm1 - 30.0 * f0 + 16.0 * fp1 - fp2) / (12.0 * step * step);
    const double hh = h0 * h0 + h1 * h1;
    const double aniso = (h0 * h0 * t0 * t0 + h1 * h1 * t1 * t1) / t2;
    out[idx] = f0 + (aniso * (d2 - 2.0 * d1) + d1 * hh) / (12.0 * t2);
  }
}

// Continuous Fourier transform of an isotropic xi (eq. Periodicboxmodes), one workgroup per
// distinct squared frequency s of the box:
//   2-D: P(k) = 2 pi int_0^R r J0(k r) xi(r) dr,  3-D: P(k) = (4 pi / k) int_0^R r sin(k r) xi(r) dr,
// k = sqrt(s) kscale, over uniform panels of width min(pi / (2k), scale / 2) (a quarter of the
// oscillation and half the length scale of xi) with kHankelNodes Gauss-Legendre nodes each.
// R puts the exponential cut-off of xi at e^-40.  xi is ln(1 + omega) when lognormal != 0.
__global__ void __launch_bounds__(kQThreads) k_hankel(const int64_t* __restrict__ svals, double kscale, int ndim,
                                                       int kind, double p0, double p1, double p2, double p3,
                                                       int lognormal, double scale, double R, HankelRule g,
                                                       double* __restrict__ pvals) {
  const int64_t j = blockIdx.x;
  const double k = sqrt((double)svals[j]) * kscale;
  const double dl = fmin(M_PI / (2.0 * k), 0.5 * scale);
  const int64_t npan = (int64_t)ceil(R / dl);
  double acc = 0.0;
  for (int64_t p = threadIdx.x; p < npan; p += kQThreads) {
    const double a = (double)p * dl;
    double part = 0.0;
    for (int i = 0; i < kHankelNodes; ++i) {
      const double r = a + g.x[i] * dl;
      double xi = omega_iso(kind, p0, p1, p2, p3, r);
      if (lognormal) xi = log1p(xi);
      part += g.w[i] * r * (ndim == 2 ? j0(k * r) : sin(k * r)) * xi;
    }
    acc += part;
  }
  __shared__ double red[kQThreads];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int t = kQThreads / 2; t > 0; t >>= 1) {
    if ((int)threadIdx.x < t) red[threadIdx.x] += red[threadIdx.x + t];
    __syncthreads();
  }
  if (threadIdx.x == 0) pvals[j] = red[0] * dl * (ndim == 2 ? 2.0 * M_PI : 4.0 * M_PI / k);
}

// lambda on the box octant q_i in [0, half] (row-major): P(s) / h^d for s = sum q_i^2 > 0, and 0
// for the DC mode.
__global__ void k_fill_box_octant(int ndim, int32_t O, const int32_t* __restrict__ sidx,
                                  const double* __restrict__ pvals, double inv_hd, double* __restrict__ lam) {
  int64_t n = O;
  for (int d = 1; d < ndim; ++d) n *= O;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t rest = idx, s = 0;
    for (int d = 0; d < ndim; ++d) {
      const int64_t q = rest % O;
      rest /= O;
      s += q * q;
    }
    lam[idx] = s == 0 ? 0.0 : pvals[sidx[s]] * inv_hd;
  }
}

__global__ void k_log1p(double* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = log1p(p[i]);
}

}  // namespace

hipError_t launch_lag_cell_average(const int32_t* O, const double* h, int kind, const double* p, const CellQuad& q,
                                   double near_cells, double log_step, double* out, hipStream_t s) {
  const double hmax = h[0] > h[1] ? h[0] : h[1];
  const double rn = near_cells * hmax;
  const double rn2 = rn * rn;
  // lags with l_i h_i >= rn are never near: the near kernel covers the box below that
  const int64_t b0 = (int64_t)ceil(rn / h[0]) + 1, b1 = (int64_t)ceil(rn / h[1]) + 1;
  const unsigned g0 = (unsigned)(b0 < O[0] ? b0 : O[0]), g1 = (unsigned)(b1 < O[1] ? b1 : O[1]);
  hipLaunchKernelGGL(k_lag_near, dim3(g0, g1), dim3(kQThreads), 0, s, O[0], O[1], h[0], h[1], rn2, kind, p[0], p[1],
                     p[2], p[3], q, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nl = (int64_t)O[0] * O[1];
  const int blocks = (int)((nl + 255) / 256 < 65536 ? (nl + 255) / 256 : 65536);
  hipLaunchKernelGGL(k_lag_far, dim3(blocks), dim3(256), 0, s, O[0], O[1], h[0], h[1], rn2, kind, p[0], p[1], p[2],
                     p[3], log_step, out);
  return hipGetLastError();
}

hipError_t launch_box_spectrum(int ndim, int32_t half, const int64_t* svals, int64_t nvals, const int32_t* sidx,
                               double kscale, double inv_hd, int kind, const double* p, int lognormal, double scale,
                               double R, const HankelRule& g, double* pvals, double* lam, hipStream_t s) {
  hipLaunchKernelGGL(k_hankel, dim3((unsigned)nvals), dim3(kQThreads), 0, s, svals, kscale, ndim, kind, p[0], p[1],
                     p[2], p[3], lognormal, scale, R, g, pvals);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t n = half + 1;
  for (int d = 1; d < ndim; ++d) n *= half + 1;
  const int blocks = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
  hipLaunchKernelGGL(k_fill_box_octant, dim3(blocks), dim3(256), 0, s, ndim, half + 1, sidx, pvals, inv_hd, lam);
  return hipGetLastError();
}

hipError_t launch_log1p(double* p, int64_t n, hipStream_t s) {
  const int blocks = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
  hipLaunchKernelGGL(k_log1p, dim3(blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace ce
