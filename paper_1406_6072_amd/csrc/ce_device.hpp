// Device building blocks for gfx950: complex arithmetic, the Philox4x32-10
// counter generator, uniform and Box-Muller maps, radix DFTs and the in-place
// LDS Stockham stage used by every line-transform pass.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ce_internal.hpp"

namespace ce {

template <typename T>
struct cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> c_add(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> c_sub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> c_mul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> c_conj(cpx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> c_scale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by S*i (S = +1 or -1)
template <int S, typename T>
__device__ __forceinline__ cpx<T> c_rot(cpx<T> a) {
  return S > 0 ? cpx<T>{-a.y, a.x} : cpx<T>{a.y, -a.x};
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies by odd constants; the high halves are XOR-ed with the
// other two words and the round key, the key advances by two Weyl constants.
struct Words4 {
  uint32_t x0, x1, x2, x3;
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
  // The key is uniform over the wave.  The empty asm makes the compiler derive the ten
  // round keys here (scalar adds) rather than keep all twenty live across the caller's
  // loops, which overflows the scalar registers into VGPR lanes in the larger kernels.
  k0 = __builtin_amdgcn_readfirstlane(k0);
  k1 = __builtin_amdgcn_readfirstlane(k1);
  __asm__ volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t pa = (uint64_t)c0 * 0xD2511F53ull;
    const uint64_t pb = (uint64_t)c2 * 0xCD9E8D57ull;
    // three-input XOR in one instruction (gfx950 v_bitop3_b32, truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pb >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa >> 32), c3, k1, 0x96);
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = n0;
    c2 = n2;
  }
  return {c0, c1, c2, c3};
}

// Uniform in (0, 1): (x + 1/2) 2^-32.  FP64 exactly; FP32 as the single rounding
// of that value computed from float(x) (relative error below 2^-23).
__device__ __forceinline__ double unit64(uint32_t x) { return ((double)x + 0.5) * 0x1p-32; }
__device__ __forceinline__ float unit32(uint32_t x) { return __fmaf_rn((float)x, 0x1p-32f, 0x1p-33f); }
// 52-bit uniform from two words, exact in FP64.
__device__ __forceinline__ double unit52(uint32_t x0, uint32_t x1) {
  const uint64_t v = ((uint64_t)x0 << 20) | (uint64_t)(x1 >> 12);
  return ((double)v + 0.5) * 0x1p-52;
}

// Box-Muller: (r cos 2 pi u2, r sin 2 pi u2), r = sqrt(-2 ln u1).
__device__ __forceinline__ cpx<double> box_muller(double u1, double u2) {
  const double r = sqrt(-2.0 * log(u1));
  double s, c;
  sincospi(2.0 * u2, &s, &c);
  return {r * c, r * s};
}
// FP32: the hardware transcendentals -- v_log_f32 is log2 (-2 ln u = -2 ln2 log2 u) and
// v_sin_f32 / v_cos_f32 take their argument in revolutions, i.e. sin(2 pi u2) directly.
__device__ __forceinline__ cpx<float> box_muller(float u1, float u2) {
  const float r = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u1));
  return {r * __builtin_amdgcn_cosf(u2), r * __builtin_amdgcn_sinf(u2)};
}

template <typename T>
__device__ __forceinline__ cpx<T> normal_pair(uint32_t a, uint32_t b);
template <>
__device__ __forceinline__ cpx<double> normal_pair<double>(uint32_t a, uint32_t b) {
  return box_muller(unit64(a), unit64(b));
}
template <>
__device__ __forceinline__ cpx<float> normal_pair<float>(uint32_t a, uint32_t b) {
  return box_muller(unit32(a), unit32(b));
}

// ---------------------------------------------------------------------------
// LDS addressing: one padding slot every 16 elements breaks the power-of-two
// strides of the Stockham writes; lines are a pitch apart (odd offset).
__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }
__host__ __device__ inline int line_pitch(int L) { return L + (L >> 4) + 1; }

// Workgroup id -> logical tile so consecutive tiles share an XCD (and its L2):
// hardware places workgroup i on XCD i % 8.
__device__ __forceinline__ int64_t xcd_tile(int64_t i, int64_t G) {
  const int64_t q = G >> 3, rem = G & 7;
  const int64_t x = i & 7, k = i >> 3;
  return x * q + (x < rem ? x : rem) + k;
}

// ---------------------------------------------------------------------------
// Radix DFTs, X_k = sum_n v_n exp(S 2 pi i n k / R).

// cos / sin (2 pi m / 16), m = 0..15
__device__ constexpr double kC16[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440,
                                        0.38268343236508977173, 0.0, -0.38268343236508977173,
                                        -0.70710678118654752440, -0.92387953251128675613, -1.0,
                                        -0.92387953251128675613, -0.70710678118654752440,
                                        -0.38268343236508977173, 0.0, 0.38268343236508977173,
                                        0.70710678118654752440, 0.92387953251128675613};
__device__ constexpr double kS16[16] = {0.0, 0.38268343236508977173, 0.70710678118654752440,
                                        0.92387953251128675613, 1.0, 0.92387953251128675613,
                                        0.70710678118654752440, 0.38268343236508977173, 0.0,
                                        -0.38268343236508977173, -0.70710678118654752440,
                                        -0.92387953251128675613, -1.0, -0.92387953251128675613,
                                        -0.70710678118654752440, -0.38268343236508977173};

// multiply by exp(S 2 pi i m / 16) for a compile-time m in [0, 8)
template <int S, int M, typename T>
__device__ __forceinline__ cpx<T> tw16(cpx<T> a) {
  if constexpr (M == 0) {
    return a;
  } else if constexpr (M == 4) {
    return c_rot<S>(a);
  } else {
    const T c = (T)kC16[M], s = (T)(S * kS16[M]);
    return {a.x * c - a.y * s, a.x * s + a.y * c};
  }
}

template <int R, int S, typename T>
struct Pow2Dft;

template <int S, typename T>
struct Pow2Dft<1, S, T> {
  static __device__ __forceinline__ void run(cpx<T>*) {}
};

template <int S, typename T>
struct Pow2Dft<2, S, T> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    const cpx<T> a = v[0], b = v[1];
    v[0] = c_add(a, b);
    v[1] = c_sub(a, b);
  }
};

template <int R, int S, typename T>
struct Pow2Dft {
  template <int K>
  static __device__ __forceinline__ void combine(cpx<T>* v, const cpx<T>* e, const cpx<T>* o) {
    if constexpr (K < R / 2) {
      const cpx<T> t = tw16<S, K*(16 / R)>(o[K]);
      v[K] = c_add(e[K], t);
      v[K + R / 2] = c_sub(e[K], t);
      combine<K + 1>(v, e, o);
    }
  }
  static __device__ __forceinline__ void run(cpx<T>* v) {
    cpx<T> e[R / 2], o[R / 2];
#pragma unroll
    for (int n = 0; n < R / 2; ++n) {
      e[n] = v[2 * n];
      o[n] = v[2 * n + 1];
    }
    Pow2Dft<R / 2, S, T>::run(e);
    Pow2Dft<R / 2, S, T>::run(o);
    combine<0>(v, e, o);
  }
};

// Odd radix R, streamed: pairs n, R-n share cosines and sines, so only
// cos/sin(2 pi m / R) for m = 1..(R-1)/2 are needed; each output pair X_k, X_{R-k} is handed to
// put(k, X) as soon as it is formed.  TAB = false: the cosines and sines are in registers (cs,
// sn); TAB = true: they are read from the line's root table where used (tw[m step] =
// exp(-2 pi i m / R)): the address is uniform over the wave, so the values come through the
// scalar cache instead of occupying (R - 1) vector registers (radices 29 and 31).
template <int R, int S, bool TAB, typename T, typename Put>
__device__ __forceinline__ void odd_dft(cpx<T>* v, const T* cs, const T* sn, const cpx<T>* __restrict__ tw, int step,
                                        Put&& put) {
  constexpr int H = (R - 1) / 2;
  // sums and differences of the pairs n, R - n replace them in place, so the live set is
  // the R inputs plus the (R - 1) / 2 cosines and sines
#pragma unroll
  for (int n = 1; n <= H; ++n) {
    const cpx<T> p = v[n], q = v[R - n];
    v[n] = c_add(p, q);
    v[R - n] = c_sub(p, q);
  }
  cpx<T> x0 = v[0];
#pragma unroll
  for (int n = 1; n <= H; ++n) x0 = c_add(x0, v[n]);
  put(0, x0);
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    cpx<T> a = v[0], b = {T(0), T(0)};
#pragma unroll
    for (int n = 1; n <= H; ++n) {
      const int m = (n * k) % R;  // compile-time after unrolling
      const int mm = m <= H ? m : R - m;
      T c, s;
      if constexpr (TAB) {
        const cpx<T> w = tw[mm * step];
        c = w.x;
        s = m <= H ? -w.y : w.y;
      } else {
        c = cs[mm];
        s = m <= H ? sn[mm] : -sn[mm];
      }
      const cpx<T> sp = v[n];
      const cpx<T> dm = v[R - n];
      a.x += sp.x * c;
      a.y += sp.y * c;
      b.x += dm.x * s;
      b.y += dm.y * s;
    }
    const cpx<T> ib = c_rot<S>(b);
    put(k, c_add(a, ib));
    put(R - k, c_sub(a, ib));
  }
}

// odd_dft with output r stored at dst[pidx(base + r Ns)] when that index is below keep.
template <int R, int S, typename T>
__device__ __forceinline__ void odd_dft_store(cpx<T>* v, const T* cs, const T* sn, cpx<T>* dst, int base, int Ns,
                                              int keep) {
  odd_dft<R, S, false>(v, cs, sn, static_cast<const cpx<T>*>(nullptr), 0, [&](int r, cpx<T> x) {
    const int o = base + r * Ns;
    if (o < keep) dst[pidx(o)] = x;
  });
}

// One in-place Stockham stage of a power-of-two line FFT with every size known
// at compile time (Govindaraju et al. 2008 indexing): butterfly j reads
// elements j + r L/R, multiplies by exp(S 2 pi i r k/(Ns R)), k = j mod Ns, and
// writes (j/Ns) Ns R + k + r Ns.  All reads precede all writes (workgroup
// barrier), so the stage is in place.  Lane count NL = L/16 (one line per NL
// threads, 16 elements each).  With HALF only outputs below L/2 are formed and
// stored (the pruned last stage).  The twiddles of a stage are read as one
// contiguous vector: stw[k (R-1) + r - 1] = exp(-2 pi i r k / (Ns R)).
template <typename T, int S, int L, int R, int Ns, bool HALF>
__device__ __forceinline__ void stage_ct(cpx<T>* line, int lane, bool active, const cpx<T>* __restrict__ stw) {
  constexpr int NL = L / kEPT > 0 ? L / kEPT : 1;
  constexpr int nb = L / R;
  constexpr int NB = (nb + NL - 1) / NL;
  constexpr bool kExact = NB * NL == nb;
  cpx<T> v[NB][R];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lane + b * NL;
    if (active && (kExact || j < nb)) {
      if constexpr (nb % 16 == 0) {
        const int base = pidx(j);
#pragma unroll
        for (int r = 0; r < R; ++r) v[b][r] = line[base + r * (nb + nb / 16)];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[b][r] = line[pidx(j + r * nb)];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lane + b * NL;
    if (active && (kExact || j < nb)) {
      const int k = j & (Ns - 1);
      if constexpr (Ns > 1) {
        const cpx<T>* w = stw + k * (R - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> t = w[r - 1];
          if (S > 0) t.y = -t.y;
          v[b][r] = c_mul(v[b][r], t);
        }
      }
      Pow2Dft<R, S, T>::run(v[b]);
      constexpr int RK = HALF ? R / 2 : R;
      const int base = (j / Ns) * Ns * R + k;
      if constexpr (Ns % 16 == 0) {
        const int pb = pidx(base);
#pragma unroll
        for (int r = 0; r < RK; ++r) line[pb + r * (Ns + Ns / 16)] = v[b][r];
      } else if constexpr (Ns == 1) {
        const int pb = pidx(base);
#pragma unroll
        for (int r = 0; r < RK; ++r) line[pb + r] = v[b][r];
      } else {
#pragma unroll
        for (int r = 0; r < RK; ++r) line[pidx(base + r * Ns)] = v[b][r];
      }
    }
  }
  __syncthreads();
}

// Butterfly j of a mixed-radix stage with span Ns: k = j mod Ns (the twiddle index) and the
// output base (j / Ns) Ns R + k.  The quotient is umulhi(j, nsm), exact for j < 4096.
__device__ __forceinline__ void stage_index(int j, int Ns, uint32_t nsm, int R, int& k, int& base) {
  const int q = Ns > 1 ? (int)__umulhi((uint32_t)j, nsm) : j;
  k = j - q * Ns;
  base = q * Ns * R + k;
}

// Out-of-place Stockham stage (src -> dst LDS lines), any supported radix; one
// butterfly at a time, so the register footprint is one radix.  The twiddles of
// butterfly j are read as one contiguous vector: stw[k (R-1) + r - 1] =
// exp(-2 pi i r k / (Ns R)) (stages with Ns > 1).
template <typename T, int R, int S>
__device__ __forceinline__ void pingpong_stage(const cpx<T>* src, cpx<T>* dst, int L, int Ns, uint32_t nsm, int lane,
                                               int nlanes, bool active, const cpx<T>* __restrict__ tw,
                                               const cpx<T>* __restrict__ stw, int keep) {
  asm volatile("" : "+v"(lane));  // per-stage lane (no indices kept live across stages)
  constexpr bool kPow2 = (R & (R - 1)) == 0;
  constexpr int H = (R - 1) / 2;
  const int nb = L / R;
  T cs[H + 1], sn[H + 1];
  if constexpr (!kPow2) {
    const int Lr = L / R;
#pragma unroll
    for (int m = 1; m <= H; ++m) {
      const cpx<T> w = tw[m * Lr];
      cs[m] = w.x;
      sn[m] = -w.y;
    }
  }
  if (active) {
    for (int j = lane; j < nb; j += nlanes) {
      cpx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = src[pidx(j + r * nb)];
      int k, base;
      stage_index(j, Ns, nsm, R, k, base);
      if (Ns > 1) {
        const cpx<T>* w = stw + k * (R - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> t = w[r - 1];
          if (S > 0) t.y = -t.y;
          v[r] = c_mul(v[r], t);
        }
      }
      if constexpr (kPow2) {
        Pow2Dft<R, S, T>::run(v);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int o = base + r * Ns;
          if (o < keep) dst[pidx(o)] = v[r];
        }
      } else {
        odd_dft_store<R, S, T>(v, cs, sn, dst, base, Ns, keep);
      }
    }
  }
  __syncthreads();
}

// In-place Stockham stage of a mixed-radix line (R = 2, 4, 8, 16 or an odd prime up to 31): each thread
// loads the R inputs of all its butterflies j = lane + b nlanes (at most ceil(kEPT / R) of
// them, since nlanes >= L / kEPT) into registers, the workgroup waits, and then each butterfly
// is twiddled, transformed and stored into the same buffer.  One LDS buffer per line (the
// ping-pong form needs two), and all of a thread's loads are in flight together.
template <typename T, int R, int S>
__device__ __forceinline__ void inplace_stage(cpx<T>* line, int L, int Ns, uint32_t nsm, int lane, int nlanes,
                                              bool active, const cpx<T>* __restrict__ tw,
                                              const cpx<T>* __restrict__ stw, int keep) {
  constexpr bool kPow2 = (R & (R - 1)) == 0;
  constexpr int H = (R - 1) / 2;
  constexpr int NB = (kEPT + R - 1) / R;
  constexpr bool kTab = R >= 29;  // cosines and sines read where used
  const int nb = L / R;
  // the lane index is made opaque per stage: otherwise the butterfly indices and LDS offsets,
  // equal in every stage of one radix, are computed once and kept live across the whole
  // transform (they spill)
  asm volatile("" : "+v"(lane));
  T cs[H + 1], sn[H + 1];
  if constexpr (!kPow2 && !kTab) {
#pragma unroll
    for (int m = 1; m <= H; ++m) {
      const cpx<T> w = tw[m * nb];
      cs[m] = w.x;
      sn[m] = -w.y;
    }
  }
  // With one pad element per 16, pidx(x + r s) = pidx(x) + r (s + s / 16) when 16 divides s:
  // then a butterfly's R inputs (stride nb) or outputs (stride Ns) are one index plus a uniform
  // stride each, instead of a padded index per element.
  const bool lin_in = (nb & 15) == 0, lin_out = (Ns & 15) == 0;
  const int nbp = nb + (nb >> 4), nsp = Ns + (Ns >> 4);
  cpx<T> v[NB][R];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lane + b * nlanes;
    if (active && j < nb) {
      if (lin_in) {
        const int p0 = pidx(j);
#pragma unroll
        for (int r = 0; r < R; ++r) v[b][r] = line[p0 + r * nbp];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[b][r] = line[pidx(j + r * nb)];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lane + b * nlanes;
    if (active && j < nb) {
      int k, base;
      stage_index(j, Ns, nsm, R, k, base);
      if (Ns > 1) {
        const cpx<T>* w = stw + k * (R - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> t = w[r - 1];
          if (S > 0) t.y = -t.y;
          v[b][r] = c_mul(v[b][r], t);
        }
      }
      if (lin_out && base + (R - 1) * Ns < keep) {
        // every output kept, at one index plus a uniform stride
        cpx<T>* o = line + pidx(base);
        auto put = [&](int r, cpx<T> x) { o[r * nsp] = x; };
        if constexpr (kPow2) {
          Pow2Dft<R, S, T>::run(v[b]);
#pragma unroll
          for (int r = 0; r < R; ++r) put(r, v[b][r]);
        } else {
          odd_dft<R, S, kTab>(v[b], cs, sn, tw, nb, put);
        }
      } else {
        auto put = [&](int r, cpx<T> x) {
          const int o = base + r * Ns;
          if (o < keep) line[pidx(o)] = x;
        };
        if constexpr (kPow2) {
          Pow2Dft<R, S, T>::run(v[b]);
#pragma unroll
          for (int r = 0; r < R; ++r) put(r, v[b][r]);
        } else {
          odd_dft<R, S, kTab>(v[b], cs, sn, tw, nb, put);
        }
      }
    }
  }
  __syncthreads();
}

// Out-of-place stage of a prime radix R >= 11 with the inputs kept in LDS instead of
// registers: each butterfly owns its R source slots, so it overwrites them with the
// twiddled pair sums v[n] + v[R-n] and differences v[n] - v[R-n], then forms each output
// pair X_k, X_{R-k} by reading them back.  The register footprint is the (R - 1) / 2
// cosines and sines plus a few accumulators, so no radix spills.
template <typename T, int R, int S>
__device__ __forceinline__ void pingpong_stage_lds(cpx<T>* src, cpx<T>* dst, int L, int Ns, uint32_t nsm, int lane,
                                                   int nlanes, bool active, const cpx<T>* __restrict__ tw,
                                                   const cpx<T>* __restrict__ stw, int keep) {
  asm volatile("" : "+v"(lane));  // per-stage lane (no indices kept live across stages)
  constexpr int H = (R - 1) / 2;
  const int nb = L / R;
  T cs[H + 1], sn[H + 1];
  {
    const int Lr = L / R;
#pragma unroll
    for (int m = 1; m <= H; ++m) {
      const cpx<T> w = tw[m * Lr];
      cs[m] = w.x;
      sn[m] = -w.y;
    }
  }
  if (active) {
    for (int j = lane; j < nb; j += nlanes) {
      int k, base;
      stage_index(j, Ns, nsm, R, k, base);
      const cpx<T>* w = stw + k * (R - 1);
      auto twiddled = [&](int r) {
        cpx<T> x = src[pidx(j + r * nb)];
        if (Ns > 1 && r > 0) {
          cpx<T> t = w[r - 1];
          if (S > 0) t.y = -t.y;
          x = c_mul(x, t);
        }
        return x;
      };
      const cpx<T> v0 = twiddled(0);
      cpx<T> x0 = v0;
#pragma unroll
      for (int n = 1; n <= H; ++n) {
        const cpx<T> p = twiddled(n), q = twiddled(R - n);
        const cpx<T> sp = c_add(p, q);
        x0 = c_add(x0, sp);
        src[pidx(j + n * nb)] = sp;
        src[pidx(j + (R - n) * nb)] = c_sub(p, q);
      }
      if (base < keep) dst[pidx(base)] = x0;
#pragma unroll
      for (int kk = 1; kk <= H; ++kk) {
        cpx<T> a = v0, b = {T(0), T(0)};
#pragma unroll
        for (int n = 1; n <= H; ++n) {
          const int m = (n * kk) % R;  // compile-time after unrolling
          const int mm = m <= H ? m : R - m;
          const T c = cs[mm];
          const T sg = m <= H ? sn[mm] : -sn[mm];
          const cpx<T> sp = src[pidx(j + n * nb)];
          const cpx<T> dm = src[pidx(j + (R - n) * nb)];
          a.x += sp.x * c;
          a.y += sp.y * c;
          b.x += dm.x * sg;
          b.y += dm.y * sg;
        }
        const cpx<T> ib = c_rot<S>(b);
        const int o1 = base + kk * Ns, o2 = base + (R - kk) * Ns;
        if (o1 < keep) dst[pidx(o1)] = c_add(a, ib);
        if (o2 < keep) dst[pidx(o2)] = c_sub(a, ib);
        // keep the sums in LDS: no hoisting of the reads above into registers
        __asm__ volatile("" ::: "memory");
      }
    }
  }
  __syncthreads();
}

// The same for any odd prime R known only at run time (the primes above 31): the direct
// O(R^2) DFT of the pair sums and differences in the butterfly's own LDS slots; the angle
// 2 pi m / R of each term comes from the line's root table, tw[m L / R], with m = n kk mod R
// advanced incrementally (the index is uniform over the wave).
template <typename T, int S>
__device__ __forceinline__ void pingpong_stage_generic(cpx<T>* src, cpx<T>* dst, int L, int R, int Ns, uint32_t nsm,
                                                       int lane, int nlanes, bool active,
                                                       const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ stw,
                                                       int keep) {
  asm volatile("" : "+v"(lane));  // per-stage lane (no indices kept live across stages)
  const int H = (R - 1) / 2;
  const int nb = L / R;
  const int Lr = L / R;
  if (active) {
    for (int j = lane; j < nb; j += nlanes) {
      int k, base;
      stage_index(j, Ns, nsm, R, k, base);
      const cpx<T>* w = stw + k * (R - 1);
      auto twiddled = [&](int r) {
        cpx<T> x = src[pidx(j + r * nb)];
        if (Ns > 1 && r > 0) {
          cpx<T> t = w[r - 1];
          if (S > 0) t.y = -t.y;
          x = c_mul(x, t);
        }
        return x;
      };
      const cpx<T> v0 = twiddled(0);
      cpx<T> x0 = v0;
      for (int n = 1; n <= H; ++n) {
        const cpx<T> p = twiddled(n), q = twiddled(R - n);
        const cpx<T> sp = c_add(p, q);
        x0 = c_add(x0, sp);
        src[pidx(j + n * nb)] = sp;
        src[pidx(j + (R - n) * nb)] = c_sub(p, q);
      }
      if (base < keep) dst[pidx(base)] = x0;
      for (int kk = 1; kk <= H; ++kk) {
        cpx<T> a = v0, b = {T(0), T(0)};
        int m = 0;
        for (int n = 1; n <= H; ++n) {
          m += kk;
          if (m >= R) m -= R;
          // cos / sin (2 pi m / R) from the root exp(-2 pi i m' / R), m' = min(m, R - m)
          const bool lo = m <= H;
          const cpx<T> r = tw[(lo ? m : R - m) * Lr];
          const T c = r.x;
          const T sg = lo ? -r.y : r.y;
          const cpx<T> sp = src[pidx(j + n * nb)];
          const cpx<T> dm = src[pidx(j + (R - n) * nb)];
          a.x += sp.x * c;
          a.y += sp.y * c;
          b.x += dm.x * sg;
          b.y += dm.y * sg;
        }
        const cpx<T> ib = c_rot<S>(b);
        const int o1 = base + kk * Ns, o2 = base + (R - kk) * Ns;
        if (o1 < keep) dst[pidx(o1)] = c_add(a, ib);
        if (o2 < keep) dst[pidx(o2)] = c_sub(a, ib);
      }
    }
  }
  __syncthreads();
}

// Power-of-two lengths: the stage sequence is fixed at compile time (one
// straight-line instantiation per length), which keeps the register
// allocation to that of a single radix and turns every LDS offset into an
// immediate.  The radices match the host factorisation: 2, 4, 8, 16, 8.4, 8.8,
// 16.8, 16.16, 16.8.4, 16.8.8, 16.16.8, 16.16.16; the per-stage twiddle tables
// follow one another in stage order in f.stw (stages with Ns > 1 only).
template <typename T, int S, int L, int Ns, bool HALF, int... Rs>
struct StaticFft;
template <typename T, int S, int L, int Ns, bool HALF>
struct StaticFft<T, S, L, Ns, HALF> {
  static __device__ __forceinline__ void run(cpx<T>*, int, bool, const cpx<T>*) {}
};
template <typename T, int S, int L, int Ns, bool HALF, int R, int... Rs>
struct StaticFft<T, S, L, Ns, HALF, R, Rs...> {
  static __device__ __forceinline__ void run(cpx<T>* a, int lane, bool active, const cpx<T>* stw) {
    stage_ct<T, S, L, R, Ns, HALF && sizeof...(Rs) == 0>(a, lane, active, stw);
    StaticFft<T, S, L, Ns * R, HALF, Rs...>::run(a, lane, active, Ns > 1 ? stw + Ns * (R - 1) : stw);
  }
};

template <typename T, int S, bool HALF>
__device__ __forceinline__ void pow2_fft_h(cpx<T>* a, int L, int lane, bool active, const cpx<T>* stw) {
  switch (L) {
    case 2: StaticFft<T, S, 2, 1, HALF, 2>::run(a, lane, active, stw); break;
    case 4: StaticFft<T, S, 4, 1, HALF, 4>::run(a, lane, active, stw); break;
    case 8: StaticFft<T, S, 8, 1, HALF, 8>::run(a, lane, active, stw); break;
    case 16: StaticFft<T, S, 16, 1, HALF, 16>::run(a, lane, active, stw); break;
    case 32: StaticFft<T, S, 32, 1, HALF, 8, 4>::run(a, lane, active, stw); break;
    case 64: StaticFft<T, S, 64, 1, HALF, 8, 8>::run(a, lane, active, stw); break;
    case 128: StaticFft<T, S, 128, 1, HALF, 16, 8>::run(a, lane, active, stw); break;
    case 256: StaticFft<T, S, 256, 1, HALF, 16, 16>::run(a, lane, active, stw); break;
    case 512: StaticFft<T, S, 512, 1, HALF, 16, 8, 4>::run(a, lane, active, stw); break;
    case 1024: StaticFft<T, S, 1024, 1, HALF, 16, 8, 8>::run(a, lane, active, stw); break;
    case 2048: StaticFft<T, S, 2048, 1, HALF, 16, 16, 8>::run(a, lane, active, stw); break;
    default: StaticFft<T, S, 4096, 1, HALF, 16, 16, 16>::run(a, lane, active, stw); break;
  }
}

template <typename T, int S>
__device__ __forceinline__ void pow2_fft(cpx<T>* a, int L, int lane, bool active, const cpx<T>* stw, int keep) {
  if (keep == L)
    pow2_fft_h<T, S, false>(a, L, lane, active, stw);
  else
    pow2_fft_h<T, S, true>(a, L, lane, active, stw);
}

// Full line FFT.  Every thread of the workgroup must call it (barriers inside);
// threads without a line pass active = false.  MIX = 0: power-of-two lengths, in place in
// buffer a, registers staged across each barrier.  MIX = 1: the stages of f.rad (radices
// 2, 4, 8, 16 and the odd primes up to 7), in place in buffer a.  MIX = 2: the same with the
// primes 11..31 too (a larger register footprint; 29 and 31 read their cosines and sines from
// the root table where used).  MIX = 3: lengths with a prime factor above 31, every stage
// ping-pong between a and b (the generic prime stage keeps its inputs in LDS).
// Returns the buffer that holds the result.
template <typename T, int S, int MIX>
__device__ __forceinline__ cpx<T>* line_fft(cpx<T>* a, cpx<T>* b, const FftDesc& f, int lane, int nlanes, bool active,
                                           int keep) {
  const cpx<T>* __restrict__ tw = static_cast<const cpx<T>*>(f.tw);
  const int L = f.L;
  int Ns = 1;
  if constexpr (!MIX) {
    (void)b;
    (void)Ns;
    (void)tw;
    pow2_fft<T, S>(a, L, lane, active, static_cast<const cpx<T>*>(f.stw), keep);
    return a;
  } else if constexpr (MIX == 1 || MIX == 2) {
    (void)b;
    const cpx<T>* __restrict__ stw0 = static_cast<const cpx<T>*>(f.stw);
    for (int s = 0; s < f.nst; ++s) {
      const int R = f.rad[s];
      const int kp = (s == f.nst - 1) ? keep : L;
      const uint32_t nm = f.nsm[s];
      const cpx<T>* sw = stw0 + f.soff[s];
      switch (R) {
        case 2: inplace_stage<T, 2, S>(a, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 4: inplace_stage<T, 4, S>(a, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 8: inplace_stage<T, 8, S>(a, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 16: inplace_stage<T, 16, S>(a, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 3: inplace_stage<T, 3, S>(a, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 5: inplace_stage<T, 5, S>(a, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        default:
          if constexpr (MIX == 1) {
            inplace_stage<T, 7, S>(a, L, Ns, nm, lane, nlanes, active, tw, sw, kp);
          } else {
            switch (R) {
              case 7: inplace_stage<T, 7, S>(a, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
              case 11: inplace_stage<T, 11, S>(a, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
              case 13: inplace_stage<T, 13, S>(a, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
              case 17: inplace_stage<T, 17, S>(a, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
              case 19: inplace_stage<T, 19, S>(a, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
              case 23: inplace_stage<T, 23, S>(a, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
              case 29: inplace_stage<T, 29, S>(a, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
              default: inplace_stage<T, 31, S>(a, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
            }
          }
          break;
      }
      Ns *= R;
    }
    return a;
  } else {
    cpx<T>* src = a;
    cpx<T>* dst = b;
    const cpx<T>* __restrict__ stw0 = static_cast<const cpx<T>*>(f.stw);
    for (int s = 0; s < f.nst; ++s) {
      const int R = f.rad[s];
      const int kp = (s == f.nst - 1) ? keep : L;
      const uint32_t nm = f.nsm[s];
      const cpx<T>* sw = stw0 + f.soff[s];
      // the primes 11..31 have their own butterflies, larger primes the generic stage
      switch (R) {
        case 2: pingpong_stage<T, 2, S>(src, dst, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 4: pingpong_stage<T, 4, S>(src, dst, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 8: pingpong_stage<T, 8, S>(src, dst, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 16: pingpong_stage<T, 16, S>(src, dst, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 3: pingpong_stage<T, 3, S>(src, dst, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 5: pingpong_stage<T, 5, S>(src, dst, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 7: pingpong_stage<T, 7, S>(src, dst, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 11: pingpong_stage_lds<T, 11, S>(src, dst, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 13: pingpong_stage_lds<T, 13, S>(src, dst, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 17: pingpong_stage_lds<T, 17, S>(src, dst, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 19: pingpong_stage_lds<T, 19, S>(src, dst, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 23: pingpong_stage_lds<T, 23, S>(src, dst, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 29: pingpong_stage_lds<T, 29, S>(src, dst, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        case 31: pingpong_stage_lds<T, 31, S>(src, dst, L, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
        default: pingpong_stage_generic<T, S>(src, dst, L, R, Ns, nm, lane, nlanes, active, tw, sw, kp); break;
      }
      cpx<T>* t = src;
      src = dst;
      dst = t;
      Ns *= R;
    }
    return src;
  }
}

}  // namespace ce
