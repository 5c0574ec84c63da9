// Host side of the C ABI declared in include/cefield.h: contexts, embedding
// plans, FFT factorisation, pass geometry, scratch memory and the entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cctype>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/cefield.h"
#include "ce_internal.hpp"

using namespace ce;

namespace {

constexpr double kDefaultNegTol = 1e-13;
constexpr size_t kLdsBudget = 80 * 1024;   // per workgroup: two workgroups fit one CU
constexpr int kMaxSide = 4096;
constexpr int kPoissonSteps = 4096;

#define CE_HIP(expr)                                   \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_status(e_);       \
  } while (0)

#define CE_TRY(expr)                                   \
  do {                                                 \
    ce_status s_ = (expr);                             \
    if (s_ != CE_OK) return s_;                        \
  } while (0)

ce_status hip_status(hipError_t e) { return e == hipErrorOutOfMemory ? CE_E_OOM : CE_E_DEVICE; }

// Launch `expr` on stream s; with profiling on, bracket it with events under `name`.
#define CE_PROF(ctx, name, s, expr)                        \
  do {                                                     \
    hipEvent_t b_ = nullptr;                               \
    if ((ctx)->prof && !(ctx)->noalloc) (ctx)->prof_begin(name, s, &b_); \
    CE_HIP(expr);                                          \
    if (b_) (void)hipEventRecord(b_, s);                   \
  } while (0)

// ---- FFT factorisation ------------------------------------------------------

bool factor_length(int L, std::vector<int>& rad) {
  rad.clear();
  if (L < 2 || L > kMaxSide) return false;
  int n = L;
  std::vector<int> odd;  // odd prime factors, ascending (any prime: those above 31 use the generic radix)
  while (n % 2 == 0 && n > 1) n /= 2;
  for (int p = 3; p * p <= n; p += 2)
    while (n % p == 0) {
      odd.push_back(p);
      n /= p;
    }
  if (n > 1) odd.push_back(n);
  n = L;
  for (int p : odd) n /= p;  // the power of two that remains
  int e = 0;
  while ((1 << e) < n) ++e;
  // the power of two in radices of at most 16 (the compile-time stage sequences of the
  // power-of-two kernels use the same split)
  std::vector<int> p2;
  int n4 = e / 4, rem = e % 4;
  if (rem == 1 && n4 >= 1) {
    for (int i = 0; i < n4 - 1; ++i) p2.push_back(16);
    p2.push_back(8);
    p2.push_back(4);
  } else if (rem == 2 && n4 >= 1) {
    for (int i = 0; i < n4 - 1; ++i) p2.push_back(16);
    p2.push_back(8);
    p2.push_back(8);
  } else {
    for (int i = 0; i < n4; ++i) p2.push_back(16);
    if (rem == 3) p2.push_back(8);
    if (rem == 2) p2.push_back(4);
    if (rem == 1) p2.push_back(2);
  }
  // mixed lengths: the power of two first, then the odd primes.  A stage writes its outputs
  // with stride Ns (the product of the radices before it), so the small-stride writes fall on
  // radices 16 and 8, whose strides the LDS padding spreads over the banks, and the odd radices
  // write runs of Ns consecutive elements
  for (int p : p2) rad.push_back(p);
  for (int p : odd) rad.push_back(p);
  if (rad.size() > (size_t)kMaxStages) return false;
  return !rad.empty();
}

// LDS elements per line: the padded line (one pad per 16 elements) plus a shift that puts
// the lines of a workgroup on different banks (FP32: 4 elements = 8 banks per line, so the
// column loads of four lines at the same position do not collide; FP64: 1 element)
int line_pitch_host(int L, size_t elem) { return L + (L >> 4) + (elem == 8 ? 4 : 1); }

// Lines of length L (FFT), K kept; A x B lines per item.  Chooses R (power of two,
// lines per workgroup) within the LDS budget and the 1024-thread limit.
// True when the line FFT of f ping-pongs between two LDS buffers: a prime radix above 31 (the
// generic prime stage keeps its inputs in LDS; every other radix runs in place).
bool mixed_radix(const FftDesc& f) {
  for (int i = 0; i < f.nst; ++i)
    if ((f.rad[i] & (f.rad[i] - 1)) && f.rad[i] > 31) return true;
  return false;
}

LineGeom make_geom(int L, int K, int64_t A, int64_t B, int64_t nitems, int64_t in_item, int64_t out_item,
                   size_t elem, bool mix, int rmin, int rmax, size_t extra_per_line = 0,
                   size_t lds_budget = kLdsBudget) {
  LineGeom g;
  g.nbuf = mix ? 2 : 1;
  g.L = L;
  g.K = K;
  g.A = A;
  g.B = B;
  g.nitems = nitems;
  g.in_item = in_item;
  g.out_item = out_item;
  g.nlanes = (L + kEPT - 1) / kEPT;
  g.lpitch = line_pitch_host(L, elem);
  const size_t per_line = (size_t)g.lpitch * elem * g.nbuf + extra_per_line;
  int R = 1;
  while (R * 2 <= rmax && (size_t)(R * 2) * per_line <= lds_budget && R * 2 * g.nlanes <= kMaxWG) R *= 2;
  if (R < rmin) R = rmin;
  g.R = R;
  const int64_t nlines = A * B;
  g.groups_per_item = (nlines + R - 1) / R;
  g.items_total = nitems;
  return g;
}


}  // namespace

// ---- launch schedules ---------------------------------------------------------------

// Launch-shape knobs of the pipeline passes (all keep the results bitwise identical): lines per
// workgroup of the noise, inner-axis, last inverse and binning passes (0 = automatic), the noise
// pass's tile order and pair blocks, and the binning pass's LDS budget.
struct Schedule {
  int lines[4] = {0, 0, 0, 0};
  int noise_order = 0;
  int noise_block = 1;
  int noise_pairs = 0;  // 0: automatic
  size_t bin_lds = kLdsBudget;
};
// Shape a schedule is tuned for: (ndim, N_0, N_1, N_2, precision).
using ScheduleKey = std::tuple<int, int, int, int, int>;

// ---- static scratch of the allocation-free entry point ----------------------------

// Device memory of ce_pipeline_run_noalloc: a file-scope device array, one copy on every device
// the library runs on, held until the process ends.  Host code never passes the array's name to
// a kernel or a copy (on the host it is only a stand-in): it uses the device address that
// hipGetSymbolAddress returns, resolved once per device with that device current.
constexpr size_t kFixedScratchBytes = size_t(1) << 30;
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
void* g_fixed_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current).
ce_status fixed_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(g_fixed_mu);
  if (!g_fixed_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return CE_E_DEVICE;
    g_fixed_ptr[device] = p;
  }
  *out = g_fixed_ptr[device];
  return CE_OK;
}
}  // namespace

// ---- context -----------------------------------------------------------------

// Constant tables shared by every context of the process, one set per device: twiddles,
// per-stage twiddles and shell mode counts.  Built on first use, never freed (they are
// small), so contexts created later (request-server slots, graphs) find them ready.
struct SharedTables {
  std::mutex mu;
  std::map<std::tuple<int, int, int>, void*> tw, stw;  // (device, L, precision)
  std::map<std::tuple<int, int, int, int, int, int, int64_t>, std::pair<int64_t*, std::vector<double>>>
      shells;  // (device, n0, n1, n2, d, nb, cell-side ratios)
};
SharedTables& shared_tables() {
  static SharedTables* t = new SharedTables();
  return *t;
}

struct ce_ctx {
  int device = 0;
  size_t budget = 0;
  size_t held = 0;  // bytes of scratch + twiddles + shell tables
  hipStream_t own = nullptr;
  hipStream_t last = nullptr;
  uint32_t* flags = nullptr;
  double* inv = nullptr;  // RN(1/k), k = 0..kPoissonSteps, for the Poisson recursion
  std::mutex mu;
  struct Buf {
    void* p = nullptr;
    size_t n = 0;
    hipStream_t used = nullptr;  // stream of the last call that used the buffer
  };
  Buf ws[14];
  // pinned host staging of batch tables; `staged` is recorded after the copy that reads it
  void* pin = nullptr;
  size_t pin_n = 0;
  hipEvent_t staged = nullptr;

  // per-kernel timing with HIP events on the launch stream
  struct ProfRec {
    const char* name;
    hipEvent_t a, b;
  };
  bool prof = false;
  // Allocation-free calls: scratch slots are carved from the library's static device array
  // (base, size) instead of being allocated; noalloc_pairs is the chunk that fits it.
  bool noalloc = false;
  int64_t noalloc_pairs = 0;
  struct Arena {
    char* base = nullptr;
    size_t size = 0, off = 0;
    void* p[14] = {};
    size_t n[14] = {};
  } arena;
  bool unpruned = false;  // inverse passes keep every embedding output (comparator form)
  // Launch schedule: the context-wide options, the schedules tuned per shape, and the one in
  // force during a call (the tuned schedule of the call's shape, else the options).  Every
  // schedule gives bitwise identical results; only the launch shape changes.
  Schedule opts;
  std::map<ScheduleKey, Schedule> tuned;
  const Schedule* active = nullptr;
  const Schedule& sch() const { return active ? *active : opts; }
  // batched pipeline: groups of different shapes run concurrently on up to batch_lanes
  // sub-contexts (own scratch and stream), forked from and joined into the caller's stream
  int batch_lanes = 4;
  std::vector<ce_ctx*> lanes;
  hipEvent_t fork = nullptr;    // recorded on the caller's stream once the batch tables are copied
  hipEvent_t joined = nullptr;  // (lane sub-contexts) recorded after the lane's last group
  std::vector<ProfRec> pending;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  std::map<std::string, std::pair<double, int64_t>> agg;

  void prof_begin(const char* name, hipStream_t s, hipEvent_t* b) {
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (!pool.empty()) {
      ev = pool.back();
      pool.pop_back();
    } else if (hipEventCreate(&ev.first) != hipSuccess || hipEventCreate(&ev.second) != hipSuccess) {
      *b = nullptr;
      return;
    }
    (void)hipEventRecord(ev.first, s);
    pending.push_back({name, ev.first, ev.second});
    *b = ev.second;
  }
  void prof_resolve() {
    for (auto& r : pending) {
      float ms = 0;
      if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        auto& e = agg[r.name];
        e.first += ms;
        e.second += 1;
      }
      pool.push_back({r.a, r.b});
    }
    pending.clear();
  }

  ce_status alloc(void** p, size_t bytes) {
    if (budget && held + bytes > budget) return CE_E_OOM;
    hipError_t e = hipMalloc(p, bytes ? bytes : 1);
    if (e != hipSuccess) return hip_status(e);
    held += bytes;
    return CE_OK;
  }
  // host -> device copy of a constant table on the context's own non-blocking stream (does
  // not wait for work that other streams have in flight)
  ce_status upload(void* dst, const void* src, size_t bytes) {
    CE_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, own));
    CE_HIP(hipStreamSynchronize(own));
    return CE_OK;
  }
  void release(void* p, size_t bytes) {
    if (p) {
      (void)hipFree(p);
      held -= bytes;
    }
  }
  // Scratch slot i with at least `bytes`, for work on the stream of the current call
  // (`last`).  Growth is stream-ordered (hipFreeAsync / hipMallocAsync on that stream), so
  // it waits for nothing but this context's earlier work; if that work ran on another
  // stream, that stream is drained first.
  ce_status scratch(int i, size_t bytes, void** out) {
    if (noalloc) {
      // a slot keeps its region for the whole call (later chunks ask for no more)
      if (arena.p[i] && arena.n[i] >= bytes) {
        *out = arena.p[i];
        return CE_OK;
      }
      const size_t need = (bytes + 255) & ~(size_t)255;
      if (arena.off + need > arena.size) return CE_E_UNSUPPORTED;
      arena.p[i] = arena.base + arena.off;
      arena.n[i] = need;
      arena.off += need;
      *out = arena.p[i];
      return CE_OK;
    }
    Buf& b = ws[i];
    const hipStream_t s = last;
    if (b.n < bytes) {
      if (b.p) {
        if (b.used != s) CE_HIP(hipStreamSynchronize(b.used));
        CE_HIP(hipFreeAsync(b.p, s));
        held -= b.n;
        b.p = nullptr;
        b.n = 0;
      }
      if (budget && held + bytes > budget) return CE_E_OOM;
      void* p = nullptr;
      const hipError_t e = hipMallocAsync(&p, bytes, s);
      if (e != hipSuccess) return hip_status(e);
      held += bytes;
      b.p = p;
      b.n = bytes;
    }
    b.used = s;
    *out = b.p;
    return CE_OK;
  }
  // table memory is the process's (shared_tables), not charged to the context budget
  ce_status table_alloc(void** p, size_t bytes) {
    const hipError_t e = hipMalloc(p, bytes ? bytes : 1);
    return e == hipSuccess ? CE_OK : hip_status(e);
  }
  ce_status twiddles(int L, int prec, const void** out) {
    SharedTables& st = shared_tables();
    std::lock_guard<std::mutex> lock(st.mu);
    auto& tw = st.tw;
    const auto key = std::make_tuple(device, L, prec);
    auto it = tw.find(key);
    if (it != tw.end()) {
      *out = it->second;
      return CE_OK;
    }
    if (noalloc) return CE_E_UNSUPPORTED;  // built with the plan; never allocated here
    const size_t elem = prec ? 16 : 8;
    std::vector<double> d(2 * (size_t)L);
    for (int k = 0; k < L; ++k) {
      // reduce the angle to the first octant for accuracy
      const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)L;
      d[2 * k] = (double)std::cos(a);
      d[2 * k + 1] = (double)-std::sin(a);
    }
    void* p = nullptr;
    CE_TRY(table_alloc(&p, elem * L));
    if (prec) {
      CE_TRY(upload(p, d.data(), elem * L));
    } else {
      std::vector<float> f(2 * (size_t)L);
      for (size_t i = 0; i < f.size(); ++i) f[i] = (float)d[i];
      CE_TRY(upload(p, f.data(), elem * L));
    }
    tw[key] = p;
    *out = p;
    return CE_OK;
  }
  // Per-stage twiddles of a power-of-two length with stage radices rad: for each stage
  // with span Ns > 1, Ns x (R-1) values exp(-2 pi i r k / (Ns R)), k < Ns, r = 1..R-1.
  ce_status stage_twiddles(int L, int prec, const std::vector<int>& rad, const void** out) {
    SharedTables& st = shared_tables();
    std::lock_guard<std::mutex> lock(st.mu);
    auto& stw = st.stw;
    const auto key = std::make_tuple(device, L, prec);
    auto it = stw.find(key);
    if (it != stw.end()) {
      *out = it->second;
      return CE_OK;
    }
    if (noalloc) return CE_E_UNSUPPORTED;
    std::vector<double> d;
    int Ns = 1;
    for (int R : rad) {
      if (Ns > 1)
        for (int k = 0; k < Ns; ++k)
          for (int r = 1; r < R; ++r) {
            const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)(r * k) /
                                  (long double)(Ns * R);
            d.push_back((double)std::cos(a));
            d.push_back((double)-std::sin(a));
          }
      Ns *= R;
    }
    if (d.empty()) d.assign(2, 0.0);
    const size_t n = d.size() / 2;
    const size_t elem = prec ? 16 : 8;
    void* p = nullptr;
    CE_TRY(table_alloc(&p, elem * n));
    if (prec) {
      CE_TRY(upload(p, d.data(), elem * n));
    } else {
      std::vector<float> f(d.size());
      for (size_t i = 0; i < f.size(); ++i) f[i] = (float)d[i];
      CE_TRY(upload(p, f.data(), elem * n));
    }
    stw[key] = p;
    *out = p;
    return CE_OK;
  }
};

struct ce_plan {
  ce_ctx* ctx = nullptr;
  int ndim = 0;
  int n[3] = {1, 1, 1};
  int M[3] = {1, 1, 1};
  double h[3] = {1, 1, 1};
  int prec = 0;
  ce_plan_info info{};
  double* lam = nullptr;  // FP64 eigenvalue octant (before clamping)
  void* sq = nullptr;     // sqrt(lambda/M^d) octant in plan precision
  int64_t noct = 0;
  size_t bytes_lam = 0, bytes_sq = 0;
};

namespace {

// The tuned schedule of a shape, if any, is in force for the duration of a call on it.
struct ScheduleScope {
  ce_ctx* c;
  const Schedule* prev;
  ScheduleScope(ce_ctx* ctx, int ndim, const int* n, int prec) : c(ctx), prev(ctx->active) {
    const auto it = c->tuned.find(ScheduleKey(ndim, n[0], ndim >= 2 ? n[1] : 1, ndim >= 3 ? n[2] : 1, prec));
    c->active = it != c->tuned.end() ? &it->second : nullptr;
  }
  ~ScheduleScope() { c->active = prev; }
};

int cap_lines(const ce_ctx* ctx, int kind, int dflt) {
  const int c = ctx->sch().lines[kind];
  return c > 0 ? c : dflt;
}

// Geometry of the binning pass (lines of length N along axis 0 of the spectra, B of them per
// item) and its record block G.  The shell sums are recorded per block of G consecutive lines,
// G = the lines per workgroup of the default schedule (LDS budget kLdsBudget, at most 32 lines)
// capped at 4: it depends only on (N, nb, precision), and every schedule uses a multiple of G
// lines per workgroup, so the spectra do not depend on the schedule.
LineGeom bin_geom(const ce_ctx* ctx, int N, int nb, int64_t B, int64_t nitems, int64_t in_item, size_t elem,
                  bool mix, int* G_out) {
  LineGeom g = make_geom(N, N, 1, B, nitems, in_item, 0, elem, mix, 1, 1);
  auto fits = [&](int R, int G, size_t budget) {
    LineGeom t = g;
    t.R = R;
    return R * t.nlanes <= kMaxWG && bin_pass_lds(t, N, nb, G, elem) <= budget;
  };
  int Rd = 1;
  while (Rd * 2 <= 32 && fits(Rd * 2, std::min(4, Rd * 2), kLdsBudget)) Rd *= 2;
  const int G = std::min(4, Rd);
  int R = G;
  const int cap = cap_lines(ctx, 3, 32);
  while (R * 2 <= cap && fits(R * 2, G, ctx->sch().bin_lds)) R *= 2;
  g.R = R;
  g.groups_per_item = (B + R - 1) / R;
  *G_out = G;
  return g;
}

// The binning pass of an N-line spectrum with nb shells fits one workgroup's LDS (one line at a time).
bool bins_fit(int N, int nb, int prec) {
  std::vector<int> rad;
  if (!factor_length(N, rad)) return true;  // reported as unsupported elsewhere
  FftDesc f;
  f.nst = (int)rad.size();
  for (int i = 0; i < f.nst; ++i) f.rad[i] = rad[i];
  const size_t elem = prec ? 16 : 8;
  LineGeom g = make_geom(N, N, 1, 1, 1, 0, 0, elem, mixed_radix(f), 1, 1);
  return bin_pass_lds(g, N, nb, 1, elem) <= kMaxLdsBytes;
}

// Stage tables of a factorisation: span, quotient multiplier and twiddle offset per stage.
void stage_layout(FftDesc& f) {
  int Ns = 1, off = 0;
  for (int s = 0; s < f.nst; ++s) {
    f.ns[s] = Ns;
    f.nsm[s] = Ns > 1 ? (uint32_t)((((uint64_t)1 << 32) + (uint64_t)Ns - 1) / (uint64_t)Ns) : 0u;
    f.soff[s] = off;
    if (Ns > 1) off += Ns * (f.rad[s] - 1);
    Ns *= f.rad[s];
  }
}

ce_status build_fft(ce_ctx* ctx, int L, int prec, FftDesc& f) {
  std::vector<int> rad;
  if (!factor_length(L, rad)) return CE_E_UNSUPPORTED;
  f.L = L;
  f.nst = (int)rad.size();
  for (int i = 0; i < f.nst; ++i) f.rad[i] = rad[i];
  stage_layout(f);
  CE_TRY(ctx->twiddles(L, prec, &f.tw));
  CE_TRY(ctx->stage_twiddles(L, prec, rad, &f.stw));
  return CE_OK;
}

ce_status check_geometry(const ce_geometry* g) {
  if (!g) return CE_E_INVALID;
  if (g->ndim < 2 || g->ndim > 3) return g->ndim == 1 ? CE_E_UNSUPPORTED : CE_E_INVALID;
  double cells = 1;
  for (int i = 0; i < g->ndim; ++i) {
    if (g->n[i] < 4 || (g->n[i] & 1)) return g->n[i] < 1 ? CE_E_INVALID : CE_E_UNSUPPORTED;
    if (!(g->h[i] > 0) || !std::isfinite(g->h[i])) return CE_E_INVALID;
    if (2 * g->n[i] > kMaxSide) return CE_E_UNSUPPORTED;
    std::vector<int> r;
    if (!factor_length((int)(2 * g->n[i]), r) || !factor_length((int)g->n[i], r)) return CE_E_UNSUPPORTED;
    cells *= 2.0 * (double)g->n[i];
  }
  if (cells >= 4294967296.0) return CE_E_UNSUPPORTED;
  return CE_OK;
}

// Every pass of a plan fits one workgroup's LDS at its smallest shape: the noise pass holds two
// lines of the first periodic axis (cells 2p and 2p + 1 share a generator call), every other
// pass one line; lengths with a prime factor above 31 need two buffers per line.
bool passes_fit(const int* M, const int* n, int ndim, int prec) {
  const size_t elem = prec ? 16 : 8;
  auto line_bytes = [&](int L) {
    std::vector<int> rad;
    if (!factor_length(L, rad)) return (size_t)0;
    bool mix = false;
    for (int r : rad) mix |= (r & (r - 1)) != 0 && r > 31;
    return (size_t)line_pitch_host(L, elem) * elem * (mix ? 2 : 1);
  };
  if (2 * line_bytes(M[0]) > kMaxLdsBytes) return false;
  for (int d = 0; d < ndim; ++d)
    if (line_bytes(M[d]) > kMaxLdsBytes || line_bytes(n[d]) > kMaxLdsBytes) return false;
  return true;
}

ce_status check_xi(const ce_geometry* g, const ce_xi* xi) {
  if (xi->kind == CE_XI_TABLE) {
    if (!xi->table) return CE_E_INVALID;
  } else if (xi->kind == CE_XI_EXP || xi->kind == CE_XI_POWEXP) {
    if (!(xi->p[1] > 0) || !std::isfinite(xi->p[0])) return CE_E_INVALID;
  } else {
    return CE_E_INVALID;
  }
  if (xi->transform & ~(CE_XI_CELL_AVERAGE | CE_XI_LOGNORMAL)) return CE_E_INVALID;
  if ((xi->transform & CE_XI_CELL_AVERAGE) && (g->ndim != 2 || xi->kind == CE_XI_TABLE)) return CE_E_UNSUPPORTED;
  return CE_OK;
}

// Gauss-Legendre nodes x and weights w on [-1, 1] (n <= 64) by Newton's method on the Legendre
// three-term recurrence, in long double.
void gauss_legendre(int n, long double* xs, long double* ws) {
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int i = 0; i < n; ++i) {
    long double x = std::cos(pi * (i + 0.75L) / (n + 0.5L));
    long double dp = 1;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1);
      const long double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-19L) break;
    }
    xs[i] = x;
    ws[i] = 2 / ((1 - x * x) * dp * dp);
  }
}

// Cell-overlap rule: kCellQuadNodes Gauss-Legendre nodes on [0, 1] mapped by
// u = (1 - cos(pi t)) / 2 (nodes clustered at both ends), with the overlap weight folded in:
// a = w (pi/2) sin(pi t) (1 - u).
const CellQuad& cell_quad() {
  static const CellQuad q = [] {
    CellQuad c{};
    const long double pi = 3.14159265358979323846264338327950288L;
    long double xs[kCellQuadNodes], ws[kCellQuadNodes];
    gauss_legendre(kCellQuadNodes, xs, ws);
    for (int i = 0; i < kCellQuadNodes; ++i) {
      const long double t = (xs[i] + 1) / 2;
      const long double u = (1 - std::cos(pi * t)) / 2;
      c.u[i] = (double)u;
      c.a[i] = (double)((ws[i] / 2) * (pi / 2) * std::sin(pi * t) * (1 - u));
    }
    return c;
  }();
  return q;
}

// Gauss-Legendre rule on the unit panel [0, 1] for the Hankel transforms.
const HankelRule& hankel_rule() {
  static const HankelRule g = [] {
    HankelRule r{};
    long double xs[kHankelNodes], ws[kHankelNodes];
    gauss_legendre(kHankelNodes, xs, ws);
    for (int i = 0; i < kHankelNodes; ++i) {
      r.x[i] = (double)((xs[i] + 1) / 2);
      r.w[i] = (double)(ws[i] / 2);
    }
    return r;
  }();
  return g;
}

constexpr double kNearCells = 15.0;   // direct overlap integral below this many cell sides
constexpr double kLogStep = 2e-3;     // step in ln r of the finite differences of eq. CoolEq

// The (transformed) lag octant of xi on the device buffer `out`, asynchronously on s.
hipError_t build_lag_octant(const ce_geometry* geom, const ce_xi* xi, double* out, hipStream_t s) {
  int32_t O[3] = {1, 1, 1};
  double h[3] = {1, 1, 1};
  int64_t noct = 1;
  for (int i = 0; i < geom->ndim; ++i) {
    O[i] = (int32_t)geom->n[i] + 1;
    h[i] = geom->h[i];
    noct *= O[i];
  }
  const double p[4] = {xi->p[0], xi->p[1], xi->p[2], xi->p[3]};
  hipError_t e;
  if (xi->kind == CE_XI_TABLE)
    e = hipMemcpyAsync(out, xi->table, sizeof(double) * (size_t)noct, hipMemcpyHostToDevice, s);
  else if (xi->transform & CE_XI_CELL_AVERAGE)
    e = launch_lag_cell_average(O, h, xi->kind, p, cell_quad(), kNearCells, kLogStep, out, s);
  else
    e = launch_lag_octant(geom->ndim, O, h, xi->kind, p, out, s);
  if (e != hipSuccess) return e;
  if (xi->transform & CE_XI_LOGNORMAL) e = launch_log1p(out, noct, s);
  return e;
}

// Cell sides of the shells: h_ref = max h_i and h_i / h_ref = a_i / c_i, the fraction of
// smallest denominator c_i <= 64 within 1e-12 relative (square cells: a_i = c_i = 1).  False
// when a ratio has no such fraction (the integer shell rule needs one).  h may be null (unit
// cells).
struct CellRatios {
  double href = 1.0;
  double rho[3] = {1.0, 1.0, 1.0};  // h_i / h_ref
  int64_t a[3] = {1, 1, 1}, c[3] = {1, 1, 1};
};
bool cell_ratios(const double* h, int ndim, CellRatios& r) {
  r = CellRatios();
  if (!h) return true;
  r.href = 0.0;
  for (int i = 0; i < ndim; ++i) r.href = std::max(r.href, h[i]);
  if (!(r.href > 0)) return false;
  for (int i = 0; i < ndim; ++i) {
    const double rho = h[i] / r.href;
    r.rho[i] = rho;
    bool found = false;
    for (int den = 1; den <= 64 && !found; ++den) {
      const double num = std::round(rho * den);
      if (num >= 1 && std::fabs(num - rho * den) <= 1e-12 * rho * den) {
        r.a[i] = (int64_t)num;
        r.c[i] = den;
        found = true;
      }
    }
    if (!found) return false;
  }
  return true;
}

// h_0^d for square (cubic) cells, else the product of the sides
double cell_volume(const double* h, int ndim) {
  bool equal = true;
  double v = 1.0;
  for (int i = 0; i < ndim; ++i) {
    equal = equal && h[i] == h[0];
    v *= h[i];
  }
  return equal ? std::pow(h[0], ndim) : v;
}

// Integer shell rule of a grid with sides n[0..ndim) and cell sides h (nullable: unit cells):
// mode q~ is in shell s - 1 for the smallest s >= 0 with (s D)^2 >= t = sum_i T_i q~_i^2, with
// D = lcm(n_i a_i) and T_i = 4 nb^2 (c_i D / (n_i a_i))^2 (CellRatios; square cells: D = lcm(n_i),
// T_i = 4 nb^2 (D / n_i)^2, the cubic rule D = N, T = 4 nb^2).  Shells are linear in |k| up to
// pi / h_ref.  False when the cell sides have no small ratio or the integers could overflow.
struct ShellRule {
  int64_t T[3] = {0, 0, 0};
  int64_t LL = 1;
  int64_t D = 1;
  CellRatios cr;
};
bool shell_rule(const int* n, int ndim, int nb, ShellRule& r, const double* h = nullptr) {
  if (!cell_ratios(h, ndim, r.cr)) return false;
  int64_t L = 1;
  for (int i = 0; i < ndim; ++i) {
    const int64_t x = (int64_t)n[i] * r.cr.a[i];
    L = L / std::gcd(L, x) * x;
    if (L > (1ll << 24)) return false;
  }
  r.D = L;
  r.LL = L * L;
  double tmax = 0;
  for (int i = 0; i < ndim; ++i) {
    const int64_t m = r.cr.c[i] * (L / ((int64_t)n[i] * r.cr.a[i]));
    r.T[i] = 4ll * nb * nb * m * m;
    tmax += (double)r.T[i] * (double)(n[i] / 2) * (double)(n[i] / 2);
  }
  // t, the edges (s D)^2 for s <= nb + 1 and their differences stay far below 2^63
  return tmax < 1e17 && (double)(nb + 2) * (nb + 2) * (double)r.LL < 1e17;
}

// Integer thresholds of user shell edges e_0 < ... < e_nb (|k|): TH_b is
// v = nb^2 D^2 (e_b h_ref / pi)^2 in FP64 (in this order), the nearest integer when v lies
// within 1e-9 v of one, else floor(v); a mode with t is in shell b when TH_b < t <= TH_{b+1}.
void shell_thresholds(const int* n, int ndim, const double* h, int nb, const double* edges,
                      std::vector<int64_t>& th) {
  ShellRule sr;
  shell_rule(n, ndim, nb, sr, h);
  const double scale = (double)((int64_t)nb * nb * sr.D * sr.D);
  th.resize(nb + 1);
  for (int b = 0; b <= nb; ++b) {
    const double x = edges[b] * sr.cr.href / M_PI;
    const double v = scale * (x * x);
    const double r = std::floor(v + 0.5);
    const double c = std::fabs(v - r) <= 1e-9 * v ? r : std::floor(v);
    th[b] = c >= 4.0e18 ? (int64_t)4e18 : (int64_t)c;
  }
}

// Shell table (nmodes and mean |k| in units of 1 / h_ref) of a grid, host, exact integers; th
// (nullable): user shells as thresholds of t; h (nullable): cell sides.
void shell_table_host(const int* n, int ndim, int nb, std::vector<int64_t>& nm, std::vector<double>& km,
                      const std::vector<int64_t>* th = nullptr, const double* h = nullptr) {
  ShellRule sr;
  shell_rule(n, ndim, nb, sr, h);
  nm.assign(nb, 0);
  std::vector<double> ks(nb, 0.0);
  const int n0 = n[0], n1 = ndim >= 2 ? n[1] : 1, n2 = ndim >= 3 ? n[2] : 1;
  for (int a = 0; a < n0; ++a) {
    const int64_t qa = a <= n0 / 2 ? a : a - n0;
    for (int b = 0; b < n1; ++b) {
      const int64_t qb = ndim >= 2 ? (b <= n1 / 2 ? b : b - n1) : 0;
      for (int c = 0; c < n2; ++c) {
        const int64_t qc = ndim >= 3 ? (c <= n2 / 2 ? c : c - n2) : 0;
        const int64_t t = sr.T[0] * qa * qa + sr.T[1] * qb * qb + sr.T[2] * qc * qc;
        int64_t bin;
        if (th) {  // number of thresholds below t, minus one
          bin = (int64_t)(std::lower_bound(th->begin(), th->end(), t) - th->begin()) - 1;
        } else {   // smallest s >= 0 with s^2 D^2 >= t
          int64_t s = (int64_t)std::sqrt((double)t / (double)sr.LL);
          while (s > 0 && (s - 1) * (s - 1) * sr.LL >= t) --s;
          while (s * s * sr.LL < t) ++s;
          bin = s - 1;
        }
        if (bin >= 0 && bin < nb) {
          nm[bin] += 1;
          // |k| h_ref = 2 pi sqrt(sum_i ((q~_i / N_i) / (h_i / h_ref))^2)
          const double fa = ((double)qa / n0) / sr.cr.rho[0], fb = ((double)qb / n1) / sr.cr.rho[1],
                       fc = ((double)qc / n2) / sr.cr.rho[2];
          ks[bin] += 2.0 * M_PI * std::sqrt(fa * fa + fb * fb + fc * fc);
        }
      }
    }
  }
  km.assign(nb, 0.0);
  for (int i = 0; i < nb; ++i) km[i] = nm[i] ? ks[i] / (double)nm[i] : NAN;
}

ce_status device_shells(ce_ctx* ctx, const int* n, int ndim, int nb, int64_t** nm_dev,
                        const std::vector<double>** km_host, const double* h = nullptr) {
  SharedTables& st = shared_tables();
  std::lock_guard<std::mutex> lock(st.mu);
  CellRatios cr;
  cell_ratios(h, ndim, cr);
  int64_t sig = 0;  // the cell-side ratios (7 bits per number)
  for (int i = 0; i < 3; ++i) sig = (sig << 14) | (cr.a[i] << 7) | cr.c[i];
  auto key = std::make_tuple(ctx->device, n[0], ndim >= 2 ? n[1] : 1, ndim >= 3 ? n[2] : 1, ndim, nb, sig);
  auto it = st.shells.find(key);
  if (it == st.shells.end()) {
    std::vector<int64_t> nm;
    std::vector<double> km;
    shell_table_host(n, ndim, nb, nm, km, nullptr, h);
    void* p = nullptr;
    CE_TRY(ctx->table_alloc(&p, sizeof(int64_t) * nb));
    CE_TRY(ctx->upload(p, nm.data(), sizeof(int64_t) * nb));
    it = st.shells.emplace(key, std::make_pair(static_cast<int64_t*>(p), km)).first;
  }
  *nm_dev = it->second.first;
  *km_host = &it->second.second;
  return CE_OK;
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

}  // namespace

// ---- entry points ---------------------------------------------------------------

namespace {

ce_status prebuild_tables(ce_ctx* ctx, const ce_plan* p);

// A new plan's FFT tables are built with it (twiddles of every length its passes use), so the
// pipeline calls on it find them ready; on failure the plan is freed (ctx locked by the caller).
ce_status with_tables(ce_ctx* ctx, ce_status st, ce_plan** out) {
  if (st != CE_OK) return st;
  st = prebuild_tables(ctx, *out);
  if (st != CE_OK) {
    ce_plan* p = *out;
    ctx->release(p->lam, p->bytes_lam);
    ctx->release(p->sq, p->bytes_sq);
    delete p;
    *out = nullptr;
  }
  return st;
}

// Shared end of plan construction: the non-negativity check of eq. condition on the FP64
// eigenvalue octant `lam` (dims O), then sqrt(lambda / M^d) in the plan precision.  Takes
// ownership of lam and of spare (nullable, released here); on success the plan keeps lam.
ce_status finish_plan(ce_ctx* ctx, std::unique_ptr<ce_plan>& plan, double* lam, double* spare, const int32_t* O,
                      double neg_tol, double sigma2, ce_plan_info* info, ce_plan** out, hipStream_t s) {
  auto fail = [&](ce_status e) {
    (void)hipStreamSynchronize(s);
    ctx->release(lam, plan->bytes_lam);
    if (spare) ctx->release(spare, plan->bytes_lam);
    return e;
  };
  const int64_t noct = plan->noct;
  double* stats = nullptr;
  unsigned long long* nneg = nullptr;
  const size_t stat_bytes = sizeof(double) * 512 + 64;
  ce_status st = ctx->alloc((void**)&stats, stat_bytes);
  if (st != CE_OK) return fail(st);
  nneg = reinterpret_cast<unsigned long long*>(stats + 512);
  std::vector<double> hs(512);
  unsigned long long hneg = 0;
  bool ok = hipMemsetAsync(nneg, 0, 8, s) == hipSuccess &&
            launch_lambda_stats(lam, plan->ndim, O, noct, stats, nneg, s) == hipSuccess &&
            hipMemcpyAsync(hs.data(), stats, sizeof(double) * 512, hipMemcpyDeviceToHost, s) == hipSuccess &&
            hipMemcpyAsync(&hneg, nneg, 8, hipMemcpyDeviceToHost, s) == hipSuccess &&
            hipStreamSynchronize(s) == hipSuccess;
  ctx->release(stats, stat_bytes);
  if (!ok) return fail(CE_E_DEVICE);
  double lmin = INFINITY, lmax = -INFINITY;
  for (int i = 0; i < 256; ++i) {
    lmin = std::min(lmin, hs[2 * i]);
    lmax = std::max(lmax, hs[2 * i + 1]);
  }
  ce_plan_info pi{};
  pi.lambda_min = lmin;
  pi.lambda_max = lmax;
  pi.sigma2 = sigma2;
  pi.n_negative = (int64_t)hneg;
  pi.n_clamped = 0;
  if (!(lmax > 0) || lmin < -neg_tol * lmax || !std::isfinite(lmin) || !std::isfinite(lmax)) {
    if (info) *info = pi;
    return fail(CE_E_NOT_PSD);
  }
  pi.n_clamped = pi.n_negative;
  // sqrt(lambda / M^d) in the plan precision (Papos2 scale folded with the 1/M^d of the inverse DFT)
  double cells = 1;
  for (int d = 0; d < plan->ndim; ++d) cells *= plan->M[d];
  plan->bytes_sq = (plan->prec ? 8 : 4) * (size_t)noct;
  st = ctx->alloc(&plan->sq, plan->bytes_sq);
  if (st != CE_OK) return fail(st);
  if (launch_sqrt_table(lam, plan->ndim, O, 1.0 / cells, plan->prec, plan->sq, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    ctx->release(plan->sq, plan->bytes_sq);
    return fail(CE_E_DEVICE);
  }
  plan->lam = lam;
  if (spare) ctx->release(spare, plan->bytes_lam);
  pi.device_bytes = plan->bytes_lam + plan->bytes_sq;
  plan->info = pi;
  if (info) *info = pi;
  *out = plan.release();
  return CE_OK;
}

}  // namespace

extern "C" {

const char* ce_status_string(ce_status s) {
  switch (s) {
    case CE_OK: return "ok";
    case CE_E_INVALID: return "invalid argument";
    case CE_E_NOT_PSD: return "embedding spectrum is negative (the embedding is not positive semi-definite)";
    case CE_E_OOM: return "out of device memory or over the context budget";
    case CE_E_UNSUPPORTED: return "unsupported geometry or option";
    case CE_E_DEVICE: return "HIP runtime error";
    case CE_E_SAMPLER: return "device-side sampler or estimator condition flagged";
  }
  return "unknown status";
}

const char* ce_version(void) { return "cefield 0.1 (gfx950)"; }

ce_status ce_ctx_create(int device, size_t hbm_budget_bytes, ce_ctx** out) {
  if (!out) return CE_E_INVALID;
  *out = nullptr;
  int n = 0;
  CE_HIP(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return CE_E_INVALID;
  CE_HIP(hipSetDevice(device));
  auto ctx = std::make_unique<ce_ctx>();
  ctx->device = device;
  ctx->budget = hbm_budget_bytes;
  CE_HIP(hipStreamCreateWithFlags(&ctx->own, hipStreamNonBlocking));
  {
    // keep memory freed by the stream-ordered scratch growth in the device's default pool
    hipMemPool_t pool = nullptr;
    CE_HIP(hipDeviceGetDefaultMemPool(&pool, device));
    uint64_t keep = UINT64_MAX;
    CE_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
  }
  {
    // the static scratch's address on this device, resolved at set-up
    void* fixed = nullptr;
    CE_TRY(fixed_scratch(device, &fixed));
  }
  void* f = nullptr;
  CE_TRY(ctx->alloc(&f, 16));
  ctx->flags = static_cast<uint32_t*>(f);
  CE_HIP(hipMemsetAsync(ctx->flags, 0, 16, ctx->own));
  CE_HIP(hipStreamSynchronize(ctx->own));
  {
    std::vector<double> inv(kPoissonSteps + 1);
    inv[0] = 0.0;
    for (int k = 1; k <= kPoissonSteps; ++k) inv[k] = 1.0 / (double)k;  // IEEE: correctly rounded
    void* p = nullptr;
    CE_TRY(ctx->alloc(&p, sizeof(double) * inv.size()));
    ctx->inv = static_cast<double*>(p);
    CE_TRY(ctx->upload(ctx->inv, inv.data(), sizeof(double) * inv.size()));
  }
  *out = ctx.release();
  return CE_OK;
}

void ce_ctx_destroy(ce_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (ce_ctx* lc : ctx->lanes) ce_ctx_destroy(lc);
  ctx->lanes.clear();
  if (ctx->fork) (void)hipEventDestroy(ctx->fork);
  if (ctx->joined) (void)hipEventDestroy(ctx->joined);
  for (auto& b : ctx->ws)
    if (b.p) (void)hipFreeAsync(b.p, nullptr);
  (void)hipDeviceSynchronize();
  ctx->prof_resolve();
  for (auto& ev : ctx->pool) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  if (ctx->flags) (void)hipFree(ctx->flags);
  if (ctx->inv) (void)hipFree(ctx->inv);
  if (ctx->pin) (void)hipHostFree(ctx->pin);
  if (ctx->staged) (void)hipEventDestroy(ctx->staged);
  if (ctx->own) (void)hipStreamDestroy(ctx->own);
  delete ctx;
}

ce_status ce_ctx_trim(ce_ctx* ctx) {
  if (!ctx) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(ctx->mu);
  for (ce_ctx* lc : ctx->lanes) CE_TRY(ce_ctx_trim(lc));
  CE_HIP(hipSetDevice(ctx->device));
  bool any = false;
  for (auto& b : ctx->ws) any |= b.p != nullptr;
  if (!any) return CE_OK;
  CE_HIP(hipDeviceSynchronize());
  for (auto& b : ctx->ws) {
    if (b.p) {
      CE_HIP(hipFreeAsync(b.p, nullptr));
      ctx->held -= b.n;
    }
    b.p = nullptr;
    b.n = 0;
  }
  CE_HIP(hipDeviceSynchronize());
  return CE_OK;
}

ce_status ce_ctx_set_profiling(ce_ctx* ctx, int32_t enable) {
  if (!ctx) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(ctx->mu);
  ctx->prof = enable != 0;
  return CE_OK;
}

ce_status ce_ctx_profile_read(ce_ctx* ctx, int32_t max, char* names, double* total_ms, int64_t* launches,
                              int32_t* n) {
  if (!ctx || !n || max < 0 || (max > 0 && (!names || !total_ms || !launches))) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  ctx->prof_resolve();
  for (ce_ctx* lc : ctx->lanes) {  // kernels the batch lanes ran for this context
    lc->prof_resolve();
    for (auto& kv : lc->agg) {
      auto& e = ctx->agg[kv.first];
      e.first += kv.second.first;
      e.second += kv.second.second;
    }
    lc->agg.clear();
  }
  int32_t i = 0;
  for (auto& kv : ctx->agg) {
    if (i >= max) break;
    std::memset(names + 32 * i, 0, 32);
    std::strncpy(names + 32 * i, kv.first.c_str(), 31);
    total_ms[i] = kv.second.first;
    launches[i] = kv.second.second;
    ++i;
  }
  *n = i;
  ctx->agg.clear();
  return CE_OK;
}

ce_status ce_ctx_set_option(ce_ctx* ctx, int32_t option, int64_t value) {
  if (!ctx) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(ctx->mu);
  switch (option) {
    case CE_OPT_UNPRUNED: ctx->unpruned = value != 0; return CE_OK;
    case CE_OPT_LINES_NOISE:
    case CE_OPT_LINES_INNER:
    case CE_OPT_LINES_LAST:
    case CE_OPT_LINES_BINS:
      if (value < 0 || value > 64 || (value & (value - 1))) return CE_E_INVALID;
      ctx->opts.lines[option - CE_OPT_LINES_NOISE] = (int)value;
      return CE_OK;
    case CE_OPT_NOISE_ORDER:
      if (value != 0 && value != 1) return CE_E_INVALID;
      ctx->opts.noise_order = (int)value;
      return CE_OK;
    case CE_OPT_BIN_LDS:
      if (value < 16384 || value > 163840) return CE_E_INVALID;
      ctx->opts.bin_lds = (size_t)value;
      return CE_OK;
    case CE_OPT_NOISE_BLOCK:
      if (value < 1 || value > 65536) return CE_E_INVALID;
      ctx->opts.noise_block = (int)value;
      return CE_OK;
    case CE_OPT_NOISE_PAIRS:
      if (value < 0 || value > 64) return CE_E_INVALID;
      ctx->opts.noise_pairs = (int)value;
      return CE_OK;
    case CE_OPT_BATCH_LANES:
      if (value < 1 || value > 16) return CE_E_INVALID;
      ctx->batch_lanes = (int)value;
      return CE_OK;
    default: return CE_E_INVALID;
  }
}

ce_status ce_ctx_check(ce_ctx* ctx, void* stream) {
  if (!ctx) return CE_E_INVALID;
  CE_HIP(hipSetDevice(ctx->device));
  hipStream_t s = stream ? as_stream(stream) : ctx->last;
  uint32_t f = 0;
  CE_HIP(hipMemcpyAsync(&f, ctx->flags, sizeof(f), hipMemcpyDeviceToHost, s));
  CE_HIP(hipStreamSynchronize(s));
  for (ce_ctx* lc : ctx->lanes)  // the batch lanes' flags (their work was joined into the caller's stream)
    if (ce_ctx_check(lc, lc->own) == CE_E_SAMPLER) f |= 1u;
  if (f) {
    CE_HIP(hipMemsetAsync(ctx->flags, 0, sizeof(uint32_t), s));
    CE_HIP(hipStreamSynchronize(s));
    return CE_E_SAMPLER;
  }
  return CE_OK;
}

ce_status ce_plan_embedding(ce_ctx* ctx, const ce_geometry* geom, const ce_xi* xi, ce_precision precision,
                            double neg_tol, ce_plan** out, ce_plan_info* info) {
  if (!ctx || !geom || !xi || !out) return CE_E_INVALID;
  *out = nullptr;
  if (precision != CE_F32 && precision != CE_F64) return CE_E_INVALID;
  CE_TRY(check_geometry(geom));
  CE_TRY(check_xi(geom, xi));
  {
    int M[3] = {1, 1, 1}, nn[3] = {1, 1, 1};
    for (int i = 0; i < geom->ndim; ++i) {
      nn[i] = (int)geom->n[i];
      M[i] = 2 * nn[i];
    }
    if (!passes_fit(M, nn, geom->ndim, precision == CE_F64 ? 1 : 0)) return CE_E_UNSUPPORTED;
  }
  if (neg_tol < 0) neg_tol = kDefaultNegTol;
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  hipStream_t s = ctx->own;

  auto plan = std::make_unique<ce_plan>();
  plan->ctx = ctx;
  plan->ndim = geom->ndim;
  plan->prec = precision == CE_F64 ? 1 : 0;
  int32_t O[3] = {1, 1, 1};
  double h[3] = {1, 1, 1};
  int64_t noct = 1;
  for (int i = 0; i < geom->ndim; ++i) {
    plan->n[i] = (int)geom->n[i];
    plan->M[i] = 2 * (int)geom->n[i];
    plan->h[i] = geom->h[i];
    O[i] = plan->n[i] + 1;
    h[i] = geom->h[i];
    noct *= O[i];
  }
  plan->noct = noct;

  double* bufA = nullptr;
  double* bufB = nullptr;
  plan->bytes_lam = sizeof(double) * noct;
  CE_TRY(ctx->alloc((void**)&bufA, plan->bytes_lam));
  ce_status st = ctx->alloc((void**)&bufB, plan->bytes_lam);
  if (st != CE_OK) {
    ctx->release(bufA, plan->bytes_lam);
    return st;
  }
  auto fail = [&](ce_status e) {
    (void)hipStreamSynchronize(s);
    ctx->release(bufA, plan->bytes_lam);
    ctx->release(bufB, plan->bytes_lam);
    return e;
  };

  // lag octant c(l) = xi(h l)  (eq. grid: lags -N..N-1, minimum image), transformed
  double sigma2 = 0;
  if (build_lag_octant(geom, xi, bufA, s) != hipSuccess ||
      hipMemcpyAsync(&sigma2, bufA, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
    return fail(CE_E_DEVICE);
  // eq. Specd: DFT over the doubled grid, separable; the lag table is even in each
  // axis so each axis is a DCT-I of the octant (length-M FFT of the even extension).
  double* src = bufA;
  double* dst = bufB;
  for (int d = 0; d < geom->ndim; ++d) {
    int64_t A = 1, B = 1;
    for (int i = 0; i < d; ++i) A *= O[i];
    for (int i = d + 1; i < geom->ndim; ++i) B *= O[i];
    FftDesc f;
    st = build_fft(ctx, plan->M[d], 1, f);
    if (st != CE_OK) return fail(st);
    LineGeom g = make_geom(plan->M[d], O[d], A, B, 1, 0, 0, 16, mixed_radix(f), 1, B > 1 ? 64 : 1024);
    DctArgs a;
    a.in = src;
    a.out = dst;
    a.M = plan->M[d];
    if (launch_dct_axis(g, f, a, s) != hipSuccess) return fail(CE_E_DEVICE);
    std::swap(src, dst);
  }
  if (hipStreamSynchronize(s) != hipSuccess) return fail(CE_E_DEVICE);  // sigma2 has arrived
  return with_tables(ctx, finish_plan(ctx, plan, src, src == bufA ? bufB : bufA, O, neg_tol, sigma2, info, out, s),
                     out);
}

ce_status ce_plan_periodic(ce_ctx* ctx, const ce_geometry* geom, int64_t box, const ce_xi* xi,
                           ce_precision precision, double neg_tol, ce_plan** out, ce_plan_info* info) {
  if (!ctx || !geom || !xi || !out) return CE_E_INVALID;
  *out = nullptr;
  if (precision != CE_F32 && precision != CE_F64) return CE_E_INVALID;
  CE_TRY(check_geometry(geom));
  CE_TRY(check_xi(geom, xi));
  const int nd = geom->ndim;
  if (box < 2 || (box & 1)) return CE_E_INVALID;
  {
    int M[3] = {1, 1, 1}, nn[3] = {1, 1, 1};
    for (int i = 0; i < nd; ++i) {
      nn[i] = (int)geom->n[i];
      M[i] = (int)std::min<int64_t>(box, kMaxSide);
    }
    if (!passes_fit(M, nn, nd, precision == CE_F64 ? 1 : 0)) return CE_E_UNSUPPORTED;
  }
  for (int i = 0; i < nd; ++i) {
    if (geom->n[i] > box) return CE_E_INVALID;
    if (geom->h[i] != geom->h[0]) return CE_E_UNSUPPORTED;
  }
  if (box > kMaxSide) return CE_E_UNSUPPORTED;
  {
    std::vector<int> r;
    if (!factor_length((int)box, r)) return CE_E_UNSUPPORTED;
  }
  if (std::pow((double)box, nd) >= 4294967296.0) return CE_E_UNSUPPORTED;
  if (xi->kind == CE_XI_TABLE || (xi->transform & CE_XI_CELL_AVERAGE)) return CE_E_UNSUPPORTED;
  if (xi->kind == CE_XI_POWEXP && !(xi->p[3] > 0)) return CE_E_UNSUPPORTED;  // needs the cut-off
  if (neg_tol < 0) neg_tol = kDefaultNegTol;
  const double h = geom->h[0];
  const double scale = xi->kind == CE_XI_EXP ? xi->p[1] : std::min(xi->p[1], xi->p[3]);
  const double R = 40.0 * (xi->kind == CE_XI_EXP ? xi->p[1] : xi->p[3]);
  const double kscale = 2.0 * M_PI / ((double)box * h);
  const int32_t half = (int32_t)(box / 2);
  // distinct squared frequencies s = sum q_i^2 on the octant and their multiplicity on the box
  const int64_t smax = (int64_t)nd * half * half;
  std::vector<double> mult(smax + 1, 0.0);
  {
    const int64_t O = half + 1;
    int64_t q[3] = {0, 0, 0};
    int64_t n = 1;
    for (int d = 0; d < nd; ++d) n *= O;
    for (int64_t idx = 0; idx < n; ++idx) {
      int64_t rest = idx, s2 = 0;
      double w = 1;
      for (int d = 0; d < nd; ++d) {
        q[d] = rest % O;
        rest /= O;
        s2 += q[d] * q[d];
        if (q[d] != 0 && q[d] != half) w *= 2;
      }
      mult[s2] += w;
    }
  }
  std::vector<int64_t> svals;
  std::vector<int32_t> sidx(smax + 1, 0);
  for (int64_t v = 1; v <= smax; ++v)
    if (mult[v] > 0) {
      sidx[v] = (int32_t)svals.size();
      svals.push_back(v);
    }
  // bound the quadrature work: panels of the largest frequency times distinct values
  const double kmax = std::sqrt((double)smax) * kscale;
  const double npan_max = std::ceil(R / std::min(M_PI / (2 * kmax), 0.5 * scale));
  if (npan_max * (double)svals.size() > 2e10) return CE_E_UNSUPPORTED;

  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  hipStream_t s = ctx->own;
  auto plan = std::make_unique<ce_plan>();
  plan->ctx = ctx;
  plan->ndim = nd;
  plan->prec = precision == CE_F64 ? 1 : 0;
  int32_t O[3] = {1, 1, 1};
  int64_t noct = 1;
  for (int i = 0; i < nd; ++i) {
    plan->n[i] = (int)geom->n[i];
    plan->M[i] = (int)box;
    plan->h[i] = h;
    O[i] = half + 1;
    noct *= O[i];
  }
  plan->noct = noct;
  plan->bytes_lam = sizeof(double) * noct;
  double* lam = nullptr;
  CE_TRY(ctx->alloc((void**)&lam, plan->bytes_lam));
  // tables for the transform: svals, sidx, pvals
  const size_t b_s = sizeof(int64_t) * svals.size(), b_i = sizeof(int32_t) * sidx.size(),
               b_p = sizeof(double) * svals.size();
  void* tab = nullptr;
  ce_status st = ctx->alloc(&tab, b_s + b_i + b_p + 64);
  if (st != CE_OK) {
    ctx->release(lam, plan->bytes_lam);
    return st;
  }
  auto* d_s = static_cast<int64_t*>(tab);
  auto* d_p = reinterpret_cast<double*>(static_cast<char*>(tab) + b_s);
  auto* d_i = reinterpret_cast<int32_t*>(static_cast<char*>(tab) + b_s + b_p);
  std::vector<double> pv(svals.size());
  double inv_hd = 1;
  for (int d = 0; d < nd; ++d) inv_hd /= h;
  const double p[4] = {xi->p[0], xi->p[1], xi->p[2], xi->p[3]};
  bool ok = ctx->upload(d_s, svals.data(), b_s) == CE_OK && ctx->upload(d_i, sidx.data(), b_i) == CE_OK &&
            launch_box_spectrum(nd, half, d_s, (int64_t)svals.size(), d_i, kscale, inv_hd, xi->kind, p,
                                (xi->transform & CE_XI_LOGNORMAL) ? 1 : 0, scale, R, hankel_rule(), d_p, lam,
                                s) == hipSuccess &&
            hipMemcpyAsync(pv.data(), d_p, b_p, hipMemcpyDeviceToHost, s) == hipSuccess &&
            hipStreamSynchronize(s) == hipSuccess;
  ctx->release(tab, b_s + b_i + b_p + 64);
  if (!ok) {
    ctx->release(lam, plan->bytes_lam);
    return CE_E_DEVICE;
  }
  // cell variance of the box field: sum over the box of lambda / M^d, in a fixed order
  double sigma2 = 0;
  for (size_t j = 0; j < svals.size(); ++j) sigma2 += mult[svals[j]] * pv[j] * inv_hd;
  sigma2 /= std::pow((double)box, nd);
  return with_tables(ctx, finish_plan(ctx, plan, lam, nullptr, O, neg_tol, sigma2, info, out, s), out);
}

ce_status ce_xi_lag_octant(ce_ctx* ctx, const ce_geometry* geom, const ce_xi* xi, double* out, void* stream) {
  if (!ctx || !geom || !xi || !out) return CE_E_INVALID;
  CE_TRY(check_geometry(geom));
  CE_TRY(check_xi(geom, xi));
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  const hipStream_t s = as_stream(stream);
  CE_HIP(build_lag_octant(geom, xi, out, s));
  if (xi->kind == CE_XI_TABLE) CE_HIP(hipStreamSynchronize(s));  // the host table is read before returning
  return CE_OK;
}

void ce_plan_release(ce_plan* plan) {
  if (!plan) return;
  ce_ctx* ctx = plan->ctx;
  std::lock_guard<std::mutex> lock(ctx->mu);
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  ctx->release(plan->lam, plan->bytes_lam);
  ctx->release(plan->sq, plan->bytes_sq);
  delete plan;
}

ce_status ce_plan_get_info(const ce_plan* plan, ce_plan_info* info) {
  if (!plan || !info) return CE_E_INVALID;
  *info = plan->info;
  return CE_OK;
}

ce_status ce_plan_eigenvalues(const ce_plan* plan, double* out, void* stream) {
  if (!plan || !out) return CE_E_INVALID;
  CE_HIP(hipSetDevice(plan->ctx->device));
  CE_HIP(hipMemcpyAsync(out, plan->lam, plan->bytes_lam, hipMemcpyDeviceToDevice, as_stream(stream)));
  return CE_OK;
}

}  // extern "C"

// ---- pipeline driver ---------------------------------------------------------------

namespace {

struct InverseSetup {
  FftDesc fM[3];   // lengths M_i
  FftDesc fN[3];   // lengths N_i
};

ce_status setup_ffts(ce_ctx* ctx, const ce_plan* p, InverseSetup& s) {
  for (int d = 0; d < p->ndim; ++d) {
    CE_TRY(build_fft(ctx, p->M[d], p->prec, s.fM[d]));
    CE_TRY(build_fft(ctx, p->n[d], p->prec, s.fN[d]));
  }
  return CE_OK;
}

ce_status prebuild_tables(ce_ctx* ctx, const ce_plan* p) {
  InverseSetup fs;
  return setup_ffts(ctx, p, fs);
}

NoiseArgs noise_args(const ce_plan* p, uint64_t seed, uint32_t rid, uint64_t first_pair) {
  NoiseArgs n;
  n.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
  n.k1 = (uint32_t)(seed >> 32);
  n.rid = rid;
  n.first_pair = first_pair;
  n.ndim = p->ndim;
  for (int d = 0; d < 3; ++d) {
    n.M[d] = d < p->ndim ? p->M[d] : 1;
    n.O[d] = d < p->ndim ? p->M[d] / 2 + 1 : 1;
  }
  n.sq = p->sq;
  return n;
}

// Inverse passes for `npairs` pairs starting at pair index first_pair, through the
// last pass whose epilogue is `epi` (rows along the last axis).
ce_status run_inverse(ce_ctx* ctx, const ce_plan* p, const InverseSetup& fs, uint64_t seed, uint32_t rid,
                      uint64_t first_pair, int64_t npairs, RowEpi epi, hipStream_t s,
                      const unsigned long long* pair_base = nullptr, const PairDesc* desc = nullptr) {
  const size_t elem = p->prec ? 16 : 8;
  const int d = p->ndim;
  // the unpruned comparator form keeps all M outputs of every axis and crops at the end
  const bool full = ctx->unpruned && epi.mode == 1;
  const int64_t M0 = p->M[0], M1 = p->M[1], M2 = d == 3 ? p->M[2] : 1;
  const int64_t K0 = full ? M0 : p->n[0], K1 = full ? M1 : p->n[1];
  NoiseArgs na = noise_args(p, seed, rid, first_pair);
  na.pair_base = pair_base;
  na.desc = desc;
  epi.pair_base = pair_base;
  epi.desc = desc;
  // pass 1: axis 0 with the noise prologue; lines b over the remaining axes
  const int64_t B1 = M1 * M2;
  const int64_t y1_item = K0 * B1;
  void* y1 = nullptr;
  CE_TRY(ctx->scratch(0, elem * (size_t)(y1_item * npairs), &y1));
  LineGeom g1 = make_geom((int)M0, (int)K0, 1, B1, npairs, 0, y1_item, elem, mixed_radix(fs.fM[0]), 2,
                          cap_lines(ctx, 0, 32));
  g1.item_minor = ctx->sch().noise_order;
  g1.item_block = ctx->sch().noise_block;
  g1.mirror_order = 1;
  // each workgroup generates pairs_wg consecutive pairs of its lines, so the octant is fetched
  // once per pairs_wg pairs; automatic: the most (at most 8) that leave 4096 workgroups.  More
  // pairs per workgroup cut the octant reads further but let the workgroups that share the
  // output's cache lines drift apart in time, so partial lines are written back more than once.
  g1.pairs_wg = ctx->sch().noise_pairs;
  if (g1.pairs_wg <= 0) {
    g1.pairs_wg = 1;
    while (g1.pairs_wg < 8 && (npairs + 2 * g1.pairs_wg - 1) / (2 * g1.pairs_wg) * g1.groups_per_item >= 4096)
      g1.pairs_wg *= 2;
  }
  g1.items_total = npairs;
  g1.nitems = (npairs + g1.pairs_wg - 1) / g1.pairs_wg;
  CE_PROF(ctx, "noise_inverse_axis0", s, launch_noise_pass(p->prec, g1, fs.fM[0], na, y1, s));
  const void* last_in = y1;
  int64_t rows = K0;
  if (d == 3) {
    // pass 2: axis 1, lines (m0, q2)
    const int64_t y2_item = K0 * K1 * M2;
    void* y2 = nullptr;
    CE_TRY(ctx->scratch(1, elem * (size_t)(y2_item * npairs), &y2));
    LineGeom g2 = make_geom((int)M1, (int)K1, K0, M2, npairs, y1_item, y2_item, elem, mixed_radix(fs.fM[1]), 1,
                            cap_lines(ctx, 1, 32));
    CE_PROF(ctx, "inverse_axis1", s, launch_line_pass(p->prec, +1, g2, fs.fM[1], y1, y2, s));
    last_in = y2;
    rows = K0 * K1;
  }
  const int last = d - 1;
  const int64_t Ml = p->M[last], Kl = full ? Ml : p->n[last];
  epi.rows_per_m0 = d == 3 ? K1 : 1;
  epi.keep0 = p->n[0];
  epi.keep1 = d == 3 ? p->n[1] : 1;
  epi.keep_last = p->n[last];
  LineGeom gl = make_geom((int)Ml, (int)Kl, rows, 1, npairs, rows * Ml, 0, elem,
                          mixed_radix(fs.fM[last]) || (epi.mode == 2 && mixed_radix(epi.fwd)), 1,
                          cap_lines(ctx, 2, std::max(2, 256 / std::max(1, (int)Ml / kEPT))));
  if (epi.mode == 2) {
    // short rows, few of them: fewer rows per workgroup until the grid has ~2048 workgroups,
    // and the epilogue's cells spread over up to 256 threads (its FP64 sampler is
    // latency-bound when a thread holds many cells)
    const int64_t rows_total = rows * npairs;
    while (gl.R > 1 && rows_total / gl.R < 2048) gl.R /= 2;
    gl.groups_per_item = (rows + gl.R - 1) / gl.R;
    gl.threads = (int)std::min<int64_t>(256, (int64_t)gl.R * Kl);
  }
  CE_PROF(ctx, epi.mode == 2 ? "inverse_last_fused" : "inverse_last_fields", s,
          launch_row_inverse(p->prec, gl, fs.fM[last], epi, last_in, s));
  return CE_OK;
}

// Forward passes after the separated first forward pass (H rows of W), ending in the
// shell sums; partials per item.
ce_status run_forward_bins(ce_ctx* ctx, int ndim, const int* n, int prec, int64_t nitems, void* H, int nb,
                           double** partials_out, int64_t* groups_out, hipStream_t s,
                           const BinArgs* window = nullptr, const int64_t* th = nullptr,
                           const double* h = nullptr) {
  const size_t elem = prec ? 16 : 8;
  const int N = n[0];
  const int W = 2 * (n[ndim - 1] / 2 + 1);
  const int64_t rows = ndim == 3 ? (int64_t)n[0] * n[1] : n[0];
  const int64_t H_item = rows * W;
  if (ndim == 3) {
    FftDesc f1;
    CE_TRY(build_fft(ctx, n[1], prec, f1));
    LineGeom g2 = make_geom(n[1], n[1], n[0], W, nitems, H_item, H_item, elem, mixed_radix(f1), 1,
                            cap_lines(ctx, 1, 32));
    CE_PROF(ctx, "forward_axis1", s, launch_line_pass(prec, -1, g2, f1, H, H, s));
  }
  FftDesc f0;
  CE_TRY(build_fft(ctx, n[0], prec, f0));
  const int64_t Bb = ndim == 3 ? (int64_t)n[1] * W : W;
  int G = 1;
  LineGeom gb = bin_geom(ctx, n[0], nb, Bb, nitems, H_item, elem, mixed_radix(f0), &G);
  if (bin_pass_lds(gb, n[0], nb, G, elem) > kMaxLdsBytes) return CE_E_UNSUPPORTED;
  const int64_t nblocks = (Bb + G - 1) / G;
  void* part = nullptr;
  CE_TRY(ctx->scratch(3, sizeof(double) * (size_t)(nitems * nblocks * 2 * nb), &part));
  BinArgs ba;
  ba.ndim = ndim;
  ba.N = N;
  ba.N1 = ndim == 3 ? n[1] : 1;
  ba.nb = nb;
  ba.W = W;
  ShellRule sr;
  if (!shell_rule(n, ndim, nb, sr, h)) return CE_E_UNSUPPORTED;
  ba.T0 = sr.T[0];
  ba.T1 = ndim == 3 ? sr.T[1] : 0;
  ba.Tl = sr.T[ndim - 1];
  ba.LL = sr.LL;
  ba.th = th;
  ba.G = G;
  ba.partials = static_cast<double*>(part);
  if (window) {
    ba.win = window->win;
    ba.ntot = window->ntot;
    ba.fsum = window->fsum;
    ba.nest = window->nest;
  }
  CE_PROF(ctx, "forward_axis0_bins", s, launch_bin_pass(prec, gb, f0, ba, H, s));
  *partials_out = ba.partials;
  *groups_out = nblocks;
  return CE_OK;
}

int64_t survey_cells(const ce_plan* p) {
  int64_t c = 1;
  for (int d = 0; d < p->ndim; ++d) c *= p->n[d];
  return c;
}

// pairs per chunk so that the scratch stays within a cap
int64_t chunk_pairs(const ce_plan* p, int64_t npairs, size_t cap) {
  const size_t elem = p->prec ? 16 : 8;
  double per = 1;
  for (int d = 0; d < p->ndim; ++d) per *= p->M[d];
  per = per / 2 * elem * 2.0;  // pass-1 and pass-2 intermediates (upper bound)
  int64_t c = (int64_t)((double)cap / per);
  if (c < 1) c = 1;
  return std::min(c, npairs);
}

constexpr size_t kScratchCap = size_t(8) << 30;

// The fused pipeline on stream s (ctx locked by the caller).  pair_base (nullable) is a
// device counter added to every pair index (graph replays advance it).
ce_status pipeline_impl(ce_ctx* ctx, const ce_plan* plan, uint64_t seed, uint32_t request_id,
                        uint64_t first_realization, int64_t count, double nbar, int32_t nbins, void* out_fields,
                        void* out_delta, int32_t* out_counts, int64_t* out_ntot, double* out_pk, double* out_cov,
                        double* out_cnorm, const unsigned long long* pair_base, hipStream_t s,
                        const float* mask = nullptr, const void* win = nullptr, const double* fsum = nullptr,
                        const double* edges = nullptr) {
  ScheduleScope scope(ctx, plan->ndim, plan->n, plan->prec);
  InverseSetup fs;
  CE_TRY(setup_ffts(ctx, plan, fs));
  const int ndim = plan->ndim;
  // masked (2-D): the expected intensity nest scales the transformed rows; the binning pass
  // forms the contrast with the window transform win and sum(f)
  const double nest = nbar > 0 ? nbar : 1.0;
  const int64_t ncells = survey_cells(plan);
  const int Nl = plan->n[ndim - 1];
  const int W = 2 * (Nl / 2 + 1);
  const int64_t rows = ncells / Nl;
  const size_t elem = plan->prec ? 16 : 8;
  const size_t relem = plan->prec ? 8 : 4;
  const int64_t npairs = (count + 1) / 2;
  const int64_t cp = ctx->noalloc ? std::min(ctx->noalloc_pairs, npairs) : chunk_pairs(plan, npairs, kScratchCap);
  void* acc = nullptr;
  CE_TRY(ctx->scratch(4, sizeof(unsigned long long) * (size_t)(2 * npairs), &acc));
  auto* ntot = static_cast<unsigned long long*>(acc);
  CE_HIP(launch_zero_u64(ntot, 2 * npairs, s));
  int64_t* nm = nullptr;
  const std::vector<double>* km = nullptr;
  // user shell edges: thresholds and shell table for this call (scratch slot 13: [th | nmodes])
  const int64_t* th_dev = nullptr;
  if (edges) {
    std::vector<int64_t> th, nmu;
    std::vector<double> kmu;
    shell_thresholds(plan->n, ndim, plan->h, nbins, edges, th);
    shell_table_host(plan->n, ndim, nbins, nmu, kmu, &th, plan->h);
    th.insert(th.end(), nmu.begin(), nmu.end());
    void* p = nullptr;
    CE_TRY(ctx->scratch(13, sizeof(int64_t) * th.size(), &p));
    CE_HIP(hipMemcpyAsync(p, th.data(), sizeof(int64_t) * th.size(), hipMemcpyHostToDevice, s));
    CE_HIP(hipStreamSynchronize(s));  // the host table goes out of scope
    th_dev = static_cast<const int64_t*>(p);
    nm = static_cast<int64_t*>(p) + (nbins + 1);
  } else if (ctx->noalloc) {
    // the shell table counted on the device into the call's scratch (no table is allocated)
    ShellRule sr;
    if (!shell_rule(plan->n, ndim, nbins, sr, plan->h)) return CE_E_UNSUPPORTED;
    void* p = nullptr;
    CE_TRY(ctx->scratch(11, sizeof(int64_t) * (size_t)nbins, &p));
    nm = static_cast<int64_t*>(p);
    const int32_t nn[3] = {plan->n[0], ndim >= 2 ? plan->n[1] : 1, ndim >= 3 ? plan->n[2] : 1};
    CE_HIP(launch_zero_u64(reinterpret_cast<unsigned long long*>(nm), nbins, s));
    CE_HIP(launch_shell_counts(nn, sr.T, sr.LL, nbins, nm, s));
  } else {
    CE_TRY(device_shells(ctx, plan->n, ndim, nbins, &nm, &km, plan->h));
  }
  const double norm = cell_volume(plan->h, ndim) / (double)ncells;
  for (int64_t j = 0; j < npairs; j += cp) {
    const int64_t np = std::min(cp, npairs - j);
    void* H = nullptr;
    CE_TRY(ctx->scratch(2, elem * (size_t)(np * rows * W), &H));
    RowEpi e;
    e.mode = 2;
    e.ncells = ncells;
    e.count = std::min<int64_t>(count - 2 * j, 2 * np);
    e.real_off = 0;
    e.fields = out_fields ? static_cast<char*>(out_fields) + relem * (size_t)(2 * j * ncells) : nullptr;
    e.delta = out_delta ? static_cast<char*>(out_delta) + relem * (size_t)(2 * j * ncells) : nullptr;
    e.counts = out_counts ? out_counts + 2 * j * ncells : nullptr;
    e.ntot = ntot + 2 * j;
    e.flags = ctx->flags;
    e.inv = ctx->inv;
    e.s2half = 0.5 * plan->info.sigma2;
    e.nbar = nbar;
    e.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
    e.k1 = (uint32_t)(seed >> 32);
    e.rid = request_id;
    e.first_pair = first_realization / 2 + j;
    e.fwd = fs.fN[ndim - 1];
    e.H = H;
    e.H_item = rows * W;
    e.mask = mask;
    e.inv_nest = 1.0 / nest;
    CE_TRY(run_inverse(ctx, plan, fs, seed, request_id, first_realization / 2 + j, np, e, s, pair_base));
    double* partials = nullptr;
    int64_t groups = 0;
    BinArgs window;
    window.win = win;
    window.ntot = ntot + 2 * j;
    window.fsum = fsum;
    window.nest = nest;
    CE_TRY(run_forward_bins(ctx, ndim, plan->n, plan->prec, np, H, nbins, &partials, &groups, s,
                            mask ? &window : nullptr, th_dev, plan->h));
    CE_PROF(ctx, "bin_reduce", s,
            launch_bin_reduce(partials, np, groups, nbins, e.count, nm, norm, mask ? 2 : 1, ntot + 2 * j, nullptr,
                              (double)ncells, out_pk + 2 * j * nbins, ctx->flags, s));
  }
  if (out_ntot) CE_HIP(launch_copy_ntot(ntot, out_ntot, count, s));
  if (count >= 2 && (out_cov || out_cnorm))
    CE_PROF(ctx, "covariance", s, launch_covariance(out_pk, count, nbins, out_cov, out_cnorm, s));
  return CE_OK;
}

// Spectra of a stack of maps described by pl (first forward pass with the contrast or field
// load, remaining forward passes, shell sums, reduction): the standalone estimator and the
// spectrum stage of the masked pipeline.
ce_status spectrum_impl(ce_ctx* ctx, int ndim, const int* n, const double* h, int prec, PairLoad pl, int64_t count,
                        int32_t nbins, double* out_pk, int64_t* out_nmodes, double* out_kmean, hipStream_t s,
                        const double* edges = nullptr) {
  ScheduleScope scope(ctx, ndim, n, prec);
  int64_t ncells = 1;
  for (int d = 0; d < ndim; ++d) ncells *= n[d];
  const int64_t nitems = (count + 1) / 2;
  const int Nl = n[ndim - 1];
  const int W = 2 * (Nl / 2 + 1);
  const int64_t rows = ncells / Nl;
  const size_t elem = prec ? 16 : 8;
  void* H = nullptr;
  CE_TRY(ctx->scratch(2, elem * (size_t)(nitems * rows * W), &H));
  pl.H = H;
  pl.H_item = rows * W;
  FftDesc fl;
  CE_TRY(build_fft(ctx, Nl, prec, fl));
  LineGeom g1 = make_geom(Nl, Nl, rows, 1, nitems, 0, 0, elem, mixed_radix(fl), 1, 1024);
  CE_PROF(ctx, "forward_rows_pair", s, launch_pair_forward(prec, g1, fl, pl, s));
  // user shell edges: thresholds and shell table for this call (scratch slot 13: [th | nmodes])
  const int64_t* th_dev = nullptr;
  int64_t* nm = nullptr;
  const std::vector<double>* km = nullptr;
  std::vector<double> km_user;
  if (edges) {
    std::vector<int64_t> th, nmu;
    shell_thresholds(n, ndim, h, nbins, edges, th);
    shell_table_host(n, ndim, nbins, nmu, km_user, &th, h);
    std::vector<int64_t> tab(th);
    tab.insert(tab.end(), nmu.begin(), nmu.end());
    void* p = nullptr;
    CE_TRY(ctx->scratch(13, sizeof(int64_t) * tab.size(), &p));
    CE_HIP(hipMemcpyAsync(p, tab.data(), sizeof(int64_t) * tab.size(), hipMemcpyHostToDevice, s));
    CE_HIP(hipStreamSynchronize(s));  // the host table goes out of scope
    th_dev = static_cast<const int64_t*>(p);
    nm = static_cast<int64_t*>(p) + (nbins + 1);
    km = &km_user;
  }
  double* partials = nullptr;
  int64_t groups = 0;
  CE_TRY(run_forward_bins(ctx, ndim, n, prec, nitems, H, nbins, &partials, &groups, s, nullptr, th_dev, h));
  if (!edges) CE_TRY(device_shells(ctx, n, ndim, nbins, &nm, &km, h));
  const double norm = cell_volume(h, ndim) / (double)ncells;
  CE_PROF(ctx, "bin_reduce", s, launch_bin_reduce(partials, nitems, groups, nbins, count, nm, norm, 0, nullptr, nullptr, (double)ncells,
                           out_pk, ctx->flags, s));
  if (out_nmodes) CE_HIP(hipMemcpyAsync(out_nmodes, nm, sizeof(int64_t) * nbins, hipMemcpyDeviceToDevice, s));
  if (out_kmean) {
    std::vector<double> k(*km);
    CellRatios cr;
    cell_ratios(h, ndim, cr);
    for (double& v : k) v /= cr.href;
    CE_HIP(hipMemcpyAsync(out_kmean, k.data(), sizeof(double) * nbins, hipMemcpyHostToDevice, s));
    CE_HIP(hipStreamSynchronize(s));
  }
  return CE_OK;
}

// Forward transform Wm of the indicator f != 0 of a mask (the spectra's row pass on the map
// [f != 0] with an empty second map, then the remaining line transforms), rows x W complex in
// the plan precision in scratch slot 12, column-major for the binning pass: [column][q0] in
// 2-D, [q1][column][q0] in 3-D (the spectra's item layout transposed over q0).
ce_status window_transform(ce_ctx* ctx, const ce_plan* plan, const float* mask, void** out, hipStream_t s) {
  ScheduleScope scope(ctx, plan->ndim, plan->n, plan->prec);
  const int ndim = plan->ndim;
  const int N0 = plan->n[0], Nl = plan->n[ndim - 1];
  const int W = 2 * (Nl / 2 + 1);
  const int64_t rows = survey_cells(plan) / Nl;
  const int64_t item = rows * W;
  const size_t elem = plan->prec ? 16 : 8;
  void* H = nullptr;
  CE_TRY(ctx->scratch(2, elem * (size_t)item, &H));
  void* Wm = nullptr;
  CE_TRY(ctx->scratch(12, elem * (size_t)item, &Wm));
  PairLoad pl;
  pl.kind = 2;
  pl.count = 1;
  pl.ncells = survey_cells(plan);
  pl.mask = mask;
  pl.H = H;
  pl.H_item = item;
  FftDesc fl, f0;
  CE_TRY(build_fft(ctx, Nl, plan->prec, fl));
  CE_TRY(build_fft(ctx, N0, plan->prec, f0));
  LineGeom g1 = make_geom(Nl, Nl, rows, 1, 1, 0, 0, elem, mixed_radix(fl), 1, 1024);
  CE_PROF(ctx, "window_rows", s, launch_pair_forward(plan->prec, g1, fl, pl, s));
  if (ndim == 3) {
    FftDesc f1;
    CE_TRY(build_fft(ctx, plan->n[1], plan->prec, f1));
    LineGeom g2 = make_geom(plan->n[1], plan->n[1], N0, W, 1, item, item, elem, mixed_radix(f1), 1,
                            cap_lines(ctx, 1, 32));
    CE_PROF(ctx, "window_axis1", s, launch_line_pass(plan->prec, -1, g2, f1, H, H, s));
  }
  LineGeom g0 = make_geom(N0, N0, 1, item / N0, 1, item, item, elem, mixed_radix(f0), 1, cap_lines(ctx, 1, 32));
  CE_PROF(ctx, "window_axis0", s, launch_line_pass(plan->prec, -1, g0, f0, H, H, s));
  CE_PROF(ctx, "window_columns", s, launch_window_columns(plan->prec, H, Wm, N0, item / N0, s));
  *out = Wm;
  return CE_OK;
}

// The pipeline on a masked survey (rate nbar f rho; delta_g = (N/f - N^)/N^ on f != 0 with
// N^ = N_tot / sum f, eq. Estim), fused: the last inverse pass transforms N / (f nest) - 1 on
// f != 0 and the binning pass completes the contrast with the window transform.
ce_status pipeline_masked_impl(ce_ctx* ctx, const ce_plan* plan, const float* mask, uint64_t seed,
                               uint32_t request_id, uint64_t first_realization, int64_t count, double nbar,
                               int32_t nbins, void* out_fields, void* out_delta, int32_t* out_counts,
                               int64_t* out_ntot, double* out_pk, double* out_cov, double* out_cnorm, hipStream_t s,
                               const double* edges = nullptr) {
  // fused: the contrast is completed in the binning pass from the window transform
  void* fsd = nullptr;
  CE_TRY(ctx->scratch(9, sizeof(double) * 257, &fsd));
  CE_HIP(launch_mask_sum(mask, survey_cells(plan), static_cast<double*>(fsd), s));
  void* win = nullptr;
  CE_TRY(window_transform(ctx, plan, mask, &win, s));
  return pipeline_impl(ctx, plan, seed, request_id, first_realization, count, nbar, nbins, out_fields, out_delta,
                       out_counts, out_ntot, out_pk, out_cov, out_cnorm, nullptr, s, mask, win,
                       static_cast<const double*>(fsd), edges);
}

ce_status pipeline_check(ce_ctx* ctx, const ce_plan* plan, uint64_t first_realization, int64_t count, double nbar,
                         int32_t nbins, const double* out_pk) {
  if (!ctx || !plan || !out_pk || count <= 0 || nbins <= 0 || (first_realization & 1)) return CE_E_INVALID;
  if (!(nbar >= 0) || !std::isfinite(nbar)) return CE_E_INVALID;
  if (plan->ctx->device != ctx->device) return CE_E_INVALID;
  if ((first_realization + (uint64_t)count + 1) / 2 > 0xFFFFFFFFull) return CE_E_INVALID;
  ShellRule sr;  // cell sides with small ratios, integers within range
  if (!shell_rule(plan->n, plan->ndim, nbins, sr, plan->h)) return CE_E_UNSUPPORTED;
  if (!bins_fit(plan->n[0], nbins, plan->prec)) return CE_E_UNSUPPORTED;  // shells beyond one workgroup's LDS
  return CE_OK;
}

// The batched pipeline: items grouped by (ndim, N, h, precision, nbins); each group runs the
// fused passes once over all its pairs with per-pair descriptors.
// A group of batch items sharing (ndim, sides, periodic sides, cell sides, precision, shells, user
// edges): every pass runs as one launch over the group's pairs.
struct Group {
  std::vector<int64_t> idx;
  int64_t pairs = 0, covs = 0;
  size_t off_desc = 0, off_slot = 0, off_cov = 0, off_th = 0;
  std::vector<int64_t> tab;  // user shells: thresholds (nbins + 1) then N_b (nbins)
};
using GroupKey = std::tuple<int, int, int, int, int, int, int, std::array<double, 3>, int, int, std::vector<double>>;

// The sub-contexts of a context's batch lanes (created on first use, same device and schedule).
ce_status ensure_lanes(ce_ctx* ctx, int nl) {
  if (!ctx->fork) CE_HIP(hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
  while ((int)ctx->lanes.size() < nl) {
    ce_ctx* lc = nullptr;
    CE_TRY(ce_ctx_create(ctx->device, 0, &lc));
    if (hipEventCreateWithFlags(&lc->joined, hipEventDisableTiming) != hipSuccess) {
      ce_ctx_destroy(lc);
      return CE_E_DEVICE;
    }
    ctx->lanes.push_back(lc);
  }
  for (ce_ctx* lc : ctx->lanes) {
    lc->opts = ctx->opts;
    lc->tuned = ctx->tuned;
    lc->prof = ctx->prof;
  }
  return CE_OK;
}

// The fused passes of one group on context c and stream s; d is the device table area.
ce_status run_batch_group(ce_ctx* c, const ce_batch_item* items, Group& g, const GroupKey& key, const char* d,
                          hipStream_t s) {
  const ce_plan* plan = items[g.idx[0]].plan;
  ScheduleScope scope(c, plan->ndim, plan->n, plan->prec);
  const int nbins = std::get<9>(key);
  const auto* ddesc = reinterpret_cast<const PairDesc*>(d + g.off_desc);
  const auto* dslot = reinterpret_cast<const SlotOut*>(d + g.off_slot);
  InverseSetup fs;
  CE_TRY(setup_ffts(c, plan, fs));
  const int ndim = plan->ndim;
  const int64_t ncells = survey_cells(plan);
  const int Nl = plan->n[ndim - 1];
  const int W = 2 * (Nl / 2 + 1);
  const int64_t rows = ncells / Nl;
  const size_t elem = plan->prec ? 16 : 8;
  const int64_t npairs = g.pairs;
  const int64_t cp = chunk_pairs(plan, npairs, kScratchCap);
  void* acc = nullptr;
  CE_TRY(c->scratch(4, sizeof(unsigned long long) * (size_t)(2 * npairs), &acc));
  auto* ntot = static_cast<unsigned long long*>(acc);
  CE_HIP(launch_zero_u64(ntot, 2 * npairs, s));
  int64_t* nm = nullptr;
  const int64_t* th = nullptr;
  if (!g.tab.empty()) {
    th = reinterpret_cast<const int64_t*>(d + g.off_th);
    nm = reinterpret_cast<int64_t*>(const_cast<char*>(d) + g.off_th) + (nbins + 1);
  } else {
    const std::vector<double>* km = nullptr;
    CE_TRY(device_shells(c, plan->n, ndim, nbins, &nm, &km, plan->h));
  }
  const double norm = cell_volume(plan->h, ndim) / (double)ncells;
  for (int64_t j = 0; j < npairs; j += cp) {
    const int64_t np = std::min(cp, npairs - j);
    void* H = nullptr;
    CE_TRY(c->scratch(2, elem * (size_t)(np * rows * W), &H));
    RowEpi e;
    e.mode = 2;
    e.ncells = ncells;
    e.count = 2 * np;
    e.ntot = ntot + 2 * j;
    e.flags = c->flags;
    e.inv = c->inv;
    e.fwd = fs.fN[ndim - 1];
    e.H = H;
    e.H_item = rows * W;
    CE_TRY(run_inverse(c, plan, fs, 0, 0, 0, np, e, s, nullptr, ddesc + j));
    double* partials = nullptr;
    int64_t ngroups = 0;
    CE_TRY(run_forward_bins(c, ndim, plan->n, plan->prec, np, H, nbins, &partials, &ngroups, s, nullptr, th,
                            plan->h));
    CE_PROF(c, "bin_reduce", s,
            launch_bin_reduce(partials, np, ngroups, nbins, 2 * np, nm, norm, 1, ntot + 2 * j, dslot + 2 * j,
                              (double)ncells, nullptr, c->flags, s));
  }
  if (g.covs)
    CE_PROF(c, "covariance", s,
            launch_covariance_batch(reinterpret_cast<const CovItem*>(d + g.off_cov), g.covs, nbins, s));
  return CE_OK;
}

ce_status pipeline_batch_impl(ce_ctx* ctx, const ce_batch_item* items, int64_t n, hipStream_t s) {
  std::map<GroupKey, Group> groups;
  for (int64_t i = 0; i < n; ++i) {
    const ce_batch_item& it = items[i];
    if (!it.plan) return CE_E_INVALID;
    CE_TRY(pipeline_check(ctx, it.plan, it.first_realization, it.count, it.nbar, it.nbins, it.out_pk));
    std::vector<double> ev;
    if (it.kedges) {
      for (int b = 0; b <= it.nbins; ++b)
        if (!std::isfinite(it.kedges[b]) || it.kedges[b] < 0 || (b > 0 && !(it.kedges[b] > it.kedges[b - 1])))
          return CE_E_INVALID;
      ev.assign(it.kedges, it.kedges + it.nbins + 1);
    }
    const ce_plan* pl = it.plan;
    const std::array<double, 3> hs{pl->h[0], pl->ndim >= 2 ? pl->h[1] : 0.0, pl->ndim >= 3 ? pl->h[2] : 0.0};
    Group& g = groups[std::make_tuple(pl->ndim, pl->n[0], pl->n[1], pl->n[2], pl->M[0], pl->M[1], pl->M[2], hs,
                                      pl->prec, (int)it.nbins, std::move(ev))];
    g.idx.push_back(i);
    g.pairs += (it.count + 1) / 2;
    if (it.count >= 2 && (it.out_cov || it.out_cnorm)) g.covs++;
  }
  // one table area: per group [PairDesc x pairs][SlotOut x 2 pairs][CovItem x covs]
  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t bytes = 0;
  for (auto& kv : groups) {
    Group& g = kv.second;
    g.off_desc = bytes;
    bytes = align(bytes + sizeof(PairDesc) * (size_t)g.pairs);
    g.off_slot = bytes;
    bytes = align(bytes + sizeof(SlotOut) * (size_t)(2 * g.pairs));
    g.off_cov = bytes;
    bytes = align(bytes + sizeof(CovItem) * (size_t)g.covs);
    const std::vector<double>& ev = std::get<10>(kv.first);
    if (!ev.empty()) {
      const ce_plan* p = items[g.idx[0]].plan;
      const int nbins = std::get<9>(kv.first);
      std::vector<int64_t> nmu;
      std::vector<double> kmu;
      shell_thresholds(p->n, p->ndim, p->h, nbins, ev.data(), g.tab);
      shell_table_host(p->n, p->ndim, nbins, nmu, kmu, &g.tab, p->h);
      g.tab.insert(g.tab.end(), nmu.begin(), nmu.end());
      g.off_th = bytes;
      bytes = align(bytes + sizeof(int64_t) * g.tab.size());
    }
  }
  if (!ctx->staged) CE_HIP(hipEventCreateWithFlags(&ctx->staged, hipEventDisableTiming));
  CE_HIP(hipEventSynchronize(ctx->staged));  // the previous batch's tables have been copied
  if (ctx->pin_n < bytes) {
    if (ctx->pin) CE_HIP(hipHostFree(ctx->pin));
    ctx->pin = nullptr;
    ctx->pin_n = 0;
    if (hipHostMalloc(&ctx->pin, bytes) != hipSuccess) {
      ctx->pin = nullptr;
      return CE_E_OOM;
    }
    ctx->pin_n = bytes;
  }
  void* dtab = nullptr;
  CE_TRY(ctx->scratch(5, bytes, &dtab));
  char* h = static_cast<char*>(ctx->pin);
  char* d = static_cast<char*>(dtab);
  for (auto& kv : groups) {
    Group& g = kv.second;
    auto* desc = reinterpret_cast<PairDesc*>(h + g.off_desc);
    auto* slot = reinterpret_cast<SlotOut*>(h + g.off_slot);
    auto* cov = reinterpret_cast<CovItem*>(h + g.off_cov);
    int64_t pi = 0, ci = 0;
    for (int64_t i : g.idx) {
      const ce_batch_item& it = items[i];
      const ce_plan* p = it.plan;
      const int64_t ncells = survey_cells(p);
      const size_t relem = p->prec ? 8 : 4;
      for (int64_t j = 0; 2 * j < it.count; ++j, ++pi) {
        PairDesc pd;
        pd.sq = p->sq;
        pd.counts = it.out_counts ? it.out_counts + 2 * j * ncells : nullptr;
        pd.fields = it.out_fields ? static_cast<char*>(it.out_fields) + relem * (size_t)(2 * j * ncells) : nullptr;
        pd.delta = it.out_delta ? static_cast<char*>(it.out_delta) + relem * (size_t)(2 * j * ncells) : nullptr;
        pd.k0 = (uint32_t)(it.seed & 0xFFFFFFFFu);
        pd.k1 = (uint32_t)(it.seed >> 32);
        pd.rid = it.request_id;
        pd.pair = (uint32_t)(it.first_realization / 2 + (uint64_t)j);
        pd.s2half = 0.5 * p->info.sigma2;
        pd.nbar = it.nbar;
        pd.nreal = it.count - 2 * j >= 2 ? 2 : 1;
        desc[pi] = pd;
        for (int hh = 0; hh < 2; ++hh) {
          SlotOut so;
          if (hh < pd.nreal) {
            so.pk = it.out_pk + (2 * j + hh) * it.nbins;
            so.ntot = it.out_ntot ? it.out_ntot + 2 * j + hh : nullptr;
          }
          slot[2 * pi + hh] = so;
        }
      }
      if (it.count >= 2 && (it.out_cov || it.out_cnorm)) cov[ci++] = CovItem{it.out_pk, it.count, it.out_cov, it.out_cnorm};
    }
    if (!g.tab.empty()) std::memcpy(h + g.off_th, g.tab.data(), sizeof(int64_t) * g.tab.size());
  }
  CE_HIP(hipMemcpyAsync(dtab, ctx->pin, bytes, hipMemcpyHostToDevice, s));
  CE_HIP(hipEventRecord(ctx->staged, s));
  // Groups are independent: with several lanes they run concurrently, each lane a sub-context
  // (its own scratch, flags and non-blocking stream) forked from s after the tables arrive and
  // joined back into s; the largest groups are dealt first, each to the least-loaded lane.
  // A group's results do not depend on the lane or the order, so they stay bitwise those of
  // the per-item calls.
  std::vector<Group*> order;
  for (auto& kv : groups) order.push_back(&kv.second);
  std::vector<double> work(order.size());
  for (size_t i = 0; i < order.size(); ++i) {
    const ce_plan* p = items[order[i]->idx[0]].plan;
    double emb = 1;
    for (int d = 0; d < p->ndim; ++d) emb *= p->M[d];
    work[i] = emb * (double)order[i]->pairs;
  }
  std::vector<size_t> byw(order.size());
  for (size_t i = 0; i < byw.size(); ++i) byw[i] = i;
  std::stable_sort(byw.begin(), byw.end(), [&](size_t a, size_t b) { return work[a] > work[b]; });
  const int nl = (int)std::min<size_t>((size_t)ctx->batch_lanes, order.size());
  if (nl <= 1) {
    for (auto& kv : groups) CE_TRY(run_batch_group(ctx, items, kv.second, kv.first, d, s));
    return CE_OK;
  }
  CE_TRY(ensure_lanes(ctx, nl));
  std::vector<double> load(nl, 0.0);
  std::vector<std::vector<size_t>> assign(nl);
  for (size_t i : byw) {
    const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[l] += work[i];
    assign[l].push_back(i);
  }
  std::vector<const void*> keys(order.size());
  {
    size_t i = 0;
    for (auto& kv : groups) keys[i++] = &kv.first;
  }
  CE_HIP(hipEventRecord(ctx->fork, s));
  ce_status st = CE_OK;
  size_t depth = 0;
  for (int l = 0; l < nl; ++l) {
    ce_ctx* lc = ctx->lanes[l];
    lc->last = lc->own;
    if (st == CE_OK && hipStreamWaitEvent(lc->own, ctx->fork, 0) != hipSuccess) st = CE_E_DEVICE;
    depth = std::max(depth, assign[l].size());
  }
  // the groups are enqueued round-robin over the lanes, so every lane has work on the device
  // while the host is still enqueueing the rest
  for (size_t p = 0; p < depth && st == CE_OK; ++p)
    for (int l = 0; l < nl && st == CE_OK; ++l)
      if (p < assign[l].size()) {
        const size_t i = assign[l][p];
        st = run_batch_group(ctx->lanes[l], items, *order[i], *static_cast<const GroupKey*>(keys[i]), d,
                             ctx->lanes[l]->own);
      }
  // the joins are recorded even after a failure, so s never waits on an unrecorded event
  for (int l = 0; l < nl; ++l) {
    ce_ctx* lc = ctx->lanes[l];
    if (hipEventRecord(lc->joined, lc->own) != hipSuccess || hipStreamWaitEvent(s, lc->joined, 0) != hipSuccess)
      st = st == CE_OK ? CE_E_DEVICE : st;
  }
  return st;
}

}  // namespace

extern "C" {

ce_status ce_pipeline_run_batch(ce_ctx* ctx, const ce_batch_item* items, int64_t n, void* stream) {
  if (!ctx || (n > 0 && !items) || n < 0) return CE_E_INVALID;
  if (n == 0) return CE_OK;
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  ctx->last = s;
  return pipeline_batch_impl(ctx, items, n, s);
}

ce_status ce_generate_fields(ce_ctx* ctx, const ce_plan* plan, uint64_t seed, uint32_t request_id,
                             uint64_t first_realization, int64_t count, void* out_fields, void* stream) {
  if (!ctx || !plan || !out_fields || count <= 0 || (first_realization & 1)) return CE_E_INVALID;
  if (plan->ctx != ctx) return CE_E_INVALID;
  if ((first_realization + (uint64_t)count + 1) / 2 > 0xFFFFFFFFull) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  ctx->last = s;
  ScheduleScope scope(ctx, plan->ndim, plan->n, plan->prec);
  InverseSetup fs;
  CE_TRY(setup_ffts(ctx, plan, fs));
  const int64_t npairs = (count + 1) / 2;
  const int64_t cp = chunk_pairs(plan, npairs, kScratchCap);
  const int64_t ncells = survey_cells(plan);
  const size_t elem = plan->prec ? 8 : 4;
  for (int64_t j = 0; j < npairs; j += cp) {
    const int64_t np = std::min(cp, npairs - j);
    RowEpi e;
    e.mode = 1;
    e.ncells = ncells;
    e.count = std::min<int64_t>(count - 2 * j, 2 * np);
    e.real_off = 0;
    e.fields = static_cast<char*>(out_fields) + elem * (size_t)(2 * j * ncells);
    CE_TRY(run_inverse(ctx, plan, fs, seed, request_id, first_realization / 2 + j, np, e, s));
  }
  return CE_OK;
}

ce_status ce_lognormal_poisson(ce_ctx* ctx, const ce_plan* plan, const void* fields, int64_t count, double nbar,
                               const float* mask_f, uint64_t seed, uint32_t request_id, uint64_t first_realization,
                               void* out_delta, int32_t* out_counts, int64_t* out_ntot, void* stream) {
  if (!ctx || !plan || !fields || !out_counts || count <= 0) return CE_E_INVALID;
  if (!(nbar >= 0) || !std::isfinite(nbar)) return CE_E_INVALID;
  if ((first_realization + (uint64_t)count) / 2 > 0xFFFFFFFFull) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  ctx->last = s;
  const int64_t ncells = survey_cells(plan);
  void* acc = nullptr;
  CE_TRY(ctx->scratch(4, sizeof(unsigned long long) * (size_t)count, &acc));
  auto* ntot = static_cast<unsigned long long*>(acc);
  CE_HIP(launch_zero_u64(ntot, count, s));
  CE_PROF(ctx, "lognormal_poisson", s, launch_lognormal_poisson(plan->prec, fields, count, ncells, 0.5 * plan->info.sigma2, nbar, mask_f,
                                  (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), request_id,
                                  first_realization, out_delta, out_counts, ntot, ctx->inv, ctx->flags, s));
  if (out_ntot) CE_HIP(launch_copy_ntot(ntot, out_ntot, count, s));
  return CE_OK;
}

ce_status ce_shell_table(const ce_geometry* geom, int32_t nbins, int64_t* nmodes, double* kmean) {
  if (!geom || !nmodes || !kmean || nbins <= 0) return CE_E_INVALID;
  if (geom->ndim < 1 || geom->ndim > 3) return CE_E_INVALID;
  for (int i = 0; i < geom->ndim; ++i)
    if (geom->n[i] < 2 || (geom->n[i] & 1) || !(geom->h[i] > 0)) return CE_E_INVALID;
  int n[3] = {1, 1, 1};
  for (int i = 0; i < geom->ndim; ++i) n[i] = (int)geom->n[i];
  ShellRule sr;
  if (!shell_rule(n, geom->ndim, nbins, sr, geom->h)) return CE_E_UNSUPPORTED;
  std::vector<int64_t> nm;
  std::vector<double> km;
  shell_table_host(n, geom->ndim, nbins, nm, km, nullptr, geom->h);
  for (double& v : km) v /= sr.cr.href;
  std::memcpy(nmodes, nm.data(), sizeof(int64_t) * nbins);
  std::memcpy(kmean, km.data(), sizeof(double) * nbins);
  return CE_OK;
}

ce_status ce_fft_factors(int32_t length, int32_t* radices, int32_t* nstages) {
  if (!radices || !nstages) return CE_E_INVALID;
  std::vector<int> r;
  if (!factor_length(length, r)) return CE_E_UNSUPPORTED;
  *nstages = (int32_t)r.size();
  for (size_t i = 0; i < r.size(); ++i) radices[i] = r[i];
  return CE_OK;
}

static ce_status estimate_common(ce_ctx* ctx, const ce_geometry* geom, ce_precision precision, ce_map_kind kind,
                                 const void* maps, int64_t count, const int64_t* ntot, const float* mask_f,
                                 int32_t nbins, const double* edges, double* out_pk, int64_t* out_nmodes,
                                 double* out_kmean, void* stream) {
  if (!ctx || !geom || !maps || !out_pk || count <= 0 || nbins <= 0) return CE_E_INVALID;
  if (precision != CE_F32 && precision != CE_F64) return CE_E_INVALID;
  if (kind != CE_MAP_FIELD && kind != CE_MAP_COUNTS_DELTAG) return CE_E_INVALID;
  CE_TRY(check_geometry(geom));
  {
    int nn[3] = {1, 1, 1};
    for (int i = 0; i < geom->ndim; ++i) nn[i] = (int)geom->n[i];
    ShellRule sr;
    if (!shell_rule(nn, geom->ndim, nbins, sr, geom->h)) return CE_E_UNSUPPORTED;
    if (!bins_fit(nn[0], nbins, precision == CE_F64 ? 1 : 0)) return CE_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  ctx->last = s;
  const int prec = precision == CE_F64 ? 1 : 0;
  const int ndim = geom->ndim;
  int n[3] = {1, 1, 1};
  int64_t ncells = 1;
  for (int d = 0; d < ndim; ++d) {
    n[d] = (int)geom->n[d];
    ncells *= n[d];
  }

  PairLoad pl;
  pl.kind = kind == CE_MAP_FIELD ? 0 : 1;
  pl.maps = maps;
  pl.count = count;
  pl.ncells = ncells;
  pl.mask = mask_f;
  if (pl.kind == 1) {
    if (mask_f) {
      void* fs = nullptr;
      CE_TRY(ctx->scratch(9, sizeof(double) * 257, &fs));
      CE_HIP(launch_mask_sum(mask_f, ncells, static_cast<double*>(fs), s));
      pl.fsum = static_cast<const double*>(fs);
    }
    if (ntot) {
      pl.ntot = ntot;
    } else {
      void* acc = nullptr;
      CE_TRY(ctx->scratch(4, sizeof(unsigned long long) * (size_t)count * 2, &acc));
      auto* u = static_cast<unsigned long long*>(acc);
      auto* sgn = reinterpret_cast<int64_t*>(u + count);
      CE_HIP(launch_zero_u64(u, count, s));
      CE_HIP(launch_count_totals(static_cast<const int32_t*>(maps), count, ncells, u, s));
      CE_HIP(launch_copy_ntot(u, sgn, count, s));
      pl.ntot = sgn;
    }
  }
  return spectrum_impl(ctx, ndim, n, geom->h, prec, pl, count, nbins, out_pk, out_nmodes, out_kmean, s, edges);
}

ce_status ce_estimate_pk(ce_ctx* ctx, const ce_geometry* geom, ce_precision precision, ce_map_kind kind,
                         const void* maps, int64_t count, const int64_t* ntot, const float* mask_f, int32_t nbins,
                         double* out_pk, int64_t* out_nmodes, double* out_kmean, void* stream) {
  return estimate_common(ctx, geom, precision, kind, maps, count, ntot, mask_f, nbins, nullptr, out_pk, out_nmodes,
                         out_kmean, stream);
}

ce_status ce_estimate_pk_edges(ce_ctx* ctx, const ce_geometry* geom, ce_precision precision, ce_map_kind kind,
                               const void* maps, int64_t count, const int64_t* ntot, const float* mask_f,
                               int32_t nbins, const double* kedges, double* out_pk, int64_t* out_nmodes,
                               double* out_kmean, void* stream) {
  if (!kedges || nbins <= 0) return CE_E_INVALID;
  for (int b = 0; b <= nbins; ++b)
    if (!std::isfinite(kedges[b]) || kedges[b] < 0 || (b > 0 && !(kedges[b] > kedges[b - 1]))) return CE_E_INVALID;
  return estimate_common(ctx, geom, precision, kind, maps, count, ntot, mask_f, nbins, kedges, out_pk, out_nmodes,
                         out_kmean, stream);
}

ce_status ce_pk_covariance(ce_ctx* ctx, const double* pk, int64_t count, int32_t nbins, double* out_cov,
                           double* out_cnorm, void* stream) {
  if (!ctx || !pk || count < 2 || nbins <= 0) return CE_E_INVALID;
  if (!out_cov && !out_cnorm) return CE_OK;
  CE_HIP(hipSetDevice(ctx->device));
  CE_HIP(launch_covariance(pk, count, nbins, out_cov, out_cnorm, as_stream(stream)));
  return CE_OK;
}

ce_status ce_cic_predict(ce_ctx* ctx, const float* mask_f, int64_t cells, double nbar, double sigma2_A,
                         int32_t nhist, double* out_pred, void* stream) {
  if (!ctx || !out_pred || cells <= 0 || nhist < 1 || nhist > CE_CIC_MAX_BINS) return CE_E_INVALID;
  if (!(nbar > 0) || !std::isfinite(nbar) || !(sigma2_A > 0) || !std::isfinite(sigma2_A)) return CE_E_INVALID;
  // the rule over the log-density A ~ N(-s2/2, s2): Gauss-Legendre panels on mu +- 12 sigma,
  // of width at most sigma / 2 and 1 / sqrt(nhist) (the relative width of the Poisson pmf of the
  // largest count), 8 nodes each, weights times the normal density
  const double mu = -0.5 * sigma2_A, sg = std::sqrt(sigma2_A);
  double wid = std::min(0.5 * sg, 1.0 / std::sqrt((double)nhist));
  const int panels = (int)std::ceil(24.0 * sg / wid);
  wid = 24.0 * sg / panels;
  const HankelRule& g = hankel_rule();  // 8 Gauss-Legendre nodes on [0, 1]
  const int nq = panels * kHankelNodes;
  std::vector<double> host(2 * (size_t)nq + 2 * (size_t)nhist);
  for (int p = 0; p < panels; ++p)
    for (int i = 0; i < kHankelNodes; ++i) {
      const double a = mu - 12.0 * sg + wid * (p + g.x[i]);
      const double z = (a - mu) / sg;
      host[(size_t)p * kHankelNodes + i] = a;
      host[(size_t)nq + (size_t)p * kHankelNodes + i] =
          g.w[i] * wid * std::exp(-0.5 * z * z) / std::sqrt(2.0 * M_PI * sigma2_A);
    }
  for (int n = 0; n < nhist; ++n) {
    host[2 * (size_t)nq + n] = std::lgamma((double)n + 1.0);
    host[2 * (size_t)nq + nhist + n] = 1.0 / (double)(n + 1);  // 1 / N for N = n + 1
  }
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  ctx->last = s;
  const int64_t bx = cic_predict_blocks(cells, nq);
  void* p = nullptr;
  CE_TRY(ctx->scratch(11, sizeof(double) * (host.size() + (size_t)nq * bx * nhist), &p));
  double* tab = static_cast<double*>(p);
  CE_HIP(hipMemcpyAsync(tab, host.data(), sizeof(double) * host.size(), hipMemcpyHostToDevice, s));
  CE_HIP(hipStreamSynchronize(s));  // the host table goes out of scope
  CE_PROF(ctx, "cic_predict", s,
          launch_cic_predict(mask_f, cells, nbar, tab, tab + nq, nq, tab + 2 * nq, nhist, tab + host.size(), out_pred,
                             s));
  return CE_OK;
}

ce_status ce_cumulative_information(ce_ctx* ctx, const double* cnorm, int32_t nbins, double* out_info,
                                    void* stream) {
  if (!ctx || !cnorm || !out_info || nbins < 1 || nbins > CE_INFO_MAX_BINS) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  ctx->last = s;
  void* work = nullptr;
  CE_TRY(ctx->scratch(10, sizeof(double) * (size_t)nbins * (size_t)nbins, &work));
  CE_PROF(ctx, "cumulative_information", s,
          launch_cumulative_information(cnorm, nbins, static_cast<double*>(work), out_info, s));
  return CE_OK;
}

ce_status ce_cic_histogram(ce_ctx* ctx, const int32_t* counts, int64_t cells, int64_t count, const float* mask_f,
                           int32_t nhist, int64_t* out_hist, void* stream) {
  if (!ctx || !counts || !out_hist || cells <= 0 || count <= 0) return CE_E_INVALID;
  if (nhist < 1 || nhist > CE_CIC_MAX_BINS) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  ctx->last = s;
  CE_PROF(ctx, "cic_histogram", s,
          launch_cic_histogram(counts, mask_f, cells, count, nhist, reinterpret_cast<unsigned long long*>(out_hist),
                               s));
  return CE_OK;
}

ce_status ce_astar_map(ce_ctx* ctx, const int32_t* counts, int64_t cells, int64_t count, const float* mask_f,
                       double nbar, double sigma2_A, int32_t subtract_mean, ce_precision precision, void* out_map,
                       double* out_mean, void* stream) {
  if (!ctx || !counts || !out_map || cells <= 0 || count <= 0) return CE_E_INVALID;
  if (precision != CE_F32 && precision != CE_F64) return CE_E_INVALID;
  if (!(nbar > 0) || !std::isfinite(nbar) || !(sigma2_A > 0) || !std::isfinite(sigma2_A)) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  ctx->last = s;
  double* mean = out_mean;
  double* part = nullptr;
  if (subtract_mean || out_mean) {
    void* p = nullptr;
    CE_TRY(ctx->scratch(8, sizeof(double) * (size_t)astar_partials(cells, count), &p));
    part = static_cast<double*>(p);
    if (!mean) {
      CE_TRY(ctx->scratch(9, sizeof(double) * (size_t)count, &p));
      mean = static_cast<double*>(p);
    }
  }
  CE_PROF(ctx, "astar_map", s,
          launch_astar(precision == CE_F64 ? 1 : 0, counts, mask_f, cells, count, nbar, sigma2_A, subtract_mean != 0,
                       out_map, part, mean, s));
  return CE_OK;
}

ce_status ce_pipeline_run(ce_ctx* ctx, const ce_plan* plan, uint64_t seed, uint32_t request_id,
                          uint64_t first_realization, int64_t count, double nbar, int32_t nbins, void* out_fields,
                          void* out_delta, int32_t* out_counts, int64_t* out_ntot, double* out_pk, double* out_cov,
                          double* out_cnorm, void* stream) {
  CE_TRY(pipeline_check(ctx, plan, first_realization, count, nbar, nbins, out_pk));
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  ctx->last = s;
  return pipeline_impl(ctx, plan, seed, request_id, first_realization, count, nbar, nbins, out_fields, out_delta,
                       out_counts, out_ntot, out_pk, out_cov, out_cnorm, nullptr, s);
}

ce_status ce_pipeline_run_noalloc(ce_ctx* ctx, const ce_plan* plan, uint64_t seed, uint32_t request_id,
                                  uint64_t first_realization, int64_t count, double nbar, int32_t nbins,
                                  void* out_fields, void* out_delta, int32_t* out_counts, int64_t* out_ntot,
                                  double* out_pk, double* out_cov, double* out_cnorm, void* stream) {
  CE_TRY(pipeline_check(ctx, plan, first_realization, count, nbar, nbins, out_pk));
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  void* base = nullptr;
  CE_TRY(fixed_scratch(ctx->device, &base));
  // the pairs per chunk that fit the array: per call the N_tot accumulators (2 per pair) and the
  // shell table; per pair the pass intermediates and the shell records of the binning pass
  const int ndim = plan->ndim;
  const size_t elem = plan->prec ? 16 : 8;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const int64_t npairs = (count + 1) / 2;
  const int64_t M1 = plan->M[1], M2 = ndim == 3 ? plan->M[2] : 1;
  const int64_t y1 = (int64_t)plan->n[0] * M1 * M2;
  const int64_t y2 = ndim == 3 ? (int64_t)plan->n[0] * plan->n[1] * M2 : 0;
  const int Nl = plan->n[ndim - 1];
  const int64_t W = 2 * (Nl / 2 + 1);
  const int64_t hrow = survey_cells(plan) / Nl * W;
  const int64_t Bb = ndim == 3 ? (int64_t)plan->n[1] * W : W;
  std::vector<int> rad;
  FftDesc f0;
  if (!factor_length(plan->n[0], rad)) return CE_E_UNSUPPORTED;
  f0.nst = (int)rad.size();
  for (int i = 0; i < f0.nst; ++i) f0.rad[i] = rad[i];
  int G = 1;
  (void)bin_geom(ctx, plan->n[0], nbins, Bb, 1, 0, elem, mixed_radix(f0), &G);
  const int64_t rec = (Bb + G - 1) / G * 2 * nbins;  // shell records per pair (doubles)
  const size_t fixed = al(sizeof(unsigned long long) * 2 * (size_t)npairs) + al(sizeof(int64_t) * (size_t)nbins);
  const size_t per_pair = elem * (size_t)(y1 + y2 + hrow) + sizeof(double) * (size_t)rec;
  if (fixed + per_pair + 4 * 256 > kFixedScratchBytes) return CE_E_UNSUPPORTED;  // one pair does not fit
  int64_t cp = (int64_t)((kFixedScratchBytes - fixed - 4 * 256) / per_pair);
  cp = std::max<int64_t>(1, std::min(cp, npairs));
  hipStream_t s = as_stream(stream);
  ctx->last = s;
  ctx->noalloc = true;
  ctx->noalloc_pairs = cp;
  ctx->arena = ce_ctx::Arena();
  ctx->arena.base = static_cast<char*>(base);
  ctx->arena.size = kFixedScratchBytes;
  const ce_status st = pipeline_impl(ctx, plan, seed, request_id, first_realization, count, nbar, nbins, out_fields,
                                     out_delta, out_counts, out_ntot, out_pk, out_cov, out_cnorm, nullptr, s);
  ctx->noalloc = false;
  return st;
}

ce_status ce_pipeline_run_edges(ce_ctx* ctx, const ce_plan* plan, const float* mask_f, uint64_t seed,
                                uint32_t request_id, uint64_t first_realization, int64_t count, double nbar, int32_t nbins,
                                const double* kedges, void* out_fields, void* out_delta, int32_t* out_counts,
                                int64_t* out_ntot, double* out_pk, double* out_cov, double* out_cnorm, void* stream) {
  CE_TRY(pipeline_check(ctx, plan, first_realization, count, nbar, nbins, out_pk));
  if (!kedges) return CE_E_INVALID;
  for (int b = 0; b <= nbins; ++b)
    if (!std::isfinite(kedges[b]) || kedges[b] < 0 || (b > 0 && !(kedges[b] > kedges[b - 1]))) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  ctx->last = s;
  if (mask_f)
    return pipeline_masked_impl(ctx, plan, mask_f, seed, request_id, first_realization, count, nbar, nbins,
                                out_fields, out_delta, out_counts, out_ntot, out_pk, out_cov, out_cnorm, s, kedges);
  return pipeline_impl(ctx, plan, seed, request_id, first_realization, count, nbar, nbins, out_fields, out_delta,
                       out_counts, out_ntot, out_pk, out_cov, out_cnorm, nullptr, s, nullptr, nullptr, nullptr,
                       kedges);
}

ce_status ce_pipeline_run_masked(ce_ctx* ctx, const ce_plan* plan, const float* mask_f, uint64_t seed,
                                 uint32_t request_id, uint64_t first_realization, int64_t count, double nbar,
                                 int32_t nbins, void* out_fields, void* out_delta, int32_t* out_counts,
                                 int64_t* out_ntot, double* out_pk, double* out_cov, double* out_cnorm, void* stream) {
  if (!mask_f)
    return ce_pipeline_run(ctx, plan, seed, request_id, first_realization, count, nbar, nbins, out_fields, out_delta,
                           out_counts, out_ntot, out_pk, out_cov, out_cnorm, stream);
  CE_TRY(pipeline_check(ctx, plan, first_realization, count, nbar, nbins, out_pk));
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  ctx->last = s;
  return pipeline_masked_impl(ctx, plan, mask_f, seed, request_id, first_realization, count, nbar, nbins, out_fields,
                              out_delta, out_counts, out_ntot, out_pk, out_cov, out_cnorm, s);
}

// ---- prepared masks ------------------------------------------------------------------

struct ce_mask {
  ce_ctx* ctx = nullptr;
  int ndim = 0, prec = 0;
  int n[3] = {1, 1, 1};
  double* fsum = nullptr;  // sum of f, then the workgroup partials (257 doubles)
  void* win = nullptr;     // window transform of [f != 0], column-major
  size_t win_bytes = 0;
  hipEvent_t ready = nullptr;  // recorded after the work that writes fsum and win
};

ce_status ce_mask_prepare(ce_ctx* ctx, const ce_plan* plan, const float* mask_f, void* stream, ce_mask** out) {
  if (!ctx || !plan || !mask_f || !out) return CE_E_INVALID;
  *out = nullptr;
  if (plan->ctx->device != ctx->device) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  ctx->last = s;
  auto m = std::make_unique<ce_mask>();
  m->ctx = ctx;
  m->ndim = plan->ndim;
  m->prec = plan->prec;
  for (int d = 0; d < plan->ndim; ++d) m->n[d] = plan->n[d];
  const int Nl = plan->n[plan->ndim - 1];
  m->win_bytes = (size_t)(plan->prec ? 16 : 8) * (size_t)(survey_cells(plan) / Nl) * (size_t)(2 * (Nl / 2 + 1));
  CE_TRY(ctx->alloc(reinterpret_cast<void**>(&m->fsum), sizeof(double) * 257));
  ce_status st = ctx->alloc(&m->win, m->win_bytes);
  if (st != CE_OK) {
    ctx->release(m->fsum, sizeof(double) * 257);
    return st;
  }
  auto fail = [&](ce_status e) {
    (void)hipStreamSynchronize(s);
    if (m->ready) (void)hipEventDestroy(m->ready);
    ctx->release(m->win, m->win_bytes);
    ctx->release(m->fsum, sizeof(double) * 257);
    return e;
  };
  if (hipEventCreateWithFlags(&m->ready, hipEventDisableTiming) != hipSuccess) return fail(CE_E_DEVICE);
  if (launch_mask_sum(mask_f, survey_cells(plan), m->fsum, s) != hipSuccess) return fail(CE_E_DEVICE);
  void* w = nullptr;
  st = window_transform(ctx, plan, mask_f, &w, s);
  if (st != CE_OK) return fail(st);
  if (hipMemcpyAsync(m->win, w, m->win_bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(CE_E_DEVICE);
  // runs on any stream wait for this event before reading the handle
  if (hipEventRecord(m->ready, s) != hipSuccess) return fail(CE_E_DEVICE);
  *out = m.release();
  return CE_OK;
}

void ce_mask_release(ce_mask* m) {
  if (!m) return;
  {
    std::lock_guard<std::mutex> lock(m->ctx->mu);
    (void)hipSetDevice(m->ctx->device);
    (void)hipEventSynchronize(m->ready);
    m->ctx->release(m->win, m->win_bytes);  // hipFree waits for the work that reads it
    m->ctx->release(m->fsum, sizeof(double) * 257);
    (void)hipEventDestroy(m->ready);
  }
  delete m;
}

ce_status ce_pipeline_run_prepared(ce_ctx* ctx, const ce_plan* plan, const float* mask_f, const ce_mask* mask,
                                   uint64_t seed, uint32_t request_id, uint64_t first_realization, int64_t count,
                                   double nbar, int32_t nbins, const double* kedges, void* out_fields,
                                   void* out_delta, int32_t* out_counts, int64_t* out_ntot, double* out_pk,
                                   double* out_cov, double* out_cnorm, void* stream) {
  CE_TRY(pipeline_check(ctx, plan, first_realization, count, nbar, nbins, out_pk));
  if (!mask_f || !mask || mask->ctx->device != ctx->device || mask->ndim != plan->ndim || mask->prec != plan->prec)
    return CE_E_INVALID;
  for (int d = 0; d < plan->ndim; ++d)
    if (mask->n[d] != plan->n[d]) return CE_E_INVALID;
  if (kedges)
    for (int b = 0; b <= nbins; ++b)
      if (!std::isfinite(kedges[b]) || kedges[b] < 0 || (b > 0 && !(kedges[b] > kedges[b - 1]))) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  ctx->last = s;
  // the handle may have been prepared on another stream: its window and sum must be complete
  CE_HIP(hipStreamWaitEvent(s, mask->ready, 0));
  return pipeline_impl(ctx, plan, seed, request_id, first_realization, count, nbar, nbins, out_fields, out_delta,
                       out_counts, out_ntot, out_pk, out_cov, out_cnorm, nullptr, s, mask_f, mask->win, mask->fsum,
                       kedges);
}

// ---- captured pipeline ------------------------------------------------------------

struct ce_graph {
  ce_ctx* ctx = nullptr;  // private context: the graph's kernels use its scratch
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  unsigned long long* base = nullptr;
};

ce_status ce_pipeline_graph_create(ce_ctx* ctx, const ce_plan* plan, uint64_t seed, uint32_t request_id,
                                   uint64_t first_realization, int64_t count, double nbar, int32_t nbins,
                                   void* out_fields, void* out_delta, int32_t* out_counts, int64_t* out_ntot,
                                   double* out_pk, double* out_cov, double* out_cnorm, ce_graph** out) {
  if (!out) return CE_E_INVALID;
  *out = nullptr;
  CE_TRY(pipeline_check(ctx, plan, first_realization, count, nbar, nbins, out_pk));
  if (count & 1) return CE_E_INVALID;
  auto g = std::make_unique<ce_graph>();
  CE_TRY(ce_ctx_create(ctx->device, ctx->budget, &g->ctx));
  auto fail = [&](ce_status st) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    ce_ctx_destroy(g->ctx);
    g->ctx = nullptr;
    return st;
  };
  ce_ctx* c = g->ctx;
  std::lock_guard<std::mutex> lock(c->mu);
  if (hipStreamCreate(&g->cap) != hipSuccess) return fail(CE_E_DEVICE);
  void* b = nullptr;
  ce_status st = c->alloc(&b, 64);
  if (st != CE_OK) return fail(st);
  g->base = static_cast<unsigned long long*>(b);
  if (hipMemset(g->base, 0, 8) != hipSuccess) return fail(CE_E_DEVICE);
  // size the scratch (no allocation may happen inside the capture)
  st = pipeline_impl(c, plan, seed, request_id, first_realization, count, nbar, nbins, out_fields, out_delta,
                     out_counts, out_ntot, out_pk, out_cov, out_cnorm, g->base, g->cap);
  if (st != CE_OK) return fail(st);
  if (hipStreamSynchronize(g->cap) != hipSuccess) return fail(CE_E_DEVICE);
  if (hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return fail(CE_E_DEVICE);
  st = pipeline_impl(c, plan, seed, request_id, first_realization, count, nbar, nbins, out_fields, out_delta,
                     out_counts, out_ntot, out_pk, out_cov, out_cnorm, g->base, g->cap);
  const hipError_t adv = launch_advance(g->base, (unsigned long long)(count / 2), g->cap);
  const hipError_t end = hipStreamEndCapture(g->cap, &g->graph);
  if (st != CE_OK) return fail(st);
  if (adv != hipSuccess || end != hipSuccess) return fail(CE_E_DEVICE);
  if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) return fail(CE_E_DEVICE);
  *out = g.release();
  return CE_OK;
}

ce_status ce_pipeline_graph_launch(ce_graph* g, void* stream) {
  if (!g) return CE_E_INVALID;
  CE_HIP(hipSetDevice(g->ctx->device));
  CE_HIP(hipGraphLaunch(g->exec, as_stream(stream)));
  return CE_OK;
}

void ce_pipeline_graph_destroy(ce_graph* g) {
  if (!g) return;
  (void)hipSetDevice(g->ctx->device);
  (void)hipDeviceSynchronize();
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->cap) (void)hipStreamDestroy(g->cap);
  ce_ctx_destroy(g->ctx);
  delete g;
}

ce_status ce_debug_philox(uint64_t seed, const uint32_t ctr[4], int64_t n_calls, uint32_t* out_words, void* stream) {
  if (!ctr || !out_words || n_calls <= 0) return CE_E_INVALID;
  CE_HIP(launch_debug_philox((uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), ctr, n_calls, out_words,
                             as_stream(stream)));
  return CE_OK;
}

ce_status ce_debug_noise(const ce_plan* plan, uint64_t seed, uint32_t request_id, uint64_t pair, void* out,
                         void* stream) {
  if (!plan || !out || pair > 0xFFFFFFFFull) return CE_E_INVALID;
  CE_HIP(hipSetDevice(plan->ctx->device));
  int64_t cells = 1;
  for (int d = 0; d < plan->ndim; ++d) cells *= plan->M[d];
  const NoiseArgs n = noise_args(plan, seed, request_id, 0);
  CE_HIP(launch_debug_noise(plan->prec, n, pair, cells, out, as_stream(stream)));
  return CE_OK;
}

}  // extern "C"

// ---- autotuner ----------------------------------------------------------------------

namespace {

ScheduleKey shape_key(int ndim, const int64_t* n, int prec) {
  return ScheduleKey(ndim, (int)n[0], ndim >= 2 ? (int)n[1] : 1, ndim >= 3 ? (int)n[2] : 1, prec);
}

Schedule from_public(const ce_schedule& p) {
  Schedule s;
  s.lines[0] = p.lines_noise;
  s.lines[1] = p.lines_inner;
  s.lines[2] = p.lines_last;
  s.lines[3] = p.lines_bins;
  s.noise_order = p.noise_order;
  s.noise_block = p.noise_block;
  s.noise_pairs = p.noise_pairs;
  s.bin_lds = (size_t)p.bin_lds;
  return s;
}

void to_public(const Schedule& s, ce_schedule* p) {
  p->lines_noise = s.lines[0];
  p->lines_inner = s.lines[1];
  p->lines_last = s.lines[2];
  p->lines_bins = s.lines[3];
  p->noise_order = s.noise_order;
  p->noise_block = s.noise_block;
  p->noise_pairs = s.noise_pairs;
  p->reserved = 0;
  p->bin_lds = (int64_t)s.bin_lds;
}

bool valid_schedule(const ce_schedule& p) {
  for (int v : {p.lines_noise, p.lines_inner, p.lines_last, p.lines_bins})
    if (v < 0 || v > 64 || (v & (v - 1))) return false;
  return (p.noise_order == 0 || p.noise_order == 1) && p.noise_block >= 1 && p.noise_block <= 65536 &&
         p.noise_pairs >= 0 && p.noise_pairs <= 64 && p.bin_lds >= 16384 && p.bin_lds <= 163840;
}

bool same(const Schedule& a, const Schedule& b) {
  return std::equal(std::begin(a.lines), std::end(a.lines), std::begin(b.lines)) && a.noise_order == b.noise_order &&
         a.noise_block == b.noise_block && a.noise_pairs == b.noise_pairs && a.bin_lds == b.bin_lds;
}

// A minimal reader for the schedule file this library writes: objects, arrays, numbers, strings.
struct JsonReader {
  const std::string& t;
  size_t i = 0;
  bool ok = true;
  explicit JsonReader(const std::string& text) : t(text) {}
  void ws() {
    while (i < t.size() && std::isspace((unsigned char)t[i])) ++i;
  }
  bool eat(char c) {
    ws();
    if (i < t.size() && t[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  std::string str() {
    ws();
    std::string s;
    if (i >= t.size() || t[i] != '"') {
      ok = false;
      return s;
    }
    for (++i; i < t.size() && t[i] != '"'; ++i) s.push_back(t[i]);
    if (i < t.size()) ++i;
    return s;
  }
  double num() {
    ws();
    const char* b = t.c_str() + i;
    char* e = nullptr;
    const double v = std::strtod(b, &e);
    if (e == b) ok = false;
    i += (size_t)(e - b);
    return v;
  }
  // skips any value
  void skip() {
    ws();
    if (i >= t.size()) {
      ok = false;
      return;
    }
    if (t[i] == '"') {
      str();
    } else if (t[i] == '{' || t[i] == '[') {
      const char close = t[i] == '{' ? '}' : ']';
      ++i;
      if (eat(close)) return;
      do {
        if (close == '}') {
          str();
          if (!eat(':')) ok = false;
        }
        skip();
      } while (ok && eat(','));
      if (!eat(close)) ok = false;
    } else if (t.compare(i, 4, "true") == 0 || t.compare(i, 4, "null") == 0) {
      i += 4;
    } else if (t.compare(i, 5, "false") == 0) {
      i += 5;
    } else {
      num();
    }
  }
};

}  // namespace

extern "C" {

ce_status ce_schedule_set(ce_ctx* ctx, const ce_geometry* geom, ce_precision precision, const ce_schedule* schedule) {
  if (!ctx || !geom || (precision != CE_F32 && precision != CE_F64)) return CE_E_INVALID;
  CE_TRY(check_geometry(geom));
  std::lock_guard<std::mutex> lock(ctx->mu);
  const ScheduleKey key = shape_key(geom->ndim, geom->n, precision == CE_F64 ? 1 : 0);
  if (!schedule) {
    ctx->tuned.erase(key);
    return CE_OK;
  }
  if (!valid_schedule(*schedule)) return CE_E_INVALID;
  ctx->tuned[key] = from_public(*schedule);
  return CE_OK;
}

ce_status ce_schedule_get(ce_ctx* ctx, const ce_geometry* geom, ce_precision precision, ce_schedule* out) {
  if (!ctx || !geom || !out || (precision != CE_F32 && precision != CE_F64)) return CE_E_INVALID;
  CE_TRY(check_geometry(geom));
  std::lock_guard<std::mutex> lock(ctx->mu);
  const auto it = ctx->tuned.find(shape_key(geom->ndim, geom->n, precision == CE_F64 ? 1 : 0));
  if (it == ctx->tuned.end()) return CE_E_INVALID;
  *out = ce_schedule{};
  to_public(it->second, out);
  return CE_OK;
}

ce_status ce_autotune(ce_ctx* ctx, const ce_plan* plan, int64_t count, double nbar, int32_t nbins, int32_t reps,
                      ce_schedule* out) {
  const double outputs_are_private = 0;  // pipeline_check wants a spectrum pointer; the tuner has its own
  CE_TRY(pipeline_check(ctx, plan, 0, count, nbar, nbins, &outputs_are_private));
  if (reps < 1 || reps > 100) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(ctx->mu);
  CE_HIP(hipSetDevice(ctx->device));
  const int64_t cells = survey_cells(plan);
  // private outputs (the timed steps write counts, N_tot, P(k) and the covariance, as the fused
  // workload does)
  const size_t b_pk = sizeof(double) * (size_t)(count * nbins), b_c = sizeof(int32_t) * (size_t)(count * cells),
               b_n = sizeof(int64_t) * (size_t)count, b_cov = sizeof(double) * (size_t)nbins * nbins;
  char* buf = nullptr;
  CE_TRY(ctx->alloc(reinterpret_cast<void**>(&buf), b_pk + b_c + b_n + b_cov + 1024));
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&](ce_status st) {
    if (s) (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    ctx->release(buf, b_pk + b_c + b_n + b_cov + 1024);
    return st;
  };
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess)
    return cleanup(CE_E_DEVICE);
  auto* pk = reinterpret_cast<double*>(buf);
  auto* cnt = reinterpret_cast<int32_t*>(buf + b_pk + 256);
  auto* nt = reinterpret_cast<int64_t*>(buf + b_pk + b_c + 512);
  auto* cov = reinterpret_cast<double*>(buf + b_pk + b_c + b_n + 768);
  const ScheduleKey key = shape_key(plan->ndim, std::array<int64_t, 3>{plan->n[0], plan->n[1], plan->n[2]}.data(),
                                    plan->prec);
  ctx->tuned.erase(key);
  const bool prof = ctx->prof;
  ctx->prof = false;
  ctx->last = s;
  // median event time of `reps` steps under schedule sc (one untimed step first)
  auto time_sched = [&](const Schedule& sc, double* ms) -> ce_status {
    ctx->tuned[key] = sc;
    std::vector<float> t;
    for (int r = 0; r <= reps; ++r) {
      CE_HIP(hipEventRecord(e0, s));
      CE_TRY(pipeline_impl(ctx, plan, 1, 0, 0, count, nbar, nbins, nullptr, nullptr, cnt, nt, pk, cov, nullptr,
                           nullptr, s));
      CE_HIP(hipEventRecord(e1, s));
      CE_HIP(hipEventSynchronize(e1));
      float m = 0;
      CE_HIP(hipEventElapsedTime(&m, e0, e1));
      if (r) t.push_back(m);
    }
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return CE_OK;
  };
  // coordinate descent from the default schedule over each knob's candidates, twice
  const Schedule dflt = ctx->opts;
  Schedule best = dflt;
  double best_ms = 0, dflt_ms = 0;
  ce_status st = time_sched(best, &dflt_ms);
  best_ms = dflt_ms;
  struct Knob {
    int which;
    std::vector<int64_t> vals;
  };
  std::vector<Knob> knobs = {{0, {2, 4, 8, 16, 32}}, {2, {1, 2, 4, 8}}, {3, {1, 2, 4, 8, 16}},
                             {4, {81920, 163840}},   {5, {1, 2, 4, 8, 16}}, {6, {0, 1}},
                             {7, {0, 1, 4}}};
  if (plan->ndim == 3) knobs.push_back({1, {1, 2, 4, 8, 16, 32}});
  for (int pass = 0; pass < 2 && st == CE_OK; ++pass)
    for (const Knob& k : knobs)
      for (int64_t v : k.vals) {
        if (st != CE_OK) break;
        Schedule c = best;
        if (k.which <= 3)
          c.lines[k.which] = (int)v;
        else if (k.which == 4)
          c.bin_lds = (size_t)v;
        else if (k.which == 5)
          c.noise_block = (int)v;
        else if (k.which == 7)
          c.noise_pairs = (int)v;
        else
          c.noise_order = (int)v;
        if (same(c, best)) continue;
        double ms = 0;
        st = time_sched(c, &ms);
        if (st == CE_OK && ms < 0.99 * best_ms) {
          best = c;
          best_ms = ms;
        }
      }
  ctx->prof = prof;
  if (st != CE_OK) {
    ctx->tuned.erase(key);
    return cleanup(st);
  }
  ctx->tuned[key] = best;
  if (out) {
    *out = ce_schedule{};
    to_public(best, out);
    out->ms = best_ms;
    out->default_ms = dflt_ms;
  }
  return cleanup(CE_OK);
}

ce_status ce_schedule_save(ce_ctx* ctx, const char* path) {
  if (!ctx || !path) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(ctx->mu);
  hipDeviceProp_t prop{};
  CE_HIP(hipGetDeviceProperties(&prop, ctx->device));
  std::string arch(prop.gcnArchName);
  arch = arch.substr(0, arch.find(':'));
  std::string js = "{\"format\": \"cefield-schedules\", \"version\": 1, \"arch\": \"" + arch + "\", \"entries\": [";
  bool first = true;
  for (const auto& kv : ctx->tuned) {
    const auto& k = kv.first;
    const Schedule& sc = kv.second;
    char line[512];
    std::snprintf(line, sizeof(line),
                  "%s\n  {\"ndim\": %d, \"n\": [%d, %d, %d], \"precision\": \"%s\", \"lines\": [%d, %d, %d, %d], "
                  "\"noise_order\": %d, \"noise_block\": %d, \"noise_pairs\": %d, \"bin_lds\": %zu}",
                  first ? "" : ",", std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k),
                  std::get<4>(k) ? "f64" : "f32", sc.lines[0], sc.lines[1], sc.lines[2], sc.lines[3], sc.noise_order,
                  sc.noise_block, sc.noise_pairs, sc.bin_lds);
    js += line;
    first = false;
  }
  js += "\n]}\n";
  FILE* f = std::fopen(path, "w");
  if (!f) return CE_E_INVALID;
  const bool ok = std::fwrite(js.data(), 1, js.size(), f) == js.size();
  return std::fclose(f) == 0 && ok ? CE_OK : CE_E_INVALID;
}

ce_status ce_schedule_load(ce_ctx* ctx, const char* path) {
  if (!ctx || !path) return CE_E_INVALID;
  FILE* f = std::fopen(path, "r");
  if (!f) return CE_E_INVALID;
  std::string text;
  char chunk[4096];
  size_t got;
  while ((got = std::fread(chunk, 1, sizeof(chunk), f)) > 0) text.append(chunk, got);
  std::fclose(f);
  JsonReader r(text);
  std::map<ScheduleKey, Schedule> found;
  if (!r.eat('{')) return CE_E_INVALID;
  bool format_ok = false;
  do {
    const std::string key = r.str();
    if (!r.eat(':')) return CE_E_INVALID;
    if (key == "format") {
      format_ok = r.str() == "cefield-schedules";
    } else if (key == "entries") {
      if (!r.eat('[')) return CE_E_INVALID;
      if (!r.eat(']')) {
        do {
          if (!r.eat('{')) return CE_E_INVALID;
          ce_geometry g{};
          int prec = -1;
          ce_schedule p{};
          p.noise_block = 1;
          p.noise_pairs = 0;
          p.bin_lds = (int64_t)kLdsBudget;
          do {
            const std::string f2 = r.str();
            if (!r.eat(':')) return CE_E_INVALID;
            if (f2 == "ndim") {
              g.ndim = (int32_t)r.num();
            } else if (f2 == "n") {
              if (!r.eat('[')) return CE_E_INVALID;
              for (int i = 0; i < 3; ++i) {
                g.n[i] = (int64_t)r.num();
                if (i < 2 && !r.eat(',')) return CE_E_INVALID;
              }
              if (!r.eat(']')) return CE_E_INVALID;
            } else if (f2 == "precision") {
              const std::string pv = r.str();
              prec = pv == "f64" ? 1 : pv == "f32" ? 0 : -1;
            } else if (f2 == "lines") {
              if (!r.eat('[')) return CE_E_INVALID;
              int32_t* dst[4] = {&p.lines_noise, &p.lines_inner, &p.lines_last, &p.lines_bins};
              for (int i = 0; i < 4; ++i) {
                *dst[i] = (int32_t)r.num();
                if (i < 3 && !r.eat(',')) return CE_E_INVALID;
              }
              if (!r.eat(']')) return CE_E_INVALID;
            } else if (f2 == "noise_order") {
              p.noise_order = (int32_t)r.num();
            } else if (f2 == "noise_block") {
              p.noise_block = (int32_t)r.num();
            } else if (f2 == "noise_pairs") {
              p.noise_pairs = (int32_t)r.num();
            } else if (f2 == "bin_lds") {
              p.bin_lds = (int64_t)r.num();
            } else {
              r.skip();
            }
          } while (r.ok && r.eat(','));
          if (!r.ok || !r.eat('}')) return CE_E_INVALID;
          for (int i = 0; i < 3; ++i) g.h[i] = 1.0;
          if (prec < 0 || check_geometry(&g) != CE_OK || !valid_schedule(p)) return CE_E_INVALID;
          found[shape_key(g.ndim, g.n, prec)] = from_public(p);
        } while (r.eat(','));
        if (!r.eat(']')) return CE_E_INVALID;
      }
    } else {
      r.skip();
    }
  } while (r.ok && r.eat(','));
  if (!r.ok || !r.eat('}') || !format_ok) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(ctx->mu);
  for (auto& kv : found) ctx->tuned[kv.first] = kv.second;
  return CE_OK;
}

}  // extern "C"
