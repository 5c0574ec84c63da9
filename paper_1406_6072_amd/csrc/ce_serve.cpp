// Request loop of the generator (host C++): continuous batching of field
// requests of different geometries.  Requests wait in a queue; a scheduler thread
// admits a group of requests whenever one of the slots (a context + stream each) is
// free, their plans are in the cache and their scratch fits the HBM budget; a group
// runs as one batched pipeline call, groups run concurrently on their slots' streams,
// so work of requests that arrive while others are on the GPU overlaps with them.  Plans (the sqrt(lambda)
// octant of a (geometry, xi, precision) key) are built by a planner thread on a
// stream of their own and kept in an LRU cache on the device shared by all slots;
// a request whose plan is being built does not hold up the requests behind it
// (admission looks ahead over the first kLookahead queued requests, oldest first).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/cefield.h"

namespace {

using Clock = std::chrono::steady_clock;
constexpr size_t kLookahead = 64;
constexpr size_t kMaxLatencies = 1 << 20;  // latency samples kept for the percentiles

struct PlanEntry {
  std::string key;
  ce_plan* plan = nullptr;
  size_t bytes = 0;
  int users = 0;  // slots running a request with this plan
};

struct Req {
  uint64_t ticket = 0;
  ce_request r{};
  std::vector<double> table;  // copy of a tabulated xi
  std::vector<double> edges;  // copy of the user shell edges (empty: the default shells)
  std::string key;
  Clock::time_point arrival;
  int state = 0;  // 0 queued, 1 running, 2 done, 3 failed, 4 cancelled
  ce_status status = CE_OK;
  double latency_ms = 0;
  size_t scratch = 0;
  bool planned = false;  // this request started the build of its plan
};

struct Slot {
  ce_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  std::vector<std::shared_ptr<Req>> reqs;  // the group running on the slot (empty: free)
  std::vector<PlanEntry*> plans;
  size_t scratch_held = 0;
  bool busy() const { return !reqs.empty(); }
};

// A free slot takes the oldest admissible request and, behind it, up to max_group - 1 more
// from the lookahead window whose scratch is at most kGroupScratch each, run as one batched
// call (one launch per pass and shape for the whole group); larger requests run alone.
constexpr int kMaxGroup = 256;
constexpr size_t kGroupScratch = size_t(256) << 20;

std::string plan_key(const ce_request& r, const std::vector<double>& table) {
  std::string k;
  auto put = [&](const void* p, size_t n) { k.append(static_cast<const char*>(p), n); };
  put(&r.geom.ndim, sizeof(r.geom.ndim));
  for (int i = 0; i < r.geom.ndim && i < 3; ++i) {
    put(&r.geom.n[i], sizeof(r.geom.n[i]));
    put(&r.geom.h[i], sizeof(r.geom.h[i]));
  }
  put(&r.xi.kind, sizeof(r.xi.kind));
  put(r.xi.p, sizeof(r.xi.p));
  put(&r.xi.transform, sizeof(r.xi.transform));
  put(&r.precision, sizeof(r.precision));
  if (!table.empty()) put(table.data(), table.size() * sizeof(double));
  return k;
}

// Upper bound of the pipeline scratch for `count` realizations (chunks of at most 8 GiB).
size_t scratch_bytes(const ce_request& r) {
  const size_t elem = r.precision == CE_F64 ? 16 : 8;
  double emb = 1, cells = 1;
  for (int i = 0; i < r.geom.ndim && i < 3; ++i) {
    emb *= 2.0 * (double)r.geom.n[i];
    cells *= (double)r.geom.n[i];
  }
  const double per_pair = emb / 2 * elem * 2.0 + cells * elem * 1.1;
  const double pairs = (double)((r.realizations + 1) / 2);
  const double cap = 8.0 * (1ull << 30) + cells * elem * 1.1 * pairs;
  return (size_t)std::min(per_pair * pairs, cap) + ((size_t)1 << 20);
}

}  // namespace

struct ce_server {
  int device = 0;
  ce_server_config cfg{};
  ce_ctx* plan_ctx = nullptr;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv;       // scheduler: submissions, plans ready, stop
  std::condition_variable plan_cv;  // planner: jobs, stop
  std::deque<std::shared_ptr<Req>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Req>> all;
  std::deque<uint64_t> finished;  // tickets in the order they reached a final state
  std::list<PlanEntry> cache;      // front = most recently used
  std::unordered_map<std::string, std::list<PlanEntry>::iterator> index;
  std::deque<std::shared_ptr<Req>> plan_jobs;  // one request per key being planned
  std::unordered_set<std::string> planning;
  std::unordered_map<std::string, ce_status> plan_failed;
  size_t cache_bytes = 0;
  size_t held = 0;  // slot scratch + cached plans
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker, planner;
  std::vector<double> lat;
  size_t lat_next = 0;
  ce_server_stats st{};
  Clock::time_point t0;

  PlanEntry* find_plan(const std::string& key) {
    auto it = index.find(key);
    if (it == index.end()) return nullptr;
    cache.splice(cache.begin(), cache, it->second);
    return &cache.front();
  }
  // drop least-recently-used plans nobody runs until `need` more bytes fit the budget (and,
  // for a plan, the plan cache)
  bool make_room(size_t need, bool plan) {
    while (held + need > cfg.hbm_budget_bytes || (plan && cache_bytes + need > cfg.plan_cache_bytes)) {
      auto it = cache.end();
      bool found = false;
      while (it != cache.begin()) {
        --it;
        if (it->users == 0) {
          found = true;
          break;
        }
      }
      if (!found) return false;
      ce_plan_release(it->plan);
      cache_bytes -= it->bytes;
      held -= it->bytes;
      index.erase(it->key);
      cache.erase(it);
    }
    return true;
  }
  void record_latency(double ms) {
    if (lat.size() < kMaxLatencies) {
      lat.push_back(ms);
    } else {
      lat[lat_next] = ms;
      lat_next = (lat_next + 1) % kMaxLatencies;
    }
  }
  void fail(Req& q, ce_status why) {
    q.status = why;
    q.latency_ms = std::chrono::duration<double, std::milli>(Clock::now() - q.arrival).count();
    q.state = 3;
    st.failed++;
    finished.push_back(q.ticket);
  }

  void complete(Slot& s) {
    // one check of the slot's context covers the group (a device-side sampler flag fails
    // every request of the group that ran with it)
    const ce_status status = ce_ctx_check(s.ctx, s.stream);
    for (auto& qp : s.reqs) {
      auto& q = *qp;
      if (q.state != 1) continue;  // failed at launch
      q.status = status;
      q.latency_ms = std::chrono::duration<double, std::milli>(Clock::now() - q.arrival).count();
      q.state = status == CE_OK ? 2 : 3;
      finished.push_back(q.ticket);
      if (status == CE_OK) {
        st.completed++;
        record_latency(q.latency_ms);
      } else {
        st.failed++;
      }
    }
    for (PlanEntry* pe : s.plans) pe->users--;
    s.plans.clear();
    s.reqs.clear();
  }

  // Reserve q's scratch on slot s (on top of `want`, the scratch of the group so far); false
  // when it does not fit, with *never set when it cannot fit even with nothing else running.
  bool reserve(Slot& s, const Req& q, size_t want, bool first, bool* never) {
    *never = false;
    const size_t total = want + q.scratch;
    const size_t extra = total > s.scratch_held ? total - s.scratch_held : 0;
    bool room = make_room(extra, false);
    if (!room && first) {
      // give back the scratch that idle slots keep cached, then try again
      for (auto& o : slots)
        if (&o != &s && !o.busy() && o.scratch_held && ce_ctx_trim(o.ctx) == CE_OK) {
          held -= o.scratch_held;
          o.scratch_held = 0;
        }
      room = make_room(extra, false);
    }
    if (!room) {
      if (first) {
        bool busy = false;
        for (auto& o : slots) busy |= o.busy();
        *never = !busy;
      }
      return false;
    }
    held += extra;
    s.scratch_held += extra;
    return true;
  }

  // Run the group picked for slot s on its stream.
  void launch(Slot& s) {
    st.launches++;
    st.largest_group = std::max(st.largest_group, (int64_t)s.reqs.size());
    for (size_t k = 0; k < s.reqs.size(); ++k) {
      Req& q = *s.reqs[k];
      if (q.planned)
        st.cache_misses++;
      else
        st.cache_hits++;
      q.state = 1;
    }
    auto run_alone = [&](Req& q, PlanEntry* pe) {
      const ce_request& r = q.r;
      double* cov = r.realizations >= 2 ? r.out_cov : nullptr;
      if (!q.edges.empty())
        return ce_pipeline_run_edges(s.ctx, pe->plan, nullptr, r.seed, r.request_id, 0, r.realizations, r.nbar,
                                     r.nbins, q.edges.data(), r.out_fields, r.out_delta, r.out_counts, r.out_ntot,
                                     r.out_pk, cov, nullptr, s.stream);
      return ce_pipeline_run(s.ctx, pe->plan, r.seed, r.request_id, 0, r.realizations, r.nbar, r.nbins,
                             r.out_fields, r.out_delta, r.out_counts, r.out_ntot, r.out_pk, cov, nullptr, s.stream);
    };
    std::vector<ce_status> rs(s.reqs.size(), CE_OK);
    bool batched = false;
    if (s.reqs.size() > 1) {
      std::vector<ce_batch_item> items(s.reqs.size());
      for (size_t k = 0; k < s.reqs.size(); ++k) {
        const ce_request& r = s.reqs[k]->r;
        ce_batch_item& it = items[k];
        it.plan = s.plans[k]->plan;
        it.seed = r.seed;
        it.request_id = r.request_id;
        it.first_realization = 0;
        it.count = r.realizations;
        it.nbar = r.nbar;
        it.nbins = r.nbins;
        it.out_pk = r.out_pk;
        it.out_counts = r.out_counts;
        it.out_ntot = r.out_ntot;
        it.out_cov = r.realizations >= 2 ? r.out_cov : nullptr;
        it.out_cnorm = nullptr;
        it.kedges = s.reqs[k]->edges.empty() ? nullptr : s.reqs[k]->edges.data();
        it.out_fields = r.out_fields;
        it.out_delta = r.out_delta;
      }
      // an invalid item makes the batch launch nothing: then every request runs alone, so a
      // failing request fails alone
      batched = ce_pipeline_run_batch(s.ctx, items.data(), (int64_t)items.size(), s.stream) == CE_OK;
    }
    if (!batched)
      for (size_t k = 0; k < s.reqs.size(); ++k) rs[k] = run_alone(*s.reqs[k], s.plans[k]);
    const bool recorded = hipEventRecord(s.done, s.stream) == hipSuccess;
    size_t kept = 0;
    for (size_t k = 0; k < s.reqs.size(); ++k) {
      const ce_status why = rs[k] != CE_OK ? rs[k] : (recorded ? CE_OK : CE_E_DEVICE);
      if (why != CE_OK) {
        fail(*s.reqs[k], why);
        s.plans[k]->users--;
      } else {
        s.reqs[kept] = s.reqs[k];
        s.plans[kept] = s.plans[k];
        ++kept;
      }
    }
    s.reqs.resize(kept);
    s.plans.resize(kept);
  }

  // At most one admission onto the free slot s (a group of requests), from the first
  // kLookahead queued requests, oldest first.
  bool admit_one(Slot& s) {
    bool progress = false;
    size_t want = 0;
    for (size_t i = 0; i < queue.size() && i < kLookahead;) {
      const std::shared_ptr<Req> q = queue[i];
      if (q->state == 4) {  // cancelled
        finished.push_back(q->ticket);
        queue.erase(queue.begin() + (std::ptrdiff_t)i);
        progress = true;
        continue;
      }
      auto f = plan_failed.find(q->key);
      if (f != plan_failed.end()) {
        queue.erase(queue.begin() + (std::ptrdiff_t)i);
        fail(*q, f->second);
        progress = true;
        continue;
      }
      PlanEntry* pe = find_plan(q->key);
      if (!pe) {
        if (!planning.count(q->key)) {
          planning.insert(q->key);
          q->planned = true;
          plan_jobs.push_back(q);
          plan_cv.notify_one();
        }
        ++i;
        continue;
      }
      const bool first = s.reqs.empty();
      if (!first && (int)s.reqs.size() >= cfg.max_group) break;  // the group is full
      if (!first && q->scratch > kGroupScratch) {  // a large request waits for a slot of its own
        ++i;
        continue;
      }
      pe->users++;  // pinned while making room
      bool never = false;
      if (reserve(s, *q, want, first, &never)) {
        want += q->scratch;
        s.reqs.push_back(q);
        s.plans.push_back(pe);
        queue.erase(queue.begin() + (std::ptrdiff_t)i);
        progress = true;
        if (q->scratch > kGroupScratch) break;  // a large request runs alone
        continue;
      }
      pe->users--;
      if (!first) break;  // the group is complete
      if (never) {  // nothing runs and it still does not fit: it can never be admitted
        queue.erase(queue.begin() + (std::ptrdiff_t)i);
        fail(*q, CE_E_OOM);
        return true;
      }
      st.admission_stalls++;  // the oldest request with a plan waits for memory; keep the order
      return progress;
    }
    if (!s.reqs.empty()) launch(s);
    return progress;
  }

  // queue the plan builds of the first kLookahead requests, so plans are built while every
  // slot is busy
  void prefetch_plans() {
    for (size_t i = 0; i < queue.size() && i < kLookahead; ++i) {
      const std::shared_ptr<Req>& q = queue[i];
      if (q->state == 4 || index.count(q->key) || planning.count(q->key) || plan_failed.count(q->key)) continue;
      planning.insert(q->key);
      q->planned = true;
      plan_jobs.push_back(q);
      plan_cv.notify_one();
    }
  }

  void loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lock(mu);
    while (true) {
      bool progress = false;
      if (!queue.empty()) prefetch_plans();
      for (auto& s : slots)
        if (s.busy() && hipEventQuery(s.done) != hipErrorNotReady) {  // done, or failed: complete() reports it
          complete(s);
          progress = true;
        }
      for (auto& s : slots)
        if (!s.busy() && !queue.empty()) progress |= admit_one(s);
      bool busy = false;
      for (auto& s : slots) busy |= s.busy();
      if (stop && !busy && queue.empty()) break;
      if (!progress) {
        if (busy)
          cv.wait_for(lock, std::chrono::microseconds(20));
        else
          cv.wait_for(lock, std::chrono::milliseconds(5));
      }
    }
  }

  void plan_loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lock(mu);
    while (true) {
      if (plan_jobs.empty()) {
        if (stop) break;
        plan_cv.wait(lock);
        continue;
      }
      const std::shared_ptr<Req> q = plan_jobs.front();
      plan_jobs.pop_front();
      ce_xi xi = q->r.xi;
      if (!q->table.empty()) xi.table = q->table.data();
      const ce_geometry geom = q->r.geom;
      const ce_precision prec = q->r.precision;
      lock.unlock();
      ce_plan* p = nullptr;
      ce_plan_info info{};
      const ce_status ps = ce_plan_embedding(plan_ctx, &geom, &xi, prec, -1.0, &p, &info);
      lock.lock();
      planning.erase(q->key);
      if (ps == CE_OK) {
        (void)make_room(info.device_bytes, true);  // best effort: plans in use are never dropped
        cache.push_front(PlanEntry{q->key, p, info.device_bytes, 0});
        index[q->key] = cache.begin();
        cache_bytes += info.device_bytes;
        held += info.device_bytes;
      } else {
        st.cache_misses++;
        plan_failed[q->key] = ps;
      }
      cv.notify_one();
    }
  }
};

extern "C" {

ce_status ce_server_create(int device, const ce_server_config* cfg, ce_server** out) {
  if (!out) return CE_E_INVALID;
  *out = nullptr;
  auto s = std::make_unique<ce_server>();
  s->device = device;
  s->cfg = cfg ? *cfg : ce_server_config{};
  if (s->cfg.slots <= 0) s->cfg.slots = 4;
  if (s->cfg.slots > 32) return CE_E_INVALID;
  if (s->cfg.max_group <= 0) s->cfg.max_group = kMaxGroup;
  if (s->cfg.max_group > kMaxGroup) return CE_E_INVALID;
  if (s->cfg.hbm_budget_bytes == 0) {
    // three quarters of the device memory free at creation
    size_t free_b = 0, total_b = 0;
    if (hipSetDevice(device) != hipSuccess || hipMemGetInfo(&free_b, &total_b) != hipSuccess) return CE_E_DEVICE;
    s->cfg.hbm_budget_bytes = free_b / 4 * 3;
  }
  if (s->cfg.plan_cache_bytes == 0) s->cfg.plan_cache_bytes = std::min((size_t)32 << 30, s->cfg.hbm_budget_bytes / 4);
  ce_status st = ce_ctx_create(device, 0, &s->plan_ctx);
  if (st != CE_OK) return st;
  s->slots.resize(s->cfg.slots);
  for (auto& sl : s->slots) {
    st = ce_ctx_create(device, 0, &sl.ctx);
    if (st == CE_OK && (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
                        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess))
      st = CE_E_DEVICE;
    if (st != CE_OK) {
      for (auto& x : s->slots) {
        if (x.done) (void)hipEventDestroy(x.done);
        if (x.stream) (void)hipStreamDestroy(x.stream);
        if (x.ctx) ce_ctx_destroy(x.ctx);
      }
      ce_ctx_destroy(s->plan_ctx);
      return st;
    }
  }
  s->t0 = Clock::now();
  ce_server* raw = s.release();
  raw->worker = std::thread([raw] { raw->loop(); });
  raw->planner = std::thread([raw] { raw->plan_loop(); });
  *out = raw;
  return CE_OK;
}

namespace {
// A queued copy of *r (a tabulated xi copied), or nullptr when r is invalid.
std::shared_ptr<Req> make_request(const ce_request* r) {
  if (!r || !r->out_pk || r->realizations <= 0 || r->nbins <= 0) return nullptr;
  auto q = std::make_shared<Req>();
  q->arrival = Clock::now();
  q->r = *r;
  if (r->xi.kind == CE_XI_TABLE) {
    if (!r->xi.table || r->geom.ndim < 1 || r->geom.ndim > 3) return nullptr;
    double n = 1;
    for (int i = 0; i < r->geom.ndim; ++i) n *= (double)(r->geom.n[i] + 1);
    q->table.assign(r->xi.table, r->xi.table + (size_t)n);
    q->r.xi.table = nullptr;
  }
  if (r->kedges) {
    q->edges.assign(r->kedges, r->kedges + r->nbins + 1);
    for (size_t b = 0; b < q->edges.size(); ++b)
      if (!std::isfinite(q->edges[b]) || q->edges[b] < 0 || (b > 0 && !(q->edges[b] > q->edges[b - 1])))
        return nullptr;
  }
  q->r.kedges = nullptr;
  q->key = plan_key(q->r, q->table);
  q->scratch = scratch_bytes(q->r);
  return q;
}
}  // namespace

ce_status ce_server_submit(ce_server* s, const ce_request* r, uint64_t* ticket) {
  return ce_server_submit_many(s, r, 1, ticket);
}

ce_status ce_server_submit_many(ce_server* s, const ce_request* r, int64_t n, uint64_t* tickets) {
  if (!s || !r || !tickets || n <= 0) return CE_E_INVALID;
  std::vector<std::shared_ptr<Req>> qs((size_t)n);
  for (int64_t k = 0; k < n; ++k)
    if (!(qs[(size_t)k] = make_request(r + k))) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(s->mu);
  if (s->stop) return CE_E_INVALID;
  for (int64_t k = 0; k < n; ++k) {
    auto& q = qs[(size_t)k];
    q->ticket = s->next_ticket++;
    tickets[k] = q->ticket;
    s->queue.push_back(q);
    s->all[q->ticket] = q;
    s->st.submitted++;
  }
  s->cv.notify_one();
  return CE_OK;
}

ce_status ce_server_poll(ce_server* s, uint64_t ticket, int32_t* state, ce_status* status, double* latency_ms) {
  if (!s || !state) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return CE_E_INVALID;
  const Req& q = *it->second;
  *state = q.state;
  if (status) *status = q.status;
  if (latency_ms) *latency_ms = q.latency_ms;
  if (q.state >= 2) s->all.erase(it);
  return CE_OK;
}

ce_status ce_server_drain(ce_server* s, int32_t max, uint64_t* tickets, int32_t* states, ce_status* statuses,
                          double* latency_ms, int32_t* n) {
  if (!s || !n || max < 0 || (max > 0 && !tickets)) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(s->mu);
  int32_t k = 0;
  while (k < max && !s->finished.empty()) {
    const uint64_t t = s->finished.front();
    s->finished.pop_front();
    auto it = s->all.find(t);
    if (it == s->all.end()) continue;  // already returned by ce_server_poll
    const Req& q = *it->second;
    tickets[k] = t;
    if (states) states[k] = q.state;
    if (statuses) statuses[k] = q.status;
    if (latency_ms) latency_ms[k] = q.latency_ms;
    s->all.erase(it);
    ++k;
  }
  *n = k;
  return CE_OK;
}

ce_status ce_server_cancel(ce_server* s, uint64_t ticket) {
  if (!s) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return CE_E_INVALID;
  Req& q = *it->second;
  if (q.state != 0) return CE_E_INVALID;  // only queued requests can be cancelled
  q.state = 4;
  q.status = CE_E_INVALID;
  return CE_OK;
}

ce_status ce_server_stats_read(ce_server* s, ce_server_stats* out) {
  if (!s || !out) return CE_E_INVALID;
  std::lock_guard<std::mutex> lock(s->mu);
  *out = s->st;
  std::vector<double> v = s->lat;
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) { return v[std::min(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5))]; };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
  }
  out->elapsed_s = std::chrono::duration<double>(Clock::now() - s->t0).count();
  out->held_bytes = s->held;
  out->queued = (int64_t)s->queue.size();
  return CE_OK;
}

void ce_server_destroy(ce_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    s->stop = true;
    for (auto& q : s->queue) {
      q->state = 4;
      q->status = CE_E_INVALID;
    }
    s->queue.clear();
    s->plan_jobs.clear();
    s->cv.notify_one();
    s->plan_cv.notify_one();
  }
  if (s->worker.joinable()) s->worker.join();
  if (s->planner.joinable()) s->planner.join();
  for (auto& pe : s->cache) ce_plan_release(pe.plan);
  for (auto& x : s->slots) {
    (void)hipStreamSynchronize(x.stream);
    (void)hipEventDestroy(x.done);
    (void)hipStreamDestroy(x.stream);
    ce_ctx_destroy(x.ctx);
  }
  ce_ctx_destroy(s->plan_ctx);
  delete s;
}

}  // extern "C"
