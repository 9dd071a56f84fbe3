// C ABI of the MB4 request server (see include/mb4.h): solve requests of
// different lattice sizes and step counts served on one GPU with continuous
// batching.
//
// Requests wait in a FIFO queue.  A request is admitted as soon as a slot
// (max_active) and a contiguous range of the device arena (first fit over
// free site ranges) are free: its potential and initial state are uploaded
// into the arena and it becomes a member of the multi-lattice engine
// (mb4_engine.hip).  Every poll runs one batch of steps for all active
// requests together: each request advances min(batch_steps, its remaining
// steps) steps with its own Newton loop, in the same launches as the others.
// Finished (or failed) requests are retired: their state is copied back, the
// arena range is freed, and queued requests take their place in the next
// poll.  A request's trajectory is bit for bit the one a single state gives
// it (same kernels, each site computed from its own lattice only).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <unordered_map>
#include <vector>

#include "mb4.h"
#include "mb4_engine.h"

using mb4::MemberDesc;
using mb4::rt::fail;
namespace eng = mb4::engine;

namespace {

constexpr int64_t kMaxSites = int64_t(1) << 28;
constexpr int kMaxBatchSteps = 32;

bool all_finite(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(v[i])) return false;
  return true;
}

struct Request {
  MemberDesc desc{};
  std::vector<double> V, p, q;  // inputs until admission, then the result
  int64_t steps = 0, done = 0;
  int32_t status = MB4_REQ_QUEUED;
  int32_t error = 0;
  int32_t last_iters = 0;
  double t_submit = 0, t_admit = -1, t_done = -1;
  double e_start = 0, e_end = 0;
};

// First-fit allocator of site ranges [0, capacity).
class Arena {
 public:
  explicit Arena(size_t capacity) { free_[0] = capacity; }
  bool alloc(size_t n, long long* base) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *base = it->first;
        const long long start = it->first + static_cast<long long>(n);
        const size_t rest = it->second - n;
        free_.erase(it);
        if (rest > 0) free_[start] = rest;
        used_ += n;
        return true;
      }
    }
    return false;
  }
  void release(long long base, size_t n) {
    auto it = free_.emplace(base, n).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + static_cast<long long>(it->second) == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + static_cast<long long>(prev->second) == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
    used_ -= n;
  }
  size_t used() const { return used_; }

 private:
  std::map<long long, size_t> free_;
  size_t used_ = 0;
};

}  // namespace

struct mb4_server {
  eng::Engine* engine = nullptr;
  size_t capacity = 0;
  int max_active = 0;
  int batch_steps = 0;
  Arena* arena = nullptr;
  std::unordered_map<int64_t, Request> reqs;
  std::deque<int64_t> queue;
  std::vector<int64_t> active;  // member order of the engine
  bool members_changed = false;
  int64_t next_id = 1;
  std::chrono::steady_clock::time_point t0;
  int64_t batches = 0;
  double site_steps = 0;
};

namespace {

double now(const mb4_server* s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

int check(const mb4_server* s) {
  if (s == nullptr) return fail(MB4_EINVAL, "server is NULL");
  return MB4_OK;
}

Request* find(mb4_server* s, int64_t id) {
  auto it = s->reqs.find(id);
  return it == s->reqs.end() ? nullptr : &it->second;
}

// Copies the result back, records the final energy and frees the range.
int retire(mb4_server* s, int64_t id, bool failed) {
  Request& r = s->reqs[id];
  const size_t n = size_t(r.desc.nx) * r.desc.ny;
  r.p.resize(n);
  r.q.resize(n);
  int rc = eng::download(s->engine, r.desc.base, n, r.p.data(), r.q.data());
  double comp[6] = {0, 0, 0, 0, 0, 0};
  if (rc == MB4_OK) rc = eng::energy_of(s->engine, r.desc, comp);
  r.e_end = comp[0];
  s->arena->release(r.desc.base, n);
  r.status = failed ? MB4_REQ_FAILED : MB4_REQ_DONE;
  r.error = failed ? MB4_ENOCONV : 0;
  r.t_done = now(s);
  s->members_changed = true;
  return rc;
}

}  // namespace

extern "C" {

int mb4_server_create(uint64_t arena_bytes, int32_t max_active, int32_t batch_steps,
                      const mb4_options* opt, mb4_server** out) {
  if (out == nullptr) return fail(MB4_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_active < 1 || max_active > 65536)
    return fail(MB4_EINVAL, "max_active must be in [1, 65536]");
  if (batch_steps < 1 || batch_steps > kMaxBatchSteps)
    return fail(MB4_EINVAL, "batch_steps must be in [1, %d]", kMaxBatchSteps);
  mb4_options o;
  mb4_options_default(&o);
  if (opt != nullptr) {
    if (!isfinite(opt->eps) || opt->eps < 0.0 || opt->eps >= 1.0)
      return fail(MB4_EINVAL, "eps must be in [0, 1)");
    if (opt->max_newton < 0 || opt->max_newton > mb4::kMaxNewton)
      return fail(MB4_EINVAL, "max_newton must be in [0, %d]", mb4::kMaxNewton);
    if (opt->inner_sweeps < 0 || opt->inner_sweeps > mb4::kMaxFusedSweeps)
      return fail(MB4_EINVAL, "inner_sweeps of a server must be in [0, %d]",
                  mb4::kMaxFusedSweeps);
    if ((opt->flags & MB4_FLAG_SPECTRAL_SOLVE) != 0)
      return fail(MB4_EINVAL, "spectral stage solves are for single states (mb4_create)");
    if ((opt->flags & ~(MB4_FLAG_NO_GRAPHS | MB4_FLAG_RELATIVE_EPS | MB4_FLAG_FP32_SOLVE)) != 0)
      return fail(MB4_EINVAL, "unknown bits in flags");
    if (opt->eps > 0.0) o.eps = opt->eps;
    if (opt->max_newton > 0) o.max_newton = opt->max_newton;
    if (opt->inner_sweeps > 0) o.inner_sweeps = opt->inner_sweeps;
    o.stream = opt->stream;
    o.flags = opt->flags;
  }
  const bool fp32 = (o.flags & MB4_FLAG_FP32_SOLVE) != 0;
  // Fixed part: step records, member tables; the rest of the arena holds
  // member sites (energy partial sums: 1/256 of a site's share).
  const size_t fixed = size_t(kMaxBatchSteps) * max_active * (o.max_newton + 1) * 8 +
                       size_t(max_active) * 120 + (size_t(1) << 20);
  const size_t per_site = eng::bytes_per_site() + 1;
  if (arena_bytes <= fixed || (arena_bytes - fixed) / per_site < 9)
    return fail(MB4_EINVAL, "arena_bytes too small");
  const size_t capacity = std::min<size_t>((arena_bytes - fixed) / per_site, size_t(INT32_MAX));
  if (size_t(kMaxBatchSteps) * size_t(max_active) * size_t(o.max_newton + 1) > size_t(INT32_MAX))
    return fail(MB4_EINVAL, "max_active * (max_newton + 1) too large for the step records");

  mb4_server* s = new (std::nothrow) mb4_server();
  if (s == nullptr) return fail(MB4_ENOMEM, "host allocation failed");
  // Membership changes between batches, so batches are launched directly
  // rather than captured into graphs.
  eng::Config cfg{o.eps,
                  (o.flags & MB4_FLAG_RELATIVE_EPS) != 0,
                  o.max_newton,
                  o.inner_sweeps,
                  fp32,
                  false,
                  static_cast<hipStream_t>(o.stream),
                  capacity,
                  max_active};
  const int rc = eng::create(cfg, &s->engine);
  if (rc != MB4_OK) {
    delete s;
    return rc;
  }
  s->arena = new (std::nothrow) Arena(capacity);
  if (s->arena == nullptr) {
    eng::destroy(s->engine);
    delete s;
    return fail(MB4_ENOMEM, "host allocation failed");
  }
  s->capacity = capacity;
  s->max_active = max_active;
  s->batch_steps = batch_steps;
  s->t0 = std::chrono::steady_clock::now();
  *out = s;
  return MB4_OK;
}

void mb4_server_destroy(mb4_server* s) {
  if (s == nullptr) return;
  eng::destroy(s->engine);
  delete s->arena;
  delete s;
}

double mb4_server_clock(const mb4_server* s) { return s == nullptr ? -1.0 : now(s); }

int mb4_server_submit(mb4_server* s, const mb4_lattice* lat, const double* potential,
                      const mb4_nonlinearity* nl, double h, const double* p, const double* q,
                      int64_t steps, int64_t* id) {
  const int rc = check(s);
  if (rc != MB4_OK) return rc;
  if (lat == nullptr || potential == nullptr || nl == nullptr || p == nullptr || q == nullptr ||
      id == nullptr)
    return fail(MB4_EINVAL, "NULL argument");
  if (lat->nx < 3 || lat->ny < 3) return fail(MB4_EINVAL, "nx, ny must be >= 3");
  const int64_t sites = int64_t(lat->nx) * int64_t(lat->ny);
  if (sites > kMaxSites || size_t(sites) > s->capacity)
    return fail(MB4_EINVAL, "request of %lld sites can never fit the arena (%zu sites)",
                static_cast<long long>(sites), s->capacity);
  if (!isfinite(lat->t_hop) || !isfinite(lat->diag_shift) || !isfinite(nl->g))
    return fail(MB4_EINVAL, "t_hop, diag_shift and g must be finite");
  if (!isfinite(h) || h == 0.0) return fail(MB4_EINVAL, "h must be finite and non-zero");
  if (steps < 0) return fail(MB4_EINVAL, "steps must be >= 0");
  const size_t n = size_t(sites);
  if (!all_finite(potential, n) || !all_finite(p, n) || !all_finite(q, n))
    return fail(MB4_EINVAL, "non-finite input");
  Request r;
  r.desc = MemberDesc{lat->nx, lat->ny, lat->t_hop, lat->diag_shift, nl->g, h, 0};
  r.V.assign(potential, potential + n);
  r.p.assign(p, p + n);
  r.q.assign(q, q + n);
  r.steps = steps;
  r.t_submit = now(s);
  const int64_t rid = s->next_id++;
  s->reqs.emplace(rid, std::move(r));
  s->queue.push_back(rid);
  *id = rid;
  return MB4_OK;
}

int mb4_server_poll(mb4_server* s, int32_t* queued, int32_t* active) {
  int rc = check(s);
  if (rc != MB4_OK) return rc;
  // Admission, FIFO: the head of the queue waits for a slot and a range.
  while (!s->queue.empty() && int(s->active.size()) < s->max_active) {
    Request& r = s->reqs[s->queue.front()];
    const size_t n = size_t(r.desc.nx) * r.desc.ny;
    long long base = 0;
    if (!s->arena->alloc(n, &base)) break;
    r.desc.base = base;
    rc = eng::upload(s->engine, base, n, r.V.data(), r.p.data(), r.q.data());
    double comp[6] = {0, 0, 0, 0, 0, 0};
    if (rc == MB4_OK) rc = eng::energy_of(s->engine, r.desc, comp);
    if (rc != MB4_OK) {
      s->arena->release(base, n);
      return rc;
    }
    r.e_start = comp[0];
    r.V.clear();
    r.V.shrink_to_fit();
    r.t_admit = now(s);
    r.status = MB4_REQ_ACTIVE;
    const int64_t id = s->queue.front();
    s->queue.pop_front();
    if (r.steps == 0) {
      rc = retire(s, id, false);
      if (rc != MB4_OK) return rc;
      continue;
    }
    s->active.push_back(id);
    s->members_changed = true;
  }
  if (s->members_changed) {
    std::vector<MemberDesc> members;
    members.reserve(s->active.size());
    for (int64_t id : s->active) members.push_back(s->reqs[id].desc);
    rc = eng::set_members(s->engine, members);
    if (rc != MB4_OK) return rc;
    s->members_changed = false;
  }
  if (!s->active.empty()) {
    const size_t m = s->active.size();
    std::vector<int64_t> remaining(m), before(m);
    std::vector<int> iters(m, 0), failed;
    for (size_t i = 0; i < m; ++i) {
      const Request& r = s->reqs[s->active[i]];
      remaining[i] = before[i] = r.steps - r.done;
      iters[i] = r.last_iters;
    }
    rc = eng::run_batch(s->engine, remaining, iters, failed, s->batch_steps);
    if (rc != MB4_OK) return rc;
    ++s->batches;
    std::vector<char> is_failed(m, 0);
    for (int f : failed) is_failed[size_t(f)] = 1;
    // Every finished request leaves the active list, even if copying one
    // back fails: its range is free again, so it must not stay a member.
    std::vector<int64_t> still;
    int first_err = MB4_OK;
    for (size_t i = 0; i < m; ++i) {
      Request& r = s->reqs[s->active[i]];
      r.done += before[i] - remaining[i];
      r.last_iters = iters[i];
      s->site_steps += double(before[i] - remaining[i]) * r.desc.nx * r.desc.ny;
      if (is_failed[i] || r.done >= r.steps) {
        rc = retire(s, s->active[i], is_failed[i] != 0);
        if (rc != MB4_OK && first_err == MB4_OK) first_err = rc;
      } else {
        still.push_back(s->active[i]);
      }
    }
    s->active.swap(still);
    if (first_err != MB4_OK) return first_err;
  }
  if (queued) *queued = int32_t(s->queue.size());
  if (active) *active = int32_t(s->active.size());
  return MB4_OK;
}

int mb4_server_request(mb4_server* s, int64_t id, mb4_request_info* info) {
  const int rc = check(s);
  if (rc != MB4_OK) return rc;
  if (info == nullptr) return fail(MB4_EINVAL, "info is NULL");
  const Request* r = find(s, id);
  if (r == nullptr) return fail(MB4_EINVAL, "unknown request %lld", static_cast<long long>(id));
  info->status = r->status;
  info->nx = r->desc.nx;
  info->ny = r->desc.ny;
  info->steps = r->steps;
  info->steps_done = r->done;
  info->t_submit = r->t_submit;
  info->t_admit = r->t_admit;
  info->t_done = r->t_done;
  info->energy_start = r->e_start;
  info->energy_end = r->e_end;
  info->last_newton_iters = r->last_iters;
  info->error = r->error;
  return MB4_OK;
}

int mb4_server_result(mb4_server* s, int64_t id, double* p, double* q) {
  const int rc = check(s);
  if (rc != MB4_OK) return rc;
  if (p == nullptr || q == nullptr) return fail(MB4_EINVAL, "p and q must not be NULL");
  const Request* r = find(s, id);
  if (r == nullptr) return fail(MB4_EINVAL, "unknown request %lld", static_cast<long long>(id));
  if (r->status != MB4_REQ_DONE && r->status != MB4_REQ_FAILED)
    return fail(MB4_EINVAL, "request %lld has not finished", static_cast<long long>(id));
  memcpy(p, r->p.data(), sizeof(double) * r->p.size());
  memcpy(q, r->q.data(), sizeof(double) * r->q.size());
  return MB4_OK;
}

int mb4_server_release(mb4_server* s, int64_t id) {
  const int rc = check(s);
  if (rc != MB4_OK) return rc;
  const Request* r = find(s, id);
  if (r == nullptr) return fail(MB4_EINVAL, "unknown request %lld", static_cast<long long>(id));
  if (r->status != MB4_REQ_DONE && r->status != MB4_REQ_FAILED)
    return fail(MB4_EINVAL, "request %lld has not finished", static_cast<long long>(id));
  s->reqs.erase(id);
  return MB4_OK;
}

int mb4_server_stats(const mb4_server* s, mb4_server_info* st) {
  const int rc = check(s);
  if (rc != MB4_OK) return rc;
  if (st == nullptr) return fail(MB4_EINVAL, "st is NULL");
  st->capacity_sites = int64_t(s->capacity);
  st->used_sites = int64_t(s->arena->used());
  st->queued = int32_t(s->queue.size());
  st->active = int32_t(s->active.size());
  st->batches = s->batches;
  st->site_steps = s->site_steps;
  return MB4_OK;
}

}  // extern "C"
