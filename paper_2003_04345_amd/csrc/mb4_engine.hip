// Engine of the multi-lattice front ends: member lattices at site offsets of
// capacity-sized fields, advanced together by Algorithm 1 of Sakai et al.
// (arXiv 2003.04345), each member with its own Newton loop.
//
// One launch per Newton phase covers every member: a block finds its member
// through a prefix table of block counts (Multi in mb4_internal.h), so
// members of any size share the launch.  Steps are batched as for a single
// state: up to kBatch steps, each with the predicted number of iterations,
// are enqueued (or replayed from a captured graph), and one read-back of all
// members' step records accepts each member's steps in order.  A member whose
// step needs more iterations keeps u_0 for the rest of the batch (its later
// steps repeat that step and change nothing); the next batch is built for
// more iterations and the member catches up, while members that are done
// skip their launches (todo[m]).
#include "mb4_engine.h"

#include <float.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "mb4.h"

namespace mb4 {
namespace engine {

using rt::fail;

namespace {

constexpr int kBatch = 32;
constexpr int kInitialPrediction = 3;

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(MB4_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

double bits_to_double(unsigned long long b) {
  double d;
  memcpy(&d, &b, sizeof d);
  return d;
}

enum { kFirst = 0, kIter = 1, kFinal = 2, kEnergy = 3 };

}  // namespace

struct Engine {
  Config cfg{};
  int rec_len = 0;
  int device = 0;
  hipStream_t q = nullptr;  // cfg.stream, or the capture stream
  hipStream_t cap_stream = nullptr;
  bool use_graphs = true;
  int region = kRegion32x32;
  std::vector<void*> allocs;
  std::vector<void*> host_allocs;

  double* V = nullptr;
  double2* u0 = nullptr;   // every member's state between batches
  double2* u0b = nullptr;  // the other u_0 buffer of a batch
  double2* Xa[3] = {nullptr, nullptr, nullptr};  // Newton iterates X^l (StepOut)
  double2* Xb[3] = {nullptr, nullptr, nullptr};
  MemberDesc* d_desc = nullptr;
  int* d_block0 = nullptr;  // 4 prefix tables of max_members + 1
  int blocks[4] = {0, 0, 0, 0};
  // Block -> member tables of the 4 classes, one after the other from
  // member_of_at[c], filled on the device from d_block0.
  int* d_member_of = nullptr;
  size_t member_of_cap = 0;
  size_t member_of_at[4] = {0, 0, 0, 0};
  int* d_todo = nullptr;
  int* h_todo = nullptr;
  unsigned long long* ring = nullptr;    // [kBatch][max_members][rec_len]
  unsigned long long* h_ring = nullptr;  // pinned
  double* partials = nullptr;
  size_t partials_blocks = 0;
  double* d_energy = nullptr;  // 6 per member

  std::vector<MemberDesc> desc;
  int predicted = kInitialPrediction;
  int lower_batches = 0;

  // Persistent form (launch_member_run): workers and their members.
  bool persistent = false;
  int cus = 0;
  int workers = 0;
  int* d_order = nullptr;   // [max_members]
  int* d_wfirst = nullptr;  // [wfirst_cap]
  size_t wfirst_cap = 0;
  int* d_conv = nullptr;    // [kBatch][max_members]: outcome of each step
  int* h_conv = nullptr;    // pinned
  int* d_pred = nullptr;    // [max_members]: each member's predicted iterations

  struct GraphEntry {
    int count, iters;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
};

namespace {

int dalloc(Engine* e, void** p, size_t bytes) {
  const hipError_t err = hipMalloc(p, std::max<size_t>(bytes, 8));
  if (err != hipSuccess)
    return fail(MB4_ENOMEM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(err));
  e->allocs.push_back(*p);
  return MB4_OK;
}

int halloc(Engine* e, void** p, size_t bytes) {
  const hipError_t err = hipHostMalloc(p, std::max<size_t>(bytes, 8), hipHostMallocDefault);
  if (err != hipSuccess)
    return fail(MB4_ENOMEM, "hipHostMalloc of %zu bytes failed: %s", bytes,
                hipGetErrorString(err));
  e->host_allocs.push_back(*p);
  return MB4_OK;
}

void drop_graphs(Engine* e) {
  for (auto& g : e->graphs) (void)hipGraphExecDestroy(g.exec);
  e->graphs.clear();
}

int tiles(int n, int t) { return (n + t - 1) / t; }

void member_blocks(const Engine* e, const MemberDesc& d, int out[4]) {
  int tx, ty;
  first_solve_tile(e->region, e->cfg.sweeps, &tx, &ty);
  out[kFirst] = tiles(d.nx, tx) * tiles(d.ny, ty);
  iterate_tile(e->region, e->cfg.sweeps, &tx, &ty);
  out[kIter] = tiles(d.nx, tx) * tiles(d.ny, ty);
  out[kFinal] = tiles(d.nx * d.ny, kFinalSites);
  energy_tile(&tx, &ty);
  out[kEnergy] = tiles(d.nx, tx) * tiles(d.ny, ty);
}

int plan_workers(Engine* e);

// Prefix tables of the four launch classes for the current members and
// region, a large enough energy scratch and, in the persistent form, the
// workers' members.
int upload_blocks(Engine* e) {
  const int n = int(e->desc.size());
  const int stride = e->cfg.max_members + 1;
  std::vector<int> tab(size_t(4) * stride, 0);
  for (int m = 0; m < n; ++m) {
    int b[4];
    member_blocks(e, e->desc[m], b);
    for (int c = 0; c < 4; ++c) {
      const int64_t next = int64_t(tab[size_t(c) * stride + m]) + b[c];
      if (next > INT32_MAX / 2) return fail(MB4_EINVAL, "the members need too many blocks");
      tab[size_t(c) * stride + m + 1] = int(next);
    }
  }
  for (int c = 0; c < 4; ++c) e->blocks[c] = tab[size_t(c) * stride + n];
  HIP_TRY(hipMemcpy(e->d_block0, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice));
  // Block -> member tables, so that a block of a launch finds its member with
  // one load instead of a binary search over the members.
  size_t total = 0;
  for (int c = 0; c < 4; ++c) {
    e->member_of_at[c] = total;
    total += size_t(e->blocks[c]);
  }
  if (total > e->member_of_cap) {
    if (e->d_member_of != nullptr) {
      (void)hipFree(e->d_member_of);
      e->allocs.erase(std::find(e->allocs.begin(), e->allocs.end(), e->d_member_of));
      e->d_member_of = nullptr;
      e->member_of_cap = 0;
    }
    const int rc = dalloc(e, reinterpret_cast<void**>(&e->d_member_of), sizeof(int) * total);
    if (rc != MB4_OK) return rc;
    e->member_of_cap = total;
  }
  for (int c = 0; c < 4; ++c)
    HIP_TRY(launch_member_table(e->d_block0 + size_t(c) * stride, n, e->blocks[c],
                                e->d_member_of + e->member_of_at[c], e->cfg.stream));
  if (size_t(e->blocks[kEnergy]) > e->partials_blocks) {
    if (e->partials != nullptr) {
      (void)hipFree(e->partials);
      e->allocs.erase(std::find(e->allocs.begin(), e->allocs.end(), e->partials));
      e->partials = nullptr;
    }
    const int rc = dalloc(e, reinterpret_cast<void**>(&e->partials),
                          sizeof(double) * 12 * size_t(e->blocks[kEnergy]));
    if (rc != MB4_OK) {
      e->partials_blocks = 0;
      return rc;
    }
    e->partials_blocks = size_t(e->blocks[kEnergy]);
  }
  return plan_workers(e);
}

// Members of each worker of the persistent form: largest first (by tiles of
// a Newton iteration), each to the worker with the least work so far, and
// as many workers as fit on the GPU at once (or one per member).
int plan_workers(Engine* e) {
  e->workers = 0;
  const int n = int(e->desc.size());
  if (!e->persistent || n == 0) return MB4_OK;
  const int per_cu = member_run_blocks_per_cu(e->cfg.sweeps, e->region, e->cfg.fp32);
  if (per_cu < 1)
    return fail(MB4_EINVAL, "no persistent launch for region %s with %d sweeps",
                region_name(e->region), e->cfg.sweeps);
  const int w = std::max(1, std::min(n, per_cu * std::max(e->cus, 1)));
  int ix, iy;
  iterate_tile(e->region, e->cfg.sweeps, &ix, &iy);
  std::vector<long long> cost(static_cast<size_t>(n));
  std::vector<int> by_cost(static_cast<size_t>(n));
  for (int m = 0; m < n; ++m) {
    cost[m] = (long long)tiles(e->desc[m].nx, ix) * tiles(e->desc[m].ny, iy);
    by_cost[m] = m;
  }
  std::stable_sort(by_cost.begin(), by_cost.end(),
                   [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<long long> load(static_cast<size_t>(w), 0);
  std::vector<std::vector<int>> lists(static_cast<size_t>(w));
  for (int m : by_cost) {
    const size_t k = size_t(std::min_element(load.begin(), load.end()) - load.begin());
    load[k] += cost[m];
    lists[k].push_back(m);
  }
  std::vector<int> order, wfirst(1, 0);
  for (const auto& l : lists) {
    order.insert(order.end(), l.begin(), l.end());
    wfirst.push_back(int(order.size()));
  }
  if (wfirst.size() > e->wfirst_cap) {
    if (e->d_wfirst != nullptr) {
      (void)hipFree(e->d_wfirst);
      e->allocs.erase(std::find(e->allocs.begin(), e->allocs.end(), e->d_wfirst));
      e->d_wfirst = nullptr;
      e->wfirst_cap = 0;
    }
    const int rc = dalloc(e, reinterpret_cast<void**>(&e->d_wfirst), sizeof(int) * wfirst.size());
    if (rc != MB4_OK) return rc;
    e->wfirst_cap = wfirst.size();
  }
  HIP_TRY(hipMemcpy(e->d_order, order.data(), sizeof(int) * order.size(), hipMemcpyHostToDevice));
  const std::vector<int> pred(size_t(n), std::max(1, std::min(e->predicted, e->cfg.max_newton)));
  HIP_TRY(hipMemcpy(e->d_pred, pred.data(), sizeof(int) * pred.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(e->d_wfirst, wfirst.data(), sizeof(int) * wfirst.size(),
                    hipMemcpyHostToDevice));
  e->workers = w;
  return MB4_OK;
}

Multi multi_of(const Engine* e, int cls, int step) {
  Multi mu;
  mu.desc = e->d_desc;
  mu.block0 = e->d_block0 + size_t(cls) * (e->cfg.max_members + 1);
  mu.member_of = e->d_member_of + e->member_of_at[cls];
  mu.count = int(e->desc.size());
  mu.blocks = e->blocks[cls];
  mu.todo = e->d_todo;
  mu.step = step;
  mu.rec_stride = e->rec_len;
  return mu;
}

Lattice lattice_of(const Engine* e) {
  Lattice L{};
  L.V = e->V;
  L.u0 = e->u0;
  return L;
}

Planes3 pp(double2* const* a) { return Planes3{{a[0], a[1], a[2]}}; }
CPlanes3 cp(double2* const* a) { return CPlanes3{{a[0], a[1], a[2]}}; }
double2* const* x_planes(const Engine* e, int l) { return (l & 1) ? e->Xa : e->Xb; }
double2* batch_u0(const Engine* e, int k) { return (k & 1) ? e->u0b : e->u0; }

ConvCheck conv_check(const Engine* e, const unsigned long long* rec, int prev) {
  return ConvCheck{rec, prev, e->cfg.eps, e->cfg.relative_eps};
}

// Step `step` of a batch of `count` steps, Newton iterations 1 .. iters, every
// member, with the iterate held as X^l = U^l - e (x) u_0 (StepOut).  Step k
// reads u_0 from u0 (k even) or u0b (k odd) and writes u_1 to the other
// buffer; a member's last step of the batch writes it to u0.  The final
// update of step k - 1 is fused into the first solve of step k, only the last
// step of the batch has its own final update, and the X buffers alternate
// with sigma = k * iters (so the first solve of step k does not write what
// that final update reads).
int enqueue_step(Engine* e, int step, int count, int iters) {
  Lattice L = lattice_of(e);
  double2* const src = batch_u0(e, step);
  L.u0 = src;
  const StepOut so{step == count - 1 ? e->u0 : batch_u0(e, step + 1), e->u0};
  const int members = int(e->desc.size());
  unsigned long long* rec = e->ring + size_t(step) * members * e->rec_len;
  const Multi mf = multi_of(e, kFirst, step), mi = multi_of(e, kIter, step),
              mfin = multi_of(e, kFinal, step);
  const bool f32 = e->cfg.fp32;
  const ConvCheck none{nullptr, 0, 0.0, false};
  const int sigma = (step * iters) & 1;
  auto xp = [&](int l) { return x_planes(e, l + sigma); };
  unsigned long long* const u0max = e->cfg.relative_eps ? rec : nullptr;
  if (step > 0) {
    const unsigned long long* prev = rec - size_t(members) * e->rec_len;
    const int sigma_prev = (sigma + iters) & 1;
    const PrevStep pv{batch_u0(e, step - 1), cp(x_planes(e, iters + sigma_prev)),
                      iters >= 2 ? conv_check(e, prev, iters - 1) : none,
                      conv_check(e, prev, iters), src, e->u0};
    HIP_TRY(launch_first_solve_x(L, pp(xp(1)), e->cfg.sweeps, rec + 1, u0max, e->q, {}, mf,
                                 e->region, f32, &pv));
  } else {
    HIP_TRY(launch_first_solve_x(L, pp(xp(1)), e->cfg.sweeps, rec + 1, u0max, e->q, {}, mf,
                                 e->region, f32, nullptr));
  }
  for (int l = 2; l <= iters; ++l) {
    const int j = l - 1;
    const ConvCheck chk = j >= 2 ? conv_check(e, rec, j - 1) : none;
    // A member whose step has not converged by the batch's last iteration
    // takes the step again from u_0 in the next batch, so of that
    // iteration's X only X_3 (u_1 = u_0 + X_3) is ever read.
    StepOut sol = so;
    sol.stage3_only = l == iters;
    HIP_TRY(launch_iterate(L, cp(xp(j)), pp(xp(l)), e->cfg.sweeps, rec + l, chk,
                           conv_check(e, rec, j), sol, e->q, {}, mi, e->region, f32));
  }
  if (step + 1 < count) return MB4_OK;  // step + 1 takes the final update
  const ConvCheck chk = iters >= 2 ? conv_check(e, rec, iters - 1) : none;
  HIP_TRY(launch_final_update(L, cp(xp(iters)), chk, conv_check(e, rec, iters), so, e->q, {},
                              mfin));
  return MB4_OK;
}

int enqueue_batch(Engine* e, int count, int iters) {
  if (e->persistent) {
    MemberRun run{};
    run.desc = e->d_desc;
    run.order = e->d_order;
    run.wfirst = e->d_wfirst;
    run.todo = e->d_todo;
    run.members = int(e->desc.size());
    run.conv = e->d_conv;
    run.pred = e->d_pred;
    run.u0 = e->u0;
    run.u0b = e->u0b;
    for (int i = 0; i < 3; ++i) {
      run.Xa[i] = e->Xa[i];
      run.Xb[i] = e->Xb[i];
    }
    run.eps = e->cfg.eps;
    run.relative = e->cfg.relative_eps;
    run.max_newton = e->cfg.max_newton;
    HIP_TRY(launch_member_run(lattice_of(e), run, e->workers, e->cfg.sweeps, e->region,
                              e->cfg.fp32, e->q));
    return MB4_OK;
  }
  HIP_TRY(launch_clear(e->ring, count * int(e->desc.size()) * e->rec_len, e->q));
  for (int k = 0; k < count; ++k) {
    const int rc = enqueue_step(e, k, count, iters);
    if (rc != MB4_OK) return rc;
  }
  return MB4_OK;
}

int batch_graph(Engine* e, int count, int iters, hipGraphExec_t* exec) {
  for (const auto& g : e->graphs)
    if (g.count == count && g.iters == iters) {
      *exec = g.exec;
      return MB4_OK;
    }
  if (e->cap_stream == nullptr)
    HIP_TRY(hipStreamCreateWithFlags(&e->cap_stream, hipStreamNonBlocking));
  e->q = e->cap_stream;
  HIP_TRY(hipStreamBeginCapture(e->cap_stream, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue_batch(e, count, iters);
  hipGraph_t graph = nullptr;
  const hipError_t err = hipStreamEndCapture(e->cap_stream, &graph);
  e->q = e->cfg.stream;
  if (rc != MB4_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (err != hipSuccess) return fail(MB4_EDEVICE, "graph capture: %s", hipGetErrorString(err));
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return fail(MB4_EDEVICE, "graph instantiate: %s", hipGetErrorString(ei));
  if (e->graphs.size() >= 64) {
    (void)hipGraphExecDestroy(e->graphs.front().exec);
    e->graphs.erase(e->graphs.begin());
  }
  e->graphs.push_back(Engine::GraphEntry{count, iters, ex});
  *exec = ex;
  return MB4_OK;
}

double conv_tol(const Engine* e, unsigned long long u0max_bits) {
  if (!e->cfg.relative_eps) return e->cfg.eps;
  const double u0max = bits_to_double(u0max_bits);
  return e->cfg.eps * (u0max > DBL_MIN ? u0max : DBL_MIN);
}

// First iteration <= last whose norm met the tolerance; 0 if none; -1 if a
// norm up to `last` is not finite.
int converged_iteration(const Engine* e, const unsigned long long* hrec, int last) {
  const double tol = conv_tol(e, hrec[0]);
  for (int l = 1; l <= last; ++l) {
    const double r = bits_to_double(hrec[l]);
    if (r <= tol) return l;
    if (!isfinite(r)) return -1;
  }
  return 0;
}

// Surplus iterations cost only launches that return at once; too few lose
// the rest of the batch for the member concerned.  So the prediction follows
// a batch's largest count up at once and down only after two lower batches.
void update_prediction(Engine* e, int batch_max) {
  if (batch_max >= e->predicted) {
    e->predicted = batch_max;
    e->lower_batches = 0;
  } else if (++e->lower_batches >= 2) {
    e->predicted = batch_max;
    e->lower_batches = 0;
  }
}

}  // namespace

size_t bytes_per_site() { return 8 + 2 * 16 + 2 * 48; }

int create(const Config& cfg, Engine** out) {
  *out = nullptr;
  if (cfg.capacity == 0 || cfg.capacity > size_t(INT32_MAX))
    return fail(MB4_EINVAL, "capacity must be in [1, 2^31) sites");
  if (cfg.max_members < 1) return fail(MB4_EINVAL, "max_members must be >= 1");
  if (cfg.sweeps < 1 || cfg.sweeps > kMaxFusedSweeps)
    return fail(MB4_EINVAL, "sweeps must be in [1, %d]", kMaxFusedSweeps);
  if (size_t(kBatch) * size_t(cfg.max_members) * size_t(cfg.max_newton + 1) > size_t(INT32_MAX))
    return fail(MB4_EINVAL, "members * (max_newton + 1) too large for the step records");
  Engine* e = new (std::nothrow) Engine();
  if (e == nullptr) return fail(MB4_ENOMEM, "host allocation failed");
  e->cfg = cfg;
  e->rec_len = cfg.max_newton + 1;
  e->q = cfg.stream;
  e->use_graphs = cfg.graphs;
  int rc = MB4_OK;
  hipError_t err = hipGetDevice(&e->device);
  if (err != hipSuccess) rc = fail(MB4_EDEVICE, "hipGetDevice: %s", hipGetErrorString(err));
  const size_t field = sizeof(double2) * cfg.capacity;
  if (rc == MB4_OK) rc = dalloc(e, reinterpret_cast<void**>(&e->V), sizeof(double) * cfg.capacity);
  if (rc == MB4_OK) rc = dalloc(e, reinterpret_cast<void**>(&e->u0), field);
  if (rc == MB4_OK) rc = dalloc(e, reinterpret_cast<void**>(&e->u0b), field);
  for (int i = 0; i < 3 && rc == MB4_OK; ++i) {
    rc = dalloc(e, reinterpret_cast<void**>(&e->Xa[i]), field);
    if (rc == MB4_OK) rc = dalloc(e, reinterpret_cast<void**>(&e->Xb[i]), field);
  }
  const size_t mm = size_t(cfg.max_members);
  if (rc == MB4_OK) rc = dalloc(e, reinterpret_cast<void**>(&e->d_desc), sizeof(MemberDesc) * mm);
  if (rc == MB4_OK) rc = dalloc(e, reinterpret_cast<void**>(&e->d_block0), sizeof(int) * 4 * (mm + 1));
  if (rc == MB4_OK) rc = dalloc(e, reinterpret_cast<void**>(&e->d_todo), sizeof(int) * mm);
  if (rc == MB4_OK) rc = halloc(e, reinterpret_cast<void**>(&e->h_todo), sizeof(int) * mm);
  const size_t words = size_t(kBatch) * mm * e->rec_len;
  if (rc == MB4_OK)
    rc = dalloc(e, reinterpret_cast<void**>(&e->ring), sizeof(unsigned long long) * words);
  if (rc == MB4_OK)
    rc = halloc(e, reinterpret_cast<void**>(&e->h_ring), sizeof(unsigned long long) * words);
  if (rc == MB4_OK) rc = dalloc(e, reinterpret_cast<void**>(&e->d_energy), sizeof(double) * 6 * mm);
  if (rc == MB4_OK) rc = dalloc(e, reinterpret_cast<void**>(&e->d_order), sizeof(int) * mm);
  if (rc == MB4_OK)
    rc = dalloc(e, reinterpret_cast<void**>(&e->d_conv), sizeof(int) * size_t(kBatch) * mm);
  if (rc == MB4_OK) rc = dalloc(e, reinterpret_cast<void**>(&e->d_pred), sizeof(int) * mm);
  if (rc == MB4_OK)
    rc = halloc(e, reinterpret_cast<void**>(&e->h_conv), sizeof(int) * size_t(kBatch) * mm);
  if (rc == MB4_OK) {
    err = hipDeviceGetAttribute(&e->cus, hipDeviceAttributeMultiprocessorCount, e->device);
    if (err != hipSuccess) rc = fail(MB4_EDEVICE, "CU count: %s", hipGetErrorString(err));
  }
  if (rc == MB4_OK) {
    err = hipMemset(e->u0, 0, field);
    if (err == hipSuccess) err = hipMemset(e->V, 0, sizeof(double) * cfg.capacity);
    if (err != hipSuccess) rc = fail(MB4_EDEVICE, "hipMemset: %s", hipGetErrorString(err));
  }
  if (rc == MB4_OK) rc = upload_blocks(e);
  if (rc != MB4_OK) {
    destroy(e);
    return rc;
  }
  *out = e;
  return MB4_OK;
}

void destroy(Engine* e) {
  if (e == nullptr) return;
  (void)hipSetDevice(e->device);
  (void)hipStreamSynchronize(e->cfg.stream);
  drop_graphs(e);
  if (e->cap_stream) (void)hipStreamDestroy(e->cap_stream);
  for (void* p : e->allocs) (void)hipFree(p);
  for (void* p : e->host_allocs) (void)hipHostFree(p);
  delete e;
}

int set_members(Engine* e, const std::vector<MemberDesc>& members) {
  if (members.size() > size_t(e->cfg.max_members))
    return fail(MB4_EINVAL, "more than %d members", e->cfg.max_members);
  for (const MemberDesc& d : members)
    if (d.base < 0 || size_t(d.base) + size_t(d.nx) * d.ny > e->cfg.capacity)
      return fail(MB4_EINVAL, "member sites outside the capacity");
  HIP_TRY(hipSetDevice(e->device));
  HIP_TRY(hipStreamSynchronize(e->cfg.stream));
  e->desc = members;
  if (!members.empty())
    HIP_TRY(hipMemcpy(e->d_desc, members.data(), sizeof(MemberDesc) * members.size(),
                      hipMemcpyHostToDevice));
  drop_graphs(e);
  return upload_blocks(e);
}

int member_count(const Engine* e) { return int(e->desc.size()); }

int upload(Engine* e, long long base, size_t n, const double* V, const double* p,
           const double* q) {
  HIP_TRY(hipSetDevice(e->device));
  hipStream_t s = e->cfg.stream;
  if (V != nullptr)
    HIP_TRY(hipMemcpyAsync(e->V + base, V, sizeof(double) * n, hipMemcpyHostToDevice, s));
  double* stage = reinterpret_cast<double*>(e->Xa[0] + base);  // scratch between batches
  HIP_TRY(hipMemcpyAsync(stage, p, sizeof(double) * n, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(stage + n, q, sizeof(double) * n, hipMemcpyHostToDevice, s));
  HIP_TRY(launch_interleave(stage, stage + n, e->u0 + base, int(n), s));
  HIP_TRY(hipStreamSynchronize(s));
  return MB4_OK;
}

int download(Engine* e, long long base, size_t n, double* p, double* q) {
  HIP_TRY(hipSetDevice(e->device));
  hipStream_t s = e->cfg.stream;
  double* stage = reinterpret_cast<double*>(e->Xa[0] + base);
  HIP_TRY(launch_deinterleave(e->u0 + base, stage, stage + n, int(n), s));
  HIP_TRY(hipMemcpyAsync(p, stage, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(q, stage + n, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return MB4_OK;
}

int run_batch(Engine* e, std::vector<int64_t>& remaining, std::vector<int>& last_iters,
              std::vector<int>& hard_failed, int max_steps, std::vector<char>* nonfinite) {
  hard_failed.clear();
  const int members = int(e->desc.size());
  if (members == 0) return MB4_OK;
  max_steps = std::max(1, std::min(max_steps, kBatch));
  int count = 0;
  for (int m = 0; m < members; ++m) {
    e->h_todo[m] = int(std::min<int64_t>(std::max<int64_t>(remaining[m], 0), max_steps));
    count = std::max(count, e->h_todo[m]);
  }
  if (count == 0) return MB4_OK;
  HIP_TRY(hipSetDevice(e->device));
  const int iters = std::max(1, std::min(e->predicted, e->cfg.max_newton));
  HIP_TRY(hipMemcpyAsync(e->d_todo, e->h_todo, sizeof(int) * members, hipMemcpyHostToDevice,
                         e->cfg.stream));
  hipGraphExec_t exec = nullptr;
  if (e->persistent) {
    // One launch for the batch (its graph is keyed by the step count alone).
    if (e->use_graphs && batch_graph(e, count, 0, &exec) != MB4_OK) {
      (void)hipGetLastError();
      e->use_graphs = false;
      exec = nullptr;
    }
    if (exec != nullptr) {
      HIP_TRY(hipGraphLaunch(exec, e->cfg.stream));
    } else {
      const int rc = enqueue_batch(e, count, 0);
      if (rc != MB4_OK) return rc;
    }
    HIP_TRY(hipMemcpyAsync(e->h_conv, e->d_conv, sizeof(int) * size_t(count) * members,
                           hipMemcpyDeviceToHost, e->cfg.stream));
    HIP_TRY(hipStreamSynchronize(e->cfg.stream));
    if (nonfinite) nonfinite->assign(size_t(members), 0);
    for (int m = 0; m < members; ++m) {
      for (int k = 0; k < e->h_todo[m]; ++k) {
        const int c = e->h_conv[size_t(k) * members + m];
        if (c <= 0) {
          hard_failed.push_back(m);
          if (nonfinite && c < 0) (*nonfinite)[m] = 1;
          break;
        }
        last_iters[m] = c;
        --remaining[m];
      }
    }
    return MB4_OK;
  }
  if (e->use_graphs && batch_graph(e, count, iters, &exec) != MB4_OK) {
    (void)hipGetLastError();
    e->use_graphs = false;
    exec = nullptr;
  }
  if (exec != nullptr) {
    HIP_TRY(hipGraphLaunch(exec, e->cfg.stream));
  } else {
    const int rc = enqueue_batch(e, count, iters);
    if (rc != MB4_OK) return rc;
  }
  const size_t pitch = sizeof(unsigned long long) * e->rec_len;
  HIP_TRY(hipMemcpy2DAsync(e->h_ring, pitch, e->ring, pitch,
                           sizeof(unsigned long long) * (iters + 1), size_t(count) * members,
                           hipMemcpyDeviceToHost, e->cfg.stream));
  HIP_TRY(hipStreamSynchronize(e->cfg.stream));
  // Every member's accepted steps are counted: the device states of all
  // members have moved on by exactly those steps.
  int batch_max = 1;
  bool retry = false;
  if (nonfinite) nonfinite->assign(size_t(members), 0);
  for (int m = 0; m < members; ++m) {
    for (int k = 0; k < e->h_todo[m]; ++k) {
      const unsigned long long* hrec = e->h_ring + (size_t(k) * members + m) * e->rec_len;
      const int c = converged_iteration(e, hrec, iters);
      if (c < 0) {
        hard_failed.push_back(m);
        if (nonfinite) (*nonfinite)[m] = 1;
        break;
      }
      if (c == 0) {
        if (iters >= e->cfg.max_newton) hard_failed.push_back(m);
        else retry = true;
        break;
      }
      last_iters[m] = c;
      --remaining[m];
      batch_max = std::max(batch_max, c);
    }
  }
  if (retry) {
    e->predicted = std::min(e->cfg.max_newton, std::max(iters + 1, batch_max));
    e->lower_batches = 0;
  } else {
    update_prediction(e, batch_max);
  }
  return MB4_OK;
}

int energy(Engine* e, double* out) {
  const int members = int(e->desc.size());
  if (members == 0) return MB4_OK;
  HIP_TRY(hipSetDevice(e->device));
  Multi mu = multi_of(e, kEnergy, 0);
  mu.todo = nullptr;
  HIP_TRY(launch_energy_multi(lattice_of(e), mu, e->partials, e->d_energy, e->cfg.stream));
  HIP_TRY(hipMemcpyAsync(out, e->d_energy, sizeof(double) * 6 * members, hipMemcpyDeviceToHost,
                         e->cfg.stream));
  HIP_TRY(hipStreamSynchronize(e->cfg.stream));
  return MB4_OK;
}

int energy_of(Engine* e, const MemberDesc& d, double out[6]) {
  HIP_TRY(hipSetDevice(e->device));
  const size_t need = energy_partials_count(d.nx, d.ny) / 12;
  if (need > e->partials_blocks) {
    if (e->partials != nullptr) {
      (void)hipFree(e->partials);
      e->allocs.erase(std::find(e->allocs.begin(), e->allocs.end(), e->partials));
      e->partials = nullptr;
      e->partials_blocks = 0;
    }
    const int rc = dalloc(e, reinterpret_cast<void**>(&e->partials), sizeof(double) * 12 * need);
    if (rc != MB4_OK) return rc;
    e->partials_blocks = need;
  }
  Lattice L{d.nx, d.ny, d.t, d.shift, d.g, d.h, e->V + d.base, e->u0 + d.base};
  double* dout = e->d_energy;  // member 0's slot: outside of a batch
  HIP_TRY(launch_energy(L, e->partials, dout, e->cfg.stream));
  HIP_TRY(hipMemcpyAsync(out, dout, sizeof(double) * 6, hipMemcpyDeviceToHost, e->cfg.stream));
  HIP_TRY(hipStreamSynchronize(e->cfg.stream));
  return MB4_OK;
}

bool region_usable(const Engine* e, int r) {
  if (r < 0 || r >= kRegionCount) return false;
  if (e->cfg.fp32 && r != kRegion32x32) return false;
  int tx, ty, ix, iy;
  first_solve_tile(r, e->cfg.sweeps, &tx, &ty);
  iterate_tile(r, e->cfg.sweeps, &ix, &iy);
  return tx > 0 && ty > 0 && ix > 0 && iy > 0;
}

int set_region(Engine* e, int r) {
  if (!region_usable(e, r))
    return fail(MB4_EINVAL, "region %d is not available with these options", r);
  if (r == e->region) return MB4_OK;
  HIP_TRY(hipSetDevice(e->device));
  HIP_TRY(hipStreamSynchronize(e->cfg.stream));
  const int old = e->region;
  e->region = r;
  const int rc = upload_blocks(e);
  if (rc != MB4_OK) {
    e->region = old;
    (void)upload_blocks(e);
    return rc;
  }
  drop_graphs(e);
  return MB4_OK;
}

int set_persistent(Engine* e, bool on) {
  if (on == e->persistent) return MB4_OK;
  HIP_TRY(hipSetDevice(e->device));
  HIP_TRY(hipStreamSynchronize(e->cfg.stream));
  e->persistent = on;
  const int rc = plan_workers(e);
  if (rc != MB4_OK) {
    e->persistent = !on;
    (void)plan_workers(e);
    return rc;
  }
  drop_graphs(e);
  return MB4_OK;
}

bool persistent(const Engine* e) { return e->persistent; }

int region(const Engine* e) { return e->region; }

int set_sweeps(Engine* e, int sweeps) {
  if (sweeps < 1 || sweeps > kMaxFusedSweeps)
    return fail(MB4_EINVAL, "sweeps must be in [1, %d]", kMaxFusedSweeps);
  if (sweeps == e->cfg.sweeps) return MB4_OK;
  HIP_TRY(hipSetDevice(e->device));
  HIP_TRY(hipStreamSynchronize(e->cfg.stream));
  const int old = e->cfg.sweeps;
  e->cfg.sweeps = sweeps;
  if (!region_usable(e, e->region)) {
    e->cfg.sweeps = old;
    return fail(MB4_EINVAL, "region %s leaves no tile at %d sweeps", region_name(e->region),
                sweeps);
  }
  const int rc = upload_blocks(e);
  if (rc != MB4_OK) {
    e->cfg.sweeps = old;
    (void)upload_blocks(e);
    return rc;
  }
  drop_graphs(e);
  return MB4_OK;
}

int sweeps(const Engine* e) { return e->cfg.sweeps; }

size_t u0_bytes(const Engine* e) { return sizeof(double2) * e->cfg.capacity; }

int save_u0(Engine* e, void* dst) {
  HIP_TRY(hipMemcpyAsync(dst, e->u0, u0_bytes(e), hipMemcpyDeviceToDevice, e->cfg.stream));
  HIP_TRY(hipStreamSynchronize(e->cfg.stream));
  return MB4_OK;
}

int restore_u0(Engine* e, const void* src) {
  HIP_TRY(hipMemcpyAsync(e->u0, src, u0_bytes(e), hipMemcpyDeviceToDevice, e->cfg.stream));
  HIP_TRY(hipStreamSynchronize(e->cfg.stream));
  return MB4_OK;
}

hipStream_t stream(const Engine* e) { return e->cfg.stream; }
int iteration_prediction(const Engine* e) { return e->predicted; }
void set_iteration_prediction(Engine* e, int predicted) {
  e->predicted = predicted;
  e->lower_batches = 0;
}

}  // namespace engine
}  // namespace mb4
