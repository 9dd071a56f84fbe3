// Host runtime of MB4 ensembles (see include/mb4.h): many independent
// lattice problems advanced together by Algorithm 1 of Sakai et al. (arXiv
// 2003.04345), each member with its own Newton loop.
//
// All members' fields live in ensemble-wide arrays (member m at site offset
// base[m]).  One launch per Newton phase covers every member: a block finds
// its member through a prefix table of block counts (Multi in
// mb4_internal.h), so members of any size share the launch.  Steps are
// batched as for a single state: up to kBatch steps, each with the predicted
// number of iterations, are enqueued (or replayed from a captured graph), and
// one read-back of all members' step records accepts each member's steps in
// order.  A member whose step needs more iterations keeps u_0 for the rest of
// the batch (its later steps repeat that step and change nothing); the next
// batch is built for more iterations and the member catches up, while
// members that are done skip their launches (todo[m]).
#include <float.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "mb4.h"
#include "mb4_internal.h"

using mb4::ConvCheck;
using mb4::CPlanes3;
using mb4::Lattice;
using mb4::MemberDesc;
using mb4::Multi;
using mb4::Planes3;
using mb4::rt::fail;

namespace {

constexpr double kDefaultEps = 1e-13;  // Sec. 3: epsilon = 1e-13
constexpr int kDefaultMaxNewton = 50;
constexpr int kDefaultSweeps = 3;
constexpr int kMaxMembers = 65536;
constexpr int64_t kMaxSites = int64_t(1) << 28;
constexpr int kBatch = 32;
constexpr int kInitialPrediction = 3;

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(MB4_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

bool all_finite(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(v[i])) return false;
  return true;
}

double bits_to_double(unsigned long long b) {
  double d;
  memcpy(&d, &b, sizeof d);
  return d;
}

}  // namespace

struct mb4_ensemble {
  int count = 0;
  std::vector<MemberDesc> desc;  // host copy
  size_t total = 0;              // sites of all members
  double eps = kDefaultEps;
  bool relative_eps = false;
  bool fp32 = false;  // FP32 inner stage solves (32 x 32 regions only)
  int max_newton = kDefaultMaxNewton;
  int sweeps = kDefaultSweeps;
  int rec_len = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t q = nullptr;  // stream / capture stream
  hipStream_t cap_stream = nullptr;
  bool use_graphs = true;
  int region = mb4::kRegion32x32;
  std::vector<void*> allocs;
  std::vector<void*> host_allocs;

  double* V = nullptr;
  double2* u0 = nullptr;
  double2* Ua[3] = {nullptr, nullptr, nullptr};
  double2* Ub[3] = {nullptr, nullptr, nullptr};
  double2* ra[3] = {nullptr, nullptr, nullptr};
  double2* rb[3] = {nullptr, nullptr, nullptr};
  MemberDesc* d_desc = nullptr;
  int* d_block0 = nullptr;  // 4 prefix tables of count + 1: first solve, iterate, final, energy
  int blocks[4] = {0, 0, 0, 0};
  int* d_todo = nullptr;
  int* h_todo = nullptr;
  unsigned long long* ring = nullptr;    // [kBatch][count][rec_len]
  unsigned long long* h_ring = nullptr;  // pinned
  double* partials = nullptr;
  double* d_energy = nullptr;

  std::vector<int64_t> steps_done;
  std::vector<int> last_iters;
  int predicted = kInitialPrediction;
  int lower_batches = 0;

  struct GraphEntry {
    int count, iters;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
};

namespace {

enum { kFirst = 0, kIter = 1, kFinal = 2, kEnergy = 3 };

int dalloc(mb4_ensemble* e, void** p, size_t bytes) {
  const hipError_t err = hipMalloc(p, std::max<size_t>(bytes, 8));
  if (err != hipSuccess)
    return fail(MB4_ENOMEM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(err));
  e->allocs.push_back(*p);
  return MB4_OK;
}

int halloc(mb4_ensemble* e, void** p, size_t bytes) {
  const hipError_t err = hipHostMalloc(p, std::max<size_t>(bytes, 8), hipHostMallocDefault);
  if (err != hipSuccess)
    return fail(MB4_ENOMEM, "hipHostMalloc of %zu bytes failed: %s", bytes,
                hipGetErrorString(err));
  e->host_allocs.push_back(*p);
  return MB4_OK;
}

void drop_graphs(mb4_ensemble* e) {
  for (auto& g : e->graphs) (void)hipGraphExecDestroy(g.exec);
  e->graphs.clear();
}

void free_all(mb4_ensemble* e) {
  drop_graphs(e);
  if (e->cap_stream) (void)hipStreamDestroy(e->cap_stream);
  for (void* p : e->allocs) (void)hipFree(p);
  for (void* p : e->host_allocs) (void)hipHostFree(p);
  e->allocs.clear();
  e->host_allocs.clear();
}

size_t records_words(int count, int max_newton) {
  return size_t(kBatch) * size_t(count) * size_t(max_newton + 1);
}

// Device bytes of an ensemble (see mb4.h).
size_t footprint_bytes(size_t total, int count, int max_newton, size_t energy_blocks) {
  return total * 216 + records_words(count, max_newton) * 8 + size_t(count) * 64 +
         size_t(4) * (count + 1) * sizeof(int) + energy_blocks * 12 * sizeof(double) +
         size_t(count) * 6 * sizeof(double);
}

int tiles(int n, int t) { return (n + t - 1) / t; }

// Blocks of member m in each launch class for the current region.
void member_blocks(const mb4_ensemble* e, const MemberDesc& d, int out[4]) {
  int tx, ty;
  mb4::first_solve_tile(e->region, e->sweeps, &tx, &ty);
  out[kFirst] = tiles(d.nx, tx) * tiles(d.ny, ty);
  mb4::iterate_tile(e->region, e->sweeps, &tx, &ty);
  out[kIter] = tiles(d.nx, tx) * tiles(d.ny, ty);
  out[kFinal] = tiles(d.nx * d.ny, mb4::kFinalSites);
  mb4::energy_tile(&tx, &ty);
  out[kEnergy] = tiles(d.nx, tx) * tiles(d.ny, ty);
}

bool region_usable(int region, int sweeps, bool fp32) {
  if (fp32 && region != mb4::kRegion32x32) return false;
  int tx, ty, ix, iy;
  mb4::first_solve_tile(region, sweeps, &tx, &ty);
  mb4::iterate_tile(region, sweeps, &ix, &iy);
  return tx > 0 && ty > 0 && ix > 0 && iy > 0;
}

// Prefix tables of the four launch classes, uploaded for the current region.
int upload_blocks(mb4_ensemble* e) {
  const int n = e->count;
  std::vector<int> tab(size_t(4) * (n + 1), 0);
  for (int c = 0; c < 4; ++c) tab[size_t(c) * (n + 1)] = 0;
  for (int m = 0; m < n; ++m) {
    int b[4];
    member_blocks(e, e->desc[m], b);
    for (int c = 0; c < 4; ++c) {
      const int64_t next = int64_t(tab[size_t(c) * (n + 1) + m]) + b[c];
      if (next > INT32_MAX / 2) return fail(MB4_EINVAL, "ensemble needs too many blocks");
      tab[size_t(c) * (n + 1) + m + 1] = int(next);
    }
  }
  for (int c = 0; c < 4; ++c) e->blocks[c] = tab[size_t(c) * (n + 1) + n];
  HIP_TRY(hipMemcpy(e->d_block0, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice));
  return MB4_OK;
}

Multi multi_of(const mb4_ensemble* e, int cls, int step) {
  Multi mu;
  mu.desc = e->d_desc;
  mu.block0 = e->d_block0 + size_t(cls) * (e->count + 1);
  mu.count = e->count;
  mu.blocks = e->blocks[cls];
  mu.todo = e->d_todo;
  mu.step = step;
  mu.rec_stride = e->rec_len;
  return mu;
}

Lattice lattice_of(const mb4_ensemble* e) {
  Lattice L{};
  L.V = e->V;
  L.u0 = e->u0;
  return L;
}

Planes3 pp(double2* const* a) { return Planes3{{a[0], a[1], a[2]}}; }
CPlanes3 cp(double2* const* a) { return CPlanes3{{a[0], a[1], a[2]}}; }
double2* const* u_planes(const mb4_ensemble* e, int j) { return (j % 2 == 1) ? e->Ua : e->Ub; }
double2* const* r_planes(const mb4_ensemble* e, int l) { return (l % 2 == 1) ? e->ra : e->rb; }

ConvCheck conv_check(const mb4_ensemble* e, const unsigned long long* rec, int prev) {
  return ConvCheck{rec, prev, e->eps, e->relative_eps};
}

// Step `step` of the batch, Newton iterations 1 .. iters, every member.
int enqueue_step(mb4_ensemble* e, int step, int iters) {
  const Lattice L = lattice_of(e);
  unsigned long long* rec = e->ring + size_t(step) * e->count * e->rec_len;
  const Multi mf = multi_of(e, kFirst, step), mi = multi_of(e, kIter, step),
              mfin = multi_of(e, kFinal, step);
  HIP_TRY(mb4::launch_first_solve(L, pp(r_planes(e, 1)), e->sweeps, rec + 1, rec,
                                  Planes3{{nullptr, nullptr, nullptr}}, e->q, {}, mf,
                                  e->region, e->fp32));
  for (int l = 2; l <= iters; ++l) {
    const int j = l - 1;
    const ConvCheck chk = j >= 2 ? conv_check(e, rec, j - 1) : ConvCheck{nullptr, 0, 0.0, false};
    const ConvCheck fin = conv_check(e, rec, j);
    const CPlanes3 uin = j >= 2 ? cp(u_planes(e, j - 1)) : CPlanes3{{nullptr, nullptr, nullptr}};
    HIP_TRY(mb4::launch_iterate(L, uin, pp(u_planes(e, j)), cp(r_planes(e, j)),
                                pp(r_planes(e, l)), j == 1, e->sweeps, rec + l, chk, fin, e->u0,
                                e->q, {}, mi, e->region, e->fp32));
  }
  const int j = iters;
  const ConvCheck chk = j >= 2 ? conv_check(e, rec, j - 1) : ConvCheck{nullptr, 0, 0.0, false};
  const ConvCheck fin = conv_check(e, rec, j);
  const CPlanes3 uin = j >= 2 ? cp(u_planes(e, j - 1)) : CPlanes3{{nullptr, nullptr, nullptr}};
  HIP_TRY(mb4::launch_final_update(L, uin, cp(r_planes(e, j)), j == 1, chk, fin, e->u0, e->q,
                                   {}, mfin, e->fp32));
  return MB4_OK;
}

int enqueue_batch(mb4_ensemble* e, int count, int iters) {
  HIP_TRY(mb4::launch_clear(e->ring, count * e->count * e->rec_len, e->q));
  for (int k = 0; k < count; ++k) {
    const int rc = enqueue_step(e, k, iters);
    if (rc != MB4_OK) return rc;
  }
  return MB4_OK;
}

int batch_graph(mb4_ensemble* e, int count, int iters, hipGraphExec_t* exec) {
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
  e->q = e->stream;
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
  e->graphs.push_back(mb4_ensemble::GraphEntry{count, iters, ex});
  *exec = ex;
  return MB4_OK;
}

double conv_tol(const mb4_ensemble* e, unsigned long long u0max_bits) {
  if (!e->relative_eps) return e->eps;
  const double u0max = bits_to_double(u0max_bits);
  return e->eps * (u0max > DBL_MIN ? u0max : DBL_MIN);
}

// First iteration <= last whose norm met the tolerance; 0 if none; -1 if a
// norm up to `last` is not finite.
int converged_iteration(const mb4_ensemble* e, const unsigned long long* hrec, int last) {
  const double tol = conv_tol(e, hrec[0]);
  for (int l = 1; l <= last; ++l) {
    const double r = bits_to_double(hrec[l]);
    if (r <= tol) return l;
    if (!isfinite(r)) return -1;
  }
  return 0;
}

void update_prediction(mb4_ensemble* e, int batch_max) {
  if (batch_max >= e->predicted) {
    e->predicted = batch_max;
    e->lower_batches = 0;
  } else if (++e->lower_batches >= 2) {
    e->predicted = batch_max;
    e->lower_batches = 0;
  }
}

// One batch: member m takes todo[m] <= count steps.  On return remaining[m]
// has dropped by the steps member m accepted.
int run_batch(mb4_ensemble* e, std::vector<int64_t>& remaining) {
  int count = 0;
  for (int m = 0; m < e->count; ++m) {
    e->h_todo[m] = int(std::min<int64_t>(remaining[m], kBatch));
    count = std::max(count, e->h_todo[m]);
  }
  if (count == 0) return MB4_OK;
  const int iters = std::max(1, std::min(e->predicted, e->max_newton));
  HIP_TRY(hipMemcpyAsync(e->d_todo, e->h_todo, sizeof(int) * e->count, hipMemcpyHostToDevice,
                         e->stream));
  hipGraphExec_t exec = nullptr;
  if (e->use_graphs && batch_graph(e, count, iters, &exec) != MB4_OK) {
    (void)hipGetLastError();
    e->use_graphs = false;
    exec = nullptr;
  }
  if (exec != nullptr) {
    HIP_TRY(hipGraphLaunch(exec, e->stream));
  } else {
    const int rc = enqueue_batch(e, count, iters);
    if (rc != MB4_OK) return rc;
  }
  const size_t pitch = sizeof(unsigned long long) * e->rec_len;
  HIP_TRY(hipMemcpy2DAsync(e->h_ring, pitch, e->ring, pitch,
                           sizeof(unsigned long long) * (iters + 1), size_t(count) * e->count,
                           hipMemcpyDeviceToHost, e->stream));
  HIP_TRY(hipStreamSynchronize(e->stream));
  // Every member's accepted steps are counted before a failure is reported:
  // the device states of all members have moved on by exactly those steps.
  int batch_max = 1;
  int failed = -1, nonfinite = -1;
  for (int m = 0; m < e->count; ++m) {
    for (int k = 0; k < e->h_todo[m]; ++k) {
      const unsigned long long* hrec = e->h_ring + (size_t(k) * e->count + m) * e->rec_len;
      const int c = converged_iteration(e, hrec, iters);
      if (c <= 0) {
        if (c < 0 && nonfinite < 0) nonfinite = m;
        if (failed < 0) failed = m;
        break;
      }
      e->last_iters[m] = c;
      ++e->steps_done[m];
      --remaining[m];
      batch_max = std::max(batch_max, c);
    }
  }
  if (nonfinite >= 0)
    return fail(MB4_ENOCONV, "member %d: non-finite Newton update (step %lld)", nonfinite,
                static_cast<long long>(e->steps_done[nonfinite] + 1));
  if (failed >= 0) {
    if (iters >= e->max_newton)
      return fail(MB4_ENOCONV, "member %d: no convergence in %d Newton iterations (step %lld)",
                  failed, e->max_newton, static_cast<long long>(e->steps_done[failed] + 1));
    e->predicted = std::min(e->max_newton, std::max(iters + 1, batch_max));
    e->lower_batches = 0;
  } else {
    update_prediction(e, batch_max);
  }
  return MB4_OK;
}

int check(const mb4_ensemble* e) {
  if (e == nullptr) return fail(MB4_EINVAL, "ensemble is NULL");
  return MB4_OK;
}

int check_member(const mb4_ensemble* e, int32_t m) {
  int rc = check(e);
  if (rc != MB4_OK) return rc;
  if (m < 0 || m >= e->count) return fail(MB4_EINVAL, "member %d out of range", m);
  return MB4_OK;
}

int use_device(const mb4_ensemble* e) {
  HIP_TRY(hipSetDevice(e->device));
  return MB4_OK;
}

}  // namespace

extern "C" {

int mb4_ensemble_create(int32_t count, const mb4_lattice* lattices,
                        const double* const* potentials, const mb4_nonlinearity* nonlinearities,
                        const double* h, const mb4_options* opt, mb4_ensemble** out) {
  if (out == nullptr) return fail(MB4_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 1 || count > kMaxMembers)
    return fail(MB4_EINVAL, "count must be in [1, %d]", kMaxMembers);
  if (lattices == nullptr || potentials == nullptr || nonlinearities == nullptr || h == nullptr)
    return fail(MB4_EINVAL, "NULL argument array");
  mb4_options o;
  mb4_options_default(&o);
  if (opt != nullptr) {
    if (!isfinite(opt->eps) || opt->eps < 0.0 || opt->eps >= 1.0)
      return fail(MB4_EINVAL, "eps must be in [0, 1)");
    if (opt->max_newton < 0 || opt->max_newton > mb4::kMaxNewton)
      return fail(MB4_EINVAL, "max_newton must be in [0, %d]", mb4::kMaxNewton);
    if (opt->inner_sweeps < 0 || opt->inner_sweeps > mb4::kMaxFusedSweeps)
      return fail(MB4_EINVAL, "inner_sweeps of an ensemble must be in [0, %d]",
                  mb4::kMaxFusedSweeps);
    if ((opt->flags & ~(MB4_FLAG_NO_GRAPHS | MB4_FLAG_RELATIVE_EPS | MB4_FLAG_FP32_SOLVE)) != 0)
      return fail(MB4_EINVAL, "unknown bits in flags");
    if (opt->eps > 0.0) o.eps = opt->eps;
    if (opt->max_newton > 0) o.max_newton = opt->max_newton;
    if (opt->inner_sweeps > 0) o.inner_sweeps = opt->inner_sweeps;
    o.stream = opt->stream;
    o.mem_budget = opt->mem_budget;
    o.flags = opt->flags;
  }
  std::vector<MemberDesc> desc(static_cast<size_t>(count));
  size_t total = 0;
  for (int m = 0; m < count; ++m) {
    const mb4_lattice& lat = lattices[m];
    if (lat.nx < 3 || lat.ny < 3) return fail(MB4_EINVAL, "member %d: nx, ny must be >= 3", m);
    const int64_t sites = int64_t(lat.nx) * int64_t(lat.ny);
    if (sites > kMaxSites) return fail(MB4_EINVAL, "member %d has more than 2^28 sites", m);
    if (!isfinite(lat.t_hop) || !isfinite(lat.diag_shift))
      return fail(MB4_EINVAL, "member %d: t_hop and diag_shift must be finite", m);
    if (!isfinite(nonlinearities[m].g)) return fail(MB4_EINVAL, "member %d: g must be finite", m);
    if (!isfinite(h[m]) || h[m] == 0.0)
      return fail(MB4_EINVAL, "member %d: h must be finite and non-zero", m);
    if (potentials[m] == nullptr) return fail(MB4_EINVAL, "member %d: potential is NULL", m);
    if (!all_finite(potentials[m], size_t(sites)))
      return fail(MB4_EINVAL, "member %d: potential has non-finite entries", m);
    desc[m] = MemberDesc{lat.nx, lat.ny, lat.t_hop, lat.diag_shift, nonlinearities[m].g, h[m],
                         static_cast<long long>(total)};
    total += size_t(sites);
  }
  if (total > size_t(INT32_MAX)) return fail(MB4_EINVAL, "ensemble has more than 2^31 sites");
  if (records_words(count, o.max_newton) > size_t(INT32_MAX))
    return fail(MB4_EINVAL, "count * (max_newton + 1) too large for the step records");
  size_t energy_blocks = 0;
  {
    int tx, ty;
    mb4::energy_tile(&tx, &ty);
    for (const auto& d : desc) energy_blocks += size_t(tiles(d.nx, tx)) * tiles(d.ny, ty);
  }
  const size_t need = footprint_bytes(total, count, o.max_newton, energy_blocks);
  if (o.mem_budget != 0 && need > o.mem_budget)
    return fail(MB4_ENOMEM, "ensemble needs %zu bytes, above mem_budget %llu", need,
                static_cast<unsigned long long>(o.mem_budget));

  mb4_ensemble* e = new (std::nothrow) mb4_ensemble();
  if (e == nullptr) return fail(MB4_ENOMEM, "host allocation failed");
  e->count = count;
  e->desc = std::move(desc);
  e->total = total;
  e->eps = o.eps;
  e->relative_eps = (o.flags & MB4_FLAG_RELATIVE_EPS) != 0;
  e->fp32 = (o.flags & MB4_FLAG_FP32_SOLVE) != 0;
  e->max_newton = o.max_newton;
  e->sweeps = o.inner_sweeps;
  e->rec_len = o.max_newton + 1;
  e->stream = static_cast<hipStream_t>(o.stream);
  e->q = e->stream;
  e->use_graphs = (o.flags & MB4_FLAG_NO_GRAPHS) == 0;
  e->steps_done.assign(size_t(count), 0);
  e->last_iters.assign(size_t(count), 0);

  int rc = MB4_OK;
  hipError_t err = hipGetDevice(&e->device);
  if (err != hipSuccess) rc = fail(MB4_EDEVICE, "hipGetDevice: %s", hipGetErrorString(err));
  const size_t field = sizeof(double2) * total;
  if (rc == MB4_OK) rc = dalloc(e, reinterpret_cast<void**>(&e->V), sizeof(double) * total);
  if (rc == MB4_OK) rc = dalloc(e, reinterpret_cast<void**>(&e->u0), field);
  for (int i = 0; i < 3 && rc == MB4_OK; ++i) {
    rc = dalloc(e, reinterpret_cast<void**>(&e->Ua[i]), field);
    if (rc == MB4_OK) rc = dalloc(e, reinterpret_cast<void**>(&e->Ub[i]), field);
    if (rc == MB4_OK) rc = dalloc(e, reinterpret_cast<void**>(&e->ra[i]), field);
    if (rc == MB4_OK) rc = dalloc(e, reinterpret_cast<void**>(&e->rb[i]), field);
  }
  if (rc == MB4_OK)
    rc = dalloc(e, reinterpret_cast<void**>(&e->d_desc), sizeof(MemberDesc) * count);
  if (rc == MB4_OK)
    rc = dalloc(e, reinterpret_cast<void**>(&e->d_block0), sizeof(int) * 4 * (count + 1));
  if (rc == MB4_OK) rc = dalloc(e, reinterpret_cast<void**>(&e->d_todo), sizeof(int) * count);
  if (rc == MB4_OK) rc = halloc(e, reinterpret_cast<void**>(&e->h_todo), sizeof(int) * count);
  const size_t words = records_words(count, o.max_newton);
  if (rc == MB4_OK)
    rc = dalloc(e, reinterpret_cast<void**>(&e->ring), sizeof(unsigned long long) * words);
  if (rc == MB4_OK)
    rc = halloc(e, reinterpret_cast<void**>(&e->h_ring), sizeof(unsigned long long) * words);
  if (rc == MB4_OK)
    rc = dalloc(e, reinterpret_cast<void**>(&e->partials),
                sizeof(double) * 12 * std::max<size_t>(energy_blocks, 1));
  if (rc == MB4_OK)
    rc = dalloc(e, reinterpret_cast<void**>(&e->d_energy), sizeof(double) * 6 * count);
  if (rc == MB4_OK) {
    std::vector<double> vall(total);
    for (int m = 0; m < count; ++m)
      memcpy(vall.data() + e->desc[m].base, potentials[m],
             sizeof(double) * size_t(e->desc[m].nx) * e->desc[m].ny);
    err = hipMemcpy(e->V, vall.data(), sizeof(double) * total, hipMemcpyHostToDevice);
    if (err == hipSuccess)
      err = hipMemcpy(e->d_desc, e->desc.data(), sizeof(MemberDesc) * count,
                      hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemset(e->u0, 0, field);
    if (err != hipSuccess) rc = fail(MB4_EDEVICE, "upload: %s", hipGetErrorString(err));
  }
  if (rc == MB4_OK) rc = upload_blocks(e);
  if (rc != MB4_OK) {
    free_all(e);
    delete e;
    return rc;
  }
  *out = e;
  return MB4_OK;
}

void mb4_ensemble_destroy(mb4_ensemble* e) {
  if (e == nullptr) return;
  (void)hipSetDevice(e->device);
  (void)hipStreamSynchronize(e->stream);
  free_all(e);
  delete e;
}

int32_t mb4_ensemble_size(const mb4_ensemble* e) { return e == nullptr ? -1 : e->count; }

int mb4_ensemble_set_state(mb4_ensemble* e, int32_t m, const double* p, const double* q) {
  int rc = check_member(e, m);
  if (rc != MB4_OK) return rc;
  if (p == nullptr || q == nullptr) return fail(MB4_EINVAL, "p and q must not be NULL");
  const MemberDesc& d = e->desc[m];
  const size_t n = size_t(d.nx) * d.ny;
  if (!all_finite(p, n) || !all_finite(q, n)) return fail(MB4_EINVAL, "state has non-finite entries");
  if ((rc = use_device(e)) != MB4_OK) return rc;
  double* stage = reinterpret_cast<double*>(e->Ua[0]);  // scratch between steps
  HIP_TRY(hipMemcpyAsync(stage, p, sizeof(double) * n, hipMemcpyHostToDevice, e->stream));
  HIP_TRY(hipMemcpyAsync(stage + n, q, sizeof(double) * n, hipMemcpyHostToDevice, e->stream));
  HIP_TRY(mb4::launch_interleave(stage, stage + n, e->u0 + d.base, int(n), e->stream));
  HIP_TRY(hipStreamSynchronize(e->stream));
  e->steps_done[m] = 0;
  e->last_iters[m] = 0;
  return MB4_OK;
}

int mb4_ensemble_get_state(mb4_ensemble* e, int32_t m, double* p, double* q) {
  int rc = check_member(e, m);
  if (rc != MB4_OK) return rc;
  if (p == nullptr || q == nullptr) return fail(MB4_EINVAL, "p and q must not be NULL");
  if ((rc = use_device(e)) != MB4_OK) return rc;
  const MemberDesc& d = e->desc[m];
  const size_t n = size_t(d.nx) * d.ny;
  double* stage = reinterpret_cast<double*>(e->Ua[0]);
  HIP_TRY(mb4::launch_deinterleave(e->u0 + d.base, stage, stage + n, int(n), e->stream));
  HIP_TRY(hipMemcpyAsync(p, stage, sizeof(double) * n, hipMemcpyDeviceToHost, e->stream));
  HIP_TRY(hipMemcpyAsync(q, stage + n, sizeof(double) * n, hipMemcpyDeviceToHost, e->stream));
  HIP_TRY(hipStreamSynchronize(e->stream));
  return MB4_OK;
}

int mb4_ensemble_step(mb4_ensemble* e, int64_t nsteps) {
  int rc = check(e);
  if (rc != MB4_OK) return rc;
  if (nsteps < 0) return fail(MB4_EINVAL, "nsteps must be >= 0");
  if ((rc = use_device(e)) != MB4_OK) return rc;
  std::vector<int64_t> remaining(size_t(e->count), nsteps);
  for (;;) {
    bool left = false;
    for (int64_t r : remaining) left = left || r > 0;
    if (!left) return MB4_OK;
    rc = run_batch(e, remaining);
    if (rc != MB4_OK) return rc;
  }
}

int mb4_ensemble_energy_components(mb4_ensemble* e, double* out) {
  int rc = check(e);
  if (rc != MB4_OK) return rc;
  if (out == nullptr) return fail(MB4_EINVAL, "out is NULL");
  if ((rc = use_device(e)) != MB4_OK) return rc;
  const Multi mu = multi_of(e, kEnergy, 0);
  Multi me = mu;
  me.todo = nullptr;
  HIP_TRY(mb4::launch_energy_multi(lattice_of(e), me, e->partials, e->d_energy, e->stream));
  HIP_TRY(hipMemcpyAsync(out, e->d_energy, sizeof(double) * 6 * e->count, hipMemcpyDeviceToHost,
                         e->stream));
  HIP_TRY(hipStreamSynchronize(e->stream));
  return MB4_OK;
}

int mb4_ensemble_member_stats(const mb4_ensemble* e, int32_t m, int64_t* steps_done,
                              int32_t* newton_iters) {
  const int rc = check_member(e, m);
  if (rc != MB4_OK) return rc;
  if (steps_done) *steps_done = e->steps_done[m];
  if (newton_iters) *newton_iters = e->last_iters[m];
  return MB4_OK;
}

int mb4_ensemble_set_region(mb4_ensemble* e, int32_t region) {
  int rc = check(e);
  if (rc != MB4_OK) return rc;
  if (region < 0 || region >= mb4::kRegionCount)
    return fail(MB4_EINVAL, "region must be in [0, %d)", int(mb4::kRegionCount));
  if (!region_usable(region, e->sweeps, e->fp32))
    return fail(MB4_EINVAL, "region %s leaves no tile at %d sweeps", mb4::region_name(region),
                e->sweeps);
  if (region == e->region) return MB4_OK;
  if ((rc = use_device(e)) != MB4_OK) return rc;
  HIP_TRY(hipStreamSynchronize(e->stream));
  const int old = e->region;
  e->region = region;
  rc = upload_blocks(e);
  if (rc != MB4_OK) {
    e->region = old;
    (void)upload_blocks(e);
    return rc;
  }
  drop_graphs(e);
  return MB4_OK;
}

int32_t mb4_ensemble_region(const mb4_ensemble* e) { return e == nullptr ? -1 : e->region; }

int mb4_ensemble_tune(mb4_ensemble* e, int32_t steps, int32_t* best, double* ms_per_step) {
  int rc = check(e);
  if (rc != MB4_OK) return rc;
  if (steps < 1) return fail(MB4_EINVAL, "steps must be >= 1");
  if ((rc = use_device(e)) != MB4_OK) return rc;
  const size_t field = sizeof(double2) * e->total;
  void* backup = nullptr;
  HIP_TRY(hipMalloc(&backup, field));
  const std::vector<int64_t> done0 = e->steps_done;
  const std::vector<int> iters0 = e->last_iters;
  const int pred0 = e->predicted, lower0 = e->lower_batches, region0 = e->region;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  double times[mb4::kRegionCount];
  int chosen = region0;
  double best_ms = -1.0;
  // Member states and counters go back after every trial; the iteration
  // prediction learnt in the untimed pass is kept for the timed one, and
  // reset at the end.
  auto restore = [&]() -> hipError_t {
    e->steps_done = done0;
    e->last_iters = iters0;
    return hipMemcpyAsync(e->u0, backup, field, hipMemcpyDeviceToDevice, e->stream);
  };
  hipError_t err = hipMemcpyAsync(backup, e->u0, field, hipMemcpyDeviceToDevice, e->stream);
  if (err == hipSuccess) err = hipEventCreate(&t0);
  if (err == hipSuccess) err = hipEventCreate(&t1);
  if (err != hipSuccess) rc = fail(MB4_EDEVICE, "tune setup: %s", hipGetErrorString(err));
  for (int r = 0; r < mb4::kRegionCount && rc == MB4_OK; ++r) {
    times[r] = -1.0;
    if (!region_usable(r, e->sweeps, e->fp32)) continue;
    rc = mb4_ensemble_set_region(e, r);
    // One untimed pass (graph capture, caches), then the timed one.
    if (rc == MB4_OK) rc = mb4_ensemble_step(e, std::min<int64_t>(steps, kBatch));
    if (rc == MB4_OK && (err = restore()) != hipSuccess)
      rc = fail(MB4_EDEVICE, "tune restore: %s", hipGetErrorString(err));
    if (rc == MB4_OK && (err = hipEventRecord(t0, e->stream)) != hipSuccess)
      rc = fail(MB4_EDEVICE, "tune event: %s", hipGetErrorString(err));
    if (rc == MB4_OK) rc = mb4_ensemble_step(e, steps);
    if (rc == MB4_OK && (err = hipEventRecord(t1, e->stream)) != hipSuccess)
      rc = fail(MB4_EDEVICE, "tune event: %s", hipGetErrorString(err));
    if (rc == MB4_OK && (err = hipEventSynchronize(t1)) != hipSuccess)
      rc = fail(MB4_EDEVICE, "tune event: %s", hipGetErrorString(err));
    float ms = 0.0f;
    if (rc == MB4_OK && (err = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess)
      rc = fail(MB4_EDEVICE, "tune event: %s", hipGetErrorString(err));
    if (rc == MB4_OK && (err = restore()) != hipSuccess)
      rc = fail(MB4_EDEVICE, "tune restore: %s", hipGetErrorString(err));
    if (rc == MB4_OK) {
      times[r] = double(ms) / steps;
      if (best_ms < 0.0 || times[r] < best_ms) {
        best_ms = times[r];
        chosen = r;
      }
    }
  }
  const int rc_sel = mb4_ensemble_set_region(e, rc == MB4_OK ? chosen : region0);
  if (rc != MB4_OK) (void)restore();
  e->predicted = pred0;
  e->lower_batches = lower0;
  (void)hipStreamSynchronize(e->stream);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  (void)hipFree(backup);
  if (rc != MB4_OK) return rc;
  if (rc_sel != MB4_OK) return rc_sel;
  if (best) *best = chosen;
  if (ms_per_step)
    for (int r = 0; r < mb4::kRegionCount; ++r) ms_per_step[r] = times[r];
  return MB4_OK;
}

}  // extern "C"
