// Host runtime and C ABI of the MB4 integrator (see include/mb4.h).
//
// A state owns the device fields of one lattice problem and drives
// Algorithm 1 of Sakai et al. (arXiv 2003.04345) on one stream:
//   per step, Newton iterations l = 1, 2, ..., each = stage solve (k
//   block-Jacobi sweeps, the three stages in one launch, which also records
//   ||r^l||_inf; in iteration 1 it builds the residual at U^0 = e_3 (x) u_0
//   itself) + update pass.  The update pass of the iteration whose norm meets
//   the tolerance writes u_1 = U_{c_3} over u_0 (Sec. 2.2, last paragraph:
//   c_3 = 1); the others apply the Newton update and form the next residual.
//   Every kernel of iteration l >= 2 returns at once when ||r^{l-1}||_inf
//   already met the tolerance.  Since the buffers a step uses depend only on
//   its place in the batch (u_0 alternates between two buffers and returns
//   to the first at the batch's end), up to kBatch steps are enqueued back to
//   back with the previous step's iteration count, and one read-back of
//   their statistics per batch tells the host where each converged (see
//   run_batch for the rare step that needs more iterations).
#include <float.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "mb4.h"
#include "mb4_internal.h"
#include "mb4_spectral.h"

using mb4::CPlanes3;
using mb4::ConvCheck;
using mb4::Lattice;
using mb4::Planes3;

namespace {

constexpr double kDefaultEps = 1e-13;  // Sec. 3: epsilon = 1e-13
constexpr int kDefaultMaxNewton = 50;
constexpr int kDefaultSweeps = 3;
constexpr int kMaxSweeps = 64;
constexpr int64_t kMaxSites = int64_t(1) << 28;
constexpr int kInitialPrediction = 3;
constexpr int kBatch = 32;  // steps enqueued per host round trip

thread_local std::string g_detail;

using mb4::rt::fail;

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

// Kernel classes for timing.  Update passes are recorded as kUpdateResidual
// and classified when the step is decided: iteration 1 (which starts from
// U = e_3 (x) u_0 and reads no U), later iterations, and the final update.
enum KernelClass {
  kFirstSolve = 0,
  kStageSolve = 1,
  kSweep = 2,
  kUpdateResidualFirst = 3,
  kUpdateResidual = 4,
  kFinalUpdate = 5,
  kIterateFirst = 6,
  kIterate = 7,
  kFinalFirst = 8,  // final update of a step fused with the next first solve
  kIterateLast = 9,  // the batch's last iteration: writes only X_3 (see below)
  kFinalEnd = 10,   // recorded as such, counted as kFinalUpdate
};
constexpr int kKernelClasses = 10;
const char* const kKernelNames[kKernelClasses] = {
    "stage_solve_first", "stage_solve", "stage_sweep", "update_residual_first",
    "update_residual",   "final_update", "iterate_first", "iterate",
    "final_first",       "iterate_last"};

}  // namespace

struct mb4_state {
  int nx = 0, ny = 0;
  size_t sites = 0;
  double t = 0, shift = 0, g = 0, h = 0;
  double eps = kDefaultEps;
  bool relative_eps = false;  // eps scaled by ||u_0||_inf
  bool fp32 = false;          // FP32 inner stage solves
  bool spectral = false;      // spectrally preconditioned stage solves
  double kappa0 = 0.0;        // their preconditioner's on-site value
  double2* twx = nullptr;     // their twiddles, nx and ny entries
  double2* twy = nullptr;
  int max_newton = kDefaultMaxNewton;
  uint64_t mem_budget = 0;  // 0: no limit
  int sweeps = kDefaultSweeps;
  int region = mb4::kRegion32x32;  // solve-region shape of the fused path
  hipStream_t stream = nullptr;
  // Stream the step kernels are enqueued to: `stream`, or cap_stream while a
  // batch is being captured into a graph.
  hipStream_t q = nullptr;
  hipStream_t cap_stream = nullptr;
  bool use_graphs = true;
  // Instantiated graphs of whole batches, keyed by (steps, iterations); the
  // time step and buffers are baked into their kernel arguments, so
  // mb4_set_h drops them.
  struct GraphEntry {
    int count, iters;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  int device = 0;
  std::vector<void*> device_allocs;
  std::vector<void*> host_allocs;
  double* V = nullptr;
  double* gs = nullptr;    // per-site nonlinearity g_j, allocated on first use
  bool gs_on = false;      // the kernels read gs instead of g
  double2* u0 = nullptr;
  double2* u0b = nullptr;  // second u_0 buffer of the fused path's batches
  double2* Ua[3] = {nullptr, nullptr, nullptr};
  double2* Ub[3] = {nullptr, nullptr, nullptr};
  double2* phib[3] = {nullptr, nullptr, nullptr};
  double2* ra[3] = {nullptr, nullptr, nullptr};
  double2* rb[3] = {nullptr, nullptr, nullptr};
  // Newton statistics: a ring of kBatch step records of rec_len words
  // (rec[0] = ||u_0||_inf, rec[l] = ||r^l||_inf, l = 1 .. max_newton), one
  // per step of a batch, cleared when the batch starts; h_ring is its pinned
  // host copy.  dbg_rec serves the kernel-level entry points.
  unsigned long long* ring = nullptr;
  unsigned long long* h_ring = nullptr;
  unsigned long long* dbg_rec = nullptr;
  unsigned long long* h_dbg = nullptr;
  int rec_len = 0;
  std::vector<double> last_res;  // ||r^l||_inf of the last accepted step
  double* partials = nullptr;
  double* eout = nullptr;
  double* h_eout = nullptr;  // pinned, 6 doubles
  // Per-kernel timing (mb4_profile_*): events bracketing launches of the
  // current step, collected once the step is decided.
  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Rec {
    int cls, step, iter;
    hipEvent_t a, b;
  };
  std::vector<Rec> prof_pending;
  int64_t prof_launches[kKernelClasses] = {};
  double prof_ms[kKernelClasses] = {};
  int64_t steps_done = 0;
  int last_iters = 0;
  int last_sweeps = 0;
  double last_rnorm = 0.0;
  int predicted = kInitialPrediction;
  int lower_batches = 0;  // batches in a row whose largest count was below it
};

namespace {

// Device-side test "Newton iteration `prev` of the step recorded at `rec`
// met the tolerance".
ConvCheck conv_check(const mb4_state* s, const unsigned long long* rec, int prev) {
  return ConvCheck{rec, prev, s->eps, s->relative_eps};
}

// Device bytes of a state: V (8 B/site), two u_0 buffers (2 x 16) and two
// stage-increment fields (2 x 48), plus the statistics records and the
// energy partial sums.  The plain path (more than four sweeps, the spectral
// solves, mb4_stage_solve beyond four sweeps) also needs the transformed
// residual (48) and two stage-correction fields (2 x 48), allocated when
// first needed.
constexpr size_t kFusedBytesPerSite = 136;
constexpr size_t kPlainBytesPerSite = 144;

size_t footprint_bytes(size_t sites, int nx, int ny, int max_newton, bool plain) {
  return sites * (kFusedBytesPerSite + (plain ? kPlainBytesPerSite : 0)) +
         size_t(kBatch + 1) * size_t(max_newton + 1) * 8 +
         mb4::energy_partials_count(nx, ny) * sizeof(double) + 8 * sizeof(double);
}

// Device bytes of a state with (plain) the plain path's fields and (site_g)
// a per-site nonlinearity.
size_t state_bytes(const mb4_state* s, bool plain, bool site_g) {
  return footprint_bytes(s->sites, s->nx, s->ny, s->max_newton, plain) +
         (site_g ? s->sites * sizeof(double) : 0);
}

int dalloc(mb4_state* s, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(e == hipErrorOutOfMemory ? MB4_ENOMEM : MB4_EDEVICE, "hipMalloc(%zu): %s", bytes,
                hipGetErrorString(e));
  }
  s->device_allocs.push_back(*p);
  return MB4_OK;
}

// The plain path's fields (Phibar, and rbar ping-pong), allocated on first
// use within the state's memory budget.
int ensure_plain_fields(mb4_state* s) {
  if (s->phib[0] != nullptr) return MB4_OK;
  if (s->mem_budget != 0 && state_bytes(s, true, s->gs != nullptr) > s->mem_budget)
    return fail(MB4_ENOMEM, "the plain path needs %zu bytes per site more, above mem_budget %llu",
                kPlainBytesPerSite, static_cast<unsigned long long>(s->mem_budget));
  const size_t field = s->sites * sizeof(double2);
  int rc = MB4_OK;
  for (int i = 0; i < 3 && rc == MB4_OK; ++i) {
    rc = dalloc(s, reinterpret_cast<void**>(&s->phib[i]), field);
    if (rc == MB4_OK) rc = dalloc(s, reinterpret_cast<void**>(&s->ra[i]), field);
    if (rc == MB4_OK) rc = dalloc(s, reinterpret_cast<void**>(&s->rb[i]), field);
  }
  if (rc != MB4_OK) {
    // Leave none of them half-made: the next call tries again.
    for (int i = 0; i < 3; ++i)
      for (double2** f : {&s->phib[i], &s->ra[i], &s->rb[i]}) {
        if (*f == nullptr) continue;
        (void)hipFree(*f);
        s->device_allocs.erase(std::find(s->device_allocs.begin(), s->device_allocs.end(),
                                         static_cast<void*>(*f)));
        *f = nullptr;
      }
  }
  return rc;
}

int halloc(mb4_state* s, void** p, size_t bytes) {
  hipError_t e = hipHostMalloc(p, bytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(MB4_EDEVICE, "hipHostMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  s->host_allocs.push_back(*p);
  return MB4_OK;
}

void drop_graphs(mb4_state* s) {
  for (auto& g : s->graphs) (void)hipGraphExecDestroy(g.exec);
  s->graphs.clear();
}

void free_all(mb4_state* s) {
  drop_graphs(s);
  if (s->cap_stream != nullptr) (void)hipStreamDestroy(s->cap_stream);
  s->cap_stream = nullptr;
  for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
  s->ev_pool.clear();
  for (void* p : s->device_allocs) (void)hipFree(p);
  for (void* p : s->host_allocs) (void)hipHostFree(p);
  s->device_allocs.clear();
  s->host_allocs.clear();
}

Lattice lattice_of(const mb4_state* s) {
  Lattice L;
  L.nx = s->nx;
  L.ny = s->ny;
  L.t = s->t;
  L.shift = s->shift;
  L.g = s->g;
  L.h = s->h;
  L.V = s->V;
  L.u0 = s->u0;
  L.gs = s->gs_on ? s->gs : nullptr;
  return L;
}

Planes3 P(double2* const (&a)[3]) { return Planes3{{a[0], a[1], a[2]}}; }
CPlanes3 C(double2* const (&a)[3]) { return CPlanes3{{a[0], a[1], a[2]}}; }

Planes3 planes_of(double* base, size_t sites) {
  double2* b = reinterpret_cast<double2*>(base);
  return Planes3{{b, b + sites, b + 2 * sites}};
}

CPlanes3 cplanes_of(const double* base, size_t sites) {
  const double2* b = reinterpret_cast<const double2*>(base);
  return CPlanes3{{b, b + sites, b + 2 * sites}};
}

int use_device(const mb4_state* s) {
  HIP_TRY(hipSetDevice(s->device));
  return MB4_OK;
}

int prof_event(mb4_state* s, hipEvent_t* ev) {
  if (s->ev_used == s->ev_pool.size()) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    s->ev_pool.push_back(e);
  }
  *ev = s->ev_pool[s->ev_used++];
  return MB4_OK;
}

// Adds the durations of the recorded launches to the per-class totals.
// Step k of the batch converged at iteration m[k] (0: it did not); its
// launches of later iterations returned at once and are not counted, and its
// update pass of iteration m[k] counts as the final update.
int prof_collect(mb4_state* s, const std::vector<int>& m) {
  for (const auto& r : s->prof_pending) {
    const int mk = (r.step < int(m.size())) ? m[r.step] : 0;
    if (mk > 0 && r.iter > mk) continue;
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    int cls = r.cls;
    if (cls == kUpdateResidual || cls == kIterate || cls == kIterateLast) {
      if (r.iter == mk)
        cls = kFinalUpdate;
      else if (cls != kIterateLast && r.iter == 1)
        cls = cls == kUpdateResidual ? kUpdateResidualFirst : kIterateFirst;
    } else if (cls == kFinalEnd) {
      if (r.iter != mk) continue;  // returned at once
      cls = kFinalUpdate;
    }
    s->prof_launches[cls] += 1;
    s->prof_ms[cls] += ms;
  }
  s->prof_pending.clear();
  s->ev_used = 0;
  return MB4_OK;
}

// Events for one launch: a fresh pair from the pool when profiling (the
// launch records its own start/stop timestamps), none otherwise.
int launch_events(mb4_state* s, int cls, int step, int iter, mb4::LaunchEvents* ev) {
  *ev = mb4::LaunchEvents{};
  if (!s->prof_on) return MB4_OK;
  int rc = prof_event(s, &ev->start);
  if (rc == MB4_OK) rc = prof_event(s, &ev->stop);
  if (rc != MB4_OK) return rc;
  s->prof_pending.push_back(mb4_state::Rec{cls, step, iter, ev->start, ev->stop});
  return MB4_OK;
}

// Enqueues one kernel launch; `expr` may use the LaunchEvents `ev_`.
#define LAUNCH(s, cls, step, iter, expr)                          \
  do {                                                            \
    mb4::LaunchEvents ev_;                                        \
    const int rc_ = launch_events((s), (cls), (step), (iter), &ev_); \
    if (rc_ != MB4_OK) return rc_;                                \
    HIP_TRY(expr);                                                \
  } while (0)

// Enqueues the stage solve of Newton iteration `iter` of step `step` of the
// batch (record `rec`): up to four block-Jacobi sweeps from r = 0 in one
// temporally blocked pass into ra (in iteration 1 with the residual at U^0
// built in place), then any further sweeps one pass each, alternating between
// rb and ra.  The pass that produces the solution records ||r^iter||_inf in
// rec[iter].  `*result` receives the planes that hold the solution.
int enqueue_spectral_solve(mb4_state* s, const Lattice& L, int step, int iter,
                           unsigned long long* rec, double2* const** result);

int enqueue_solve(mb4_state* s, const Lattice& L, int step, int iter, unsigned long long* rec,
                  double2* const** result) {
  if (s->spectral) return enqueue_spectral_solve(s, L, step, iter, rec, result);
  const ConvCheck chk = iter >= 2 ? conv_check(s, rec, iter - 1) : ConvCheck{nullptr, 0, 0.0, false};
  const int fused = std::min(s->sweeps, mb4::kMaxFusedSweeps);
  const bool extra = s->sweeps > fused;
  unsigned long long* rslot = rec + iter;
  if (iter == 1) {
    const Planes3 store = extra ? P(s->phib) : Planes3{{nullptr, nullptr, nullptr}};
    LAUNCH(s, kFirstSolve, step, iter,
           mb4::launch_first_solve(L, P(s->ra), fused, extra ? nullptr : rslot, rec, store,
                                   s->q, ev_));
  } else {
    LAUNCH(s, kStageSolve, step, iter,
           mb4::launch_stage_solve(L, C(s->phib), P(s->ra), fused, extra ? nullptr : rslot, chk,
                                   s->q, ev_));
  }
  double2* const* cur = s->ra;
  for (int k = fused; k < s->sweeps; ++k) {
    double2* const(&out)[3] = (cur == s->ra) ? s->rb : s->ra;
    const CPlanes3 in{{cur[0], cur[1], cur[2]}};
    LAUNCH(s, kSweep, step, iter,
           mb4::launch_stage_sweep(L, C(s->phib), in, P(out),
                                   k == s->sweeps - 1 ? rslot : nullptr, chk, s->q, ev_));
    cur = out;
  }
  *result = cur;
  return MB4_OK;
}

// Spectrally preconditioned stage solve of Newton iteration `iter` (see
// mb4_spectral.hip): s->sweeps Richardson iterations into ra, with rb as the
// transform buffer.  In iteration 1 the residual at U^0 = e_3 (x) u_0 comes
// first, from the one-sweep first solve (which stores it in phib and records
// ||u_0||_inf; its own solution goes to rb and is not used).  The last
// Richardson iteration records ||r^iter||_inf in rec[iter].
int enqueue_spectral_solve(mb4_state* s, const Lattice& L, int step, int iter,
                           unsigned long long* rec, double2* const** result) {
  const ConvCheck none{nullptr, 0, 0.0, false};
  const ConvCheck chk = iter >= 2 ? conv_check(s, rec, iter - 1) : none;
  if (iter == 1)
    LAUNCH(s, kFirstSolve, step, 1,
           mb4::launch_first_solve(L, P(s->rb), 1, nullptr, rec, P(s->phib), s->q, ev_));
  const mb4::SpectralArgs sa{s->kappa0, s->twx, s->twy};
  LAUNCH(s, kStageSolve, step, iter,
         mb4::launch_spectral_pass(0, L, C(s->phib), P(s->rb), P(s->ra), sa, nullptr, chk, s->q,
                                   ev_));
  for (int k = 0; k < s->sweeps; ++k) {
    const bool last = k == s->sweeps - 1;
    LAUNCH(s, kSweep, step, iter,
           mb4::launch_spectral_pass(1, L, C(s->phib), P(s->rb), P(s->ra), sa, nullptr, chk,
                                     s->q, ev_));
    LAUNCH(s, kSweep, step, iter,
           mb4::launch_spectral_pass(last ? 3 : 2, L, C(s->phib), P(s->rb), P(s->ra), sa,
                                     last ? rec + iter : nullptr, chk, s->q, ev_));
  }
  *result = s->ra;
  return MB4_OK;
}

CPlanes3 cp(double2* const* a) { return CPlanes3{{a[0], a[1], a[2]}}; }
Planes3 pp(double2* const* a) { return Planes3{{a[0], a[1], a[2]}}; }

// Fused path (at most four sweeps): the iterate of Newton iteration l is
// X^l = U^l - e (x) u_0 (see mb4::StepOut), in Ua (l + sigma odd) or Ub.
// Iteration 1's stage solve is the first-solve kernel, iteration l's (l >= 2)
// is part of the pass that forms the residual of iteration l - 1
// (k_iterate), and a step's u_1 is written by the pass after the iteration
// that met the tolerance.
//
// Batch step k of `count` reads u_0 from u0 (k even) or u0b (k odd) and
// writes u_1 to the other buffer, the last step to u0, so that a batch ends
// where it started.  The final update of step k - 1 is fused into the first
// solve of step k (prev_rec: step k - 1's record); only the last step has a
// final-update pass of its own (emit_final).  sigma = k * iters alternates the
// X buffers so that the first solve of step k does not write the X that step
// k - 1's final update reads.
double2* const* x_planes(mb4_state* s, int l) { return (l & 1) ? s->Ua : s->Ub; }
double2* batch_u0(mb4_state* s, int k) { return (k & 1) ? s->u0b : s->u0; }

int enqueue_iterations_fused(mb4_state* s, int step, int count, unsigned long long* rec,
                             int first, int last, int sigma = 0,
                             const unsigned long long* prev_rec = nullptr,
                             bool emit_final = true, bool last_is_final = false) {
  Lattice L = lattice_of(s);
  double2* const src = batch_u0(s, step);
  L.u0 = src;
  mb4::StepOut so{step == count - 1 ? s->u0 : batch_u0(s, step + 1), s->u0};
  const ConvCheck none{nullptr, 0, 0.0, false};
  auto xp = [&](int l) { return x_planes(s, l + sigma); };
  for (int l = first; l <= last; ++l) {
    if (l == 1) {
      unsigned long long* const u0max = s->relative_eps ? rec : nullptr;
      if (prev_rec != nullptr) {
        // Step k - 1 ran `last` iterations too, with sigma_{k-1} = sigma - last
        // (mod 2), so its X^last sits in x_planes(last + sigma_{k-1}).
        const int sigma_prev = (sigma + last) & 1;
        const mb4::PrevStep pv{batch_u0(s, step - 1), cp(x_planes(s, last + sigma_prev)),
                               last >= 2 ? conv_check(s, prev_rec, last - 1) : none,
                               conv_check(s, prev_rec, last), src, s->u0};
        LAUNCH(s, kFinalFirst, step, 1,
               mb4::launch_first_solve_x(L, pp(xp(1)), s->sweeps, rec + 1, u0max, s->q, ev_,
                                         mb4::Multi{}, s->region, s->fp32, &pv));
      } else {
        LAUNCH(s, kFirstSolve, step, 1,
               mb4::launch_first_solve_x(L, pp(xp(1)), s->sweeps, rec + 1, u0max, s->q, ev_,
                                         mb4::Multi{}, s->region, s->fp32, nullptr));
      }
      continue;
    }
    const int j = l - 1;  // the iteration whose residual this pass forms
    const ConvCheck chk = j >= 2 ? conv_check(s, rec, j - 1) : none;
    // In a batch, a step that has not converged by its last iteration is
    // done again from u_0 (step_single), so of that iteration's X only X_3,
    // which u_1 = u_0 + X_3 takes, is ever read.
    mb4::StepOut sol = so;
    sol.stage3_only = last_is_final && l == last;
    LAUNCH(s, sol.stage3_only ? kIterateLast : kIterate, step, j,
           mb4::launch_iterate(L, cp(xp(j)), pp(xp(l)), s->sweeps, rec + l, chk,
                               conv_check(s, rec, j), sol, s->q, ev_, mb4::Multi{},
                               s->region, s->fp32));
  }
  if (!emit_final) return MB4_OK;
  const ConvCheck chk = last >= 2 ? conv_check(s, rec, last - 1) : none;
  LAUNCH(s, kFinalEnd, step, last,
         mb4::launch_final_update(L, cp(xp(last)), chk, conv_check(s, rec, last), so, s->q, ev_));
  return MB4_OK;
}

// Iterations first .. last of a single step (u_0 and u_1 in s->u0).
int enqueue_iterations(mb4_state* s, const Lattice& L, int step, unsigned long long* rec,
                       int first, int last) {
  if (s->sweeps <= mb4::kMaxFusedSweeps && !s->spectral)
    return enqueue_iterations_fused(s, 0, 1, rec, first, last);
  for (int l = first; l <= last; ++l) {
    double2* const* rfin = nullptr;
    const int rc = enqueue_solve(s, L, step, l, rec, &rfin);
    if (rc != MB4_OK) return rc;
    const ConvCheck chk = (l >= 2) ? conv_check(s, rec, l - 1) : ConvCheck{nullptr, 0, 0.0, false};
    const ConvCheck fin = conv_check(s, rec, l);
    // Iteration l writes X = U - e (x) u_0 into Ua (l odd) or Ub (l even) and
    // reads the other.
    double2* const(&uout)[3] = (l % 2 == 1) ? s->Ua : s->Ub;
    double2* const(&uin)[3] = (l % 2 == 1) ? s->Ub : s->Ua;
    const CPlanes3 rbar{{rfin[0], rfin[1], rfin[2]}};
    LAUNCH(s, kUpdateResidual, step, l,
           mb4::launch_update_residual(L, C(uin), P(uout), rbar, true, l == 1, P(s->phib),
                                       nullptr, chk, fin, s->u0, s->q, ev_, true));
  }
  return MB4_OK;
}

// Newton tolerance of a step whose record starts with ||u_0||_inf bits.
double conv_tol(const mb4_state* s, unsigned long long u0max_bits) {
  if (!s->relative_eps) return s->eps;
  const double u0max = bits_to_double(u0max_bits);
  return s->eps * (u0max > DBL_MIN ? u0max : DBL_MIN);
}

// First iteration <= last whose norm in host record hrec met the tolerance;
// 0 if none; -1 if a norm up to `last` is not finite.
int converged_iteration(const mb4_state* s, const unsigned long long* hrec, int last) {
  const double tol = conv_tol(s, hrec[0]);
  for (int l = 1; l <= last; ++l) {
    const double r = bits_to_double(hrec[l]);
    if (r <= tol) return l;
    if (!isfinite(r)) return -1;
  }
  return 0;
}

void accept(mb4_state* s, const unsigned long long* hrec, int m) {
  s->last_iters = m;
  s->last_sweeps = m * s->sweeps;
  s->last_rnorm = bits_to_double(hrec[m]);
  s->last_res.assign(size_t(m), 0.0);
  for (int l = 1; l <= m; ++l) s->last_res[l - 1] = bits_to_double(hrec[l]);
  ++s->steps_done;
}

// Iterations the next batch is built for.  A batch built for more iterations
// than a step needs costs little (the surplus launches return at once), one
// built for fewer loses the rest of the batch; so the prediction follows the
// largest count of the last batch up at once and down only after two batches
// in a row stayed below it.
void update_prediction(mb4_state* s, int batch_max) {
  if (batch_max >= s->predicted) {
    s->predicted = batch_max;
    s->lower_batches = 0;
  } else if (++s->lower_batches >= 2) {
    s->predicted = batch_max;
    s->lower_batches = 0;
  }
}

// Fast path: `count` <= kBatch steps enqueued back to back, each with
// `iters` Newton iterations, and one read-back for all of them.  A step that
// converged in time wrote u_1 over u_0, so the next step starts from it.  If
// step k did not converge in time, u_0 kept its value, the later steps of the
// batch repeated step k's computation exactly (every kernel is
// deterministic) and changed nothing; *accepted = k tells the caller where to
// continue.
// Enqueues the whole batch (statistics cleared, then every step) on s->q.
int enqueue_batch(mb4_state* s, int count, int iters) {
  const Lattice L = lattice_of(s);
  HIP_TRY(mb4::launch_clear(s->ring, count * s->rec_len, s->q));
  const bool fused = s->sweeps <= mb4::kMaxFusedSweeps && !s->spectral;
  for (int k = 0; k < count; ++k) {
    unsigned long long* rec = s->ring + size_t(k) * s->rec_len;
    const int rc =
        fused ? enqueue_iterations_fused(s, k, count, rec, 1, iters, (k * iters) & 1,
                                         k > 0 ? rec - s->rec_len : nullptr, k == count - 1,
                                         true)
              : enqueue_iterations(s, L, k, rec, 1, iters);
    if (rc != MB4_OK) return rc;
  }
  return MB4_OK;
}

// The graph of a batch of `count` steps with `iters` iterations each,
// captured on first use.
int batch_graph(mb4_state* s, int count, int iters, hipGraphExec_t* exec) {
  for (const auto& g : s->graphs)
    if (g.count == count && g.iters == iters) {
      *exec = g.exec;
      return MB4_OK;
    }
  if (s->cap_stream == nullptr)
    HIP_TRY(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
  s->q = s->cap_stream;
  HIP_TRY(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue_batch(s, count, iters);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(s->cap_stream, &graph);
  s->q = s->stream;
  if (rc != MB4_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return fail(MB4_EDEVICE, "graph capture: %s", hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return fail(MB4_EDEVICE, "graph instantiate: %s", hipGetErrorString(ei));
  if (s->graphs.size() >= 64) {  // keep the cache bounded
    (void)hipGraphExecDestroy(s->graphs.front().exec);
    s->graphs.erase(s->graphs.begin());
  }
  s->graphs.push_back(mb4_state::GraphEntry{count, iters, ex});
  *exec = ex;
  return MB4_OK;
}

int run_batch(mb4_state* s, int count, int iters, int* accepted) {
  // Graphs replay the same launches with less host work per kernel; while
  // profiling, kernels are launched one by one with their timing events.
  hipGraphExec_t exec = nullptr;
  if (s->use_graphs && !s->prof_on && batch_graph(s, count, iters, &exec) != MB4_OK) {
    // A runtime that cannot capture these launches: run eagerly from now on.
    (void)hipGetLastError();
    s->use_graphs = false;
    exec = nullptr;
  }
  if (exec != nullptr) {
    HIP_TRY(hipGraphLaunch(exec, s->stream));
  } else {
    const int rc = enqueue_batch(s, count, iters);
    if (rc != MB4_OK) return rc;
  }
  const int words = count * s->rec_len;
  HIP_TRY(hipMemcpyAsync(s->h_ring, s->ring, sizeof(unsigned long long) * words,
                         hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  std::vector<int> m(size_t(count), 0);
  int k = 0;
  for (; k < count; ++k) {
    const unsigned long long* hrec = s->h_ring + size_t(k) * s->rec_len;
    const int mk = converged_iteration(s, hrec, iters);
    if (mk <= 0) break;
    m[k] = mk;
    accept(s, hrec, mk);
  }
  *accepted = k;
  if (k > 0) update_prediction(s, *std::max_element(m.begin(), m.begin() + k));
  return prof_collect(s, m);
}

// Slow path: one step with batches of iterations until it converges or
// max_newton is reached (Sec. 2.2: failure is reported, h is not changed).
int step_single(mb4_state* s) {
  const Lattice L = lattice_of(s);
  unsigned long long* rec = s->ring;
  HIP_TRY(mb4::launch_clear(rec, s->rec_len, s->q));
  int done = 0;
  int batch = std::max(1, std::min(s->predicted + 1, s->max_newton));
  for (;;) {
    const int upto = std::min(done + batch, s->max_newton);
    int rc = enqueue_iterations(s, L, 0, rec, done + 1, upto);
    if (rc != MB4_OK) return rc;
    HIP_TRY(hipMemcpyAsync(s->h_ring, rec, sizeof(unsigned long long) * (upto + 1),
                           hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const int m = converged_iteration(s, s->h_ring, upto);
    if (m > 0) {
      accept(s, s->h_ring, m);
      update_prediction(s, m);
      return prof_collect(s, std::vector<int>{m});
    }
    if (m < 0) {
      (void)prof_collect(s, std::vector<int>{0});
      return fail(MB4_ENOCONV, "non-finite Newton update (step %lld)",
                  static_cast<long long>(s->steps_done + 1));
    }
    if (upto >= s->max_newton) {
      (void)prof_collect(s, std::vector<int>{0});
      return fail(MB4_ENOCONV,
                  "no convergence in %d Newton iterations (||r||_inf = %.3e, tol %.3e)",
                  s->max_newton, bits_to_double(s->h_ring[upto]),
                  conv_tol(s, s->h_ring[0]));
    }
    done = upto;
    batch = 2;
  }
}

int check_state(const mb4_state* s) {
  if (s == nullptr) return fail(MB4_EINVAL, "state is NULL");
  return MB4_OK;
}

}  // namespace

int mb4::rt::fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_detail = buf;
  return code;
}

extern "C" {

void mb4_options_default(mb4_options* opt) {
  if (opt == nullptr) return;
  memset(opt, 0, sizeof(*opt));
  opt->eps = kDefaultEps;
  opt->max_newton = kDefaultMaxNewton;
  opt->inner_sweeps = kDefaultSweeps;
  opt->stream = nullptr;
  opt->mem_budget = 0;
}

int mb4_create(const mb4_lattice* lattice, const double* potential,
               const mb4_nonlinearity* nonlinearity, double h, const mb4_options* opt,
               mb4_state** out) {
  if (out == nullptr) return fail(MB4_EINVAL, "out is NULL");
  *out = nullptr;
  if (lattice == nullptr || potential == nullptr || nonlinearity == nullptr)
    return fail(MB4_EINVAL, "lattice, potential and nonlinearity must not be NULL");
  if (lattice->nx < 3 || lattice->ny < 3)
    return fail(MB4_EINVAL, "lattice sides must be >= 3 (got %d x %d)", lattice->nx, lattice->ny);
  const int64_t sites = int64_t(lattice->nx) * int64_t(lattice->ny);
  if (sites > kMaxSites) return fail(MB4_EINVAL, "lattice has more than 2^28 sites");
  if (!isfinite(lattice->t_hop) || !isfinite(lattice->diag_shift))
    return fail(MB4_EINVAL, "t_hop and diag_shift must be finite");
  if (!isfinite(nonlinearity->g)) return fail(MB4_EINVAL, "g must be finite");
  if (!isfinite(h) || h == 0.0) return fail(MB4_EINVAL, "h must be finite and non-zero");
  mb4_options o;
  mb4_options_default(&o);
  if (opt != nullptr) {
    if (!isfinite(opt->eps) || opt->eps < 0.0 || opt->eps >= 1.0)
      return fail(MB4_EINVAL, "eps must be in [0, 1)");
    if (opt->max_newton < 0 || opt->max_newton > mb4::kMaxNewton)
      return fail(MB4_EINVAL, "max_newton must be in [0, %d]", mb4::kMaxNewton);
    if (opt->inner_sweeps < 0 || opt->inner_sweeps > kMaxSweeps)
      return fail(MB4_EINVAL, "inner_sweeps must be in [0, %d]", kMaxSweeps);
    if (opt->eps > 0.0) o.eps = opt->eps;
    if (opt->max_newton > 0) o.max_newton = opt->max_newton;
    if (opt->inner_sweeps > 0) o.inner_sweeps = opt->inner_sweeps;
    o.stream = opt->stream;
    o.mem_budget = opt->mem_budget;
    if ((opt->flags & ~(MB4_FLAG_NO_GRAPHS | MB4_FLAG_RELATIVE_EPS | MB4_FLAG_FP32_SOLVE |
                        MB4_FLAG_SPECTRAL_SOLVE)) != 0)
      return fail(MB4_EINVAL, "unknown bits in flags");
    o.flags = opt->flags;
    if ((o.flags & MB4_FLAG_FP32_SOLVE) != 0 && o.inner_sweeps > mb4::kMaxFusedSweeps)
      return fail(MB4_EINVAL, "FP32 inner solves take at most %d sweeps",
                  mb4::kMaxFusedSweeps);
    if ((o.flags & MB4_FLAG_SPECTRAL_SOLVE) != 0) {
      if ((o.flags & MB4_FLAG_FP32_SOLVE) != 0)
        return fail(MB4_EINVAL, "spectral stage solves are FP64 only");
      if (lattice->nx > mb4::kMaxSpectralSide || lattice->ny > mb4::kMaxSpectralSide)
        return fail(MB4_EINVAL, "spectral stage solves take sides up to %d",
                    mb4::kMaxSpectralSide);
    }
  }
  if (!all_finite(potential, size_t(sites)))
    return fail(MB4_EINVAL, "potential has non-finite entries");
  const bool plain = o.inner_sweeps > mb4::kMaxFusedSweeps || (o.flags & MB4_FLAG_SPECTRAL_SOLVE);
  const size_t need =
      footprint_bytes(size_t(sites), lattice->nx, lattice->ny, o.max_newton, plain);
  if (o.mem_budget != 0 && need > o.mem_budget)
    return fail(MB4_ENOMEM, "state needs %zu bytes, above mem_budget %llu", need,
                static_cast<unsigned long long>(o.mem_budget));

  mb4_state* s = new (std::nothrow) mb4_state();
  if (s == nullptr) return fail(MB4_ENOMEM, "host allocation failed");
  s->nx = lattice->nx;
  s->ny = lattice->ny;
  s->sites = size_t(sites);
  s->t = lattice->t_hop;
  s->shift = lattice->diag_shift;
  s->g = nonlinearity->g;
  s->h = h;
  s->eps = o.eps;
  s->max_newton = o.max_newton;
  s->mem_budget = o.mem_budget;
  s->sweeps = o.inner_sweeps;
  s->stream = static_cast<hipStream_t>(o.stream);
  s->q = s->stream;
  s->use_graphs = (o.flags & MB4_FLAG_NO_GRAPHS) == 0;
  s->relative_eps = (o.flags & MB4_FLAG_RELATIVE_EPS) != 0;
  s->fp32 = (o.flags & MB4_FLAG_FP32_SOLVE) != 0;
  s->spectral = (o.flags & MB4_FLAG_SPECTRAL_SOLVE) != 0;

  int rc = MB4_OK;
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) rc = fail(MB4_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  const size_t field = s->sites * sizeof(double2);
  auto alloc_field = [&](double2** p) {
    if (rc == MB4_OK) rc = dalloc(s, reinterpret_cast<void**>(p), field);
  };
  if (rc == MB4_OK) rc = dalloc(s, reinterpret_cast<void**>(&s->V), s->sites * sizeof(double));
  alloc_field(&s->u0);
  alloc_field(&s->u0b);
  for (int i = 0; i < 3; ++i) {
    alloc_field(&s->Ua[i]);
    alloc_field(&s->Ub[i]);
  }
  if (rc == MB4_OK && plain) rc = ensure_plain_fields(s);
  s->rec_len = s->max_newton + 1;
  const size_t ring_bytes = size_t(kBatch) * s->rec_len * sizeof(unsigned long long);
  if (rc == MB4_OK) rc = dalloc(s, reinterpret_cast<void**>(&s->ring), ring_bytes);
  if (rc == MB4_OK) rc = dalloc(s, reinterpret_cast<void**>(&s->dbg_rec), 2 * sizeof(unsigned long long));
  if (rc == MB4_OK)
    rc = dalloc(s, reinterpret_cast<void**>(&s->partials),
                mb4::energy_partials_count(s->nx, s->ny) * sizeof(double));
  if (rc == MB4_OK) rc = dalloc(s, reinterpret_cast<void**>(&s->eout), 8 * sizeof(double));
  if (rc == MB4_OK && s->spectral) {
    // The preconditioner's constant part: the mean potential plus the shift,
    // and the DFT twiddles e^{-2 pi i m / n} (rounded once from long double).
    std::vector<double> vs(potential, potential + s->sites);
    std::sort(vs.begin(), vs.end(), [](double a, double b) { return fabs(a) < fabs(b); });
    long double sum = 0.0L;
    for (double v : vs) sum += v;
    s->kappa0 = double(sum / (long double)s->sites) + s->shift;
    rc = dalloc(s, reinterpret_cast<void**>(&s->twx), sizeof(double2) * size_t(s->nx));
    if (rc == MB4_OK) rc = dalloc(s, reinterpret_cast<void**>(&s->twy), sizeof(double2) * size_t(s->ny));
    for (int axis = 0; axis < 2 && rc == MB4_OK; ++axis) {
      const int n = axis == 0 ? s->nx : s->ny;
      std::vector<double2> tw(static_cast<size_t>(n));
      const long double pi = 3.141592653589793238462643383279502884L;
      for (int m = 0; m < n; ++m) {
        const long double ang = -2.0L * pi * (long double)m / (long double)n;
        tw[size_t(m)] = make_double2(double(cosl(ang)), double(sinl(ang)));
      }
      e = hipMemcpy(axis == 0 ? s->twx : s->twy, tw.data(), sizeof(double2) * size_t(n),
                    hipMemcpyHostToDevice);
      if (e != hipSuccess) rc = fail(MB4_EDEVICE, "twiddle upload: %s", hipGetErrorString(e));
    }
  }
  if (rc == MB4_OK) rc = halloc(s, reinterpret_cast<void**>(&s->h_ring), ring_bytes);
  if (rc == MB4_OK) rc = halloc(s, reinterpret_cast<void**>(&s->h_dbg), 2 * sizeof(unsigned long long));
  if (rc == MB4_OK) rc = halloc(s, reinterpret_cast<void**>(&s->h_eout), 8 * sizeof(double));
  if (rc == MB4_OK) {
    e = hipMemcpyAsync(s->V, potential, s->sites * sizeof(double), hipMemcpyHostToDevice,
                       s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->u0, 0, field, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->ring, 0, ring_bytes, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) rc = fail(MB4_EDEVICE, "initial upload: %s", hipGetErrorString(e));
  }
  if (rc != MB4_OK) {
    free_all(s);
    delete s;
    return rc;
  }
  *out = s;
  return MB4_OK;
}

void mb4_destroy(mb4_state* state) {
  if (state == nullptr) return;
  (void)hipSetDevice(state->device);
  (void)hipStreamSynchronize(state->stream);
  free_all(state);
  delete state;
}

int mb4_set_state(mb4_state* s, const double* p, const double* q) {
  int rc = check_state(s);
  if (rc != MB4_OK) return rc;
  if (p == nullptr || q == nullptr) return fail(MB4_EINVAL, "p and q must not be NULL");
  if (!all_finite(p, s->sites) || !all_finite(q, s->sites))
    return fail(MB4_EINVAL, "state has non-finite entries");
  if ((rc = use_device(s)) != MB4_OK) return rc;
  std::vector<double> buf(2 * s->sites);
  for (size_t i = 0; i < s->sites; ++i) {
    buf[2 * i] = p[i];
    buf[2 * i + 1] = q[i];
  }
  HIP_TRY(hipMemcpyAsync(s->u0, buf.data(), buf.size() * sizeof(double), hipMemcpyHostToDevice,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->steps_done = 0;
  s->predicted = kInitialPrediction;
  s->lower_batches = 0;
  return MB4_OK;
}

int mb4_get_state(mb4_state* s, double* p, double* q) {
  int rc = check_state(s);
  if (rc != MB4_OK) return rc;
  if (p == nullptr || q == nullptr) return fail(MB4_EINVAL, "p and q must not be NULL");
  if ((rc = use_device(s)) != MB4_OK) return rc;
  std::vector<double> buf(2 * s->sites);
  HIP_TRY(hipMemcpyAsync(buf.data(), s->u0, buf.size() * sizeof(double), hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  for (size_t i = 0; i < s->sites; ++i) {
    p[i] = buf[2 * i];
    q[i] = buf[2 * i + 1];
  }
  return MB4_OK;
}

int mb4_set_state_device(mb4_state* s, const double* d_p, const double* d_q) {
  int rc = check_state(s);
  if (rc != MB4_OK) return rc;
  if (d_p == nullptr || d_q == nullptr) return fail(MB4_EINVAL, "d_p and d_q must not be NULL");
  if ((rc = use_device(s)) != MB4_OK) return rc;
  HIP_TRY(mb4::launch_interleave(d_p, d_q, s->u0, int(s->sites), s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->steps_done = 0;
  s->predicted = kInitialPrediction;
  s->lower_batches = 0;
  return MB4_OK;
}

int mb4_get_state_device(mb4_state* s, double* d_p, double* d_q) {
  int rc = check_state(s);
  if (rc != MB4_OK) return rc;
  if (d_p == nullptr || d_q == nullptr) return fail(MB4_EINVAL, "d_p and d_q must not be NULL");
  if ((rc = use_device(s)) != MB4_OK) return rc;
  HIP_TRY(mb4::launch_deinterleave(s->u0, d_p, d_q, int(s->sites), s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return MB4_OK;
}

int mb4_step(mb4_state* s, int64_t nsteps) {
  int rc = check_state(s);
  if (rc != MB4_OK) return rc;
  if (nsteps < 0) return fail(MB4_EINVAL, "nsteps must be >= 0");
  if ((rc = use_device(s)) != MB4_OK) return rc;
  int64_t left = nsteps;
  while (left > 0) {
    const int count = int(std::min<int64_t>(left, kBatch));
    const int iters = std::max(1, std::min(s->predicted, s->max_newton));
    int accepted = 0;
    rc = run_batch(s, count, iters, &accepted);
    if (rc != MB4_OK) return rc;
    left -= accepted;
    if (accepted < count) {
      rc = step_single(s);
      if (rc != MB4_OK) return rc;
      --left;
    }
  }
  return MB4_OK;
}

int mb4_energy_components(mb4_state* s, double out[6]) {
  int rc = check_state(s);
  if (rc != MB4_OK) return rc;
  if (out == nullptr) return fail(MB4_EINVAL, "out must not be NULL");
  if ((rc = use_device(s)) != MB4_OK) return rc;
  HIP_TRY(mb4::launch_energy(lattice_of(s), s->partials, s->eout, s->stream));
  HIP_TRY(hipMemcpyAsync(s->h_eout, s->eout, 6 * sizeof(double), hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  for (int k = 0; k < 6; ++k) out[k] = s->h_eout[k];
  return MB4_OK;
}

int mb4_energy(mb4_state* s, double* H) {
  if (H == nullptr) return fail(MB4_EINVAL, "H must not be NULL");
  double comp[6];
  const int rc = mb4_energy_components(s, comp);
  if (rc == MB4_OK) *H = comp[0];
  return rc;
}

int mb4_set_nonlinearity_sites(mb4_state* s, const double* g) {
  int rc = check_state(s);
  if (rc != MB4_OK) return rc;
  if (g == nullptr) {
    if (s->gs_on) drop_graphs(s);
    s->gs_on = false;
    return MB4_OK;
  }
  if (!all_finite(g, s->sites)) return fail(MB4_EINVAL, "every g_j must be finite");
  rc = use_device(s);
  if (rc != MB4_OK) return rc;
  if (s->gs == nullptr) {
    if (s->mem_budget != 0 && state_bytes(s, s->phib[0] != nullptr, true) > s->mem_budget)
      return fail(MB4_ENOMEM, "a per-site nonlinearity needs 8 bytes per site more, above "
                  "mem_budget %llu", static_cast<unsigned long long>(s->mem_budget));
    rc = dalloc(s, reinterpret_cast<void**>(&s->gs), s->sites * sizeof(double));
    if (rc != MB4_OK) return rc;
  }
  HIP_TRY(hipMemcpyAsync(s->gs, g, s->sites * sizeof(double), hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  // Captured batches hold the lattice, and with it whether g_j is read.
  drop_graphs(s);
  s->gs_on = true;
  return MB4_OK;
}

int mb4_set_h(mb4_state* s, double h) {
  int rc = check_state(s);
  if (rc != MB4_OK) return rc;
  if (!isfinite(h) || h == 0.0) return fail(MB4_EINVAL, "h must be finite and non-zero");
  if (h != s->h) drop_graphs(s);
  s->h = h;
  return MB4_OK;
}

int mb4_set_region(mb4_state* s, int32_t region) {
  const int rc = check_state(s);
  if (rc != MB4_OK) return rc;
  if (region < 0 || region >= MB4_REGION_COUNT)
    return fail(MB4_EINVAL, "region must be in [0, %d)", MB4_REGION_COUNT);
  if (s->fp32 && region != MB4_REGION_32x32)
    return fail(MB4_EINVAL, "FP32 inner solves are built for MB4_REGION_32x32 only");
  if (region != s->region) drop_graphs(s);
  s->region = region;
  return MB4_OK;
}

int32_t mb4_region(const mb4_state* s) { return s == nullptr ? -1 : s->region; }

int mb4_set_sweeps(mb4_state* s, int32_t sweeps) {
  const int rc = check_state(s);
  if (rc != MB4_OK) return rc;
  if (sweeps < 1 || sweeps > kMaxSweeps)
    return fail(MB4_EINVAL, "sweeps must be in [1, %d]", kMaxSweeps);
  if (s->fp32 && sweeps > mb4::kMaxFusedSweeps)
    return fail(MB4_EINVAL, "FP32 inner solves take at most %d sweeps", mb4::kMaxFusedSweeps);
  if (sweeps > mb4::kMaxFusedSweeps) {
    int prc = use_device(s);
    if (prc == MB4_OK) prc = ensure_plain_fields(s);
    if (prc != MB4_OK) return prc;
  }
  if (sweeps != s->sweeps) drop_graphs(s);
  s->sweeps = sweeps;
  return MB4_OK;
}

int32_t mb4_sweeps(const mb4_state* s) { return s == nullptr ? -1 : s->sweeps; }

int mb4_tune(mb4_state* s, int32_t steps, int32_t* best_region, int32_t* best_sweeps,
             double* ms_per_step) {
  int rc = check_state(s);
  if (rc != MB4_OK) return rc;
  if (steps < 1 || steps > 1024) return fail(MB4_EINVAL, "steps must be in [1, 1024]");
  if (s->spectral)
    return fail(MB4_EINVAL,
                "mb4_tune covers block-Jacobi sweeps; set the Richardson count with "
                "mb4_set_sweeps");
  if ((rc = use_device(s)) != MB4_OK) return rc;
  void* backup = nullptr;
  hipError_t err = hipMalloc(&backup, s->sites * sizeof(double2));
  if (err != hipSuccess) return fail(MB4_ENOMEM, "tune backup: %s", hipGetErrorString(err));
  // Everything a trial changes: u_0 (device) and the step counters.
  const int region0 = s->region, sweeps0 = s->sweeps;
  const int64_t done0 = s->steps_done;
  const int iters0 = s->last_iters, lsw0 = s->last_sweeps;
  const double rn0 = s->last_rnorm;
  const std::vector<double> res0 = s->last_res;
  const int pred0 = s->predicted, lower0 = s->lower_batches;
  // Trials are not part of the run: they stay out of the kernel profile.
  const bool prof0 = s->prof_on;
  s->prof_on = false;
  auto restore = [&]() -> int {
    s->steps_done = done0;
    s->last_iters = iters0;
    s->last_sweeps = lsw0;
    s->last_rnorm = rn0;
    s->last_res = res0;
    HIP_TRY(hipMemcpyAsync(s->u0, backup, s->sites * sizeof(double2), hipMemcpyDeviceToDevice,
                           s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return MB4_OK;
  };
  if (ms_per_step != nullptr)
    for (int k = 0; k < 4 * MB4_REGION_COUNT; ++k) ms_per_step[k] = -1.0;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if ((err = hipMemcpyAsync(backup, s->u0, s->sites * sizeof(double2), hipMemcpyDeviceToDevice,
                            s->stream)) != hipSuccess ||
      (err = hipEventCreate(&t0)) != hipSuccess || (err = hipEventCreate(&t1)) != hipSuccess)
    rc = fail(MB4_EDEVICE, "tune set-up: %s", hipGetErrorString(err));
  int best_r = region0, best_s = sweeps0, pred_best = pred0;
  double best_ms = -1.0;
  for (int sw = 2; sw <= mb4::kMaxFusedSweeps && rc == MB4_OK; ++sw) {
    for (int reg = 0; reg < MB4_REGION_COUNT && rc == MB4_OK; ++reg) {
      if (mb4_set_region(s, reg) != MB4_OK || mb4_set_sweeps(s, sw) != MB4_OK) continue;
      s->predicted = pred0;
      s->lower_batches = lower0;
      // One untimed pass (graph capture, caches, the iteration prediction),
      // then the timed one.  A pair under which a step does not converge is
      // skipped.
      int trc = mb4_step(s, steps);
      if (trc == MB4_OK) trc = restore();
      if (trc == MB4_OK && (err = hipEventRecord(t0, s->stream)) != hipSuccess)
        trc = fail(MB4_EDEVICE, "tune event: %s", hipGetErrorString(err));
      if (trc == MB4_OK) trc = mb4_step(s, steps);
      if (trc == MB4_OK && (err = hipEventRecord(t1, s->stream)) != hipSuccess)
        trc = fail(MB4_EDEVICE, "tune event: %s", hipGetErrorString(err));
      if (trc == MB4_OK && (err = hipEventSynchronize(t1)) != hipSuccess)
        trc = fail(MB4_EDEVICE, "tune event: %s", hipGetErrorString(err));
      float ms = 0.0f;
      if (trc == MB4_OK && (err = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess)
        trc = fail(MB4_EDEVICE, "tune event: %s", hipGetErrorString(err));
      const int pred = s->predicted;
      if (trc != MB4_OK && trc != MB4_ENOCONV) {
        rc = trc;
        break;
      }
      if ((rc = restore()) != MB4_OK) break;
      if (trc != MB4_OK) continue;
      const double t = double(ms) / steps;
      if (ms_per_step != nullptr) ms_per_step[(sw - 1) * MB4_REGION_COUNT + reg] = t;
      if (best_ms < 0.0 || t < best_ms) {
        best_ms = t;
        best_r = reg;
        best_s = sw;
        pred_best = pred;
      }
    }
  }
  if (rc != MB4_OK) {
    (void)restore();
    best_r = region0;
    best_s = sweeps0;
    pred_best = pred0;
  }
  (void)mb4_set_region(s, best_r);
  (void)mb4_set_sweeps(s, best_s);
  s->predicted = pred_best;
  s->lower_batches = 0;
  s->prof_on = prof0;
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  (void)hipFree(backup);
  if (rc != MB4_OK) return rc;
  if (best_region) *best_region = best_r;
  if (best_sweeps) *best_sweeps = best_s;
  return MB4_OK;
}

int64_t mb4_steps_done(const mb4_state* s) { return s == nullptr ? -1 : s->steps_done; }

int mb4_last_stats(const mb4_state* s, int32_t* newton_iters, int32_t* inner_sweeps,
                   double* last_rnorm) {
  int rc = check_state(s);
  if (rc != MB4_OK) return rc;
  if (newton_iters) *newton_iters = s->last_iters;
  if (inner_sweeps) *inner_sweeps = s->last_sweeps;
  if (last_rnorm) *last_rnorm = s->last_rnorm;
  return MB4_OK;
}

int mb4_last_residuals(const mb4_state* s, double* out, int32_t n, int32_t* count) {
  int rc = check_state(s);
  if (rc != MB4_OK) return rc;
  if (n < 0 || (n > 0 && out == nullptr)) return fail(MB4_EINVAL, "bad output buffer");
  const int m = std::min(n, int(s->last_res.size()));
  for (int l = 0; l < m; ++l) out[l] = s->last_res[size_t(l)];
  if (count) *count = m;
  return MB4_OK;
}

int mb4_profile_enable(mb4_state* s, int32_t enable) {
  int rc = check_state(s);
  if (rc != MB4_OK) return rc;
  s->prof_on = enable != 0;
  s->prof_pending.clear();
  s->ev_used = 0;
  for (int k = 0; k < kKernelClasses; ++k) {
    s->prof_launches[k] = 0;
    s->prof_ms[k] = 0.0;
  }
  return MB4_OK;
}

int32_t mb4_profile_classes(void) { return kKernelClasses; }

const char* mb4_profile_name(int32_t cls) {
  return (cls >= 0 && cls < kKernelClasses) ? kKernelNames[cls] : "";
}

int mb4_profile_read(const mb4_state* s, int32_t cls, int64_t* launches, double* total_ms) {
  int rc = check_state(s);
  if (rc != MB4_OK) return rc;
  if (cls < 0 || cls >= kKernelClasses) return fail(MB4_EINVAL, "no kernel class %d", cls);
  if (launches) *launches = s->prof_launches[cls];
  if (total_ms) *total_ms = s->prof_ms[cls];
  return MB4_OK;
}

int mb4_newton_update(mb4_state* s, double* d_U, const double* d_rbar, double* d_phibar,
                      double* rnorm) {
  int rc = check_state(s);
  if (rc != MB4_OK) return rc;
  if (d_U == nullptr || d_phibar == nullptr)
    return fail(MB4_EINVAL, "d_U and d_phibar must not be NULL");
  if ((rc = use_device(s)) != MB4_OK) return rc;
  const bool has_r = d_rbar != nullptr;
  const CPlanes3 uin = cplanes_of(d_U, s->sites);
  const CPlanes3 rin = has_r ? cplanes_of(d_rbar, s->sites) : CPlanes3{{nullptr, nullptr, nullptr}};
  const ConvCheck none{nullptr, 0, 0.0, false};
  HIP_TRY(mb4::launch_clear(s->dbg_rec, 2, s->stream));
  HIP_TRY(mb4::launch_update_residual(lattice_of(s), uin, P(s->Ua), rin, has_r, false,
                                      planes_of(d_phibar, s->sites), s->dbg_rec + 1, none, none,
                                      nullptr, s->stream));
  if (has_r) {
    // The pass cannot update U in place (other blocks read its halo), so the
    // result goes through the state's stage buffer.
    const Planes3 uout = planes_of(d_U, s->sites);
    for (int i = 0; i < 3; ++i)
      HIP_TRY(hipMemcpyAsync(uout.s[i], s->Ua[i], s->sites * sizeof(double2),
                             hipMemcpyDeviceToDevice, s->stream));
  }
  HIP_TRY(hipMemcpyAsync(s->h_dbg, s->dbg_rec, 2 * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (rnorm) *rnorm = bits_to_double(s->h_dbg[1]);
  return MB4_OK;
}

int mb4_stage_solve(mb4_state* s, const double* d_phibar, double* d_rbar, int32_t sweeps) {
  int rc = check_state(s);
  if (rc != MB4_OK) return rc;
  if (d_phibar == nullptr || d_rbar == nullptr)
    return fail(MB4_EINVAL, "d_phibar and d_rbar must not be NULL");
  if (sweeps < 1 || sweeps > kMaxSweeps)
    return fail(MB4_EINVAL, "sweeps must be in [1, %d]", kMaxSweeps);
  if ((rc = use_device(s)) != MB4_OK) return rc;
  if (sweeps > mb4::kMaxFusedSweeps && (rc = ensure_plain_fields(s)) != MB4_OK) return rc;
  const Lattice L = lattice_of(s);
  const CPlanes3 ph = cplanes_of(d_phibar, s->sites);
  const Planes3 ext = planes_of(d_rbar, s->sites);
  const ConvCheck none{nullptr, 0, 0.0, false};
  const int fused = std::min(int(sweeps), mb4::kMaxFusedSweeps);
  // Same kernels as a Newton iteration; the last pass writes the caller's
  // planes.
  Planes3 prev = (fused == sweeps) ? ext : P(s->ra);
  HIP_TRY(mb4::launch_stage_solve(L, ph, prev, fused, nullptr, none, s->stream));
  for (int k = fused; k < sweeps; ++k) {
    const Planes3 out =
        (k == sweeps - 1) ? ext : ((prev.s[0] == s->ra[0]) ? P(s->rb) : P(s->ra));
    const CPlanes3 in{{prev.s[0], prev.s[1], prev.s[2]}};
    HIP_TRY(mb4::launch_stage_sweep(L, ph, in, out, nullptr, none, s->stream));
    prev = out;
  }
  HIP_TRY(hipStreamSynchronize(s->stream));
  return MB4_OK;
}

const char* mb4_strerror(int code) {
  switch (code) {
    case MB4_OK:
      return "success";
    case MB4_EINVAL:
      return "invalid argument";
    case MB4_ENOMEM:
      return "out of memory or above the memory budget";
    case MB4_EDEVICE:
      return "HIP runtime error";
    case MB4_ENOCONV:
      return "simplified Newton iteration did not converge";
    default:
      return "unknown status code";
  }
}

const char* mb4_error_detail(void) { return g_detail.c_str(); }

}  // extern "C"
