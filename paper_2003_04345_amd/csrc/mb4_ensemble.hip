// C ABI of MB4 ensembles (see include/mb4.h): a fixed set of independent
// lattice problems stored one after the other and advanced together by the
// multi-lattice engine (mb4_engine.hip), each member with its own Newton loop
// (Algorithm 1 of Sakai et al., arXiv 2003.04345).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "mb4.h"
#include "mb4_engine.h"

using mb4::MemberDesc;
using mb4::rt::fail;
namespace eng = mb4::engine;

namespace {

constexpr int kMaxMembers = 65536;
constexpr int64_t kMaxSites = int64_t(1) << 28;
constexpr int kBatch = 32;

bool all_finite(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(v[i])) return false;
  return true;
}

}  // namespace

struct mb4_ensemble {
  eng::Engine* engine = nullptr;
  std::vector<MemberDesc> desc;
  size_t total = 0;
  std::vector<int64_t> steps_done;
  std::vector<int> last_iters;
};

namespace {

int check(const mb4_ensemble* e) {
  if (e == nullptr) return fail(MB4_EINVAL, "ensemble is NULL");
  return MB4_OK;
}

int check_member(const mb4_ensemble* e, int32_t m) {
  const int rc = check(e);
  if (rc != MB4_OK) return rc;
  if (m < 0 || m >= int(e->desc.size())) return fail(MB4_EINVAL, "member %d out of range", m);
  return MB4_OK;
}

// Device bytes of an ensemble (see mb4.h).
size_t footprint_bytes(size_t total, int count, int max_newton) {
  return total * eng::bytes_per_site() + size_t(kBatch) * count * (max_newton + 1) * 8 +
         size_t(count) * 120 + total / 256 * 12 * sizeof(double);
}

// A launch configuration the autotuner tries.
struct Shape {
  int region = mb4::kRegion32x32;
  int sweeps = 3;
  bool persistent = false;  // one launch per batch (mb4_ensemble_set_persistent)
};

// Times `steps` steps of the ensemble under each shape (one untimed pass
// first: graph capture, caches, the iteration prediction), restoring every
// member's state and counters after each trial.  times[k] receives ms per
// step of shapes[k], or -1 where the shape leaves no tile, is not built
// (FP32 solves: 32 x 32 only) or has fewer than min_sweeps sweeps.  The
// fastest shape is selected, with the iteration prediction its trial
// learnt; on an error the original shape and prediction come back.
int tune_shapes(mb4_ensemble* e, int32_t steps, const std::vector<Shape>& shapes,
                std::vector<double>* times, Shape* chosen, int min_sweeps = 1) {
  eng::Engine* g = e->engine;
  const hipStream_t s = eng::stream(g);
  void* backup = nullptr;
  hipError_t err = hipMalloc(&backup, eng::u0_bytes(g));
  if (err != hipSuccess) return fail(MB4_ENOMEM, "tune backup: %s", hipGetErrorString(err));
  const std::vector<int64_t> done0 = e->steps_done;
  const std::vector<int> iters0 = e->last_iters;
  const Shape shape0{eng::region(g), eng::sweeps(g), eng::persistent(g)};
  const int pred0 = eng::iteration_prediction(g);
  hipEvent_t t0 = nullptr, t1 = nullptr;
  times->assign(shapes.size(), -1.0);
  *chosen = shape0;
  int pred_best = pred0;
  double best_ms = -1.0;
  auto restore = [&]() {
    e->steps_done = done0;
    e->last_iters = iters0;
    return eng::restore_u0(g, backup);
  };
  auto select = [&](const Shape& sh) {
    // Sweeps first when they shrink (the tile grows), region first otherwise.
    int rc = MB4_OK;
    if (sh.sweeps < eng::sweeps(g)) {
      rc = eng::set_sweeps(g, sh.sweeps);
      if (rc == MB4_OK) rc = eng::set_region(g, sh.region);
    } else {
      rc = eng::set_region(g, sh.region);
      if (rc == MB4_OK) rc = eng::set_sweeps(g, sh.sweeps);
    }
    if (rc == MB4_OK) rc = eng::set_persistent(g, sh.persistent);
    return rc;
  };
  int rc = eng::save_u0(g, backup);
  if (rc == MB4_OK && ((err = hipEventCreate(&t0)) != hipSuccess ||
                       (err = hipEventCreate(&t1)) != hipSuccess))
    rc = fail(MB4_EDEVICE, "tune events: %s", hipGetErrorString(err));
  for (size_t k = 0; k < shapes.size() && rc == MB4_OK; ++k) {
    const Shape& sh = shapes[k];
    if (sh.sweeps < min_sweeps) continue;
    // Usable: the region exists in this precision and leaves a tile at these
    // sweeps (checked by selecting it; a refusal only skips the shape).
    if (select(sh) != MB4_OK) {
      rc = select(shape0);
      continue;
    }
    eng::set_iteration_prediction(g, pred0);
    // One untimed pass (graph capture, caches), then the timed one.
    rc = mb4_ensemble_step(e, std::min<int64_t>(steps, kBatch));
    if (rc == MB4_OK) rc = restore();
    if (rc == MB4_OK && (err = hipEventRecord(t0, s)) != hipSuccess)
      rc = fail(MB4_EDEVICE, "tune event: %s", hipGetErrorString(err));
    if (rc == MB4_OK) rc = mb4_ensemble_step(e, steps);
    if (rc == MB4_OK && (err = hipEventRecord(t1, s)) != hipSuccess)
      rc = fail(MB4_EDEVICE, "tune event: %s", hipGetErrorString(err));
    if (rc == MB4_OK && (err = hipEventSynchronize(t1)) != hipSuccess)
      rc = fail(MB4_EDEVICE, "tune event: %s", hipGetErrorString(err));
    float ms = 0.0f;
    if (rc == MB4_OK && (err = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess)
      rc = fail(MB4_EDEVICE, "tune event: %s", hipGetErrorString(err));
    const int pred = eng::iteration_prediction(g);
    if (rc == MB4_OK) rc = restore();
    if (rc == MB4_OK) {
      (*times)[k] = double(ms) / steps;
      if (best_ms < 0.0 || (*times)[k] < best_ms) {
        best_ms = (*times)[k];
        *chosen = sh;
        pred_best = pred;
      }
    }
  }
  const int rc_sel = select(rc == MB4_OK ? *chosen : shape0);
  if (rc != MB4_OK) (void)restore();
  eng::set_iteration_prediction(g, rc == MB4_OK ? pred_best : pred0);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  (void)hipFree(backup);
  if (rc != MB4_OK) return rc;
  return rc_sel;
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
    if ((opt->flags & MB4_FLAG_SPECTRAL_SOLVE) != 0)
      return fail(MB4_EINVAL, "spectral stage solves are for single states (mb4_create)");
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
  if (size_t(kBatch) * size_t(count) * size_t(o.max_newton + 1) > size_t(INT32_MAX))
    return fail(MB4_EINVAL, "count * (max_newton + 1) too large for the step records");
  const bool fp32 = (o.flags & MB4_FLAG_FP32_SOLVE) != 0;
  const size_t need = footprint_bytes(total, count, o.max_newton);
  if (o.mem_budget != 0 && need > o.mem_budget)
    return fail(MB4_ENOMEM, "ensemble needs %zu bytes, above mem_budget %llu", need,
                static_cast<unsigned long long>(o.mem_budget));

  mb4_ensemble* e = new (std::nothrow) mb4_ensemble();
  if (e == nullptr) return fail(MB4_ENOMEM, "host allocation failed");
  eng::Config cfg{o.eps,
                  (o.flags & MB4_FLAG_RELATIVE_EPS) != 0,
                  o.max_newton,
                  o.inner_sweeps,
                  fp32,
                  (o.flags & MB4_FLAG_NO_GRAPHS) == 0,
                  static_cast<hipStream_t>(o.stream),
                  total,
                  count};
  int rc = eng::create(cfg, &e->engine);
  if (rc == MB4_OK) rc = eng::set_members(e->engine, desc);
  if (rc == MB4_OK) {
    std::vector<double> zero;
    for (int m = 0; m < count && rc == MB4_OK; ++m) {
      const size_t n = size_t(desc[m].nx) * desc[m].ny;
      zero.assign(n, 0.0);
      rc = eng::upload(e->engine, desc[m].base, n, potentials[m], zero.data(), zero.data());
    }
  }
  if (rc != MB4_OK) {
    eng::destroy(e->engine);
    delete e;
    return rc;
  }
  e->desc = std::move(desc);
  e->total = total;
  e->steps_done.assign(size_t(count), 0);
  e->last_iters.assign(size_t(count), 0);
  *out = e;
  return MB4_OK;
}

void mb4_ensemble_destroy(mb4_ensemble* e) {
  if (e == nullptr) return;
  eng::destroy(e->engine);
  delete e;
}

int32_t mb4_ensemble_size(const mb4_ensemble* e) {
  return e == nullptr ? -1 : int32_t(e->desc.size());
}

int mb4_ensemble_set_state(mb4_ensemble* e, int32_t m, const double* p, const double* q) {
  int rc = check_member(e, m);
  if (rc != MB4_OK) return rc;
  if (p == nullptr || q == nullptr) return fail(MB4_EINVAL, "p and q must not be NULL");
  const MemberDesc& d = e->desc[m];
  const size_t n = size_t(d.nx) * d.ny;
  if (!all_finite(p, n) || !all_finite(q, n))
    return fail(MB4_EINVAL, "state has non-finite entries");
  rc = eng::upload(e->engine, d.base, n, nullptr, p, q);
  if (rc != MB4_OK) return rc;
  e->steps_done[m] = 0;
  e->last_iters[m] = 0;
  return MB4_OK;
}

int mb4_ensemble_get_state(mb4_ensemble* e, int32_t m, double* p, double* q) {
  const int rc = check_member(e, m);
  if (rc != MB4_OK) return rc;
  if (p == nullptr || q == nullptr) return fail(MB4_EINVAL, "p and q must not be NULL");
  const MemberDesc& d = e->desc[m];
  return eng::download(e->engine, d.base, size_t(d.nx) * d.ny, p, q);
}

int mb4_ensemble_step(mb4_ensemble* e, int64_t nsteps) {
  int rc = check(e);
  if (rc != MB4_OK) return rc;
  if (nsteps < 0) return fail(MB4_EINVAL, "nsteps must be >= 0");
  const size_t n = e->desc.size();
  std::vector<int64_t> remaining(n, nsteps);
  std::vector<int> failed;
  std::vector<char> nonfinite;
  for (;;) {
    bool left = false;
    for (int64_t r : remaining) left = left || r > 0;
    if (!left) return MB4_OK;
    const std::vector<int64_t> before = remaining;
    rc = eng::run_batch(e->engine, remaining, e->last_iters, failed, kBatch, &nonfinite);
    if (rc != MB4_OK) return rc;
    for (size_t m = 0; m < n; ++m) e->steps_done[m] += before[m] - remaining[m];
    if (!failed.empty()) {
      const int m = failed.front();
      return nonfinite[m]
                 ? fail(MB4_ENOCONV, "member %d: non-finite Newton update (step %lld)", m,
                        static_cast<long long>(e->steps_done[m] + 1))
                 : fail(MB4_ENOCONV,
                        "member %d: no convergence in the allowed Newton iterations (step %lld)",
                        m, static_cast<long long>(e->steps_done[m] + 1));
    }
  }
}

int mb4_ensemble_energy_components(mb4_ensemble* e, double* out) {
  const int rc = check(e);
  if (rc != MB4_OK) return rc;
  if (out == nullptr) return fail(MB4_EINVAL, "out is NULL");
  return eng::energy(e->engine, out);
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
  const int rc = check(e);
  if (rc != MB4_OK) return rc;
  return eng::set_region(e->engine, region);
}

int32_t mb4_ensemble_region(const mb4_ensemble* e) {
  return e == nullptr ? -1 : eng::region(e->engine);
}

int mb4_ensemble_set_sweeps(mb4_ensemble* e, int32_t sweeps) {
  const int rc = check(e);
  if (rc != MB4_OK) return rc;
  return eng::set_sweeps(e->engine, sweeps);
}

int32_t mb4_ensemble_sweeps(const mb4_ensemble* e) {
  return e == nullptr ? -1 : eng::sweeps(e->engine);
}

int mb4_ensemble_tune(mb4_ensemble* e, int32_t steps, int32_t* best, double* ms_per_step) {
  int rc = check(e);
  if (rc != MB4_OK) return rc;
  if (steps < 1) return fail(MB4_EINVAL, "steps must be >= 1");
  const int sw = eng::sweeps(e->engine);
  const bool pe = eng::persistent(e->engine);
  std::vector<Shape> shapes;
  for (int r = 0; r < mb4::kRegionCount; ++r) shapes.push_back(Shape{r, sw, pe});
  std::vector<double> times;
  Shape chosen{};
  rc = tune_shapes(e, steps, shapes, &times, &chosen);
  if (rc != MB4_OK) return rc;
  if (best) *best = chosen.region;
  if (ms_per_step)
    for (int r = 0; r < mb4::kRegionCount; ++r) ms_per_step[r] = times[size_t(r)];
  return MB4_OK;
}

int mb4_ensemble_tune_all(mb4_ensemble* e, int32_t steps, int32_t* best_region,
                          int32_t* best_sweeps, double* ms_per_step) {
  int rc = check(e);
  if (rc != MB4_OK) return rc;
  if (steps < 1) return fail(MB4_EINVAL, "steps must be >= 1");
  const bool pe = eng::persistent(e->engine);
  std::vector<Shape> shapes;
  for (int sw = 1; sw <= mb4::kMaxFusedSweeps; ++sw)
    for (int r = 0; r < mb4::kRegionCount; ++r) shapes.push_back(Shape{r, sw, pe});
  std::vector<double> times;
  Shape chosen{};
  rc = tune_shapes(e, steps, shapes, &times, &chosen, /*min_sweeps=*/2);
  if (rc != MB4_OK) return rc;
  if (best_region) *best_region = chosen.region;
  if (best_sweeps) *best_sweeps = chosen.sweeps;
  if (ms_per_step)
    for (size_t k = 0; k < times.size(); ++k) ms_per_step[k] = times[k];
  return MB4_OK;
}

int mb4_ensemble_set_persistent(mb4_ensemble* e, int32_t on) {
  const int rc = check(e);
  if (rc != MB4_OK) return rc;
  return eng::set_persistent(e->engine, on != 0);
}

int32_t mb4_ensemble_persistent(const mb4_ensemble* e) {
  return e == nullptr ? -1 : (eng::persistent(e->engine) ? 1 : 0);
}

int mb4_ensemble_tune_launch(mb4_ensemble* e, int32_t steps, int32_t* persistent,
                             double* ms_per_step) {
  int rc = check(e);
  if (rc != MB4_OK) return rc;
  if (steps < 1) return fail(MB4_EINVAL, "steps must be >= 1");
  const int r = eng::region(e->engine), sw = eng::sweeps(e->engine);
  const std::vector<Shape> shapes{Shape{r, sw, false}, Shape{r, sw, true}};
  std::vector<double> times;
  Shape chosen{};
  rc = tune_shapes(e, steps, shapes, &times, &chosen);
  if (rc != MB4_OK) return rc;
  if (persistent) *persistent = chosen.persistent ? 1 : 0;
  if (ms_per_step)
    for (size_t k = 0; k < times.size(); ++k) ms_per_step[k] = times[k];
  return MB4_OK;
}

}  // extern "C"
