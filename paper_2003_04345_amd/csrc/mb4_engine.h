// Internal engine of the multi-lattice front ends (mb4_ensemble_*,
// mb4_server_*): a set of member lattices at site offsets of capacity-sized
// device fields, advanced together batch by batch with one launch per Newton
// phase (see mb4_engine.hip).  Not part of the public ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "mb4_internal.h"

namespace mb4 {
namespace engine {

struct Config {
  double eps;
  bool relative_eps;
  int max_newton;
  int sweeps;            // 1 .. kMaxFusedSweeps
  bool fp32;             // FP32 inner stage solves
  bool graphs;           // replay batches from captured graphs
  hipStream_t stream;
  size_t capacity;       // sites of every field
  int max_members;
};

struct Engine;

// Bytes of device memory per site of capacity: V, two u_0 buffers and two
// Newton-iterate fields (X^l, three stages each).
size_t bytes_per_site();

int create(const Config& cfg, Engine** out);
void destroy(Engine* e);

// Replaces the member set; each member's sites [base, base + nx*ny) must lie
// inside the capacity and not overlap another member's.  Per-member
// statistics restart.
int set_members(Engine* e, const std::vector<MemberDesc>& members);
int member_count(const Engine* e);

// V and psi = p + i q of the sites [base, base + n) from host arrays (copied).
int upload(Engine* e, long long base, size_t n, const double* V, const double* p,
           const double* q);
// psi of the sites [base, base + n) to host arrays.
int download(Engine* e, long long base, size_t n, double* p, double* q);

// One batch: member m takes min(remaining[m], max_steps) steps (max_steps
// <= 32).  remaining[m] drops by the steps member m accepted and
// last_iters[m] receives the Newton iterations of its last accepted step.
// A member whose step fails for good (a non-finite update, or no convergence
// in max_newton iterations) is listed in hard_failed and keeps its last
// accepted step; a member that needs more iterations than the batch was built
// for is retried in the next batch with more.
int run_batch(Engine* e, std::vector<int64_t>& remaining, std::vector<int>& last_iters,
              std::vector<int>& hard_failed, int max_steps, std::vector<char>* nonfinite = nullptr);

// Energy components of every member, out[6 m + k].
int energy(Engine* e, double* out);
// Energy components of one lattice at sites [base, ...) (any member or not).
int energy_of(Engine* e, const MemberDesc& d, double out[6]);

// One persistent launch per batch (launch_member_run) instead of one launch
// per Newton phase; the results are the same bit for bit.  Refused when the
// current region and sweeps have no persistent build.
int set_persistent(Engine* e, bool on);
bool persistent(const Engine* e);

int set_region(Engine* e, int region);
int region(const Engine* e);
bool region_usable(const Engine* e, int region);
// Block-Jacobi sweeps per stage solve (1 .. kMaxFusedSweeps); the current
// region must leave a tile at the new count.
int set_sweeps(Engine* e, int sweeps);
int sweeps(const Engine* e);

// u_0 of the whole capacity to / from a device buffer (autotuning trials).
int save_u0(Engine* e, void* dst);
int restore_u0(Engine* e, const void* src);
size_t u0_bytes(const Engine* e);
hipStream_t stream(const Engine* e);
int iteration_prediction(const Engine* e);
void set_iteration_prediction(Engine* e, int predicted);

}  // namespace engine
}  // namespace mb4
