// Internal interface between the MB4 runtime (mb4_runtime.hip) and its HIP
// kernels (mb4_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mb4 {

// Largest Newton iteration count a state may request.
constexpr int kMaxNewton = 1000;

// Statistics of one step live in a record of unsigned 64-bit words:
// rec[0] = ||u_0||_inf, rec[l] = ||r^l||_inf for Newton iteration l >= 1.
// Non-negative doubles are stored as their IEEE bit patterns, so that an
// unsigned atomicMax is an exact, order-independent maximum (and a NaN, whose
// patterns sort above +inf, survives it).

// The lattice problem as the kernels see it: periodic nx x ny, hopping -t on
// the four links, on-site A_jj = V_j + shift, nonlinearity g (or g_j per
// site), time step h.
struct Lattice {
  int nx, ny;
  double t, shift, g, h;
  const double* V;     // [nx*ny]
  const double2* u0;   // [nx*ny] (p, q)
  const double* gs = nullptr;  // [nx*ny] g_j per site, or NULL: g at every site
};

// Three planes of a stage field (element type double2, or float2 for the
// stage corrections of the FP32 inner solves).
template <class T2>
struct PlanesOf {
  T2* s[3];
};

template <class T2>
struct CPlanesOf {
  const T2* s[3];
};

using Planes3 = PlanesOf<double2>;
using CPlanes3 = CPlanesOf<double2>;

// Convergence test of Newton iteration `prev`:
// ||r^prev||_inf <= eps * max(||u_0||_inf, DBL_MIN).  Kernels of iteration l
// return at once when iteration l-1 passed it; the update pass of iteration l
// turns into the final update when iteration l passed it.
struct ConvCheck {
  const unsigned long long* rec;  // step record; NULL: the test is false
  int prev;                       // iteration whose norm decides
  double eps;                     // ||r^prev||_inf <= eps (Algorithm 1) ...
  bool relative;                  // ... or <= eps * ||u_0||_inf (rec[0])
};

// Several independent lattices ("members") advanced by the same launches.
// Member m's sites are [base, base + nx*ny) of ensemble-wide fields, whose
// planes are all members' sites long; its step record starts rec_stride words
// after member m-1's.  A block finds its member in member_of (one load), or
// by binary search in block0 when there is no such table.
struct MemberDesc {
  int nx, ny;
  double t, shift, g, h;
  long long base;
};

struct Multi {
  const MemberDesc* desc = nullptr;  // device [count]; NULL: the Lattice argument alone
  const int* block0 = nullptr;       // device [count + 1]: first block of each member
  const int* member_of = nullptr;    // device [blocks]: member of each block (or NULL)
  int count = 0;
  int blocks = 0;                    // blocks of the launch (block0[count])
  const int* todo = nullptr;         // device [count]: steps of the batch each member takes
  int step = 0;                      // step of the batch this launch belongs to
  int rec_stride = 0;                // record words between consecutive members
};

// Region shapes of the temporally blocked solve kernels (positions per
// block, two per thread).
enum Region : int { kRegion32x32 = 0, kRegion64x16 = 1, kRegion32x16 = 2, kRegionCount = 3 };
const char* region_name(int region);

// Output tile of the first-iteration solve and of the fused iteration for a
// region and sweeps (1..4); sites per block of the final update and of the
// energy partial sums.
void first_solve_tile(int region, int sweeps, int* tx, int* ty);
void iterate_tile(int region, int sweeps, int* tx, int* ty);
constexpr int kFinalSites = 256;
void energy_tile(int* tx, int* ty);

// Optional timestamps of one launch (both NULL: untimed).
struct LaunchEvents {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};

// Kernel launchers (each enqueues on `stream`; return hipSuccess or an error).
// p[0 .. n) = 0 (a kernel, so that it may sit in a captured graph).
hipError_t launch_clear(unsigned long long* p, int n, hipStream_t stream);

// member_of[b] = m for every block b in [block0[m], block0[m + 1]), m < count,
// b < blocks = block0[count] (the table Multi::member_of points into).
hipError_t launch_member_table(const int* block0, int count, int blocks, int* member_of,
                               hipStream_t stream);

// The launchers below that take a Multi run every member of it when mu.desc is
// not NULL: the Lattice then carries ensemble-wide V and u0, planes and
// records are those of member 0, and `region` picks the solve-region shape.
// Members with todo[m] <= mu.step do nothing.

// Newton iteration 1, stage solve: `sweeps` (1..4) block-Jacobi sweeps of
// (I - h lambda_i J) r_i = -Phibar_i with Phibar_i = -h TC_i f(u_0) (the
// residual at U^0 = e_3 (x) u_0) built in place, into rout.  Records
// ||u_0||_inf in *u0max_slot and ||(T (x) I) r||_inf in *rslot (each if not NULL),
// and writes that Phibar to phib_out when phib_out.s[0] is not NULL.
hipError_t launch_first_solve(const Lattice& lat, Planes3 rout, int sweeps,
                              unsigned long long* rslot, unsigned long long* u0max_slot,
                              Planes3 phib_out, hipStream_t stream, LaunchEvents ev = {});

// Newton iteration l >= 2 (or a kernel-level call), stage solve: `sweeps`
// (1..4) block-Jacobi sweeps from r = 0 for the three stage systems
// (I - h lambda_i J) r_i = -phib_i in one temporally blocked pass;
// ||(T (x) I) r||_inf to *rslot if not NULL.
constexpr int kMaxFusedSweeps = 4;
hipError_t launch_stage_solve(const Lattice& lat, CPlanes3 phib, Planes3 rout, int sweeps,
                              unsigned long long* rslot, ConvCheck check, hipStream_t stream,
                              LaunchEvents ev = {});

// One more block-Jacobi sweep from the iterate rin (rin and rout must not
// alias); ||(T (x) I) rout||_inf to *rslot if not NULL.
hipError_t launch_stage_sweep(const Lattice& lat, CPlanes3 phib, CPlanes3 rin, Planes3 rout,
                              unsigned long long* rslot, ConvCheck check, hipStream_t stream,
                              LaunchEvents ev = {});

// Update pass of one Newton iteration.  Skipped when `check` says an earlier
// iteration converged.  If `fin` says this iteration converged (its norm was
// recorded by the stage solve): u0_out <- U_3 + (T rbar)_3 (base U_3 = Uin[2],
// or u_0 if from_u0), site by site, and nothing else.  Otherwise:
// Uout <- base + (T (x) I) rbar (base = Uin, or e_3 (x) u_0 if from_u0), then
// phib <- (T^-1 (x) I) Phi(Uout); ||(T (x) I) rbar||_inf goes to *rslot if not
// NULL.  Uin and Uout must not alias (blocks read the halo of Uin while
// others write Uout).  Uout is not written when !from_u0 && !has_rbar.
// xform: the stage fields hold X = U - e (x) u_0 instead of U (from_u0 then
// means X = 0), as on the fused path; the final update is u_0 + X_3 + (T
// rbar)_3.  Rounding then stays at the size of X, not of U, which matters
// for stiff kinetic operators.
hipError_t launch_update_residual(const Lattice& lat, CPlanes3 Uin, Planes3 Uout, CPlanes3 rbar,
                                  bool has_rbar, bool from_u0, Planes3 phib,
                                  unsigned long long* rslot, ConvCheck check, ConvCheck fin,
                                  double2* u0_out, hipStream_t stream, LaunchEvents ev = {},
                                  bool xform = false);

// ---------------------------------------------------------------------------
// The fused path (at most four sweeps per stage solve) holds the Newton
// iterate of a step as its increment over u_0, X^l = U^l - e (x) u_0
// (Eq. MB4_6 summed: X^l = (T (x) I)(rbar^1 + ... + rbar^l), X^0 = 0), so
// that an iteration reads u_0, V and X^{l-1} and writes only X^l.  u_1 =
// u_0 + X_3 (Sec. 2.2: c_3 = 1).
//
// Within a batch of steps u_0 alternates between two buffers: step k reads
// Lattice::u0 and sends its u_1 to `next` (the other buffer), except that the
// last step a member takes in the batch (k = todo[m] - 1 with a Multi; the
// caller passes next = home on the batch's last step otherwise) sends it to
// `home`, where the batch started.  Writes to next are never read by the same
// launch; u_1 goes to `home` site by site only (final updates), so home may
// be the step's own u_0.
struct StepOut {
  double2* next;
  double2* home;
  // launch_iterate writes only X_3 of X^{iter+1}: the caller takes the step
  // again from u_0 if iteration iter + 1 does not converge, so X_1 and X_2
  // of that iterate are never read.
  bool stage3_only = false;
};

// The final update of the previous step, fused into the first solve of the
// next.  Unless the previous step converged before its last iteration (`chk`
// holds: an update pass already wrote its u_1, which is this step's u_0), the
// region's u_0 is formed from the previous step's u_0 and X (u_0 + X_3 if it
// converged at its last iteration, `fin`; u_0 itself if it did not converge,
// so that the step repeats), and each block writes it for its tile to `next`,
// a writable alias of this step's Lattice::u0.  With a Multi, the records are
// member 0's, and a member whose previous step was its last in the batch gets
// only that final update, written to `home`.
struct PrevStep {
  const double2* u0;  // u_0 of the previous step
  CPlanes3 X;         // its X at the last iteration
  ConvCheck chk, fin;
  double2* next;
  double2* home;
};

// Newton iteration 1 of the fused path: as launch_first_solve, the residual at
// X^0 = 0 built in place and `sweeps` (1..4) block-Jacobi sweeps, writing
// X^1 = (T (x) I) rbar^1 to xout (and its norm to *rslot).  prev: the fused
// final update of the previous step (NULL: none).
//
// fp32: the FP32 inner stage solves.  The block-Jacobi sweeps, the 2x2 block
// inverses and the right-hand side -Phibar are rounded to and computed in
// FP32; the residual Phi, the stage quadrature, X, the update and the norms
// stay FP64.  Only the 32 x 32 region exists in this precision.
hipError_t launch_first_solve_x(const Lattice& lat, Planes3 xout, int sweeps,
                                unsigned long long* rslot, unsigned long long* u0max_slot,
                                hipStream_t stream, LaunchEvents ev, const Multi& mu, int region,
                                bool fp32, const PrevStep* prev);

// Newton iteration `iter` >= 1 of the fused path fused with the stage solve
// of iteration iter + 1: unless `check` says an earlier iteration converged
// (then nothing) or `fin` says iteration iter converged (then u_1 = u_0 +
// X^iter_3 to so, site by site), Phibar of U^iter = u_0 + Xin, `sweeps` (1..4)
// block-Jacobi sweeps of the stage systems, Xout <- Xin + (T (x) I) rbar^{iter+1}
// and ||(T (x) I) rbar^{iter+1}||_inf into *rnext.  Xin and Xout must not alias.
hipError_t launch_iterate(const Lattice& lat, CPlanes3 Xin, Planes3 Xout, int sweeps,
                          unsigned long long* rnext, ConvCheck check, ConvCheck fin, StepOut so,
                          hipStream_t stream, LaunchEvents ev = {}, const Multi& mu = {},
                          int region = kRegion32x32, bool fp32 = false);

// Final update of the last step of a batch, site by site: unless `check` says
// an update pass already wrote u_1, u_1 = u_0 + X_3 if `fin` holds, u_0
// otherwise (the step did not converge), to so.
hipError_t launch_final_update(const Lattice& lat, CPlanes3 X, ConvCheck check, ConvCheck fin,
                               StepOut so, hipStream_t stream, LaunchEvents ev = {},
                               const Multi& mu = {});

// ---------------------------------------------------------------------------
// A batch of the multi-lattice engine as one persistent launch.  Each block
// is a worker that owns whole members, order[wfirst[w] .. wfirst[w + 1]),
// and takes each of them through its todo[m] steps one after the other,
// every Newton iteration of a step included (Algorithm 1's loop runs on the
// device, up to max_newton iterations, with the stopping test of ConvCheck).
// A member's tiles are only ever touched by its own block, so the block's
// barriers order one phase (a Newton iteration over all tiles) before the
// next, and no grid-wide synchronisation exists.  Step k of a member reads
// u_0 from u0 (k even) or u0b (k odd) and sends u_1 on through the fused
// first solve of step k + 1, the last step's u_1 going to u0 (home); X^l
// alternates between Xa and Xb.  conv[k * members + m] receives the
// outcome of step k: the iteration it converged at (>= 1), 0 if it had not
// converged after max_newton iterations, -1 if an update was not finite.
// A member stops at such a failed step and keeps its u_0 in u0.  pred[m] is
// the member's predicted iteration count, carried from batch to batch: that
// iteration writes only X_3 of its iterate, and a step that needs more is
// taken again from its u_0 with one more (as the per-phase form does in its
// next batch), so the results do not depend on the prediction.
struct MemberRun {
  const MemberDesc* desc;  // device [members]
  const int* order;        // device: members, worker after worker
  const int* wfirst;       // device [workers + 1]
  const int* todo;         // device [members]: steps of the batch
  int members;
  int* conv;               // device [steps][members]
  int* pred;               // device [members]
  double2* u0;
  double2* u0b;
  double2* Xa[3];
  double2* Xb[3];
  double eps;
  bool relative;
  int max_newton;
};

// lat carries the ensemble-wide V (and per-site g, if any); `workers`
// blocks.  Region and sweeps as for launch_iterate.
hipError_t launch_member_run(const Lattice& lat, const MemberRun& run, int workers, int sweeps,
                             int region, bool fp32, hipStream_t stream, LaunchEvents ev = {});

// Blocks of launch_member_run that are resident on one CU at a time (0 if
// the shape is not built).
int member_run_blocks_per_cu(int sweeps, int region, bool fp32);

// (p, q) arrays <-> interleaved double2 field of n sites.
hipError_t launch_interleave(const double* p, const double* q, double2* out, int n,
                             hipStream_t stream);
hipError_t launch_deinterleave(const double2* in, double* p, double* q, int n,
                               hipStream_t stream);

// Energy components: H, U_K, U_I, U_E, sum n, sum n^2 into out[6] (device),
// through `partials` (device scratch of energy_partials_count(nx, ny) doubles).
size_t energy_partials_count(int nx, int ny);
hipError_t launch_energy(const Lattice& lat, double* partials, double* out,
                         hipStream_t stream);
// The same with psi given as two device planes p, q of nx*ny doubles (lat.u0
// unused).
hipError_t launch_energy_planes(const Lattice& lat, const double* p, const double* q,
                                double* partials, double* out, hipStream_t stream);
// The same for every member of a Multi (block0 over energy tiles): out[6 m + k];
// partials holds 12 doubles per block.
hipError_t launch_energy_multi(const Lattice& lat, const Multi& mu, double* partials,
                               double* out, hipStream_t stream);

// Host runtime: records `fmt` as the calling thread's error detail (what
// mb4_error_detail returns) and returns `code`.
namespace rt {
int fail(int code, const char* fmt, ...);
}  // namespace rt

}  // namespace mb4
