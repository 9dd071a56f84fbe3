/*
 * mb4.h - C ABI of the MI355X (gfx950) MB4 integrator for the periodic 2D
 * lattice nonlinear Schroedinger-type equation.
 *
 * Method: Sakai, Kudo, Imachi, Miyatake, Hoshi, Yamamoto, "A Parallelizable
 * Energy-Preserving Integrator MB4 and Its Application to Quantum-Mechanical
 * Wavepacket Dynamics", arXiv 2003.04345 (Sec. 2.2, Sec. 2.3, Algorithm 1).
 *
 * Problem.  psi in C^{nx*ny}, site (x, y) at index y*nx + x (x fastest, as in
 * Sec. 2.1).  The flow is
 *     i dpsi/dt = (K + V) psi + g |psi|^2 psi,
 * with K = -t_hop on the four periodic nearest-neighbour links plus
 * diag_shift on the diagonal, and V the on-site potential.  In the paper's
 * notation (Eq. dNLS) this is gamma = -g; its K = -Laplacian_h (Eq.
 * Kdefinition) is t_hop = 1/h_x^2, diag_shift = 4/h_x^2.  With
 * u = (p, q) = (Re psi, Im psi) the flow is u' = S grad H(u) (Eqs. EOM1,
 * EOM2) with S = [[0, I], [-I, 0]] and
 *     H = 1/2 (p^T A p + q^T A q) + g/4 sum_j |psi_j|^4,   A = K + V,
 * which is half of the paper's H (Eqs. U_K - U_E) and gives the same flow.
 *
 * One call of mb4_step advances one MB4 step per requested step: the
 * simplified Newton iteration on the stage system (Eqs. Phidefinition,
 * Newton1) with the Jacobian frozen at u_0 (Eq. Jacobian2), decoupled by the
 * eigendecomposition of E into three stage solves (Eqs. MB4_4 - MB4_6) that
 * run concurrently in one kernel, until ||r^l||_inf <= eps (Algorithm 1; or
 * eps * ||u_0||_inf with MB4_FLAG_RELATIVE_EPS), then u_1 = U_{c_3}
 * (c_3 = 1).  All arithmetic is IEEE double on the GPU, except the inner
 * stage solves under MB4_FLAG_FP32_SOLVE.
 *
 * Conventions for every entry point.
 *  - Return value: MB4_OK (0) or a negative MB4_E* code; mb4_strerror gives a
 *    static string, mb4_error_detail a message for the calling thread's last
 *    failure.
 *  - Arguments are validated on the host before any device call, so invalid
 *    calls return MB4_EINVAL even on a machine without a GPU.
 *  - "host" pointers are ordinary CPU memory, read (or written) during the
 *    call only; the library copies what it keeps and never retains caller
 *    pointers.  "device" pointers are GPU memory of the state's device.
 *  - A state is used by one host thread at a time.  All its work runs on the
 *    stream given at creation (NULL is the null stream); every entry point
 *    returns after that work is complete.
 */
#ifndef MB4_H
#define MB4_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define MB4_API __attribute__((visibility("default")))
#else
#define MB4_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

#define MB4_OK 0
#define MB4_EINVAL (-1)   /* invalid argument: NULL, non-finite, size limits */
#define MB4_ENOMEM (-2)   /* footprint above mem_budget or allocation failed */
#define MB4_EDEVICE (-3)  /* a HIP runtime call failed */
#define MB4_ENOCONV (-4)  /* simplified Newton did not converge (Sec. 2.2) */

/* Periodic lattice.  nx, ny >= 3; nx * ny <= 2^28.  t_hop and diag_shift
 * finite. */
typedef struct {
  int32_t nx, ny;
  double t_hop;
  double diag_shift;
} mb4_lattice;

/* Cubic on-site nonlinearity g |psi|^2 psi (g = -gamma of the paper). */
typedef struct {
  double g;
} mb4_nonlinearity;

/* Solver options; pass NULL for all defaults, or start from
 * mb4_options_default().  Zero in a numeric field selects its default. */
typedef struct {
  double eps;            /* Newton tolerance: the loop stops once ||r^l||_inf <= eps
                            (Algorithm 1; default 1e-13, the epsilon of Sec. 3),
                            or <= eps * ||u_0||_inf with MB4_FLAG_RELATIVE_EPS */
  int32_t max_newton;    /* Newton iterations before MB4_ENOCONV; default 50, <= 1000 */
  int32_t inner_sweeps;  /* block-Jacobi sweeps per stage solve (Richardson iterations
                            with MB4_FLAG_SPECTRAL_SOLVE); default 3, <= 64 */
  void* stream;          /* hipStream_t for all work of the state; NULL = null stream */
  uint64_t mem_budget;   /* bytes of device memory the state may allocate; 0 = no limit */
  uint32_t flags;        /* MB4_FLAG_* bits; 0 = defaults */
} mb4_options;

/* mb4_options.flags: launch every kernel from the host instead of replaying
 * captured HIP graphs of whole batches of steps (same results, bit for bit;
 * graphs are never used while profiling is enabled). */
#define MB4_FLAG_NO_GRAPHS 1u
/* mb4_options.flags: read eps relative to ||u_0||_inf of each step instead of
 * as an absolute bound (for states whose amplitude is far from 1). */
#define MB4_FLAG_RELATIVE_EPS 2u
/* mb4_options.flags: FP32 inner stage solves.  The block-Jacobi sweeps of
 * the stage systems (Eq. MB4_5), their 2x2 block inverses and right-hand
 * sides run in FP32 (the stage corrections rbar never leave the chip); the
 * residual Phi, the stage quadrature, the Newton update U + (T (x) I) rbar,
 * its norm and the energy stay FP64, so the step converges to the same FP64
 * root.  At most 4 inner sweeps; mb4_newton_update and mb4_stage_solve stay
 * FP64. */
#define MB4_FLAG_FP32_SOLVE 4u
/* mb4_options.flags: spectrally preconditioned stage solves, for kinetic
 * operators too stiff for block-Jacobi sweeps (the continuum -Delta_h of
 * Sec. 3: t_hop = 1/h_x^2, diag_shift = 4 t_hop, where h lambda_i t_hop
 * reaches ~10).  Each stage system of Eq. MB4_5 is solved by inner_sweeps
 * Richardson iterations preconditioned by its constant-coefficient part (the
 * hopping, diag_shift and the mean potential), which the 2D discrete Fourier
 * transform diagonalises; one iteration contracts the error by at most
 * h |lambda_i| times the largest on-site deviation (V - mean V plus the
 * nonlinear Jacobian).  Sides up to 1024, FP64 only (not with
 * MB4_FLAG_FP32_SOLVE), up to 64 iterations; single states only.  The
 * kernel-level mb4_newton_update and mb4_stage_solve keep their block-Jacobi
 * form. */
#define MB4_FLAG_SPECTRAL_SOLVE 8u

typedef struct mb4_state mb4_state;

/* Fills *opt with the defaults.  NULL-safe. */
MB4_API void mb4_options_default(mb4_options* opt);

/* Creates a state on the current HIP device.
 *  lattice, nonlinearity: host structs as above.
 *  potential: host array of nx*ny finite doubles V_j (copied).
 *  h: time step, finite and non-zero (negative steps run backwards).
 *  opt: NULL or options.
 *  out: receives the new state; set to NULL on failure.
 * The initial state psi is zero until mb4_set_state*.  Device memory: 136
 * bytes per site (potential, two u_0 buffers, two fields of stage
 * increments) plus a few kilobytes; 144 bytes per site more (the
 * transformed residual and two stage-correction fields) once the state runs
 * more than four inner sweeps or the spectral solves, or mb4_stage_solve
 * with more than four sweeps, allocated on first use within mem_budget.
 * Errors: MB4_EINVAL, MB4_ENOMEM, MB4_EDEVICE. */
MB4_API int mb4_create(const mb4_lattice* lattice, const double* potential,
               const mb4_nonlinearity* nonlinearity, double h,
               const mb4_options* opt, mb4_state** out);

/* Frees all device memory of the state.  NULL-safe. */
MB4_API void mb4_destroy(mb4_state* state);

/* Sets psi = p + i q from host arrays of nx*ny finite doubles (copied) and
 * resets the step counter.  Errors: MB4_EINVAL, MB4_EDEVICE. */
MB4_API int mb4_set_state(mb4_state* state, const double* p, const double* q);

/* Copies psi to host arrays p, q of nx*ny doubles. */
MB4_API int mb4_get_state(mb4_state* state, double* p, double* q);

/* As mb4_set_state / mb4_get_state with device arrays of nx*ny doubles. The
 * caller orders its own work on these arrays with the state's stream.  No
 * finiteness check is made on device input. */
MB4_API int mb4_set_state_device(mb4_state* state, const double* d_p, const double* d_q);
MB4_API int mb4_get_state_device(mb4_state* state, double* d_p, double* d_q);

/* Advances nsteps >= 0 MB4 steps (Algorithm 1, time loop).  Each step is
 * all-or-nothing: if the Newton loop of a step does not reach the tolerance
 * within max_newton iterations (or produces a non-finite update), the call
 * returns MB4_ENOCONV and the state keeps the last accepted step;
 * mb4_steps_done tells how far the run got, and the caller may lower h with
 * mb4_set_h and continue (Sec. 2.2 advises this remedy). */
MB4_API int mb4_step(mb4_state* state, int64_t nsteps);

/* H of the current state, in the convention above (Sec. 2.1, Eqs. U_K - U_E,
 * halved).  Summed on the GPU in a fixed order with compensated (TwoSum)
 * arithmetic. */
MB4_API int mb4_energy(mb4_state* state, double* H);

/* out[0..5] = H, U_K, U_I, U_E, sum |psi|^2, sum |psi|^4 with
 * U_K = psi^H K psi / 2, U_I = g/4 sum |psi|^4, U_E = psi^H V psi / 2;
 * sum |psi|^4 is the participation ratio of Sec. 3.2. */
MB4_API int mb4_energy_components(mb4_state* state, double out[6]);

/* The six components of mb4_energy_components for a field given on the
 * device, without a state and without allocating anything: for callers that
 * cannot call hipMalloc (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The per-tile partial sums go to a
 * fixed device array of the library (3 MiB on each GPU it runs on, held
 * until the process ends), so the lattice may have at most 32768 tiles of
 * 64 x 4 sites, ceil(nx/64) * ceil(ny/4) <= 32768 (8,388,608 sites of full
 * tiles, e.g. 2048 x 4096); larger ones return MB4_EINVAL.
 *  lattice, nonlinearity: host structs as for mb4_create.
 *  d_potential, d_p, d_q: device arrays of nx*ny doubles (V, Re psi, Im psi),
 *    read.
 *  d_out: device array of 6 doubles, written: H, U_K, U_I, U_E, sum |psi|^2,
 *    sum |psi|^4, the same values, bit for bit, as mb4_energy_components of a
 *    state holding this field.
 *  stream: hipStream_t the kernels are enqueued on (NULL: null stream).
 * Unlike the other entry points it only enqueues: the results are in d_out
 * once the stream reaches them.  Every call on one GPU uses that GPU's one
 * array, which is fully overwritten before it is read, so calls whose work
 * may overlap on one GPU (other streams, other host threads) race; order
 * them on one stream.  The first call on a device looks up the array's
 * address there.  Errors: MB4_EINVAL (before any device call), MB4_EDEVICE. */
MB4_API int mb4_energy_components_noalloc(const mb4_lattice* lattice,
                                          const mb4_nonlinearity* nonlinearity,
                                          const double* d_potential, const double* d_p,
                                          const double* d_q, double* d_out, void* stream);

/* Site-dependent nonlinearity (the Appendix's U_I = -1/2 sum_i gamma_i n_i^2,
 * here g_i = -gamma_i): the flow becomes i psi_j' = ((K + V) psi)_j +
 * g_j |psi_j|^2 psi_j, and H's U_I = 1/4 sum_j g_j |psi_j|^4, which MB4
 * conserves as before.  g: host array of nx*ny finite doubles (copied), or
 * NULL to return to the uniform g of mb4_create.  The first call allocates
 * 8 bytes per site of device memory within mem_budget.  Single states only;
 * the ensemble and server keep one g per member.  Errors: MB4_EINVAL,
 * MB4_ENOMEM, MB4_EDEVICE. */
MB4_API int mb4_set_nonlinearity_sites(mb4_state* state, const double* g);

/* Changes the time step (finite, non-zero). */
MB4_API int mb4_set_h(mb4_state* state, double h);

/* Steps accepted since the last mb4_set_state*; -1 for NULL. */
MB4_API int64_t mb4_steps_done(const mb4_state* state);

/* Statistics of the last accepted step: Newton iterations, block-Jacobi
 * sweeps per stage solve summed over the iterations, and ||r||_inf of the
 * last Newton update.  Any output pointer may be NULL. */
MB4_API int mb4_last_stats(const mb4_state* state, int32_t* newton_iters,
                   int32_t* inner_sweeps, double* last_rnorm);

/* ||r^l||_inf of the Newton updates l = 1 .. n of the last accepted step into
 * out[0 .. n-1] (Algorithm 1, convergence measure r); *count receives
 * min(n, iterations).  out may be NULL when n == 0. */
MB4_API int mb4_last_residuals(const mb4_state* state, double* out, int32_t n,
                               int32_t* count);

/* Per-kernel timing for measurement (the per-phase breakdown of Sec. 3.2).
 * While enabled, each kernel launch of mb4_step is bracketed by HIP events on
 * the state's stream and its duration is added to its kernel class; launches
 * of Newton iterations after convergence (which return at once) are not
 * counted.  Enabling resets the accumulators.  Classes are numbered
 * 0 .. mb4_profile_classes()-1; mb4_profile_name gives a static name. */
MB4_API int mb4_profile_enable(mb4_state* state, int32_t enable);
MB4_API int32_t mb4_profile_classes(void);
MB4_API const char* mb4_profile_name(int32_t kernel_class);
MB4_API int mb4_profile_read(const mb4_state* state, int32_t kernel_class,
                             int64_t* launches, double* total_ms);

/* Kernel-level entry points, for callers that drive the Newton loop
 * themselves and for testing each kernel against a reference.  Stage fields
 * are three stage-major planes of nx*ny sites, each site an interleaved
 * (p, q) pair: element (i, site, comp) at d[(i*nx*ny + site)*2 + comp].
 *
 * mb4_newton_update: U <- U + (T (x) I) rbar if d_rbar != NULL (Eq. MB4_6
 * and the update of Eq. Newton1), then d_phibar <- (T^-1 (x) I) Phi(U)
 * (Eqs. Phidefinition, MB4_4) at the state's current psi as u_0, with the
 * linear stage integrals by E (Eq. fKu2) and the cubic ones by 6-node
 * Gauss-Legendre (exact for Eq. fIu2).  If rnorm != NULL it receives
 * ||(T (x) I) rbar||_inf (0 when d_rbar is NULL).  d_U is read and written,
 * d_rbar read, d_phibar written; all device. */
MB4_API int mb4_newton_update(mb4_state* state, double* d_U, const double* d_rbar,
                      double* d_phibar, double* rnorm);

/* mb4_stage_solve: approximate solutions of the three decoupled stage
 * systems (I - h lambda_i J) rbar_i = -phibar_i (Eq. MB4_5) with J frozen at
 * the state's psi (Eqs. JL, JR): exact 2x2 on-site block inverses and
 * `sweeps` >= 1 block-Jacobi sweeps over the hopping links, starting from
 * rbar = 0.  d_phibar read, d_rbar written; both device. */
MB4_API int mb4_stage_solve(mb4_state* state, const double* d_phibar, double* d_rbar,
                    int32_t sweeps);

/* ------------------------------------------------------------------------
 * Launch shape of the fused block-Jacobi path (inner_sweeps <= 4).
 *
 * Shapes of the solve regions (positions per block; the output tile is the
 * region less the halo the sweeps need).  All give identical results; the
 * speed depends on the lattice size, which mb4_tune and mb4_ensemble_tune
 * measure. */
#define MB4_REGION_32x32 0
#define MB4_REGION_64x16 1
#define MB4_REGION_32x16 2
#define MB4_REGION_COUNT 3

/* Selects the solve-region shape of a state (MB4_REGION_*; MB4_REGION_32x32
 * at creation); with MB4_FLAG_FP32_SOLVE only MB4_REGION_32x32 is built.
 * mb4_region returns it (-1 for NULL).  Errors: MB4_EINVAL. */
MB4_API int mb4_set_region(mb4_state* state, int32_t region);
MB4_API int32_t mb4_region(const mb4_state* state);

/* Inner iterations per stage solve (Eq. MB4_5) of a state, as inner_sweeps
 * of mb4_options: block-Jacobi sweeps (1 .. 64; at most 4 with
 * MB4_FLAG_FP32_SOLVE), or Richardson iterations with
 * MB4_FLAG_SPECTRAL_SOLVE.  The stage solves are inexact inner solves of the
 * simplified Newton iteration, so the count changes the number of Newton
 * iterations, not the root.  More than four sweeps allocate the plain
 * path's fields (see mb4_create) if the state has none yet.  mb4_sweeps
 * returns it (-1 for NULL).  Errors: MB4_EINVAL, MB4_ENOMEM, MB4_EDEVICE. */
MB4_API int mb4_set_sweeps(mb4_state* state, int32_t sweeps);
MB4_API int32_t mb4_sweeps(const mb4_state* state);

/* Autotuner of a state: times `steps` (1 .. 1024) steps under every region
 * shape and 2 .. 4 sweeps (one untimed pass first), keeps the fastest pair,
 * and restores the state, the step count and the statistics, so the run
 * continues as if it had not been called.  A pair under which a step does
 * not converge is skipped.  ms_per_step (may be NULL) receives
 * 4 * MB4_REGION_COUNT times in ms per step, index
 * (sweeps - 1) * MB4_REGION_COUNT + region, negative for a pair not timed;
 * *best_region and *best_sweeps (either may be NULL) the pair kept.  Uses
 * 16 bytes per site of temporary device memory.  Not with
 * MB4_FLAG_SPECTRAL_SOLVE.  Errors: MB4_EINVAL, MB4_ENOMEM, MB4_EDEVICE (the
 * state is restored and keeps its shape). */
MB4_API int mb4_tune(mb4_state* state, int32_t steps, int32_t* best_region,
                     int32_t* best_sweeps, double* ms_per_step);

/* ------------------------------------------------------------------------
 * Ensembles: many independent lattice problems (disorder realisations, say)
 * advanced together.  Every Newton phase of every member runs in one launch
 * over all members' tiles, with the same kernels and arithmetic as a single
 * state, so a member's trajectory is bit for bit the one mb4_step gives for
 * it alone.  Steps are replayed from HIP graphs as for a single state.  Each
 * member converges and is accepted on its own (Algorithm 1 per member);
 * members that need more Newton iterations do not hold the others back
 * beyond the batch in which it happens.
 *
 * Member fields are stored one after the other: 136 bytes per site
 * (potential, two u_0 buffers, two Newton-iterate fields of three stages)
 * plus the step records (8 * 32 * (max_newton + 1) bytes per member). */
typedef struct mb4_ensemble mb4_ensemble;

/* Creates an ensemble of `count` (1 .. 65536) members on the current device.
 *  lattices, nonlinearities, h: host arrays of `count` entries, each as for
 *    mb4_create (h finite and non-zero).
 *  potentials: host array of `count` pointers, member m's to nx*ny finite
 *    doubles (copied).
 *  opt: as for mb4_create, except that inner_sweeps must be at most 4 (one
 *    temporally blocked pass per stage solve); NULL for the defaults.
 * Members start at psi = 0.  Region MB4_REGION_32x32 until set or tuned.
 * Errors: MB4_EINVAL (before any device work), MB4_ENOMEM, MB4_EDEVICE. */
MB4_API int mb4_ensemble_create(int32_t count, const mb4_lattice* lattices,
                                const double* const* potentials,
                                const mb4_nonlinearity* nonlinearities, const double* h,
                                const mb4_options* opt, mb4_ensemble** out);

/* Frees the ensemble's device memory.  NULL-safe. */
MB4_API void mb4_ensemble_destroy(mb4_ensemble* ens);

/* Number of members; -1 for NULL. */
MB4_API int32_t mb4_ensemble_size(const mb4_ensemble* ens);

/* psi of member m from / to host arrays of its nx*ny doubles; setting resets
 * the member's step counter.  Errors: MB4_EINVAL (bad member, NULL, or
 * non-finite input), MB4_EDEVICE. */
MB4_API int mb4_ensemble_set_state(mb4_ensemble* ens, int32_t member, const double* p,
                                   const double* q);
MB4_API int mb4_ensemble_get_state(mb4_ensemble* ens, int32_t member, double* p, double* q);

/* Advances every member by nsteps >= 0 steps.  Steps are all-or-nothing per
 * member.  If a member's Newton loop fails (max_newton iterations or a
 * non-finite update), the call returns MB4_ENOCONV; that member keeps its
 * last accepted step, others may be further on, and
 * mb4_ensemble_member_stats tells where each one is. */
MB4_API int mb4_ensemble_step(mb4_ensemble* ens, int64_t nsteps);

/* out[6 m + k] = the six components of mb4_energy_components for member m;
 * out holds 6 * count doubles. */
MB4_API int mb4_ensemble_energy_components(mb4_ensemble* ens, double* out);

/* Steps accepted by member m since its last set_state, and the Newton
 * iterations of its last accepted step.  Either pointer may be NULL. */
MB4_API int mb4_ensemble_member_stats(const mb4_ensemble* ens, int32_t member,
                                      int64_t* steps_done, int32_t* newton_iters);

/* Selects the solve-region shape (MB4_REGION_*); with MB4_FLAG_FP32_SOLVE
 * only MB4_REGION_32x32 is built. */
MB4_API int mb4_ensemble_set_region(mb4_ensemble* ens, int32_t region);
MB4_API int32_t mb4_ensemble_region(const mb4_ensemble* ens);

/* Autotuner: times `steps` (>= 1) steps of the ensemble with each region
 * shape whose tiles are non-empty, keeps the fastest, and restores every
 * member's state and counters, so the run continues as if it had not been
 * called.  ms_per_step (may be NULL) receives MB4_REGION_COUNT times in ms
 * per step (negative for a shape not tried); *best (may be NULL) the shape
 * kept.  Uses 16 bytes per site of temporary device memory. */
MB4_API int mb4_ensemble_tune(mb4_ensemble* ens, int32_t steps, int32_t* best,
                              double* ms_per_step);

/* Block-Jacobi sweeps per stage solve of every member (1 .. 4; the stage
 * solves, Eq. MB4_5, are inexact inner solves of the simplified Newton
 * iteration, so the count changes the number of Newton iterations, not the
 * root).  mb4_ensemble_sweeps returns it (-1 for NULL).
 * Errors: MB4_EINVAL (out of range, or the region leaves no tile). */
MB4_API int mb4_ensemble_set_sweeps(mb4_ensemble* ens, int32_t sweeps);
MB4_API int32_t mb4_ensemble_sweeps(const mb4_ensemble* ens);

/* Autotuner over region shape and sweeps together: as mb4_ensemble_tune,
 * for every shape and 2 .. 4 sweeps, keeping the fastest pair (fewer sweeps
 * cost less per Newton iteration but may need more iterations).
 * ms_per_step (may be NULL) receives 4 * MB4_REGION_COUNT times, index
 * (sweeps - 1) * MB4_REGION_COUNT + region, negative for a pair not tried;
 * *best_region and *best_sweeps (either may be NULL) the pair kept. */
MB4_API int mb4_ensemble_tune_all(mb4_ensemble* ens, int32_t steps, int32_t* best_region,
                                  int32_t* best_sweeps, double* ms_per_step);

/* Launch form of the ensemble's batches (Algorithm 1's time loop and
 * Newton loop for every member).  on = 0 (the default): one launch per
 * Newton phase for all members, the batch of up to 32 steps replayed from a
 * captured graph, each step built for a predicted number of iterations.
 * on != 0: one persistent launch per batch, in which each block owns whole
 * members and runs every step and every Newton iteration of them itself,
 * deciding convergence on the device, so that no iteration is predicted and
 * none is wasted.  Both forms use the same tile kernels and give the same
 * results bit for bit.  mb4_ensemble_persistent returns the form (-1 for
 * NULL).  Errors: MB4_EINVAL, MB4_EDEVICE. */
MB4_API int mb4_ensemble_set_persistent(mb4_ensemble* ens, int32_t on);
MB4_API int32_t mb4_ensemble_persistent(const mb4_ensemble* ens);

/* Autotuner over the launch form: as mb4_ensemble_tune, timing the
 * per-phase form and the persistent form at the current region and sweeps
 * and keeping the faster.  ms_per_step (may be NULL) receives the two times
 * (per-phase first); *persistent (may be NULL) the form kept (0 or 1). */
MB4_API int mb4_ensemble_tune_launch(mb4_ensemble* ens, int32_t steps, int32_t* persistent,
                                     double* ms_per_step);

/* ------------------------------------------------------------------------
 * Serving: solve requests of different lattice sizes and step counts on one
 * GPU with continuous batching.  Requests wait in a FIFO queue and are
 * admitted as soon as an active slot and a contiguous range of the server's
 * device arena are free (admission by HBM footprint).  Each mb4_server_poll
 * runs one batch for all active requests together: every request advances
 * min(batch_steps, remaining) steps in the same launches as the others, with
 * its own Newton loop.  Finished requests are retired and their memory taken
 * by the next ones.  A request's result is bit for bit what mb4_step gives
 * it alone with the same options.  One host thread per server. */
typedef struct mb4_server mb4_server;

#define MB4_REQ_QUEUED 0
#define MB4_REQ_ACTIVE 1
#define MB4_REQ_DONE 2
#define MB4_REQ_FAILED 3

typedef struct {
  int32_t status;              /* MB4_REQ_* */
  int32_t nx, ny;
  int64_t steps, steps_done;
  double t_submit, t_admit, t_done; /* mb4_server_clock seconds; -1 if not yet */
  double energy_start;         /* H at admission (mb4_energy convention) */
  double energy_end;           /* H when retired */
  int32_t last_newton_iters;   /* Newton iterations of the last accepted step */
  int32_t error;               /* MB4_ENOCONV for a failed request, else 0 */
} mb4_request_info;

typedef struct {
  int64_t capacity_sites, used_sites;
  int32_t queued, active;
  int64_t batches;
  double site_steps;           /* lattice-site-steps completed */
} mb4_server_info;

/* Creates a server on the current device whose device memory stays within
 * arena_bytes (member fields: 136 bytes per site, plus step records).  max_active (1 .. 65536) bounds
 * the requests on the GPU at once, batch_steps (1 .. 32) the steps per poll.
 * opt as for mb4_ensemble_create (inner_sweeps <= 4; mem_budget ignored).
 * Errors: MB4_EINVAL, MB4_ENOMEM, MB4_EDEVICE. */
MB4_API int mb4_server_create(uint64_t arena_bytes, int32_t max_active, int32_t batch_steps,
                              const mb4_options* opt, mb4_server** out);
MB4_API void mb4_server_destroy(mb4_server* srv);

/* Seconds since the server was created (the clock of mb4_request_info). */
MB4_API double mb4_server_clock(const mb4_server* srv);

/* Queues a request: lattice, potential (nx*ny), nonlinearity and h as for
 * mb4_create, initial psi = p + i q (nx*ny each), and steps >= 0 MB4 steps.
 * All inputs are copied.  *id receives the request id.  MB4_EINVAL if the
 * request could never fit the arena. */
MB4_API int mb4_server_submit(mb4_server* srv, const mb4_lattice* lattice,
                              const double* potential, const mb4_nonlinearity* nonlinearity,
                              double h, const double* p, const double* q, int64_t steps,
                              int64_t* id);

/* One scheduling round: admit what fits, run one batch, retire what is
 * done.  queued / active (may be NULL) receive the counts afterwards.  A
 * request whose Newton loop fails is retired as MB4_REQ_FAILED; the others go
 * on. */
MB4_API int mb4_server_poll(mb4_server* srv, int32_t* queued, int32_t* active);

MB4_API int mb4_server_request(mb4_server* srv, int64_t id, mb4_request_info* info);

/* psi of a finished request (the last accepted step of a failed one) into
 * host arrays of nx*ny doubles. */
MB4_API int mb4_server_result(mb4_server* srv, int64_t id, double* p, double* q);

/* Forgets a finished request. */
MB4_API int mb4_server_release(mb4_server* srv, int64_t id);

MB4_API int mb4_server_stats(const mb4_server* srv, mb4_server_info* stats);

/* Static description of a status code. */
MB4_API const char* mb4_strerror(int code);

/* Message describing the calling thread's last failed call ("" if none). */
MB4_API const char* mb4_error_detail(void);

#ifdef __cplusplus
}
#endif

#endif /* MB4_H */
