/*
 * slh.h -- C ABI of libslh, the MI355X (gfx950) implementation of the
 * scatter-limited hybrid Monte Carlo / discrete-ordinates method for
 * time-dependent, single-group, isotropically scattering linear transport on
 * a 2-D Cartesian mesh (Krotz & McClarren, "Scatter-Limited Hybrid Monte
 * Carlo, Deterministic Transport with Quasi-Monte Carlo Sampling",
 * arXiv:2511.16821).
 *
 * The problem (Sec. 2.1, eq. (1)):
 *     (1/c) dPsi/dt + Omega.grad Psi + sigma_a Psi
 *         = sigma_s (<Psi>/(4 pi) - Psi) + Q/(4 pi)
 * on a uniform nx x ny mesh of [x_lo,x_hi] x [y_lo,y_hi] (x-y geometry,
 * invariant in z, directions on the whole unit sphere), with piecewise
 * constant sigma_s, sigma_a and angle-integrated isotropic source Q per cell,
 * zero initial data and vacuum boundaries.
 *
 * One time step (Sec. 2.2, steps 1-4):
 *   1. scatter-limited (Q)MC leg: census particles and N_p source particles
 *      with at most N_s scatters each (Sec. 2.3), track-length tallies
 *      T_pre (fewer than N_s scatters) and T_post (exactly N_s);
 *   2. DG S_N solve of the collided equation with source
 *      sigma_s/(4 pi) (phi_c + phi_post), bilinear discontinuous Galerkin,
 *      source iteration;
 *   3. remap: scatter-free (Q)MC leg from the census and N_p particles of the
 *      frozen source Q + sigma_s (phi_pre + phi_post + phi_c), tally T_R;
 *   4. the remap census is the state at t_{n+1}.
 * phi = T / (cell area * dt) is the step-averaged scalar flux (integral of
 * Psi over the sphere); phi_R is the solution of the step.  A steady-state
 * mode (slh_problem.steady) runs the same steps with an infinite time step.
 *
 * Conventions for every call:
 *   - Status codes only: no exceptions, no abort across this boundary.
 *   - Arguments are validated before anything is allocated; on error nothing
 *     is changed and slh_last_error() holds a message (thread-local).
 *   - Host arrays passed in are caller-owned and copied; output pointers are
 *     caller-owned.  Device memory of a solver is owned by the solver.
 *   - Field arrays are FP64, nx*ny long, row-major: cell (i, j) is element
 *     j*nx + i.
 *   - Work is enqueued on the HIP stream given at creation (borrowed, never
 *     destroyed); calls that return host data synchronise that stream.
 */
#ifndef SLH_H
#define SLH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SLH_ABI_VERSION 9u

typedef enum {
    SLH_OK = 0,
    SLH_E_INVALID_ARG = 1,   /* a field or parameter is out of range        */
    SLH_E_OUT_OF_MEMORY = 2, /* device allocation failed (nothing leaked)   */
    SLH_E_DEVICE = 3,        /* a HIP call failed                           */
    SLH_E_NOT_CONVERGED = 4, /* source iteration hit si_max_iter (the step
                                still completed; see slh_stats)             */
    SLH_E_NUMERIC = 5,       /* numeric fault: a non-finite weight, tally,
                                majorant or residual (slh_stats)            */
    SLH_E_REJECTED = 6,      /* serving: request does not fit the budget    */
    SLH_E_STATE = 7          /* call not valid in the object's state        */
} slh_status;

/* Arithmetic of the tracking kernels.  SLH_FP32_TRACK runs geometry,
 * distance sampling and attenuation in FP32 with cell-local coordinates;
 * tallies, balance totals, emission CDFs and the DG solve stay FP64. */
typedef enum { SLH_FP64 = 0, SLH_FP32_TRACK = 1 } slh_precision;

/* Points fed to the inverse-CDF maps (Sec. 2.4): scrambled Sobol' (QMC) or a
 * counter-based pseudo-random hash (plain MC, for comparisons). */
/* Point sets (Sec. 2.4): Owen-scrambled Sobol', pseudo-random (plain MC),
 * or Halton (the paper's set) randomised by a shift modulo 1 per stream and
 * dimension.  Dimensions past 32 are pseudo-random in every mode. */
typedef enum { SLH_SOBOL_OWEN = 0, SLH_PRNG = 1, SLH_HALTON = 2 } slh_points;

/* Which flux slh_get_flux returns (all FP64). */
typedef enum {
    SLH_FLUX_REMAP = 0,         /* phi_R, nx*ny: the solution of the step    */
    SLH_FLUX_PRE = 1,           /* phi_pre, nx*ny (step 1, n < N_s)          */
    SLH_FLUX_POST = 2,          /* phi_post, nx*ny (step 1, n = N_s)         */
    SLH_FLUX_COLLIDED_NODAL = 3 /* phi_c, 4*nx*ny: nodes (x0,y0),(x1,y0),
                                   (x0,y1),(x1,y1) of each cell             */
} slh_flux_kind;

typedef struct {
    uint32_t abi_version;          /* SLH_ABI_VERSION                        */
    int32_t nx, ny;                /* >= 1                                   */
    double x_lo, x_hi, y_lo, y_hi; /* x_hi > x_lo, y_hi > y_lo               */
    const double *sigma_s;         /* host, nx*ny, >= 0, finite              */
    const double *sigma_a;         /* host, nx*ny, >= 0, finite              */
    const double *q;               /* host, nx*ny, >= 0, angle-integrated    */
    double c;                      /* particle speed, > 0                    */
    double dt;                     /* time step, > 0                         */
    int32_t n_s;                   /* scatter limit N_s >= 0; -1: unlimited
                                      (the first leg is then plain MC, the
                                      collided solve has no source)        */
    int64_t n_particles;           /* N_p, 0..2^31: source particles per MC     */
                                   /* pass, born in proportion to the source   */
                                   /* (Sec. 2.3) and stratified by cell: with  */
                                   /* M_i = A dt (largest corner |q_i| rounded */
                                   /* up to a power of two) and w_q = sum(M) / */
                                   /* N_p (sum correctly rounded) rounded down */
                                   /* to five significant bits, cell i emits   */
                                   /* floor(r_i) or floor(r_i) + 1 particles,  */
                                   /* r_i = M_i / w_q, the second with chance  */
                                   /* frac(r_i); E[total] = sum(M) / w_q lies  */
                                   /* in [N_p, N_p 16/15)                      */
    int64_t census_cap;            /* census bank size; 0 -> n_particles     */
    int32_t sn_order;              /* even N >= 2: N^2 product directions    */
    double time_closure;           /* tau in sigma_t + tau/(c dt); 0 -> 2    */
    double si_tol;                 /* SI relative tolerance; 0 -> 1e-12      */
    int32_t si_max_iter;           /* 0 -> 200                               */
    double w_cut_rel;              /* cutoff |w| < w_cut_rel * w_q           */
    uint64_t seed;                 /* point-set seed                         */
    int32_t points;                /* slh_points                             */
    int32_t precision;             /* slh_precision                          */
    const int32_t *n_s_cell;       /* host, nx*ny, or NULL: per-cell scatter */
                                   /* limits N_s(x) (-1 unlimited, else 0..1e6),*/
                                   /* the space/material-dependent limit the  */
                                   /* paper names as its next step; n_s is    */
                                   /* then ignored.  A segment is pre-limit   */
                                   /* when the history's collision count is   */
                                   /* below its cell's limit.  Copied at      */
                                   /* slh_create.                             */
    int32_t boundary;              /* reflective sides, a bit mask of        */
                                   /* SLH_REFLECT_*; 0: vacuum everywhere.   */
                                   /* A history reaching a reflective side is */
                                   /* mirrored; the DG inflow on such a side  */
                                   /* is the previous source iteration's      */
                                   /* outflow of the mirrored direction.      */
    int32_t steady;                /* 0: time steps of dt (above).  1: steady */
                                   /* state, the infinite time step of the   */
                                   /* paper's runs (Sec. 3): dt, c and        */
                                   /* time_closure are not used, histories    */
                                   /* end only by leakage, the cutoff or the  */
                                   /* path horizon, no census is carried,     */
                                   /* phi = T / (cell area) is the flux per   */
                                   /* unit source rate, and the collided      */
                                   /* solve has sigma_e = sigma_t.  Each       */
                                   /* slh_advance step is then an independent */
                                   /* steady solve with the step's own points.*/
                                   /* With no scatter limit anywhere (pure   */
                                   /* MC) the steady step skips the collided  */
                                   /* solve and the remap: phi_R = phi_pre.   */
    double horizon;                /* steady only: path length (in units of  */
                                   /* length) at which a history ends; its    */
                                   /* weight then is booked as census and     */
                                   /* dropped.  0 -> ln(1/w_cut_rel) / min    */
                                   /* sigma_a, at which every weight is below */
                                   /* the cutoff; that needs w_cut_rel > 0    */
                                   /* and sigma_a > 0 in every cell, else     */
                                   /* horizon must be given (> 0, finite).    */
                                   /* Tallies are fixed point with a unit of  */
                                   /* 2^-61 times (total weight x horizon).   */
    int32_t si_norm;               /* source-iteration stopping test:         */
                                   /* SLH_SI_NORM_COLLIDED (0): stop when     */
                                   /* ||dphi_c|| <= si_tol ||phi_c||;         */
                                   /* SLH_SI_NORM_TOTAL (1): when ||dphi_c||  */
                                   /* <= si_tol ||phi_c + phi_pre + phi_post||*/
                                   /* (the step's whole flux), so a small     */
                                   /* collided part needs fewer sweeps.       */
                                   /* Norms are L2 over nodal values.         */
    int32_t closure;               /* collided solve (step 2):                */
                                   /* SLH_CLOSE_SN (0): DG S_N, source        */
                                   /* iteration;  SLH_CLOSE_DIFFUSION (1):    */
                                   /* cell-centred diffusion,                 */
                                   /* (sigma_a + tau/(c dt)) phi_c            */
                                   /*  - div(D grad phi_c) = sigma_s phi_post,*/
                                   /* D = 1/(3 (sigma_t + tau/(c dt))) (no    */
                                   /* tau/(c dt) in steady state), harmonic-  */
                                   /* mean faces, Marshak vacuum sides,       */
                                   /* zero-current reflective sides; solved   */
                                   /* by preconditioned conjugate gradients   */
                                   /* to |r| <= si_tol |b| within si_max_iter */
                                   /* iterations (reported as si_iterations;  */
                                   /* si_norm is not used).  phi_c is then    */
                                   /* constant in each cell.  Needs           */
                                   /* sigma_t + tau/(c dt) > 0 in every cell. */
    int32_t si_accel;              /* S_N closing stage only:                  */
                                   /* SLH_ACCEL_NONE (0): plain source        */
                                   /* iteration; SLH_ACCEL_DSA (1): diffusion  */
                                   /* synthetic acceleration, after each sweep */
                                   /* phi += delta with delta the solution of  */
                                   /* the closure's diffusion system (see      */
                                   /* closure; vacuum condition on every side, */
                                   /* since reflected inflow lags) for the     */
                                   /* source sigma_s times the cell average of */
                                   /* the sweep's change,                      */
                                   /* solved by conjugate gradients to 1e-2    */
                                   /* relative residual (at most 32 steps).    */
                                   /* Same fixed point, fewer sweeps when      */
                                   /* scattering dominates.  Needs             */
                                   /* sigma_t + tau/(c dt) > 0 in every cell.  */
    int32_t census_qmc;            /* points of the census histories (the     */
                                   /* bank is ordered by cell either way):    */
                                   /* SLH_CENSUS_HISTORY (0): a stream per    */
                                   /* history (its id), point 0, so a         */
                                   /* history's draws do not depend on the    */
                                   /* others: FP32 and FP64 tracking differ   */
                                   /* at rounding level;  SLH_CENSUS_COHORT   */
                                   /* (1): the census particles of a cell     */
                                   /* draw the points of the cell's census    */
                                   /* stream at their ranks in bank order, a  */
                                   /* low-discrepancy set per cell (QMC       */
                                   /* convergence carried across steps; a     */
                                   /* particle that another precision puts in */
                                   /* another cell re-pairs its cohort's      */
                                   /* points, so FP32 and FP64 differ at MC   */
                                   /* noise level in those cells).            */
    const double *inflow;          /* host, 2 (nx + ny) values, or NULL: the  */
                                   /* prescribed isotropic inflow G of the    */
                                   /* boundary faces (Sec. 2.1), per unit     */
                                   /* solid angle, area and time: the x_lo    */
                                   /* faces (j = 0..ny-1), the x_hi faces,    */
                                   /* the y_lo faces (i = 0..nx-1), the y_hi  */
                                   /* faces; 0 on reflective sides.  Applied  */
                                   /* in both MC legs (steps 1 and 3; the     */
                                   /* collided solve has zero boundary data): */
                                   /* face f is an emitter after the cells,   */
                                   /* majorant (pi L_f) dt pow2_ceil(|G_f|)   */
                                   /* (pi G the partial current), particles   */
                                   /* uniform along the face and in time,     */
                                   /* cosine law about the inward normal.     */
} slh_problem;

#define SLH_CENSUS_HISTORY 0
#define SLH_CENSUS_COHORT 1

#define SLH_ACCEL_NONE 0
#define SLH_ACCEL_DSA 1

#define SLH_CLOSE_SN 0
#define SLH_CLOSE_DIFFUSION 1

#define SLH_SI_NORM_COLLIDED 0
#define SLH_SI_NORM_TOTAL 1

#define SLH_REFLECT_X_LO 1
#define SLH_REFLECT_X_HI 2
#define SLH_REFLECT_Y_LO 4
#define SLH_REFLECT_Y_HI 8

/* Balance of one pass (implicit capture, Sec. 2.3), FP64 from
 * order-independent fixed-point sums: emitted = absorbed + scattered +
 * leaked + census + cutoff up to rounding of the per-particle terms. */
typedef struct {
    double emitted;      /* source + census-in weight                        */
    double absorbed;     /* integral of sigma_a w ds                         */
    double scattered;    /* integral of sigma_s w ds on post-limit segments
                            (step 1: handed to the collided stage)           */
    double leaked;       /* weight leaving through the boundary              */
    double census;       /* weight alive at t_{n+1} (steady state: at the
                            path horizon, dropped)                           */
    double cutoff;       /* weight of histories ended by the cutoff          */
    double source_w;     /* weight emitted by the source                     */
    double census_in_w;  /* weight of the census-in bank                     */
    uint64_t segments;   /* tracking-loop iterations                         */
    uint64_t particles;  /* histories started                                */
    double majorant_sum; /* sum of the cell majorants M_i, correctly rounded  */
    double weight_quantum; /* w_q of the pass's emission                      */
    uint64_t source_particles; /* particles emitted by the source              */
    uint64_t killed;     /* histories ended by the device's guard of 2^26
                            segments per history (booked as cutoff); 0 in
                            every normal run, and slh_synchronize reports
                            SLH_E_NUMERIC when it is not                    */
} slh_balance;

typedef struct {
    int64_t step;            /* steps enqueued                               */
    int32_t si_iterations;   /* last step: transport sweeps                  */
    double si_residual;      /* last step: ||dphi||/||phi|| at exit          */
    int32_t si_converged;    /* last step: 1 if residual <= si_tol           */
    int64_t census_alive;    /* last step: census candidates at t_{n+1}      */
    int64_t census_kept;     /* last step: bank size after the cap           */
    double thin_factor;      /* last step: weight factor of the cap          */
    uint64_t segments_total; /* last step, both passes                       */
    double ms_mc, ms_dg, ms_remap, ms_census; /* last step run in timing mode
                                 (slh_set_timing), stage times: emission and
                                 MC pass 1; collided solve and remap set-up;
                                 remap pass; census.  0 otherwise          */
    /* Totals since creation (or the last slh_load), for throughput and
     * roofline accounting, kept on the device.  Kernel times exist only for
     * steps run in timing mode: HIP events recorded on the solver's stream
     * immediately around each MC-pass kernel launch. */
    double ms_kernel_mc_total;      /* step-1 (scatter-limited) pass kernels */
    double ms_kernel_remap_total;   /* step-3 (remap) pass kernels           */
    uint64_t seg_mc_total;          /* segments of step-1 passes             */
    uint64_t seg_remap_total;       /* segments of step-3 passes             */
    uint64_t census_in_total;       /* census-in particles over all steps
                                       (each step's bank, which both passes
                                       read once)                            */
    uint64_t census_out_total;      /* census candidates written (step 3)    */
    uint64_t steps_total;           /* steps accounted in the totals         */
    uint64_t thin_overflow_total;   /* steps whose census draw exceeded the
                                       cap (first cap in slot order kept)   */
    uint64_t graph_launches_total;  /* HIP graphs launched: one per step (three
                                       in timing mode)                       */
    uint64_t host_waits_total;      /* host waits inside slh_advance: 0, the
                                       steps are asynchronous                */
    uint64_t killed_total;          /* histories ended by the segment guard   */
    /* Diffusion synthetic acceleration (si_accel), last step: corrections
     * solved, their conjugate-gradient iterations in total, and how many
     * stopped at the iteration limit (32) before the tolerance (1e-2): on
     * large meshes a correction is then approximate, which changes the
     * number of sweeps but not the fixed point of the iteration. */
    int32_t dsa_corrections;
    int32_t dsa_iterations;
    int32_t dsa_unconverged;
    int32_t numeric_flags;          /* OR over all steps: 1 a non-finite cell
                                       majorant or sum, 2 a non-finite history
                                       weight or tally, 4 an emission clamped
                                       to the source bank, 8 a non-finite
                                       source-iteration residual, 16 the
                                       segment guard fired (0 normally)     */
    uint64_t si_unconverged_total;  /* steps whose source iteration stopped
                                       at si_max_iter                        */
    int32_t si_batch;               /* source iterations launched per step at
                                       present (see slh_advance)             */
    int32_t pad0;
    uint64_t si_restarts_total;     /* steps run again because their batch
                                       ended before the iteration            */
} slh_stats;

typedef struct slh_solver slh_solver;

/* Allocator hooks for device memory (e.g. PyTorch's caching allocator).  Both
 * NULL -> hipMalloc / hipFree.  alloc must return memory aligned to 256 bytes
 * (as hipMalloc does), or NULL; slh_create fails with SLH_E_INVALID_ARG on a
 * misaligned block (after handing it back to free_fn). */
typedef void *(*slh_alloc_fn)(size_t bytes, void *ctx);
typedef void (*slh_free_fn)(void *ptr, void *ctx);

/* Creates a solver: validates the problem, copies the fields to the device,
 * builds the S_N quadrature and the Sobol' tables, and enqueues nothing
 * else.  hip_stream: hipStream_t to use (NULL = the null stream). */
slh_status slh_create(const slh_problem *problem, void *hip_stream, slh_alloc_fn alloc,
                      slh_free_fn free_fn, void *alloc_ctx, slh_solver **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * solver as slh_create, with every device buffer carved from a fixed static
 * scratch array of 64 MiB that each device holds for the life of the
 * process.  No hipMalloc, hipFree, pinned host allocation, event or graph is
 * created; kernels are launched directly on hip_stream, so slh_advance
 * itself may be captured by the caller.  Results are bitwise those of
 * slh_create.  SLH_E_REJECTED if slh_footprint_bytes(problem) exceeds the
 * scratch; SLH_E_STATE if the current device's scratch already holds a
 * static solver (one at a time per device, released by slh_destroy).  The
 * scratch keeps the previous solver's contents; the solver initialises
 * everything it reads.  Stage and kernel times in slh_stats are zero, and
 * slh_set_graphs(s, 1) is SLH_E_STATE. */
slh_status slh_create_static(const slh_problem *problem, void *hip_stream, slh_solver **out);

/* Enqueues n_steps >= 1 time steps (steps 1-4 above) on the solver's stream
 * and returns without waiting for the device.  Each step is one HIP graph
 * (captured on first use, once per census-bank parity and batch, and
 * replayed): the scatter-limited leg, the collided solve as a batch of
 * source iterations of which those after the device's stopping test return
 * at once, the remap leg and the census.  Nothing in a step waits for the
 * host.  The batch adapts to the iteration counts of past steps (an eighth
 * more than the last one, plus two, in multiples of four; at most
 * si_max_iter); a step whose batch ends before its iteration stops itself
 * and every step enqueued after it on the device, and the next call that
 * waits for the stream (slh_synchronize, slh_get_*, slh_save, slh_load) runs
 * them again, the stopped one with the iterations it did plus an estimate of
 * the rest from its contraction rate (si_max_iter without an estimate or
 * when it stops again) and the others with a doubled batch.  With DSA on
 * meshes above 4096 cells the conjugate-gradient steps of each correction
 * are batched the same way (a quarter more than the last step's longest
 * correction, plus two; a correction left unfinished stops the step, which
 * runs again with the limit of 32).  Results do not depend on the batches.
 * The outcome of the steps (convergence, numeric faults) is reported by
 * slh_synchronize.  Returns SLH_E_DEVICE if a launch fails. */
slh_status slh_advance(slh_solver *s, int32_t n_steps);

/* Sets the batch of source iterations of the next steps (n >= 1, at most
 * si_max_iter), and that of conjugate-gradient steps per diffusion
 * correction to n (at most 32); the adaptive rules of slh_advance take over
 * after the next wait.  For tuning and tests; results do not depend on it. */
slh_status slh_set_si_batch(slh_solver *s, int32_t n);

/* enable != 0 (the default): each step is launched as a HIP graph; 0: every
 * kernel is launched directly.  Results are identical. */
slh_status slh_set_graphs(slh_solver *s, int32_t enable);

/* enable != 0: later steps are launched as three graphs with the two MC-pass
 * kernels launched directly between HIP events, so that slh_get_stats
 * reports their kernel times and the stage times of the last step; 0 (the
 * default): one graph per step, no events.  Results are identical.
 * SLH_E_STATE for a static solver. */
slh_status slh_set_timing(slh_solver *s, int32_t enable);

/* Blocks until the solver's stream is idle, then reports the outcome of the
 * steps enqueued since the last call: SLH_E_NUMERIC if a step met a numeric
 * fault (see slh_stats.numeric_flags; the results are then not valid),
 * else SLH_E_NOT_CONVERGED if a step's source iteration stopped at
 * si_max_iter (the step was still completed), else SLH_OK. */
slh_status slh_synchronize(slh_solver *s);

/* Copies the last step's flux to host_out (FP64; nx*ny values, or 4*nx*ny
 * for SLH_FLUX_COLLIDED_NODAL).  Synchronises the stream. */
slh_status slh_get_flux(slh_solver *s, int32_t which, double *host_out);

/* Same, into device memory dev_out (enqueued on the solver's stream). */
slh_status slh_get_flux_device(slh_solver *s, int32_t which, double *dev_out);

/* Balance of the last step's pass: pass = 1 (scatter-limited leg) or 2
 * (remap).  Synchronises the stream. */
slh_status slh_get_balance(slh_solver *s, int32_t pass, slh_balance *out);

slh_status slh_get_stats(slh_solver *s, slh_stats *out);

/* Census bank at the start of the next step, host copies, global
 * coordinates.  Arrays of at least *n entries are written (any pointer may be
 * NULL); *n receives the bank size.  Synchronises the stream. */
slh_status slh_get_census(slh_solver *s, int64_t *n, double *x, double *y, double *ox,
                          double *oy, double *w, int32_t *cell, uint64_t *hid);

/* Checkpoint: the complete state between steps is the census bank, the step
 * index and the problem (zero collided initial data every step).  With
 * buf == NULL, *len receives the size needed.  The buffer records the mesh
 * size, seed, precision and bank; slh_load rejects (SLH_E_INVALID_ARG,
 * nothing changed) a buffer written for another mesh, seed or precision, a
 * bank above the cap, and particles that are not valid for this problem (a
 * cell off the mesh, a position outside its cell, a non-finite weight or one
 * above the recorded maximum). */
slh_status slh_save(slh_solver *s, void *buf, size_t *len);
slh_status slh_load(slh_solver *s, const void *buf, size_t len);

/* Device memory the solver for this problem needs, in bytes (admission).
 * Exact when sigma_s and sigma_a are given (the collided sweep's material
 * table depends on them); with NULL fields an upper bound over both sweeps. */
size_t slh_footprint_bytes(const slh_problem *problem);

void slh_destroy(slh_solver *s);

/* Message of the last failed call on this thread ("" if none). */
const char *slh_last_error(void);

/* Point function of Sec. 2.4 on the device: for k in [0, n) writes
 * out[k*n_dims + d] = P(stream, dim0 + d, index0 + k), the 32-bit point word
 * that the tracking kernels use for (time step, pass, population, key),
 * with pass in {1, 2}, population 0 = source (key = birth cell, index =
 * particle number within the cell) or 1 = census (key = history id, index
 * 0), and points an slh_points value.  dev_out is device memory of
 * n*n_dims words; enqueued on hip_stream. */
slh_status slh_qmc_points(uint64_t seed, uint64_t step, uint32_t pass, uint32_t population,
                          uint64_t cohort, uint32_t dim0, uint32_t n_dims, uint32_t index0,
                          uint32_t n, int32_t points, uint32_t *dev_out, void *hip_stream);

/* ---------------------------------------------------------------------- */
/* Serving: continuous batching of independent solves on one GPU.           */
/* ---------------------------------------------------------------------- */

typedef struct {
    size_t hbm_budget_bytes; /* admission limit on summed footprints; 0 -> 64 GiB */
    int32_t max_slots;       /* concurrently resident requests; 0 -> 8        */
    int32_t n_streams;       /* ignored: each slot has its own HIP stream     */
} slh_server_cfg;

typedef struct {
    double submit_s;  /* host clock at submit                           */
    double admit_s;   /* when the request got a slot and memory         */
    double done_s;    /* when its result was available on the host      */
    double queue_ms;  /* admit - submit                                  */
    double run_ms;    /* done - admit                                    */
    double latency_ms;/* done - submit                                   */
    uint64_t segments;/* tracking segments of the whole solve            */
} slh_latency;

typedef struct slh_server slh_server;

/* Creates a server: one device arena of hbm_budget_bytes (allocated once;
 * no device allocation happens while requests run) and max_slots worker
 * threads, each with its own HIP stream.  A worker takes the first queued
 * request (arrival order; a request that does not fit yet is passed over,
 * but once four later requests have been admitted ahead of the one at the
 * head of the queue, nothing else is admitted until it fits) whose
 * footprint fits in the arena, runs all its steps on its stream, and
 * returns its memory, so requests are admitted as slots and memory free up
 * and resident requests overlap on the device.  max_slots <= 64. */
slh_status slh_server_create(const slh_server_cfg *cfg, slh_server **out);

/* Queues a solve of n_steps steps.  The problem's arrays are copied before
 * the call returns.  SLH_E_REJECTED if its footprint alone exceeds the
 * budget; SLH_E_INVALID_ARG if the problem is invalid. */
slh_status slh_server_submit(slh_server *srv, const slh_problem *problem, int32_t n_steps,
                             uint64_t *ticket);

/* *done = 1 once the result of ticket is available. */
slh_status slh_server_poll(slh_server *srv, uint64_t ticket, int32_t *done);

/* Blocks until the ticket is done; copies the final phi_R (nx*ny FP64),
 * the remap balance of the last step and the latency record. Any output
 * pointer may be NULL.  Releases the request. */
slh_status slh_server_result(slh_server *srv, uint64_t ticket, double *flux_out,
                             slh_balance *balance, slh_latency *latency);

/* Waits for all outstanding work, then frees everything. */
void slh_server_destroy(slh_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* SLH_H */
