/*
 * lbm.h -- C ABI of liblbm, a gfx950 (MI355X) implementation of the D2Q9
 * pseudopotential multi-relaxation-time lattice Boltzmann timestep of Shan,
 * Zhu, Yao, Yin and Jiang, "Pseudopotential MRT lattice Boltzmann model for
 * cavitation bubble collapse with high density ratio" (arXiv:1605.01800).
 *
 * One timestep (lbm_step) is, in the paper's order:
 *   density rho = sum_a f_a                           (Section 2.1, after Eq. 4)
 *   Carnahan-Starling pressure p(rho)                 (Eq. 15)
 *   pseudopotential psi(rho)                          (Eq. 13, G = -1)
 *   interaction force F, 4 axis + 4 diagonal sites    (Eq. 7)
 *   velocity with the half-step force                 (Eq. 6)
 *   moments, equilibrium moments                      (Eqs. 1, 4)
 *   Li's modified source term                         (Eq. 14)
 *   relaxation in moment space                        (Eqs. 2, 3)
 *   back-transform and streaming                      (Eq. 5), periodic in x;
 *   in y periodic, or halfway bounce-back walls       (Section 4.1)
 *
 * Conventions for every call:
 *   - Device pointers are HIP device addresses on the device that was current
 *     when the handle was created; host pointers are ordinary host memory.
 *   - The caller owns every buffer it passes (workspace, outputs, stream) and
 *     keeps it alive until lbm_destroy.  The library never allocates device
 *     memory; a handle owns only host metadata and captured HIP graphs.
 *   - Work is enqueued on the handle's stream and is asynchronous unless the
 *     call says it synchronises.  A handle is not thread-safe.
 *   - Every call returns an lbm_status.  LBM_ENONFINITE is sticky: once a
 *     handle has seen a non-finite density or psi^2 < 0 it refuses to step
 *     until lbm_init_bubble, lbm_set_populations or lbm_load replaces its state.
 *   - Population layout on the device (lbm_get/set_populations): nine planes,
 *     plane a holding f_a row by row, f[a][y][x], x fastest, no padding.  The
 *     velocity order is e_0 = (0,0), e_1..4 = (1,0),(0,1),(-1,0),(0,-1),
 *     e_5..8 = (1,1),(-1,1),(-1,-1),(1,-1): axis sites first, so that the
 *     weights of Eq. 7 are w_1..4 = 1/3, w_5..8 = 1/12.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,      /* bad argument, size or combination */
    LBM_ENOMEM = -2,      /* workspace or buffer too small */
    LBM_EHIP = -3,        /* a HIP runtime call failed */
    LBM_ENONFINITE = -4,  /* non-finite rho or psi (psi^2 < 0, Eq. 13) was latched */
    LBM_ESTATE = -5       /* call not valid in the handle's current state */
} lbm_status;

typedef enum {
    LBM_FP64 = 0,         /* populations and arithmetic in binary64 */
    LBM_FP32 = 1,         /* populations and arithmetic in binary32 */
    LBM_FP32_MIXED = 2    /* binary32 populations and arithmetic; Eq. 15 and Eq. 13
                             in binary64 at sites whose density lies in the
                             spinodal interval of Eq. 15 at T (lbm_spinodals),
                             widened by a tenth of its width on each side (all
                             sites in binary32 at or above T_c) */
} lbm_precision;

/* Parameters of one instance.  Section 3.1 fixes a = 0.5, R = 1, G = -1,
 * s_rho = s_j = 1.0 and s_e = s_zeta = s_q = 1.1; Section 3.1 and 4.1 give
 * eps = 1.86 and s_nu = 1/tau_nu with tau_nu in {0.51, 0.6, 0.8}.  Eq. 15 is
 * evaluated with eta = b rho / 4; b = 4 reproduces the densities the paper
 * prints in Section 3.2.  T is the absolute temperature (lbm_critical_point
 * gives T_c). */
typedef struct {
    int32_t nx, ny;        /* lattice sites; 1 <= nx, ny <= 65536 */
    int32_t walls_y;       /* 0: periodic in y; 1: halfway bounce-back walls at
                              y = -1/2 and y = ny - 1/2 (Section 4.1) */
    int32_t precision;     /* lbm_precision */
    double a, b, R, T;     /* Eq. 15 */
    double G;              /* interaction strength, Eq. 7 and Eq. 13; < 0 */
    double eps;            /* Li's coefficient, Eq. 14 */
    double s_rho, s_e, s_zeta, s_j, s_q, s_nu;   /* Lambda of Eq. 2 as rates 1/tau */
} lbm_params;

/* A gas disc of Eq. 16, centre (x0, y0) in lattice units, radius r0. */
typedef struct {
    double x0, y0, r0;
} lbm_bubble;

#define LBM_MAX_BUBBLES 8

/* Diagnostics of the current state, all in binary64.  Sums are taken in a
 * fixed order, so they are bitwise reproducible for a given state. */
typedef struct {
    int64_t step;                       /* steps taken since the last init */
    double mass;                        /* sum of rho */
    double mom_x, mom_y;                /* sum of rho v, v of Eq. 6 */
    int32_t n_bubbles;                  /* bubbles given to lbm_init_bubble */
    int32_t nonfinite;                  /* 1 if a non-finite value was latched */
    double gas_area[LBM_MAX_BUBBLES];   /* sum of clip((rho_l-rho)/(rho_l-rho_g),0,1),
                                           each site counted for the nearest centre */
    double radius[LBM_MAX_BUBBLES];     /* sqrt(gas_area / pi) */
    double wall_p_max;                  /* max of p(rho) (Eq. 15) over the wall rows
                                           and over every step since init; walls only */
    int64_t wall_p_step;                /* step after which that maximum was seen */
} lbm_diag;

/* ---- single instance ------------------------------------------------------ */

/* Device workspace that lbm_create needs for these parameters, in bytes. */
int lbm_workspace_bytes(const lbm_params *params, size_t *bytes);

/* Creates an instance in a caller-owned device workspace of ws_bytes bytes
 * (256-byte aligned, at least lbm_workspace_bytes) and binds it to the HIP
 * stream hip_stream (a hipStream_t; NULL means the null stream).  The state is
 * undefined until lbm_init_bubble or lbm_set_populations. */
int lbm_create(const lbm_params *params, void *d_workspace, size_t ws_bytes,
               void *hip_stream, void **handle);

/* Initial state of Eq. 16 at rest (f_a = w_a rho).  With slab_rows == 0 the
 * density is the tanh profile around the nb discs in b (0 <= nb <=
 * LBM_MAX_BUBBLES), using the signed distance to the nearest disc edge; with
 * slab_rows > 0 it is a flat liquid slab of that many rows centred on
 * y = (ny-1)/2 and b is ignored.  The liquid side takes rho_l (1 + delta)
 * (Section 4.1: the liquid density is raised to drive the collapse).  With
 * noise_amp > 0 every site is then scaled by 1 + noise_amp (2u - 1), u the
 * SplitMix64 deviate of (seed XOR site index), site index y*nx + x.  rho_l and
 * rho_g are also kept for the gas-fraction diagnostics.  Resets the step
 * counter, the wall-pressure peak and the non-finite latch. */
int lbm_init_bubble(void *handle, const lbm_bubble *b, int nb, int slab_rows,
                    double rho_l, double rho_g, double W, double delta,
                    double noise_amp, uint64_t seed);

/* Initial state at rest from a density field: f_a = w_a rho (w = 4/9, 1/9,
 * 1/36), for any initial density, e.g. the uniform liquid with a perturbed
 * line of the cavitation-inception run (Section 3.2).  d_rho: nx*ny binary64
 * values on the device, row-major [y][x].  rho_l and rho_g are kept for the
 * gas-fraction diagnostics (no bubbles are assumed: n_bubbles = 0).  Resets
 * the step counter, the wall-pressure peak and the non-finite latch. */
int lbm_init_density(void *handle, const void *d_rho, double rho_l, double rho_g);

/* Enqueues n >= 0 timesteps (Eqs. 15, 13, 7, 6, 4, 14, 3, 5).  Asynchronous.
 * LBM_ESTATE while the handle is attached to a batch (step the batch) or has
 * no state yet; LBM_ENONFINITE once the latch has been read as set.
 * Results are deterministic: the same state and step counter give the same
 * bits with every tile variant, alone or in any batch.  In binary32 the rest
 * population of every site is rounded stochastically, from a hash of the
 * site and the step counter, so that each site keeps its mass on average;
 * a state restored with its step counter (lbm_load) therefore steps
 * bitwise as the original, while lbm_set_populations (which resets the
 * counter) may differ from it in the last bits. */
int lbm_step(void *handle, int64_t n);

/* Macroscopic fields of the current state and the diagnostics.  d_rho, d_ux,
 * d_uy: device arrays of nx*ny values in the handle's population precision
 * (binary32 for both binary32 modes), row-major [y][x]; d_p: nx*ny binary64
 * values of Eq. 15.  Any of the four may be NULL.  out may be NULL.
 * Synchronises the stream; returns LBM_ENONFINITE if the latch is set. */
int lbm_macros(void *handle, void *d_rho, void *d_ux, void *d_uy, void *d_p,
               lbm_diag *out);

/* Copies the current post-streaming populations to / from a device buffer of
 * 9*nx*ny values in the population precision, layout f[a][y][x].  Asynchronous.
 * The state is stored internally as deviations g_a = f_a - w_a rho_ref from the
 * rest equilibrium of a reference density (rho_l of the last lbm_init_bubble
 * or lbm_init_density, 0 for a handle never initialised); these calls convert,
 * so the buffer holds plain populations f_a.  lbm_set_populations keeps the
 * current reference and resets the step counter and the latch like an init. */
int lbm_get_populations(void *handle, void *d_out);
int lbm_set_populations(void *handle, const void *d_in);

/* Checkpoint: lbm_checkpoint_bytes gives the size of a host image holding the
 * populations, the step counter, the wall-pressure peak and the init
 * parameters; lbm_save writes it (synchronises), lbm_load restores it into a
 * handle created with the same parameters. */
int lbm_checkpoint_bytes(void *handle, size_t *bytes);
int lbm_save(void *handle, void *host_buf, size_t bytes);
int lbm_load(void *handle, const void *host_buf, size_t bytes);

/* Synchronises the stream and reports LBM_ENONFINITE if the latch is set. */
int lbm_sync(void *handle);
/* Non-blocking completion query: *done = 1 when all work enqueued for the
 * handle (on the batch's stream while it is attached) has finished, 0 while
 * some is pending.  Does not read the non-finite latch (lbm_sync does). */
int lbm_poll(void *handle, int *done);

/* Releases the handle's host metadata and graphs (not the caller's memory). */
void lbm_destroy(void *handle);

/* Static text for a status code. */
const char *lbm_strerror(int status);

/* ---- batching: many instances stepped by one launch per pass -------------- */

/* Tiles an instance with these parameters contributes to a batch work-list
 * at most (the count for the smallest tile shape). */
int lbm_tile_count(const lbm_params *params, int64_t *max_tiles);

/* Device workspace a batch of at most max_instances instances and max_tiles
 * tiles (sum of lbm_tile_count) needs, in bytes. */
int lbm_batch_workspace_bytes(int max_instances, int64_t max_tiles, size_t *bytes);

/* A batch steps every attached instance together: each pass is one launch
 * over a work-list of tiles drawn from all instances, and a chunk of steps is
 * replayed from a captured HIP graph.  All instances of a batch share one
 * precision and the batch's stream (an attached instance's own stream is not
 * used until it is detached).  The caller owns the batch workspace (256-byte
 * aligned) as for lbm_create.  Results are bitwise those of stepping each
 * instance alone. */
int lbm_batch_create(int precision, int max_instances, int64_t max_tiles, void *d_workspace,
                     size_t ws_bytes, void *hip_stream, void **batch);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call hipMalloc, harnesses that forbid
 * it): a batch like lbm_batch_create's whose workspace (instance
 * descriptors, tile work-list, latch copies) is the library's own static
 * device array instead of a caller-owned buffer, and which allocates
 * nothing: no device or pinned host memory, no captured graphs (its chunks
 * are launched directly), so every later call on it (attach, step, status,
 * destroy) allocates nothing either.  Descriptor and tile uploads, which
 * happen only when the batch changes, are copies from host memory that
 * complete before the call returns.  The instances themselves keep their
 * caller-owned workspaces (lbm_create).
 *
 * Limits: max_instances <= LBM_STATIC_MAX_INSTANCES and max_tiles <=
 * LBM_STATIC_MAX_TILES (LBM_ENOMEM beyond them); the array holds about
 * 1.1 MB on every device the library runs on, until the process ends.  One
 * such batch per device at a time: the array is shared by every call on
 * that device and keeps the last batch's contents, so a second
 * lbm_batch_create_static on the device returns LBM_ESTATE until the first
 * is destroyed (work of a destroyed batch still in flight on another stream
 * would race with the new one: destroy synchronises the batch's stream).  The
 * device is the current one; hip_stream must belong to it.  Results are
 * bitwise those of lbm_batch_create's batch. */
#define LBM_STATIC_MAX_INSTANCES 64
#define LBM_STATIC_MAX_TILES 65536
int lbm_batch_create_static(int precision, int max_instances, int64_t max_tiles, void *hip_stream,
                            void **batch);
int lbm_batch_attach(void *batch, void *handle);
int lbm_batch_detach(void *batch, void *handle);
/* n steps of every attached instance.  Asynchronous.  LBM_ENONFINITE, with
 * nothing enqueued, if an instance that would step has a latched non-finite
 * state (detach it first). */
int lbm_batch_step(void *batch, int64_t n);
/* Same, for a per-instance count: counts[i] steps for the i-th attached
 * instance (attach order); instances with fewer steps finish first and stay
 * unchanged afterwards.  Asynchronous. */
int lbm_batch_step_each(void *batch, const int64_t *counts, int n_counts);
/* Readies the batch for a following lbm_batch_step(batch, n): the descriptors
 * of the attached instances and the tile list are sent to the device as that
 * call needs them, and the HIP graphs of its chunks (the time integration of
 * Eq. 5 repeated, up to 256 steps per graph) are captured, instantiated and
 * uploaded.  Enqueues transfers but no kernel and does not advance the state.
 * The step then enqueues nothing but its graph launches, as long as nothing
 * that changes the batch (attach, detach, variant, initialisation, another
 * step count) comes between the two calls; otherwise the step does the
 * missing work itself.  Meant for timing and for latency-critical loops.
 * LBM_EINVAL for a null batch or n < 0; LBM_ENOMEM if the tiles exceed the
 * batch's max_tiles. */
int lbm_batch_prepare(void *batch, int64_t n);
int lbm_batch_size(void *batch, int *n_attached);
/* Non-blocking completion query of the batch's stream, as lbm_poll. */
int lbm_batch_poll(void *batch, int *done);
/* The non-finite latch of every attached instance as of the end of the last
 * chunk the batch stepped, in attach order, read in one transfer after the
 * batch's stream has drained: nonfinite[i] = 1 for a latched instance (which
 * then refuses further steps, alone or in a batch, until it is
 * re-initialised), 0 otherwise.  n is the length of nonfinite and must be at
 * least lbm_batch_size.  Synchronises the batch's stream. */
int lbm_batch_status(void *batch, int *nonfinite, int n);
void lbm_batch_destroy(void *batch);

/* ---- kernel variants and measurement -------------------------------------- */

/* Number of tile-shape variants and a short name for each. */
int lbm_variant_count(void);
const char *lbm_variant_name(int variant);
/* Blocks (tiles) of a fused variant's kernel that the current device holds at
 * once in the given precision mode, from the runtime's occupancy query, made
 * once per process at the first lbm_create or lbm_batch_create (0 before that,
 * and for the two-pass variants).  A fused launch whose tiles fit walks every
 * other band of tiles downwards, so that vertically neighbouring tiles, which
 * then run side by side, read their shared rows at the same time; a larger
 * launch walks every tile upwards.  Results do not depend on the walk.
 * LBM_EINVAL for an unknown variant or precision or a null blocks. */
int lbm_resident_blocks(int precision, int variant, int *blocks);
/* Selects the tile-shape variant a handle or a batch launches.  Results are
 * bitwise the same for every variant except the paired ones ("fused2-*"),
 * whose compiler contracts a few products differently (last-bit differences,
 * within 1e-14 relative in binary64 per step).  The paired variants need an even
 * nx for every instance: LBM_EINVAL otherwise, also from lbm_batch_attach of
 * an odd-nx instance to a batch using one; the autotuner skips them then. */
int lbm_set_variant(void *handle, int variant);
int lbm_batch_set_variant(void *batch, int variant);
/* on = 1: the fused single-pass kernel of the 64-column variants ("fused-*")
 * and the two-step kernel ("twostep-*", its stores to memory) store the
 * batch's populations with write-through stores (relaxed
 * agent-scope atomic stores, which leave no dirty line in the XCD's L2);
 * 0 (the default): ordinary stores.  Results are bitwise the same.  Every
 * kernel end writes back the dirty L2 lines of the whole device, so when
 * several batches run concurrently on their own streams (each launch's end
 * then also writes back the others' lines) write-through pays; a batch
 * running alone is faster without it on grids that stream from HBM, and can
 * be faster with it on grids that stay in the caches
 * (lbm_batch_tune_write_through decides by timing).  The paired and two-pass
 * variants ignore the setting.  LBM_EINVAL for a null batch or on not 0 or
 * 1. */
int lbm_batch_set_write_through(void *batch, int on);
/* Times the batch's current variant with write-through stores off and on, in
 * three passes of min(reps, 8) warm-up steps and reps timed steps each, and
 * keeps the setting with the fastest pass: *on the setting kept,
 * *ms_per_step (may be null) its time per step.  For variants that ignore the
 * setting nothing is timed: *on is the current setting, *ms_per_step NaN.
 * Which is faster depends on the workload: write-through pays where the
 * populations stay in the caches (the 24-instance 256 x 256 sweep, also as one
 * batch with the two-step kernel) and costs where they stream from HBM (an
 * 8192 x 4096 grid).  It advances the instances' state.  LBM_EINVAL for a
 * null batch or out pointer or reps < 1, LBM_ESTATE for an empty batch. */
int lbm_batch_tune_write_through(void *batch, int reps, int *on, float *ms_per_step);
/* Times every variant on the batch's current instances with HIP events, in
 * three passes of min(reps, 8) warm-up steps and reps timed steps each, scores
 * each variant by its fastest pass, selects the best and returns it with its
 * time per step.  It advances the instances' state (call it on throwaway
 * state or before initialising). */
int lbm_batch_autotune(void *batch, int reps, int *best_variant, float *ms_per_step);
/* Runs n steps of the batch with a HIP event pair around every kernel launch
 * and returns the summed device time per kernel kind (ms has 2 entries):
 * two-pass variants ms[0] density/psi pass, ms[1] force+collide+stream pass;
 * single-pass variants ms[0] = 0, ms[1] the whole step. */
int lbm_batch_step_timed(void *batch, int64_t n, float *ms);
int lbm_step_timed(void *handle, int64_t n, float *ms);

/* ---- host helpers (no device work) ---------------------------------------- */

/* Critical point of Eq. 15: dp/drho = d2p/drho2 = 0.  Host only. */
int lbm_critical_point(double a, double b, double R, double *T_c, double *rho_c,
                       double *p_c);

/* Spinodal densities of Eq. 15 at temperature T < T_c: the gas-side local
 * maximum and the liquid-side local minimum of p(rho) (dp/drho = 0), between
 * which Eq. 15 is mechanically unstable.  LBM_EINVAL at or above T_c.  Host
 * only. */
int lbm_spinodals(double a, double b, double R, double T, double *rho_sg,
                  double *rho_sl);

/* Coexisting gas and liquid densities of Eq. 15 at temperature T < T_c by the
 * Maxwell rule (Eq. 11), solved as equal pressure and equal chemical
 * potential.  Host only. */
int lbm_maxwell(double a, double b, double R, double T, double *rho_g,
                double *rho_l, double *p0);

/* Coexisting densities of the lattice model with Li's term predicted by the
 * mechanical-stability condition of Eq. 9 for a flat interface,
 * int (p0 - p) psi' / psi^(1+eps) drho = 0 between rho_g and rho_l with
 * p(rho_g) = p(rho_l) = p0 and psi of Eq. 13 (c = 1, c_s^2 = 1/3, G < 0).
 * eps = 0 is the condition without Li's term.  LBM_EINVAL when no pressure
 * satisfies it (e.g. eps = 1 below about 0.7 T_c).  Host only. */
int lbm_mechanical_stability(double a, double b, double R, double T, double G, double eps,
                             double *rho_g, double *rho_l, double *p0);

/* Plain device-to-device copy kernel of n bytes (n a multiple of 16) on a
 * stream, for calibrating the memory-traffic counters against a known byte
 * count.  Asynchronous. */
int lbm_copy_kernel(void *d_dst, const void *d_src, size_t n, void *hip_stream);

/* The current device's constant-rate clock: *tick its present value (read by
 * a one-thread kernel, waited for), *rate_hz its frequency.  Synchronous.
 * With lbm_hold_until, for timing work on several streams from one common
 * instant. */
int lbm_device_clock(uint64_t *tick, uint64_t *rate_hz);

/* Enqueues on a stream a one-thread kernel that waits until the device clock
 * (lbm_device_clock) reaches `tick`, or for at most `max_ticks` from its own
 * start (at most one second's worth; LBM_EINVAL beyond), so that holds with
 * the same `tick` on several streams release their streams together, however
 * far apart the host enqueued them.  Asynchronous. */
int lbm_hold_until(uint64_t tick, uint64_t max_ticks, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
