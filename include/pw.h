/*
 * pw.h - C ABI of the MI355X multipatch scalar-wave library (libpw).
 *
 * The library advances the scalar wave system of "PatchworkWave" (Bowen et al.,
 * arXiv 2002.00088) on one global patch (id 0) plus any number of moving local
 * patches, one classic-RK4 step at a time, on one AMD Instinct MI355X (gfx950).
 *
 * State vector per patch (Sec. 2.2, Eqs. eom1-eom3): u = [phi, Pi_t, Pi_1, Pi_2, Pi_3],
 * the one-form Pi_mu = d_mu phi in the patch's own numerical coordinates.
 *
 * Conventions common to every call
 *   - Host arrays of patch data are interior-only, FP64, laid out [5][n2][n1][n0]
 *     with n0 fastest (field-major).  They are copied in or out; the library never
 *     keeps a caller pointer.
 *   - Ownership: the library owns all device memory.  It allocates through the
 *     caller's allocator callbacks when given (pw_config.dev_alloc/dev_free), else
 *     with hipMalloc.  It runs every kernel on the caller's stream (pw_config.stream,
 *     a hipStream_t; if NULL the library creates and owns a non-blocking stream).
 *     The caller owns host arrays and its stream, and must keep the stream alive
 *     until pw_destroy.
 *   - Errors: every call returns a pw_status; < 0 is an error and pw_last_error()
 *     returns a message.  No C++ exception crosses the ABI.  A context is not
 *     thread-safe; calls on one context must not overlap.
 *   - Synchronisation: calls that return data to the host (pw_get_state with a
 *     host destination, pw_get_flags, pw_diagnostics, pw_counters) synchronise the
 *     stream.  pw_rk4_step and pw_exchange_ghosts only enqueue work.
 */
#ifndef PW_H
#define PW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pw_context pw_context; /* opaque, library-owned */
typedef int32_t pw_status;

enum {
  PW_OK = 0,
  PW_EINVAL = -1,   /* bad argument or configuration */
  PW_ENOMEM = -2,   /* device or host allocation failed */
  PW_EDEVICE = -3,  /* a HIP runtime call failed */
  PW_ESTATE = -4,   /* call not valid in the current state (e.g. no global patch) */
  PW_EOVERLAP = -5, /* two local patches cover a global cell that is not live (Sec. 2.4.2) */
  PW_EMOTION = -6   /* a patch moves max(1, buffer_width - NG) global cells or more within a
                       step: the NG+1 buffer covers one cell of motion per step and a wider
                       buffer relaxes the bound (Sec. 2.4.2) */
};

enum { PW_FP64 = 0, PW_MIXED = 1, PW_MIXED_INC = 2 }; /* precision */
enum { PW_CART = 0, PW_SPH = 1, PW_CYL = 2 };  /* patch topology */
enum { PW_STATIC = 0, PW_LINEAR = 1, PW_CIRCLE = 2 }; /* patch motion */
enum { PW_FLAG_LIVE = 0, PW_FLAG_EFFGHOST = 1, PW_FLAG_DEACT = 2 }; /* cover flags */
enum { PW_SCHED_BATCHED = 0, PW_SCHED_PER_PATCH = 1 };
enum { PW_EXACT_NONE = 0, PW_EXACT_PLANE = 1, PW_EXACT_GAUSS = 2 };

enum { PW_FORM_PAPER = 0, PW_FORM_FIRST_ORDER = 1 };  /* form of the Pi_t equation */
enum { PW_BC_EXACT = 0, PW_BC_SOMMERFELD = 1 };        /* outer boundary of the global patch */

#define PW_MAX_SV 4
#define PW_MAX_PULSES 32

/*
 * Library configuration.
 *   precision        PW_FP64: every array and operation FP64.  PW_MIXED: FP64 state
 *                    u_n, FP64 RK accumulator, FP64 donor location, Lagrange weights
 *                    and frame Jacobians; FP32 stage inputs, FP32 stencil arithmetic
 *                    (an FP32 copy of u_n feeds the first stage).  Interpolation: the
 *                    weights are formed in FP64; the x-row sums run in FP32 with the x
 *                    weights rounded to FP32 once, and the rows and layers are combined
 *                    with the FP64 y and z weights in FP64.
 *                    Accuracy of PW_FP64 against a plain FP64 evaluation of the same
 *                    scheme: per field, max |difference| over live cells below 1e-12
 *                    of the field's largest magnitude there; the one-form components
 *                    Pi_t, Pi_x, Pi_y, Pi_z, which the frame transforms mix, share one
 *                    magnitude (their largest), since a component that is small next
 *                    to the others carries their rounding.
 *                    PW_MIXED_INC: as PW_MIXED, but the accumulator carries the
 *                    increment dt sum_l b_l K_l (Table rk4) in FP32 and
 *                    u_{n+1} = u_n + increment + b_4 dt K_4 is formed in FP64.
 *   n_state_vectors  1..4 independent state vectors sharing maps and cover flags
 *                    (multiple state vectors, Sec. 1.1); each has its own wave speed
 *                    (d'Alembertian Lap - v^-2 d_t^2) and interpolation order.
 *   interp_points    points P per axis of the tensor-product Lagrange stencil, 2..6
 *                    (order P-1).  6 is the paper's stencil i_c-2..i_c+3 (Sec. 2.4,
 *                    Eq. Pijk); the stencil starts at floor(q - (P-2)/2) for the
 *                    fractional cell index q, so 5 centres on the nearest node and 2 is
 *                    linear interpolation between the two neighbouring nodes.
 *   buffer_width     live buffer under each local patch edge: 4 = NG+1 is the paper's
 *                    (Sec. 2.4.2).  1..3 is the ablation of the original Patchwork flags:
 *                    global->local stencils may then reach effective ghost cells, so each
 *                    stage fills the effective ghosts first and the local ghosts from them
 *                    (interpolation of interpolated data).  At most 16.
 *   ko_eps           Kreiss-Oliger strength (0.005 in the paper, Sec. 2.3).
 *   schedule         PW_SCHED_BATCHED: each RK stage is one launch over all patches
 *                    and the step is captured in a HIP graph when use_graph != 0.
 *                    PW_SCHED_PER_PATCH: one stencil launch per patch per stage, no graph.
 *   stream           hipStream_t of the caller (NULL: a stream owned by the library).
 *   dev_alloc/free   optional device allocator; alloc_user is passed back unchanged.
 *   pi_form          PW_FORM_PAPER (0): the Pi_t equation as in Sec. 2.2, Eqs. eom1-eom3,
 *                    with second differences of phi (g^ij d_i d_j phi, C^i d_i phi).
 *                    PW_FORM_FIRST_ORDER (1): its first-order reduction, the evolved
 *                    Psi_i = Pi_i in place of d_i phi and d_i Psi_j in place of
 *                    d_i d_j phi (Pi_t' = d_i Psi^i on a static Cartesian patch).
 *   outer_bc         PW_BC_EXACT (0): the outer ghosts of the global patch hold the
 *                    registered exact solution (the paper's analytic BCs, Sec. 3), or a
 *                    copy of the nearest interior cell if none is registered.
 *                    PW_BC_SOMMERFELD (1): the outer ghosts are evolved with the state by
 *                    the radiative condition d_t u = -v (X.grad u + u)/r for waves leaving
 *                    the origin (every field, asymptotic value 0; 4th-order centred
 *                    derivatives along interior axes, 2nd-order one-sided inward along
 *                    ghost axes).  They start from the PW_BC_EXACT value at the first
 *                    step after the state is set.  Needs a non-periodic Cartesian global patch.
 */
typedef struct {
  int32_t precision;
  int32_t n_state_vectors;
  double wave_speed[PW_MAX_SV];
  int32_t interp_points[PW_MAX_SV];
  int32_t buffer_width;
  double ko_eps;
  int32_t schedule;
  int32_t use_graph;
  void *stream;
  void *(*dev_alloc)(uint64_t bytes, void *user);
  void (*dev_free)(void *ptr, void *user);
  void *alloc_user;
  int32_t pi_form;
  int32_t outer_bc;
} pw_config;

/*
 * Patch description (Secs. 2.1 and 2.4.1): numerical box [lo,hi] of n cells per axis
 * (cell-centred), topology map M (Cartesian identity; spherical x' = (r,theta,phi),
 * M = r (sin th cos ph, sin th sin ph, cos th); cylindrical x' = (r,phi,z),
 * M = (r cos ph, r sin ph, z); Secs. 2.1, 3.3 and 3.4),
 * orientation R(t) and centre motion c(t), so that the background Cartesian
 * coordinates are X_B = c(t) + R(t) M(x').
 *   motion PW_STATIC: c = c0; PW_LINEAR: c = c0 + vel t;
 *          PW_CIRCLE: c = c0 + radius (cos(w t + phase), sin(w t + phase), 0), w = speed/radius.
 *   orientation R(t) = Q(t) R0: R0 the ZYZ Euler rotation euler_zyz, Q(t) the rotation
 *          by |spin| t about spin/|spin| (a patch rotating about its centre with
 *          angular velocity spin, background frame; spin = 0: R(t) = R0).
 *   periodic[a]: axis a wraps (the phi axis of a spherical or cylindrical patch, which
 *          must then span 2 pi; every axis of a periodic global box).  A curvilinear
 *          patch keeps its ghosts off r = 0 (and a spherical one off the poles);
 *          phi values of a non-periodic phi axis lie in (-pi, pi].
 *   sv_mask: bit s set if the patch carries state vector s.
 * The first patch created must be the global one (is_global = 1, static, unrotated,
 * centred at the origin, no spin): Cartesian, or spherical with phi as its only
 * periodic axis (Sec. 3.4).  Every later patch is a local patch.  Local patches may
 * overlap where the global cells stay live (in the buffers); a global cell covered
 * by two local patches keeps the lower id, and an overlap that reaches a non-live
 * global cell is PW_EOVERLAP.
 */
typedef struct {
  int32_t coord;
  int32_t is_global;
  int32_t n[3];
  double lo[3], hi[3];
  int32_t periodic[3];
  double euler_zyz[3];
  int32_t motion;
  double c0[3], vel[3];
  double radius, speed, phase;
  uint32_t sv_mask;
  double spin[3];
} pw_patch_desc;

/*
 * Exact solution of one state vector in the background frame, used for initial
 * data, the analytic outer boundary (Sec. 3: analytic BCs at the global edge) and
 * error norms.
 *   PW_EXACT_PLANE: phi = amp sin(kappa.X - v|kappa| t + phase) + offset  (Eq. wave_solution)
 *   PW_EXACT_GAUSS: sum of spherical pulses with phi(0) = A exp(-|X-x_c|^2/w^2), d_t phi(0) = 0.
 */
typedef struct {
  int32_t kind;
  double amp, offset, kappa[3], phase;
  int32_t n_pulses;
  double pulse_amp[PW_MAX_PULSES];
  double pulse_center[PW_MAX_PULSES][3];
  double pulse_width[PW_MAX_PULSES];
} pw_exact_desc;

/*
 * Diagnostics of one patch and state vector over its live cells (all interior cells
 * of a local patch; cells flagged PW_FLAG_LIVE on the global patch).
 *   max_abs/sum_sq:          per field
 *   err_max/err_sum_sq:      per field, against the registered exact solution (0 if none)
 *   int_rel_err:             sum over live cells of |phi - phi_e| / |phi_e| sqrt(gamma) d^3x'
 *                            (Sec. 3.2, with sqrt(gamma) = |det dX/dx'| the volume element)
 *   live_cells, volume:      live cell count and sum of sqrt(gamma) d^3x'
 *   energy:                  1/2 sum (Pi_t^2 - v^2 phi L phi) dx0 dx1 dx2, L the sum of the
 *                            4th-order second differences along the numerical axes (the
 *                            discrete energy of a static Cartesian patch)
 *   constraint_max:          max |Pi_a - D_a phi|, a = 1..3 (the constraint Psi_a = d_a phi
 *                            of the first-order system, 4th-order D_a)
 *   energy and constraint_max run over the live cells whose +-2 stencils along each
 *   numerical axis reach live interior cells only (periodic axes wrap).
 */
typedef struct {
  double max_abs[5];
  double sum_sq[5];
  double err_max[5];
  double err_sum_sq[5];
  double int_rel_err;
  double live_cells;
  double volume;
  double energy;
  double constraint_max[3];
} pw_diag;

/*
 * Skip and event counters since creation (Secs. 2.4.1-2.4.2: points that cannot be
 * interpolated are skipped and keep their lower-priority value).
 *   skip_local:   local ghost points whose global donor stencil was not all live
 *   skip_eff:     global effective ghosts whose local donor stencil left the interior
 *   skip_uncover: cells that became live at a step end and could not be interpolated
 *   n_uncover:    cells that became live at a step end
 *   steps:        RK4 steps taken
 *   skip_outer:   covered physical ghost cells of the global patch (outer ghosts
 *                 that are not periodic copies, lying in a local patch; Sec. 2.4.2,
 *                 last paragraph) whose local stencil left the interior: they keep
 *                 their boundary value
 *   n_outer:      covered physical ghost cells filled or attempted, summed over
 *                 ghost fills and state vectors
 */
typedef struct {
  int64_t skip_local, skip_eff, skip_uncover, n_uncover, steps;
  int64_t skip_outer, n_outer;
} pw_counters_t;

/* Create a context.  cfg is copied.  *out receives the context on success.
 * Validation switch: with the environment variable PW_L2G_DIRECT set to "1"
 * when the context is created, every local->global interpolation point gathers
 * its stencil straight from global memory (the path otherwise taken only by a
 * work item whose donor box cannot be staged in LDS); the results are the same
 * bitwise, the step is slower. */
pw_status pw_create(const pw_config *cfg, pw_context **out);

/* Add a patch; the first one is the global patch.  *id_out receives its id
 * (0 for the global patch, 1.. for local patches).  Allocates its device buffers.
 * PW_EINVAL if an axis has more than 1017 cells or the five padded fields of the
 * patch ([n2+6][n1+6][row pitch]) hold 2^32 elements or more (about 925^3 cells). */
pw_status pw_create_patch(pw_context *ctx, const pw_patch_desc *desc, int32_t *id_out);

/* Register the exact solution of state vector sv (copied). */
pw_status pw_set_exact(pw_context *ctx, int32_t sv, const pw_exact_desc *ex);

/* Set every patch's interior to its registered exact solution at time t0
 * (in the patch's frame) and set the current time to t0. */
pw_status pw_init_exact(pw_context *ctx, double t0);

/* Copy n_elems = 5*n0*n1*n2 FP64 values of patch `patch`, state vector sv, into the
 * library (src on the host, or on the device if src_is_device) and set the current
 * time to t0.  Cover flags are recomputed before the next step. */
pw_status pw_set_state(pw_context *ctx, int32_t patch, int32_t sv, const double *src, int64_t n_elems,
                       int32_t src_is_device, double t0);

/* Copy the interior of u (FP64) of patch/sv out, layout as pw_set_state. */
pw_status pw_get_state(pw_context *ctx, int32_t patch, int32_t sv, double *dst, int64_t n_elems,
                       int32_t dst_is_device);

/* pw_get_state into host memory for callers that cannot allocate device memory
 * (code that must not call hipMalloc: tight serving loops, harnesses that forbid
 * it).  Same arguments and layout as pw_get_state with a host destination; it
 * calls no allocator.  The state is staged through a static device array of
 * 4 Mi FP64 values (32 MiB) per GPU, held from library load until the process
 * ends: PW_EINVAL if 5*n0*n1*n2 exceeds 4194304 (use pw_get_state), PW_ESTATE
 * if the patch layout is not on the device yet (any earlier pw_init_exact,
 * pw_set_state, pw_get_state or pw_rk4_step puts it there).  Synchronises the
 * stream.  All contexts on one GPU share the array: calls that overlap on one
 * GPU (from several threads or streams) race. */
pw_status pw_get_state_noalloc(pw_context *ctx, int32_t patch, int32_t sv, double *dst, int64_t n_elems);

/* Copy u including ghost cells, [5][n2+6][n1+6][n0+6] FP64, to host memory. */
pw_status pw_get_state_full(pw_context *ctx, int32_t patch, int32_t sv, double *dst, int64_t n_elems);

/* Copy the cover flags (PW_FLAG_*, one byte per global interior cell, [n2][n1][n0])
 * and, if cover != NULL, the id of the covering local patch or -1 (Sec. 2.4.2).
 * Computes them first if the state changed since the last step. */
pw_status pw_get_flags(pw_context *ctx, uint8_t *flags, int32_t *cover, int64_t n_cells);

/* Fill the ghost cells of u at time t in the order boundary -> periodic ->
 * interpatch (Sec. 2.4, Fig. BC_order): analytic outer ghosts (or nearest copy),
 * periodic copies, then global->local and local->global interpolation with the
 * frame transform through the background frame (Secs. 2.4.1-2.4.2).  Outer
 * ghost cells of the global patch that lie in a local patch are local->global
 * targets too, over their boundary value (Sec. 2.4.2, last paragraph; not with
 * PW_BC_SOMMERFELD, which evolves them). */
pw_status pw_exchange_ghosts(pw_context *ctx, double t);

/* Advance nsteps classic-RK4 steps of size dt (Sec. 2.3, Table rk4): per stage a
 * ghost fill of the stage input at t_n + c_s dt, then the RHS of Eqs. eom1-eom3
 * with Kreiss-Oliger dissipation and the stage update on every live cell.  Cover
 * flags are computed at t_n and frozen for the step, maps follow the substep times,
 * and cells that become live at the step end are interpolated from the covering
 * local patch (Sec. 2.4.2).  Returns PW_EMOTION before launching if a patch
 * would move max(1, buffer_width - 3) global cells or more in one step,
 * PW_EOVERLAP if two local patches cover one global cell that is not live.
 * nsteps = 0 advances nothing (the flags, outer ghosts and step graph may be
 * prepared); nsteps < 0 or dt <= 0 (or NaN): PW_EINVAL. */
pw_status pw_rk4_step(pw_context *ctx, double dt, int32_t nsteps);

/* Run-time tuning parameters.  None changes a computed value: every setting
 * evaluates the same arithmetic per cell and per ghost point. */
typedef struct {
  int32_t tile_z_global; /* planes per workgroup of the stage kernel, global patch (1..512) */
  int32_t tile_z_local;  /* the same for local patches (1..512) */
  int32_t g2l_run;       /* consecutive local-ghost bricks dealt to one XCD (1..64) */
  int32_t l2g_run;       /* consecutive 64-entry effective-ghost groups dealt to one XCD (1..64) */
  int32_t global_order;  /* how the global patch's stage tiles are dealt to the eight XCDs
                            (each has its own L2): PW_ORDER_BANDS (0) eight bands of tile
                            rows, PW_ORDER_OCTANTS (1) the eight octants of the index box,
                            whose shared faces, read from two L2s, are smaller */
  int32_t chain;         /* where the stage kernels of the curvilinear local patches run in
                            the two-stream step: PW_CHAIN_GLOBAL (0) on the global chain
                            after the global stage kernel, PW_CHAIN_LOCAL_AFTER (1) on the
                            local chain after the Cartesian local patches,
                            PW_CHAIN_LOCAL_BEFORE (2) on the local chain before them */
  int32_t local_tile;    /* columns per workgroup of the stage kernel on local patches:
                            PW_TILE_32X8 (0) or PW_TILE_16X16 (1) */
  int32_t global_tile;   /* the same on the global patch: PW_TILE_32X8 (0),
                            PW_TILE_128X4 (1, 512 threads) or PW_TILE_128X8 (2, 512
                            threads, two rows of the tile per thread; PW_MIXED and
                            PW_MIXED_INC only, PW_EINVAL under PW_FP64) */
} pw_tuning;
enum { PW_ORDER_BANDS = 0, PW_ORDER_OCTANTS = 1 };
enum { PW_CHAIN_GLOBAL = 0, PW_CHAIN_LOCAL_AFTER = 1, PW_CHAIN_LOCAL_BEFORE = 2 };
enum { PW_TILE_32X8 = 0, PW_TILE_16X16 = 1, PW_TILE_128X4 = 1, PW_TILE_128X8 = 2 };

/* Current tuning parameters. */
pw_status pw_get_tuning(pw_context *ctx, pw_tuning *out);

/* Set the tuning parameters (PW_EINVAL if one is out of range).  The tile lists
 * are rebuilt and the next pw_rk4_step re-captures its graph. */
pw_status pw_set_tuning(pw_context *ctx, const pw_tuning *t);

/* Autotuner: times candidate settings on this context's own patches with HIP
 * events over steps_per_trial steps of size dt each (after one untimed step),
 * searching the two tile depths and the global tile order on a grid, then the
 * other global tile shapes (128x8 in the mixed modes only) with the global tile
 * depths, the place of the curvilinear local stage kernels, the local tile shape
 * with the local tile depths and the two run lengths, and keeps the fastest
 * (written to *best unless best is NULL).  It advances the state and
 * the time by every step it takes, so call it before setting the initial data
 * (or set it again afterwards).  On an error the previous settings are restored. */
pw_status pw_autotune(pw_context *ctx, double dt, int32_t steps_per_trial, pw_tuning *best);

/* Current coordinate time. */
pw_status pw_get_time(const pw_context *ctx, double *t);

/* Diagnostics of one patch / state vector (synchronous). */
pw_status pw_diagnostics(pw_context *ctx, int32_t patch, int32_t sv, pw_diag *out);

/* Counters (synchronous). */
pw_status pw_counters(pw_context *ctx, pw_counters_t *out);

/* Number of live cells evolved per step summed over patches and state vectors
 * (synchronous; uses the current cover flags). */
pw_status pw_live_cells(pw_context *ctx, int64_t *out);

/* Kernel classes timed by pw_kernel_times. */
enum {
  PW_K_POSE = 0,
  PW_K_GHOST_S1 = 1, /* ghost fill of stage s (s = 1..4): PW_K_GHOST_S1 + s - 1 */
  PW_K_STAGE_S1 = 5, /* RHS + RK update of stage s: PW_K_STAGE_S1 + s - 1 */
  PW_K_FLAGS = 9,    /* cover flags at t_{n+1} */
  PW_K_FINALIZE = 10, /* uncover fill, poison, flag swap */
  PW_K_GSTAGE_S1 = 11, /* the global patch's launch within PW_K_STAGE_S1 + s - 1: PW_K_GSTAGE_S1 + s - 1 */
  PW_K_G2L = 15,       /* the global -> local interpolation kernel within a ghost fill (every stage) */
  PW_K_L2G = 16,       /* the local -> global interpolation kernel within a ghost fill (every stage) */
  PW_K_NCLASS = 17
};

/* Enable (on != 0) or disable per-kernel-class timing.  While enabled, steps run
 * without the graph and every kernel class is bracketed by hipEvents on the
 * library's stream; totals accumulate until pw_kernel_times resets them. */
pw_status pw_enable_timing(pw_context *ctx, int32_t on);

/* Copy the accumulated time (ms) and launch-group count of every kernel class
 * (arrays of PW_K_NCLASS entries), then reset them (synchronous). */
pw_status pw_kernel_times(pw_context *ctx, double *total_ms, int64_t *count);

/* Message of the last error on this context (never NULL). */
const char *pw_last_error(const pw_context *ctx);

/* Free all device memory and the context.  NULL is ignored. */
void pw_destroy(pw_context *ctx);

#ifdef __cplusplus
}
#endif
#endif /* PW_H */
