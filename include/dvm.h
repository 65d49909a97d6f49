/*
 * dvm.h -- C ABI of the MI355X (gfx950) discrete-velocity solver for the
 * steady linearized BGK equation in 2-D staircase geometries.
 *
 * Method: Lindsay, Su, Liu & Wu, "Comparative study of the discrete velocity
 * and lattice Boltzmann methods for rarefied gas flows through irregular
 * channels" (arXiv:1704.03126):
 *   - linearized BGK equation, Sec. II.A, Eq. (BGK);
 *   - discrete velocities of Eq. (nonuniform_v);
 *   - source iteration of Eq. (iteration) with second-order upwind
 *     differences (text after Eq. (iteration));
 *   - diffuse walls, Eq. (diffuse2), on a staircase (Sec. II.A);
 *   - periodic inlet/outlet and the Poiseuille flow rate Q and apparent
 *     permeability k_a of Sec. III.
 *
 * Conventions shared by every call
 *   - All pointers passed in are HOST pointers unless stated otherwise.  The
 *     library copies what it needs during the call; the caller keeps
 *     ownership and no pointer is retained after the call returns.
 *   - Every device allocation is owned by the context and freed by
 *     dvm_destroy.
 *   - Grids are row-major (ny rows of nx cells), x (axis 1) is the flow
 *     direction and is always periodic.  One reference length H spans
 *     cells_per_H cells; the cell size is 1/cells_per_H.
 *   - Return values: 0 on success, a negative DVM_E* code on failure.  No
 *     exception or abort crosses the ABI; dvm_last_error() returns a message
 *     for the calling thread.  Argument checks run on the host before any
 *     device work, so a rejected call leaves the context unchanged.
 *   - Calls on one context are not thread-safe; distinct contexts are
 *     independent.  Work is issued on the stream given to dvm_create.
 */
#ifndef DVM_H
#define DVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DVM_OK 0
#define DVM_EINVAL (-1)     /* bad argument (message says which)              */
#define DVM_ENOMEM (-2)     /* device or host allocation failed               */
#define DVM_EHIP (-3)       /* a HIP runtime call failed                      */
#define DVM_ESTATE (-4)     /* call out of order (e.g. solve before geometry) */
#define DVM_ENOCONV (-5)    /* max_iter reached before the stop rule held     */
#define DVM_EDIVERGED (-6)  /* non-finite or growing iterates                 */

#define DVM_FP64 0          /* all sweeps in FP64                             */
#define DVM_FP32_REFINE 1   /* FP32 sweeps, FP64 moments + defect correction  */

#define DVM_SCHED_AUTO 0    /* wrap-around diagonal, skewed order for instances
                               whose iteration stops contracting (default)   */
#define DVM_SCHED_SKEW 1    /* sweep order with lags at periodic/strip seams only */
#define DVM_SCHED_WRAP 2    /* wrap-around diagonal: fewer steps on wide grids  */

#define DVM_ACCEL_AUTO 0    /* source iteration with extrapolation of the
                               dominant mode once its contraction rate has
                               settled (q <= 0.98; not part of the paper's
                               method); GMRES takes over an instance whose
                               iteration stops contracting, and is tried on
                               one that contracts slowly (q > 0.98 with over
                               150 iterations to go; 300 for the FP64 tails
                               of DVM_FP32_REFINE), kept while its cycles
                               together reduce the residual 1.5 x faster than
                               the plain iteration per unit of work (sweeps,
                               the orthogonalisation counted in sweep
                               equivalents: deterministic).  With
                               DVM_FP32_REFINE the FP32 correction iteration
                               is extrapolated the same way (where its
                               tolerance is far above the extrapolated FP32
                               rounding), and a correction that contracts
                               slowly (q > 0.98 with over 1000 iterations to
                               go) or not at all continues in GMRES whose
                               Krylov steps are FP32 sweeps (each cycle from
                               the FP64 residual)                            */
#define DVM_ACCEL_NONE 1    /* plain source iteration only (the paper's)      */
#define DVM_ACCEL_GMRES 2   /* restarted GMRES on the fixed-point map of the
                               iteration from the start.  Restarts are
                               deflated (see krylov_deflate); the instances of
                               a batch share the sweeps of each Arnoldi step
                               but each runs its own Arnoldi process, so a
                               batch gives every instance bitwise the result
                               of its own solve                               */

#define DVM_STATUS_RUNNING 0
#define DVM_STATUS_CONVERGED 1
#define DVM_STATUS_MAXITER 2
#define DVM_STATUS_DIVERGED 3

typedef struct dvm_ctx dvm_ctx; /* opaque, library-owned */

/* Solver settings.  A zero-initialised struct (or NULL) selects defaults. */
typedef struct {
    int precision;          /* DVM_FP64 (default) or DVM_FP32_REFINE          */
    double tol;             /* stop tolerance on the relative change of u1
                               between iterations (Sec. II.A uses 1e-5);
                               default 1e-8                                   */
    long max_iter;          /* iteration cap per solve; default 200000        */
    int block_iters;        /* iterations per captured launch block; 0 -> 32  */
    int use_graphs;         /* 1: replay blocks as HIP graphs; 0: plain launches */
    int vel_per_lane;       /* velocities per lane: 2, 4 or 8                 */
    int waves_per_block;    /* waves per workgroup: 4 or 8; supported pairs
                               (V, G): (4,8) (8,4) (4,4) (2,8).  Both 0: the
                               pair is chosen by timing a few sweeps of the
                               geometries at the first solve (per precision;
                               kept per process and in tune_cache)            */
    const char *tune_cache; /* autotune cache file (appended to) or NULL;
                               the string is copied                           */
    int profile;            /* 1: time every sweep launch with HIP events on
                               the context's stream (replaces graph replay);
                               read the totals with dvm_profile              */
    int schedule;           /* order of the cells within a sweep (the fixed
                               point does not depend on it):
                               DVM_SCHED_SKEW lags only the values that cross
                               periodic seams and 64-row strip boundaries, as
                               the paper's iteration lags its periodic seam,
                               at the price of 63 fill steps per pass;
                               DVM_SCHED_WRAP (grids with nx >= 8) sweeps a
                               wrap-around diagonal without fill steps but
                               also lags the y coupling along one diagonal
                               per strip, and the iteration can then diverge
                               (seen with a solid block inside a periodic
                               cell); DVM_SCHED_AUTO (default) starts every
                               instance on the wrap-around diagonal and moves
                               an instance that runs away there (relative
                               change of u1 not down by 5% over 64 iterations
                               while max |u1| grew by 10%, or non-finite
                               iterates) to the skewed order for good: the
                               layout is rebuilt, that instance's solve
                               restarts from zero and the other instances of
                               the call restart from their current state
                               (instances outside the call keep theirs)     */
    int accel;              /* DVM_ACCEL_AUTO (default), DVM_ACCEL_NONE or
                               DVM_ACCEL_GMRES.  GMRES drives the iteration's
                               state (moments, lagged seam, wrap and wall
                               values) with the same sweeps and reaches the
                               same fixed point; it converges where the lagged
                               iteration diverges.  AUTO hands an instance to
                               GMRES when its relative change of u1 has not
                               dropped by 0.5% over 64 iterations; a slowly
                               contracting one gets a GMRES trial (see
                               DVM_ACCEL_AUTO).  GMRES stop
                               rule: one iteration from the result changes u1
                               by eps (relative) with eps / sigma <= tol,
                               sigma the smallest singular value of the last
                               Krylov projection clamped to [1e-3, 1]         */
    int krylov_dim;         /* GMRES restart length; 0 -> 40 with deflated
                               restarts, 64 with plain ones (max 64); at large
                               delta (Kn 0.01-0.03) a plain restart of 30
                               stagnated                                     */
    int persistent;         /* 1: run each block of block_iters iterations
                               (FP64 forward and FP32 correction) as one
                               cooperative launch that stays resident: per
                               iteration the sweep's work items are drawn
                               from a device counter, then moments, records
                               and the stop rule run behind grid barriers,
                               with per-instance stop flags and iteration
                               counts on the device.  Results are bitwise
                               those of the separate launches.  Applies with
                               4 velocities per lane and 8 waves per
                               workgroup and without per-face specular or
                               gradient passes; other blocks (and profile =
                               1) use the separate launches.  0 (default):
                               separate launches, replayed as HIP graphs   */
    int krylov_deflate;     /* GMRES restarts with deflation (Morgan's
                               GMRES-DR): each cycle hands this many harmonic
                               Ritz vectors of its smallest harmonic Ritz
                               values, with its residual, to the next cycle,
                               whose Arnoldi steps extend that basis instead
                               of starting from the residual alone (the
                               slowest modes of the source iteration stay in
                               the Krylov space across restarts).  0 -> a
                               quarter of the restart length (10 of 40);
                               negative -> plain restarts; at most 31 and
                               krylov_dim/2 - 1; a complex pair is kept
                               whole (one more).  A cycle whose kept basis
                               cannot be formed to rounding restarts plainly */
    int warm_extrapolate;   /* 1: continuation for sweeps in delta.  After
                               each converged solve at a uniform delta the
                               library keeps the instance's state (two per
                               instance, device memory of two GMRES state
                               vectors); a warm solve (dvm_solve_warm) at a
                               new delta, same alpha, drive and walls, then
                               starts from the state extrapolated linearly in
                               log(delta) through the last two solutions, if
                               the step goes on in the same direction and at
                               most doubles.  Same fixed point, fewer
                               iterations.  0 (default): warm solves start
                               from the last state as it is                  */
} dvm_config;

/* Per-instance result of dvm_solve. */
typedef struct {
    long iters;             /* source iterations (FP64 + FP32 sweeps)         */
    long sweeps_fp64;       /* of which FP64 sweeps                           */
    double rel_change;      /* last relative change of u1                     */
    double est_error;       /* a-posteriori bound rel_change*r/(1-r)          */
    int status;             /* DVM_STATUS_*                                   */
    int schedule;           /* sweep order the solve ended in: DVM_SCHED_SKEW
                               or DVM_SCHED_WRAP                              */
} dvm_info;

/* Device allocator hooks of dvm_create: alloc(bytes, ud) returns device
 * memory of at least `bytes` bytes aligned to 256 bytes (NULL on failure, which
 * the calling entry point reports as DVM_ENOMEM); free_(ptr, ud) releases
 * it.  Both may be called from any entry point that touches the device
 * (dvm_solve, dvm_solve_warm, dvm_get_moments, dvm_grad) and from dvm_destroy,
 * on the calling thread.  Memory is used on the context's stream only. */
typedef void *(*dvm_alloc_fn)(size_t bytes, void *ud);
typedef void (*dvm_free_fn)(void *ptr, void *ud);

/* Create a context for n_instances independent problems sharing one
 * velocity grid of nv x nv nodes, Eq. (nonuniform_v) (nv even, 4 <= nv <= 128).
 * hip_stream: a hipStream_t, or NULL for a stream of the library's own.
 * alloc / free_ / alloc_ud: where every device buffer of the context comes
 * from (e.g. a framework's caching allocator); both NULL: hipMalloc/hipFree.
 * Exactly one of alloc and free_ NULL is DVM_EINVAL.  The context keeps the
 * two function pointers and alloc_ud (not dereferenced) until dvm_destroy.
 * On success *out receives the context; no device work happens here. */
int dvm_create(dvm_ctx **out, int nv, int n_instances, const dvm_config *cfg,
               void *hip_stream, dvm_alloc_fn alloc, dvm_free_fn free_,
               void *alloc_ud);

/* Describe instance `instance` (0-based): an nx x ny staircase geometry,
 * the "stair case" approximation of the solid surface of Sec. II.A (every
 * solid cell is a square of side 1 / cells_per_H; the faces it shares with
 * fluid cells are diffuse walls, Eq. (diffuse2)), with the periodic inlet and
 * outlet along x of Sec. II.A and Sec. III.
 *   solid[ny*nx]: host array, row-major (row y = 0 first), 1 = solid,
 *     0 = fluid; any other value is DVM_EINVAL.  Copied during the call.
 *   periodic_y: 1 for a periodic unit cell (the porous media of Sec. III),
 *     0 for a channel with walls on the outer y faces (Sec. II and the rough
 *     channel).
 *   cells_per_H: cells per reference length H (> 0, finite); the flow rate
 *     and rarefaction parameter are in units of H.
 * nx == 1 means invariant along x (plane channel); otherwise nx >= 4;
 * ny >= 4.  Every fluid component must carry flux along x (wrap around the x
 * period); fully enclosed pores are rejected with DVM_EINVAL (the problem
 * would have one null mode per pore).  Errors leave the instance as it was.
 * Replaces any previous geometry of the instance and discards its solution;
 * the device layout is rebuilt at the next solve. */
int dvm_set_geometry(dvm_ctx *ctx, int instance, int nx, int ny,
                     const uint8_t *solid, int periodic_y, double cells_per_H);

/* Rows of unequal height across the channel (the nonuniform spacing of
 * Sec. II.A, e.g. fine rows in a rough band): dy[ny] heights of the rows of
 * instance `instance` in units of H, bottom row first; NULL restores rows
 * of height 1 / cells_per_H.  cells_per_H keeps setting the x spacing.
 * Along y the upwind face value becomes h_u + r (h_u - h_uu) with
 * r = dy_u / (dy_u + dy_uu) (the paper's second-order difference on a
 * uniform grid), the flux difference is divided by the cell's own height,
 * and Q weighs u1 by dx dy.  Call after dvm_set_geometry (which resets the
 * heights); discards the instance's solution.  Such instances take the
 * per-cell path of the sweep; dvm_grad transposes the same weights.
 * DVM_EINVAL for a non-finite or non-positive height, DVM_ESTATE before
 * dvm_set_geometry. */
int dvm_set_row_heights(dvm_ctx *ctx, int instance, const double *dy);

/* What drives the flow of instance `instance` in its next solves: the
 * source pressure_gradient * xi of every fluid cell (a pressure gradient
 * along +x; 1 is the Poiseuille problem of Sec. III) and the x velocities of
 * the outer bottom and top walls of a walled channel, whose diffuse emission
 * becomes rho_w + 2 U xi (Eq. (diffuse1), U in units of v_m; the Couette
 * problem of Sec. II is pressure_gradient = 0, top velocity 1).  The
 * staircase itself is at rest.  Defaults: 1, 0, 0.  Kept across
 * dvm_set_geometry; a solve of a periodic cell (periodic_y = 1) with a
 * nonzero wall velocity fails with DVM_EINVAL.  DVM_EINVAL for non-finite
 * values. */
int dvm_set_driving(dvm_ctx *ctx, int instance, double pressure_gradient,
                    double wall_velocity_bottom, double wall_velocity_top);

/* Solve the steady problem driven as set by dvm_set_driving (by default a
 * unit pressure gradient along +x, the Poiseuille problem of Sec. III).
 *   instance >= 0: solve that instance; delta points to 1 value
 *     (delta_is_field = 0) or to ny*nx values (delta_is_field = 1, ignored in
 *     solids).
 *   instance == -1: solve every instance in one batched launch sequence;
 *     delta holds n_instances scalars (delta_is_field = 0) or the fields of
 *     all instances back to back (delta_is_field = 1); info (if non-NULL)
 *     receives n_instances records.
 * delta is the rarefaction parameter sqrt(pi)/(2 Kn) >= 0 (finite).
 * alpha in (0, 1] is the accommodation coefficient: 1 = diffuse walls of
 * Eq. (diffuse2); alpha < 1 adds Maxwell's specular share 1 - alpha.
 * Starts from h = 0 (or from the instance's previous solution when the
 * geometry is unchanged and `warm` semantics are requested with
 * dvm_solve_warm).  Returns DVM_ENOCONV if some instance hit max_iter
 * (its state is kept; calling again resumes), DVM_EDIVERGED on non-finite
 * iterates. */
int dvm_solve(dvm_ctx *ctx, int instance, const double *delta,
              int delta_is_field, double alpha, dvm_info *info);

/* As dvm_solve but starting from the instance's current state (warm start
 * along a delta sweep, or resume after DVM_ENOCONV). */
int dvm_solve_warm(dvm_ctx *ctx, int instance, const double *delta,
                   int delta_is_field, double alpha, dvm_info *info);

/* Flow rate of Sec. III, Q = (1/L) * sum over fluid of u1 dA (L = nx cells),
 * and apparent permeability k_a = sqrt(4/pi) Q Kn = Q / delta (NaN when delta
 * is a field).  k_a may be NULL.  Q of every solved instance is reduced on the
 * device (fixed summation order) at the end of each solve and kept with the
 * context, so this call does no device work.  DVM_ESTATE before the
 * instance's first solve. */
int dvm_flow_rate(const dvm_ctx *ctx, int instance, double *Q, double *k_a);

/* Moments of Sec. II.A at every cell (ny*nx each, 0 in solids): perturbed
 * density rho (gauge: zero mean over fluid cells), velocities u1, u2,
 * temperature tau, and shear stress p12 = 2 * int v1 v2 h f_eq.  Any output
 * may be NULL. */
int dvm_get_moments(const dvm_ctx *ctx, int instance, double *rho, double *u1,
                    double *u2, double *tau, double *p12);

/* For callers that cannot allocate memory during the call: code under HIP
 * stream capture, serving loops and harnesses that forbid hipMalloc.  Same
 * moments as dvm_get_moments, but every output is a DEVICE array of ny*nx
 * doubles owned by the caller (any may be NULL), written asynchronously on
 * the context's stream: the values are there once the stream has reached
 * this call (synchronize the stream, or order later work after it).  The
 * call allocates nothing, host or device: the staging it needs (the work
 * items of the shear-stress pass and the density gauge) lives in a static
 * device array of 1 MiB per GPU, set up by the context's first solve and
 * held until the process ends.  That array is shared by every call on the
 * same GPU and keeps the last call's contents: calls that overlap on one GPU
 * (other threads, other streams) race.  DVM_EINVAL if the instance needs
 * more than 65520 work items (strips x 4 x velocity groups), DVM_ESTATE
 * before the instance's first solve. */
int dvm_get_moments_noalloc(const dvm_ctx *ctx, int instance, double *rho,
                            double *u1, double *u2, double *tau, double *p12);

/* Gradient of Q by the discrete adjoint: dQ_ddelta[ny*nx] (0 in solids) with
 * respect to the per-cell rarefaction parameter, and dQ_dalpha with respect
 * to the accommodation coefficient, at the converged state of the last
 * dvm_solve of this instance.  Either output may be NULL. */
int dvm_grad(dvm_ctx *ctx, int instance, double *dQ_ddelta, double *dQ_dalpha);

/* Permeability of a porous medium from a rarefaction sweep of one geometry
 * (Sec. III): n >= 3 solves at distinct delta[i] > 0 with flow rates Q[i]
 * (dvm_flow_rate), porosity phi in (0, 1] (fluid fraction of the cell).
 * With Kn = sqrt(pi)/(2 delta) (Sec. II.A) and k_a = sqrt(4/pi) Q Kn = Q/delta:
 *   k_inf   -- the intrinsic permeability, the limit of k_a as Kn -> 0,
 *              taken as the value at Kn = 0 of the quadratic in Kn through
 *              the three samples of smallest Kn;
 *   H_star  -- the characteristic length H* = H sqrt(12 k_inf / phi), in
 *              units of H;
 *   Kn_star -- Kn* = Kn H / H* for every sample (n values);
 *   ka_ratio -- k_a / k_inf for every sample (n values);
 *   Kn      -- Kn of every sample (n values);
 *   k_a     -- k_a of every sample (n values).
 * Host-only arithmetic on host arrays; any output may be NULL.  DVM_EINVAL if
 * n < 3, a delta is not finite and > 0, two deltas coincide, phi is outside
 * (0, 1], or the extrapolated k_inf is not positive. */
int dvm_permeability(int n, const double *delta, const double *Q, double phi,
                     double *k_inf, double *H_star, double *Kn_star,
                     double *ka_ratio, double *Kn, double *k_a);

/* Kernel timings gathered while cfg.profile == 1 (HIP events on the
 * context's stream around every sweep launch of the source iteration, the
 * refinement's FP64 steps and FP32 correction iterations, and the
 * extrapolation's extra iteration; GMRES sweeps are not timed).  Launches at
 * the end of a block that find every instance stopped (and return at once)
 * are not counted. */
typedef struct {
    double sweep_ms;        /* FP64 sweep launches: total milliseconds       */
    long n_sweeps;          /*   their count                                 */
    double updates;         /*   fluid cell x velocity updates they made      */
    double other_ms;        /* moments, record and stop-rule kernels of the
                               plain FP64 iterations                          */
    double sweep32_ms;      /* FP32 sweep launches (DVM_FP32_REFINE)          */
    long n_sweeps32;
    double updates32;
    long persistent_blocks; /* blocks run as one cooperative launch
                               (persistent = 1; counted without profile too) */
    long persistent_iters;  /*   the iterations those blocks held             */
} dvm_prof;

/* Totals since the previous call (then reset); out must not be NULL. */
int dvm_profile(dvm_ctx *ctx, dvm_prof *out);

/* Sweep launch shape in use: velocities per lane and waves per workgroup of
 * the FP64 sweep and of the FP32 sweep (the latter used by
 * DVM_FP32_REFINE).  With autotuning the shapes are known after the first
 * dvm_solve; before it all four read 0.  Any output may be NULL. */
int dvm_launch_shape(const dvm_ctx *ctx, int *vel_per_lane, int *waves_per_block,
                     int *vel_per_lane32, int *waves_per_block32);

/* Release every resource of the context (NULL is ignored). */
void dvm_destroy(dvm_ctx *ctx);

/* Message of the last failed call on this thread ("" if none). */
const char *dvm_last_error(void);

/* Library version string. */
const char *dvm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DVM_H */
