/*
 * mrab.h -- C ABI of libmrab.so: SBP-SAT right-hand side of the compressible
 * Navier-Stokes equations on overlapping structured grids, advanced by the
 * multi-rate Adams-Bashforth (MRAB) scheme, on one AMD MI355X (gfx950) GPU.
 *
 * Method: Mikida, Kloeckner, Bodony, "Multi-Rate Time Integration on Overset
 * Meshes" (arXiv 1805.06607).  Each declaration names the passage that defines
 * the operation.
 *
 * Conventions
 *  - Every call returns an mr_status (0 = MR_OK) and never throws.  After an
 *    error, mr_last_error(ctx) describes it.
 *  - Grid point p = i + nx*(j + ny*k) (x fastest).  A state or right-hand side
 *    is structure-of-arrays: nv x npts doubles (nv = dim + 2: rho, rho*u_i,
 *    rho*E), variable-major.
 *  - Host arrays passed in are copied during the call; the caller keeps them.
 *  - Device pointers (states, right-hand sides, the workspace) are borrowed
 *    from the caller and must stay valid until the stream is synchronised.
 *  - All device work is enqueued on the HIP stream given to mr_create; calls
 *    marked "async" do not synchronise the host.  Setup calls may synchronise.
 *  - The library never allocates device memory: mr_finalize reports the
 *    workspace size and the caller binds one buffer with mr_bind_workspace
 *    (or, for small systems, the library's static per-device array with
 *    mr_bind_static_workspace).
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef MRAB_H
#define MRAB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mr_ctx mr_ctx;

typedef enum {
    MR_OK = 0,
    MR_ERR_ARG = -1,          /* invalid argument (null pointer, bad size or flag) */
    MR_ERR_STATE = -2,        /* call out of order (e.g. mr_rhs before binding) */
    MR_ERR_SETUP = -3,        /* invalid geometry: short run, missing donor, bad rate */
    MR_ERR_HIP = -4,          /* a HIP runtime call failed */
    MR_ERR_NONFINITE = -5,    /* the state guard found a NaN/Inf */
    MR_ERR_UNSUPPORTED = -6   /* valid but not implemented (e.g. 3D curvilinear) */
} mr_status;

enum { MR_SBP_21 = 21, MR_SBP_42 = 42 };
enum { MR_BC_PERIODIC = 0, MR_BC_INTERFACE = 1, MR_BC_FARFIELD = 2, MR_BC_WALL = 3 };
enum { MR_CARTESIAN = 0, MR_CURVILINEAR = 1 };

/* Scheme and physics parameters.
 *  sbp            MR_SBP_21 or MR_SBP_42: diagonal-norm SBP first-derivative
 *                 operator (section "The Compressible Navier-Stokes Equations on
 *                 Overset Meshes"); second derivatives apply it twice.
 *  order, hist_len  AB order n and history length m >= n (m > n: the
 *                 extended-history, minimum-norm schemes of eq. ext_ab).
 *  interp_width   donor stencil width per direction (2 bilinear, 4 cubic);
 *                 informational, the weights come with mr_set_overset or
 *                 mr_assemble_overset (whose width argument rules).
 *  gamma, Re, Pr, mu, lambda_over_mu  gas constants; T = p/rho,
 *                 c_p = gamma/(gamma-1), tau_ij as in the Appendix equations.
 *  sigma_I_iface  sigma^I of the SAT interface penalty, eq. (int) (1/2).
 *  sigma_I_bc     sigma^I of the far-field and wall penalties.
 *  T_wall         isothermal wall temperature.
 *  wall_visc      wall no-slip penalty factor: sigma = wall_visc*mu*|grad k|^2/Re.
 *  q_inf          far-field target state (nv values).
 *  cfl, dt_fixed  macrostep H = cfl * min over grids of rate * min_pt dt_pt
 *                 (eq. ts_inv, ts_visc, ts_overall) unless dt_fixed > 0.
 */
typedef struct {
    int dim;
    int sbp;
    int order, hist_len;
    int interp_width;
    double gamma, Re, Pr, mu, lambda_over_mu;
    double sigma_I_iface, sigma_I_bc, T_wall, wall_visc;
    double q_inf[5];
    double cfl, dt_fixed;
} mr_params;

/* One structured grid.
 *  n[d], periodic[d]   points and periodicity per direction (n[2] = 1 in 2D)
 *  kind                MR_CARTESIAN (origin, spacing) or MR_CURVILINEAR (coords)
 *  coords              host, dim x npts, curvilinear only (2D)
 *  coord_period[d][c]  jump of coordinate c across the seam of periodic
 *                      direction d (0 for grids whose coordinates wrap)
 *  iblank              host, npts, 1 active / 0 hole; NULL = all active
 *  face_bc[2d+s]       boundary flag of face s (0: min, 1: max) of direction d
 *  rate                right-hand-side evaluations per macrostep (r_l); every
 *                      rate must divide the largest one
 */
typedef struct {
    int n[3];
    int periodic[3];
    int kind;
    double origin[3], spacing[3];
    const double *coords;
    double coord_period[3][3];
    const int8_t *iblank;
    int face_bc[6];
    int rate;
} mr_grid_desc;

/* Create a context.  hip_stream: a hipStream_t (NULL = default stream). */
int mr_create(const mr_params *params, void *hip_stream, mr_ctx **out);

/* Add a grid; grid ids are 0, 1, ... in call order.  Splits every grid line
 * into runs of active points (closures at run ends, SAT faces at run ends:
 * the face's flag at grid faces, interface next to holes).
 * Errors: MR_ERR_ARG (bad sizes/flags), MR_ERR_SETUP (a run shorter than two
 * closures), MR_ERR_UNSUPPORTED (3D curvilinear). */
int mr_add_grid(mr_ctx *ctx, const mr_grid_desc *desc, int *grid_id);

/* Donor stencils of the receivers of recv_grid that take their data from
 * donor_grid (section "SAT-Based Interpolation": Lagrange interpolation of
 * donor data).  recv_pt[n]: receiver points (each an active point that ends a
 * run on an interface face); donor_pt[n*S], weights[n*S]: S = width^dim donor
 * points and weights per receiver.  May be called several times per pair.
 * Errors: MR_ERR_ARG (index out of range), MR_ERR_SETUP (donor point blanked). */
int mr_set_overset(mr_ctx *ctx, int recv_grid, int donor_grid, int64_t n, int stencil_size,
                   const int64_t *recv_pt, const int64_t *donor_pt, const double *weights);

/* Fractional-index callback for mr_assemble_overset: for the n physical
 * points x (dim x n doubles, component-major), write their fractional indices
 * in curvilinear grid `grid` to f (dim x n; grid point i of a direction sits
 * at i; NaN marks a point outside the grid).  Return 0, or nonzero to abort
 * the assembly. */
typedef int (*mr_locate_fn)(void *user, int grid, int64_t n, const double *x, double *f);

/* Chimera donor-receiver search and interpolation weights for every grid, in
 * place of mr_set_overset calls (section "SAT-Based Interpolation": donor
 * search, then Lagrange interpolation with weights from Lagrange shape
 * functions).  Receivers are the active points that end a run on an
 * interface face.  For each receiver, the donor is the first other grid in
 * decreasing priority[grid] (ties: lower id) whose width-point-per-direction
 * stencil, based at floor(f) - (width/2 - 1) around the receiver's fractional
 * index f, lies inside the grid (periodic directions wrap) and covers only
 * active points; weights are tensor products of the 1D Lagrange shape
 * functions on the width integer nodes (entry order x fastest).  Fractional
 * indices: on Cartesian grids (x - origin) / spacing; on curvilinear grids
 * the caller's locate (user is passed through), or with locate == NULL the
 * library's own search (the nearest grid point, then Newton iterations on the
 * grid's coordinates interpolated by 4-point Lagrange polynomials per
 * direction).  Receivers register grid by grid, per grid donor by donor in
 * priority order, ascending point order within a pair (mr_get_overset reads
 * them back).  Host only.
 * width^dim must be a power of two of at most 64 (widths 1, 2, 4; 8 in 2D).
 * On an error the stencils registered before it stay: set up a new context
 * to retry.
 * Errors: MR_ERR_ARG (width), MR_ERR_STATE (after mr_finalize, receivers
 * already registered), MR_ERR_SETUP (a receiver without a donor, the
 * callback failed). */
int mr_assemble_overset(mr_ctx *ctx, int width, const int *priority, mr_locate_fn locate, void *user);

/* The registered donor stencils of grid's receivers, in row order: with every
 * array NULL, *n is set to the number of receivers; otherwise *n must be at
 * least that number and is set to it, recv_pt[n], donor_grid[n],
 * donor_pt[n*S] and weights[n*S] (S = stencil size; any may be NULL) are
 * filled.  Host only.  Errors: MR_ERR_ARG (bad grid, *n too small). */
int mr_get_overset(const mr_ctx *ctx, int grid, int64_t *n, int64_t *recv_pt, int *donor_grid, int64_t *donor_pt,
                   double *weights);

/* Validate (every interface run end has exactly one donor stencil, every rate
 * divides the largest), build the device tables and the static rate schedule,
 * and report the workspace size in bytes. */
int mr_finalize(mr_ctx *ctx, size_t *workspace_bytes);

/* Bind caller-owned device memory (>= the reported size, 256-byte aligned),
 * upload the tables, compute metric terms on the device. */
int mr_bind_workspace(mr_ctx *ctx, void *dev_ptr, size_t bytes);

/* Size of the library's static workspace: one array of this many bytes per
 * device, held from the load of the library's code object until the process
 * ends. */
#define MR_STATIC_WORKSPACE_BYTES ((size_t)16 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, allocation-free serving loops, harnesses that forbid hipMalloc):
 * mr_bind_workspace with the library's own static array on the device of the
 * context's stream (the current device for the default stream) in place of
 * caller memory.  Calls no hipMalloc, hipFree or other allocating routine; the
 * array is cleared and the tables uploaded exactly as mr_bind_workspace does.
 * The array is shared: binding it to a context takes it from the context that
 * held it on that device, whose later calls fail with MR_ERR_STATE; calls of
 * two contexts that overlap on one device race.  Released by mr_destroy of
 * its holder.
 * Errors: MR_ERR_ARG (the reported workspace exceeds
 * MR_STATIC_WORKSPACE_BYTES: bind caller memory instead), MR_ERR_STATE (before
 * mr_finalize or already bound), MR_ERR_HIP. */
int mr_bind_static_workspace(mr_ctx *ctx);

/* Copy a grid state (device, nv x npts) into / out of the context (async).
 * After mr_set_state (or mr_set_history) macrosteps need mr_mrab_start or
 * mr_mrab_resume first (MR_ERR_STATE otherwise). */
int mr_set_state(mr_ctx *ctx, int grid, const double *dev_q);
int mr_get_state(mr_ctx *ctx, int grid, double *dev_q_out);

/* One coupled right-hand side of all grids at a common time (async):
 * donor data gathered from dev_q of the donor grids, then per grid the
 * SBP-SAT right-hand side (eq. int and the Appendix equations) into
 * dev_dqdt[g] (nv x npts; 0 at holes).  dev_q[g] and dev_dqdt[g] are device
 * pointers, one per grid, and must not alias. */
int mr_rhs(mr_ctx *ctx, double t, const double *const *dev_q, double *const *dev_dqdt);

/* Donor data of the receivers of grid g from the given donor states (async):
 * out (device) receives, per receiver, q_hat (nv) then F_hat^V_j (nv-1 each,
 * j = 0..dim-1).  For parity tests of the interpolation step. */
int mr_receiver_data(mr_ctx *ctx, int grid, const double *const *dev_q, double *dev_out);
int mr_num_receivers(const mr_ctx *ctx, int grid, int64_t *n);

/* Timestep (setup; synchronises): per-point estimate eq. (ts_visc) on the
 * current states, H = cfl * min_g rate_g * min_pt dt (or dt_fixed),
 * h = H / r_max.  Fixes H for the run. */
int mr_timestep(mr_ctx *ctx, double *h, double *H);

/* Set the macrostep H directly (h = H / r_max), instead of mr_timestep's
 * estimate; later macrosteps need mr_mrab_start or mr_mrab_resume first.
 * Errors: MR_ERR_SETUP (H not positive and finite). */
int mr_set_macrostep(mr_ctx *ctx, double H);

/* Bootstrap (section "Adams-Bashforth Integration"): single-rate RK at
 * h = H / r_max (Heun RK3 for order <= 3, classic RK4 for order 4) for
 * (m-1)*r_max steps from the current states at time t0, keeping F(y_n) at each
 * grid's history nodes; then stages the first own step of every grid. */
int mr_mrab_start(mr_ctx *ctx, double t0);

/* nsteps macrosteps of MRAB, fastest first, no re-extrapolation (section
 * "Multi-rate Adams-Bashforth Integration", Steps 1-7, generalised to nested
 * integer rates).  Async. */
int mr_mrab_macrostep(mr_ctx *ctx, int nsteps);

/* Copy history value j (0 = oldest .. hist_len-1 = newest right-hand side of
 * grid g, the values the AB combination of eq. ab_general weights) into
 * dev_out (nv x npts, async).  For checkpoints and tests. */
int mr_get_history(mr_ctx *ctx, int grid, int j, double *dev_out);

/* Set history value j of grid g from dev_in (nv x npts, async), the inverse
 * of mr_get_history.  Together with mr_set_state and mr_mrab_resume this sets
 * the whole integrator state (each grid's state and its m right-hand-side
 * values), e.g. to form step matrices by finite differences (section
 * "Procedure for Determining Discrete Stability") or to restart from a
 * checkpoint.  Errors: MR_ERR_STATE before mr_mrab_start. */
int mr_set_history(mr_ctx *ctx, int grid, int j, const double *dev_in);

/* Continue MRAB from the current states and histories at time t (async):
 * stages every grid's next own step (eq. ab_general) and the donor data of
 * the next macrostep's mid-step times, as the end of mr_mrab_start does;
 * the macrostep count restarts at 0.  Errors: MR_ERR_STATE before
 * mr_mrab_start. */
int mr_mrab_resume(mr_ctx *ctx, double t);

/* Current time and completed macrosteps. */
int mr_time(const mr_ctx *ctx, double *t, int64_t *macrosteps);

/* Checkpoint and restart of the integrator (every grid's state and its
 * hist_len right-hand-side values, the time, the completed macrosteps and
 * the macrostep H).  mr_save_bytes: the size of a checkpoint.  mr_save
 * writes one into caller-owned device memory dev_buf (a 256-byte header,
 * then per grid the state and the history values oldest first, each nv x
 * npts) and synchronises the stream; mr_load reads one back into a context
 * built from the same problem (same grids, hist_len), sets H, stages the next
 * macrostep as mr_mrab_resume does (so it may follow mr_bind_workspace
 * without mr_mrab_start), and synchronises.  Macrosteps after mr_load repeat
 * those after mr_save bit for bit.  Errors: MR_ERR_ARG (null, buffer too
 * small or misaligned), MR_ERR_STATE (save before mr_mrab_start or with a
 * state set since; load before mr_bind_workspace), MR_ERR_SETUP (the
 * checkpoint belongs to a different problem). */
int mr_save_bytes(const mr_ctx *ctx, size_t *bytes);
int mr_save(mr_ctx *ctx, void *dev_buf, size_t bytes);
int mr_load(mr_ctx *ctx, const void *dev_buf, size_t bytes);

/* AB coefficients (host, pure): spacing * alpha_j, j = 0..hist_len-1 oldest
 * first, for history nodes -(m-1)..0 in units of the step and target offset
 * tau in (0,1] (eq. vandermonde; minimum norm when hist_len > order, eq.
 * ext_ab); alpha_j is rounded to double once, then multiplied by spacing (the
 * level's step), as the integrator forms its coefficients.  out: hist_len
 * host doubles.  Errors: MR_ERR_ARG (tau outside (0,1], order or hist_len out
 * of range, spacing not positive and finite). */
int mr_ab_coeffs(int order, int hist_len, double spacing, double tau, double *out);

/* Per-launch timing of the grids' fused right-hand-side kernels with HIP
 * events recorded on the stream each launch is issued on: grid >= 0 times that
 * grid's launches, MR_ALL_GRIDS every grid's, -1 disables; at most max_events
 * launches are recorded.  mr_kernel_time synchronises and returns the summed
 * duration and the number of timed launches since the last enable;
 * mr_kernel_time_grid the same for one grid's launches (-1: all). */
enum { MR_ALL_GRIDS = -2 };
int mr_kernel_timing(mr_ctx *ctx, int grid, int max_events);
int mr_kernel_time_grid(mr_ctx *ctx, int grid, double *total_ms, int *count);
int mr_kernel_time(mr_ctx *ctx, double *total_ms, int *count);

/* Execution options (any time after mr_create; they change the launch plan,
 * not the method):
 *  "rhs_two_pass"        1: 2D grids use the gradient pass and the point-wise
 *                        right-hand-side kernel instead of the fused tile
 *                        kernel (default 0).
 *  "multi_stream"        1: inside mr_mrab_macrostep every grid's work runs on
 *                        a stream of its own, ordered against the other grids
 *                        by events only where receiver data passes between
 *                        them, so a slow grid's step overlaps a fast grid's
 *                        substeps; the call still returns with all work
 *                        ordered before later work on the context's stream
 *                        (0: everything on the context's stream; default:
 *                        on when the grids hold at least 4 Mi points in all,
 *                        where the launches are long enough to gain from it).
 *  "donor_blocks"        1: links with stencils of at most 16 entries whose
 *                        receiver chunks fit one workgroup's LDS get their
 *                        receiver rows in one launch per donor step (the
 *                        extrapolant at the points the chunk reads, the values
 *                        at its distinct donor points, the weighted sums);
 *                        0: always the values-then-gather launches, with a
 *                        separate extrapolation launch (default 1).
 *  "rhs_tile3d"          3D grids: the gradient pass and the flux pass on LDS
 *                        tiles of shape 0..3 (8x8x8, 16x8x4, 32x4x4, 16x4x4
 *                        outputs; each thread evaluates its own point once,
 *                        the halo slabs are evaluated per direction), or -1
 *                        for the point-wise kernels (default 1).  Same
 *                        formulas; results agree to rounding.
 *  "tile3d_slab"         3D tiled passes: the order in which the launch
 *                        takes its tiles.  n > 0: slabs of n tile rows along
 *                        y, each slab taken plane by plane along z, so a
 *                        tile's z neighbours are n tile rows away and their
 *                        halo data is still in the cache; 0: plain x, y, z
 *                        order (default 3).  Each output is computed alone, so
 *                        results are bitwise the same for every value.
 *  "ride_donors"         1: with one stream, the mid-step donor data of a
 *                        slower 2D grid (one chunked link) is produced inside
 *                        the launch of the next grid evaluated at the same
 *                        micro-time, in workgroups of its own, when that
 *                        grid's 2D tile has at least 256 threads; it reads
 *                        and writes nothing that evaluation touches.  0: a
 *                        launch of its own (default 1).  Bitwise the same.
 *  "graph"               reserved: 1 (replaying captured HIP graphs of whole
 *                        macrostep periods) is switched off and returns
 *                        MR_ERR_UNSUPPORTED; 0 is accepted.
 * Errors: MR_ERR_ARG (unknown name or bad value), MR_ERR_UNSUPPORTED. */
int mr_set_option(mr_ctx *ctx, const char *name, int64_t value);

/* Tile shape of a 2D grid's fused right-hand-side kernel: shape in
 * 0..MR_NUM_TILE_SHAPES-1, or -1 for the size-based default.  Every shape
 * evaluates the same formulas per output; results agree up to rounding (the
 * compiler may fuse a multiply-add differently per shape), and one shape is
 * bitwise reproducible run to run.  mr_get_tile_shape
 * reports the shape in use (-1 for 3D grids) and its tile (tx x ty outputs,
 * tm threads per output).  Errors: MR_ERR_ARG (bad grid or shape),
 * MR_ERR_UNSUPPORTED (3D grid). */
enum { MR_NUM_TILE_SHAPES = 8 };
int mr_set_tile_shape(mr_ctx *ctx, int grid, int shape);
int mr_get_tile_shape(const mr_ctx *ctx, int grid, int *shape, int *tx, int *ty, int *tm);
/* The tile of shape `shape` (0..MR_NUM_TILE_SHAPES-1): tx x ty outputs per
 * workgroup, tm threads per output; host only, no device needed.  Null
 * output pointers are skipped.  Errors: MR_ERR_ARG (shape out of range). */
int mr_tile_shape_info(int shape, int *tx, int *ty, int *tm);

/* Autotuner (setup; synchronises): for every 2D grid, time reps launches of
 * each tile shape on the current state, writing only scratch buffers, and
 * keep the fastest.  The timed launches are queued behind a short wait on the
 * device, so they run back to back and the host's launch rate does not enter
 * the timing.  Needs a bound workspace; leaves states, histories and
 * the schedule untouched. */
int mr_autotune(mr_ctx *ctx, int reps);

/* Non-finite guard: synchronises, returns MR_ERR_NONFINITE if any state holds
 * a NaN or Inf, and the largest |q| in *maxabs. */
int mr_guard(mr_ctx *ctx, double *maxabs);

/* Batches (many independent systems advanced together).  A batch holds
 * finalized 2D contexts sharing one stream and one SBP operator, whose links
 * all take the one-launch donor form; their macrosteps H and step ratios may
 * differ (every system's largest rate must divide the batch's least common
 * multiple R <= 64).  One batch macrostep advances every system by one of its
 * own macrosteps: for each of the R micro-times, one work-list launch per
 * kind of job -- donor data at the current time, fused right-hand sides (one
 * launch per tile shape and grid kind), mid-step donor data -- over all
 * systems that step then.  The launches run the same per-tile and per-chunk
 * code as each system's own mr_mrab_macrostep, so every system's result is
 * the same.  The launch plan (jobs in device memory, built on the host from
 * the systems' bookkeeping, one plan period of macrosteps) is rebuilt when a
 * system was stepped on its own, restarted, or changed its step, tile shapes
 * or options.  The library allocates nothing: mr_batch_workspace_size
 * reports the bytes the caller binds.  Errors: MR_ERR_ARG, MR_ERR_STATE (a
 * context not finalized; a system not started), MR_ERR_UNSUPPORTED (3D, the
 * gradient-pass form, two-launch donor links, mixed operators or streams). */
typedef struct mr_batch mr_batch;
int mr_batch_create(mr_ctx *const *ctxs, int n, mr_batch **out);
int mr_batch_workspace_size(const mr_batch *batch, size_t *bytes);
int mr_batch_bind_workspace(mr_batch *batch, void *dev_ptr, size_t bytes);
int mr_batch_macrostep(mr_batch *batch, int nsteps);
/* Tile shape of every right-hand side in the batch's launches (0 ..
 * MR_NUM_TILE_SHAPES-1), or -1 (default) for each grid's own shape, with
 * which every system's result equals its own macrosteps bit for bit.  A
 * batch fills the GPU with many grids at once, so large tiles (shape 0, 32 x
 * 16) usually beat the small multi-thread tiles that suit one small grid. */
int mr_batch_set_tile_shape(mr_batch *batch, int shape);
/* Autotuner of the batch's tile shape: times `reps` passes of one fused
 * right-hand side of every grid of every system (from the current states
 * into the systems' scratch buffers: states, histories and times are not
 * changed) for each candidate -- every grid's own shape (-1), then each shape
 * 0 .. MR_NUM_TILE_SHAPES-1 for all -- with HIP events around back-to-back
 * launches, keeps the fastest as the batch's shape and returns it in *shape.
 * ms (may be NULL): MR_NUM_TILE_SHAPES + 1 host doubles, the time of one pass
 * per candidate in the same order.  Synchronises the stream.
 * Errors: MR_ERR_ARG (reps outside 1..1000), MR_ERR_STATE (not bound, a
 * system not started), MR_ERR_HIP. */
int mr_batch_autotune(mr_batch *batch, int reps, int *shape, double *ms);
const char *mr_batch_last_error(const mr_batch *batch);
void mr_batch_destroy(mr_batch *batch);

/* Discrete adjoint (2D systems).  The derivative of a whole run -- the RK
 * bootstrap of mr_mrab_start from initial states y0, then nmacro MRAB
 * macrosteps at the context's macrostep H (held fixed: it is not
 * differentiated) -- of
 *     J = sum_i tau_i sum_k w_k p(q_grid(pts_k, t_i)),
 * the time integral (trapezoid rule over the objective grid's own-step times
 * from the start of the macrosteps, tau_i = its step, halved at both ends)
 * of a weighted sum of the pressure p = (gamma - 1)(rho E - rho |u|^2 / 2)
 * at listed points of one grid (a wall-pressure force when w_k = n_x ds).
 * The run the adjoint differentiates is the library's own forward pass of
 * the method, with the kernels and rounding order of mr_mrab_macrostep (the
 * fused right-hand side with the next own step, the donor-data launches, the
 * extrapolants at the donor-stencil points).  Every step of the derivative is a hand-written adjoint
 * kernel (transposed SBP rows as gathers, exact local Jacobians of the
 * pointwise flux, SAT and primitive maps by forward-mode dual numbers,
 * donor data reversed per donor and stencil point from precomputed tables,
 * so results do not depend on thread timing); macrosteps are reversed under
 * a binomial checkpointing schedule with nsnap snapshots of every grid's
 * state and history (slot 0 holds the start of the macrosteps).  The
 * library allocates nothing: mr_adj_workspace_size reports the bytes the
 * caller binds (states, histories, one macrostep's tape, the bootstrap
 * states and the snapshots).  Errors: MR_ERR_ARG, MR_ERR_STATE (call order,
 * no macrostep set), MR_ERR_UNSUPPORTED (3D grids).
 *
 * mr_adj_set_objective: host arrays, copied; points of `grid`, unique and
 *     active; n = 0 removes the objective.
 * mr_adj_rhs: lam_q = (d mr_rhs / d q)^T lamF for the coupled right-hand side
 *     at states q (device, one array per grid, SoA nv x npts), donor data at
 *     the same time included.
 * mr_adj_forward: the forward pass alone: J and (yN non-null) the final
 *     states.
 * mr_adj_gradient: grad[g] = dL/dy0[g] for L = jscale * J + sum_g <lamN[g],
 *     yN[g]> (lamN null or an entry null: zero); J, and in *nfwd the
 *     macrosteps run forward (the first pass plus the recomputations).
 *     nmacro <= 4096.
 * mr_adj_schedule: host only; the forward macrosteps the reversal of nmacro
 *     macrosteps recomputes with nsnap slots (slot 0 holding the start). */
int mr_adj_set_objective(mr_ctx *ctx, int grid, int64_t n, const int64_t *pts, const double *w);
int mr_adj_workspace_size(mr_ctx *ctx, int nsnap, size_t *bytes);
int mr_adj_bind_workspace(mr_ctx *ctx, void *dev_ptr, size_t bytes);
int mr_adj_rhs(mr_ctx *ctx, const double *const *dev_q, const double *const *dev_lamF, double *const *dev_lam_q);
int mr_adj_forward(mr_ctx *ctx, int nmacro, const double *const *dev_y0, double *const *dev_yN, double *J);
int mr_adj_gradient(mr_ctx *ctx, int nmacro, const double *const *dev_y0, const double *const *dev_lamN,
                    double jscale, double *const *dev_grad, double *J, int64_t *nfwd);
int mr_adj_schedule(int nmacro, int nsnap, int64_t *nfwd);

const char *mr_last_error(const mr_ctx *ctx);
void mr_destroy(mr_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* MRAB_H */
