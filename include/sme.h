/*
 * sme.h -- C ABI of the MI355X shallow-moment-equation (SME) time-step library.
 *
 * The library advances the hierarchy of hydrostatic shallow moment equations
 * of arXiv 2601.04826 with an explicit, first-order, path-conservative finite
 * volume scheme:
 *   - PDE template  dQ/dt + div F(Q) + B(Q) : grad Q = S(Q)               (Eq. (2))
 *   - SME flux, non-conservative matrices, friction closure       (Eq. (1), Sec. 3.4)
 *   - hydrostatic predictor then the friction ODE (Lie splitting)  (Eqs. (3a), (3d))
 *   - finite volumes for non-conservative systems, CFL time step  (Sec. 2.1.2, Sec. 3.1)
 * The calls mirror the paper's solver interface (Sec. 2.1.2): sme_init is the
 * solver's initialisation (state and auxiliary data bound to a mesh and a
 * model level), sme_run is the solve loop, sme_eigmax evaluates the model's
 * eigenvalue bound over the state for the adaptive time step.
 *
 * Numbers and layout
 *   FP64 throughout.  State Q is structure-of-arrays.  The calls that copy a
 *   state in or out (sme_set_state, sme_get_state) use Q[f * ncells + i] in the
 *   caller's cell order; the two device buffers a context is bound to use
 *   Q[f * field_stride + i] in the library's internal cell order (the caller's
 *   order on 1D and structured meshes):
 *     1D       nfields = N + 2   : (h, q_0 .. q_N),          q_k = h alpha_k
 *     2D       nfields = 2N + 3  : (h, qx_0..qx_N, qy_0..qy_N), qx_k = h alpha_k, qy_k = h beta_k
 *   Bathymetry b[i] is static.  Units: SI, kinematic (rho = 1).
 *
 * Ownership
 *   The caller owns the two device buffers of the state (the ping-pong pair
 *   of the explicit step, as in the solver's initialisation, Sec. 2.1.2, which
 *   hands out the state arrays); sme_init binds them to the context and they
 *   must outlive it.  Each step reads one and writes the other; sme_current
 *   says which one holds the state.  The context owns the rest: bathymetry in
 *   the internal order, mesh geometry, Gauss points and the time-step slots
 *   (sme_workspace_size bytes, allocated in sme_init, freed in sme_destroy).
 *   Other pointers passed in are only read during the call; host or device
 *   memory as the on_device flag says.  All device work is queued on the
 *   HIP stream given to sme_init; a call returns once its work is queued unless
 *   it returns a host value (sme_eigmax, sme_run with t_out/steps_done,
 *   sme_step with dt_used, sme_get_state into host memory), which synchronises
 *   that stream.  One context must not be used from two threads at once.
 *
 * Errors
 *   Every function returns SME_OK (0) or a negative code and never throws.
 *   sme_last_error(ctx) gives the message of the last failure on ctx;
 *   sme_strerror(code) a generic text.
 */
#ifndef SME_H
#define SME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SME_OK 0
#define SME_EINVAL (-1)    /* bad level, mesh, size or pointer                 */
#define SME_ENOMEM (-2)    /* device or host allocation failed                 */
#define SME_EHIP (-3)      /* a HIP runtime call failed (message kept)         */
#define SME_ENONPHYS (-4)  /* h <= 0 or a non-finite value appeared            */
#define SME_EMESH (-5)     /* degenerate triangle or non-manifold edge         */

#define SME_MESH_1D 1          /* nx uniform cells on [x0, x1]                   */
#define SME_MESH_2D_STRUCT 2   /* nx * ny cells, index j * nx + i                */
#define SME_MESH_2D_TRI 3      /* triangles (counter-clockwise vertex order)     */

#define SME_BC_PERIODIC 0      /* Periodic boundary (Sec. 2.1.1)                 */
#define SME_BC_EXTRAP 1        /* Extrapolation boundary (Sec. 2.1.1): copy       */
#define SME_BC_WALL 2          /* reflective wall: normal velocity mirrored       */

#define SME_MAX_LEVEL 8

typedef struct sme_ctx sme_ctx;

/* Model parameters (Sec. 3.1, Sec. 3.4).  g gravity; c_slip the slip
 * coefficient C of the bed closure sigma(0) = C u(0) (kinematic, m/s); nu the
 * kinematic viscosity of the Newtonian bulk closure (m^2/s); cfl the Courant
 * number of the adaptive step (0.45 in the paper); quad_points the number of
 * Gauss-Legendre points (1..8) on the straight path of the non-conservative
 * fluctuation; implicit_friction selects how the friction ODE of the
 * splitting (Eq. (3d)) is stepped: 0 forward Euler on the predicted state,
 * 1 backward Euler (the cell-local linear solve per moment block, stable for
 * any nu dt / h^2: the implicit source step of Sec. 2.1.2); order 1 is the
 * first-order scheme (forward Euler, cell values at the faces), order 2 the
 * second-order one on 1D and structured grids (least-squares-type limited
 * reconstruction, the compute_derivatives building block of Sec. 2.1.2:
 * minmod slopes of h + b, the momenta and b, the path fluctuation between the
 * reconstructed face values plus the one inside each cell, two-stage SSP
 * Runge-Kutta, then the friction step; the state then stays in one of the two
 * bound buffers, the other holds the first stage).  Order 2 is not available
 * on triangles, in the ensemble, with a learned closure or in sme_step_static
 * (SME_EINVAL). */
typedef struct {
    double g;
    double c_slip;
    double nu;
    double cfl;
    int quad_points;
    int implicit_friction;
    int order;
} sme_params;

/* Mesh description; all arrays are host memory, copied during sme_init.
 *   kind SME_MESH_1D        nx cells on [x0, x1]; bc[0] left, bc[1] right.
 *   kind SME_MESH_2D_STRUCT nx * ny cells on [x0,x1] x [y0,y1];
 *                           bc = {west, east, south, north}; periodic must pair.
 *   kind SME_MESH_2D_TRI    n_vert vertices vert_xy[2*v + {0,1}], n_tri
 *                           triangles tri[3*t + {0,1,2}] (CCW), at most 2^28
 *                           of them; every edge used by one triangle only is
 *                           a reflective wall. */
typedef struct {
    int kind;
    int64_t nx, ny;
    double x0, x1, y0, y1;
    int bc[4];
    int64_t n_vert, n_tri;
    const double *vert_xy;
    const int32_t *tri;
} sme_mesh;

/* Number of fields and cells a (level, mesh) pair needs, and the field stride
 * (ncells rounded up to a multiple of 256) of the state buffers sme_init
 * binds; no context and no device work.  Any output pointer may be NULL. */
int sme_layout(int level, const sme_mesh *mesh, int *nfields, int64_t *ncells, int64_t *field_stride);

/* Bytes of device memory sme_init allocates for a (level, mesh, params)
 * triple besides the caller's state buffers: bathymetry, Gauss points,
 * time-step slots, the limited slopes of the second-order scheme (1D grids,
 * and structured grids above level 6: below, the slopes are computed inside
 * the stages) and, on
 * triangles, neighbours, normals, centroids and the two cell permutations
 * (params NULL: first order).  Attaching a learned closure adds its network
 * and rates buffers. */
int sme_workspace_size(int level, const sme_mesh *mesh, const sme_params *params, size_t *bytes);

/* Create a solver for the SME of the given level (0..8) on the mesh
 * (the solver initialisation of Sec. 2.1.2: model, mesh and settings in, state
 * arrays bound).
 *   q_dev   two distinct caller-owned device buffers of the current device,
 *           256-byte aligned, each nfields * field_stride doubles (sme_layout);
 *           they stay owned by the caller and must outlive the context.  The
 *           library writes them in every step, and on triangles it also uses
 *           the one not holding the state as scratch in sme_set_state and
 *           sme_get_state.  SME_EINVAL if a pointer is NULL, not device memory
 *           of this device, misaligned or (as far as the runtime can tell)
 *           too short.
 *   b       bathymetry [ncells] in caller cell order (NULL = flat), host or
 *           device memory (b_on_device); copied.
 *   stream  hipStream_t to queue all work on (NULL = a stream of the context).
 * There is no state until sme_set_state. */
int sme_init(sme_ctx **out, int level, const sme_mesh *mesh, const sme_params *params,
             double *const q_dev[2], const double *b, int b_on_device, void *stream);

/* Load / read the state Q [nfields][ncells] (caller cell order; host memory,
 * or device memory if on_device).  sme_set_state also evaluates the eigenvalue
 * bound of the new state for the next CFL step and clears the time and step
 * counters.  On 1D and structured meshes q may also be one of the two bound
 * buffers (on_device = 1), filled by the caller with field stride
 * field_stride: that buffer then holds the state and nothing is copied. */
int sme_set_state(sme_ctx *ctx, const double *q, int on_device);
int sme_get_state(sme_ctx *ctx, double *q, int on_device);

/* Maximum wave-speed bound lam(Q, n) over all cells and face normals of the
 * current state, and the CFL step dt = cfl * min_i 2|V_i| / sum_f |e_f| lam(Q_i, n_f)
 * (Sec. 3.1 adaptive step).  Synchronises the stream.  Either pointer may be NULL. */
int sme_eigmax(sme_ctx *ctx, double *lam_max, double *dt);

/* One time step.  dt > 0 uses that step; dt <= 0 uses the CFL step of the
 * current state (computed on the device, no host round trip).  If dt_used is
 * not NULL the stream is synchronised and the step taken is returned. */
int sme_step(sme_ctx *ctx, double dt, double *dt_used);

/* n_steps CFL steps, queued as replays of a captured HIP graph.  t_end > 0
 * stops the simulated time at t_end: the last step is shortened, and the call
 * stops queueing steps once the device clock has reached t_end.  It reads the
 * clock two graphs (12 steps) behind the newest queued one, so the call blocks
 * while the device works through its queue, and up to 12 steps after t_end are
 * no-ops (a copy of the state each).  If t_out / steps_done are not NULL the stream is synchronised
 * and the simulated time since sme_set_state and the number of steps that
 * advanced the state are returned; SME_ENONPHYS is returned if a step produced
 * h <= 0 or a non-finite value (the state is then not usable).
 * A small 1D grid (at most 40 x 62 cells at levels 0-1, down to 8 x 62 at
 * level 8) whose state fits in one workgroup's LDS, with no closure attached,
 * is instead advanced by one workgroup that keeps
 * the state in LDS and takes up to 2048 steps per launch (its own step loop
 * stops at t_end; the clock is checked between launches).  The result is
 * bitwise the same as single sme_step calls.  The environment variable
 * SME_NO_LDS_RUN selects the graph path for such grids too. */
int sme_run(sme_ctx *ctx, int64_t n_steps, double t_end, double *t_out, int64_t *steps_done);

/* Simulated time and step count since sme_set_state (synchronises). */
int sme_time(sme_ctx *ctx, double *t, int64_t *steps);

/* 3D lifting of the current state (the interpolate_3d postprocessing of
 * Sec. 2.2.1; the shallow-water case is printed in Sec. 3.1): for nz sigma
 * levels zeta[l] in [0, 1] (host array, nz <= 64) and every cell, writes into
 * the device array out [5][nz][ncells] (caller cell order) the variables
 *   z = b + zeta h                                   elevation of the level
 *   u = sum_k alpha_k phi_k(zeta), v = sum_k beta_k phi_k(zeta)   (v = 0 in 1D)
 *   w = -sum_k (d_x qx_k + d_y qy_k) Phi_k(zeta) + u (d_x b + zeta d_x h)
 *       + v (d_y b + zeta d_y h)                     incompressibility with the
 *                                                    kinematic bed condition
 *   p = rho g h (1 - zeta)                           hydrostatic pressure
 * Horizontal derivatives are least-squares gradients over the cell's
 * neighbours inside the domain (central differences on uniform grids, one-sided
 * at walls and open ends; the minimum-norm gradient for a triangle with one
 * neighbour).  rho > 0 (1 gives the kinematic pressure).  Queued on the
 * context's stream; SME_EINVAL for a bad level count, a level outside [0, 1]
 * or an output that is not device memory. */
int sme_interpolate_3d(sme_ctx *ctx, int nz, const double *zeta, double rho, double *out);

/* Which of the two bound buffers (0 or 1, the index into q_dev of sme_init)
 * holds the current state; it alternates with every step. */
int sme_current(const sme_ctx *ctx);

int sme_nfields(const sme_ctx *ctx);
int64_t sme_ncells(const sme_ctx *ctx);
int sme_level(const sme_ctx *ctx);

/* The bound buffer holding the current state (q_dev[sme_current(ctx)]), in
 * the library's internal cell order (identity for 1D and structured meshes,
 * a bandwidth-reducing permutation for triangles); field f starts at element
 * f * sme_field_stride(ctx) (ncells rounded up to a multiple of 256). */
const double *sme_state_device(const sme_ctx *ctx);
int64_t sme_field_stride(const sme_ctx *ctx);

/* One step without any allocation, for callers that cannot allocate device
 * memory: code being captured into a HIP graph, tight serving loops, hosts
 * that forbid hipMalloc.  No context: the same step as sme_step on a 1D or
 * structured mesh (SME_EINVAL for triangles, which need geometry tables),
 * from the caller's state q to q_next (distinct device buffers, 256-byte
 * aligned, [nfields][field_stride] with field_stride >= ncells a multiple of
 * 256) over the bathymetry b (device, [ncells], required).  dt > 0 is used as
 * given; dt <= 0 takes the CFL step of q (computed on the device).  The
 * band height on structured grids is chosen as sme_init chooses it, so the
 * result is bitwise that of sme_step on a context holding q.
 * Scratch: the time-step slots, the non-physical-state word and the Gauss
 * points live in one static device array of 8 KiB per GPU (used from the
 * first call on a device until the process ends); its size does not depend on
 * the grid, which is limited only as sme_layout limits it.  No hipMalloc,
 * hipFree or allocating library call is made.  Work is queued on `stream`;
 * if dt_used is not NULL the stream is synchronised, the step taken is
 * returned and SME_ENONPHYS reports h <= 0 or a non-finite value in q_next.
 * Every call on a GPU shares that GPU's scratch array: calls that overlap on
 * one GPU (other streams or host threads) race and must be serialised by the
 * caller. */
int sme_step_static(int level, const sme_mesh *mesh, const sme_params *params, const double *q, double *q_next,
                    int64_t field_stride, const double *b, double dt, double *dt_used, void *stream);

/* ------------------------------------------------------------------------
 * Batched ensemble: n independent structured 2D grids (SME_MESH_2D_STRUCT) of
 * mixed size and level 0..4, advanced together by one persistent kernel launch
 * per step (captured in HIP graphs); every grid takes its own CFL step (the
 * adaptive step of Sec. 3.1 per grid).  The model parameters are shared.
 * Each grid's state is handled in its own caller order, [nfields_i][nx_i*ny_i].
 * A grid advanced in a batch is bitwise identical to the same grid advanced
 * alone by sme_run.  Errors as above; sme_batch_last_error gives the text.
 */
typedef struct sme_batch sme_batch;

/* levels[i] in 0..4, meshes[i] structured; b NULL or b[i] NULL = flat bed,
 * else b[i] host array [nx_i*ny_i].  stream as for sme_init. */
int sme_batch_init(sme_batch **out, int n, const int *levels, const sme_mesh *meshes,
                   const double *const *b, const sme_params *params, void *stream);
int sme_batch_set_state(sme_batch *bt, int inst, const double *q, int on_device);
int sme_batch_get_state(sme_batch *bt, int inst, double *q, int on_device);
/* n_steps steps of every grid; if any grid produced h <= 0 or a non-finite
 * value the call returns SME_ENONPHYS (it synchronises the stream). */
int sme_batch_run(sme_batch *bt, int64_t n_steps);
int sme_batch_time(sme_batch *bt, int inst, double *t, int64_t *steps);
int64_t sme_batch_cells(const sme_batch *bt);
/* Band height (rows per wave) used for grids of a level, and setting it. */
int sme_batch_rows(const sme_batch *bt, int level);
int sme_batch_set_rows(sme_batch *bt, int level, int rows);
/* Tile autotuner: for every level present, times candidate band heights on
 * this device with HIP events and keeps the fastest; results are cached in the
 * text file cache_path (NULL = no cache) keyed by device name, compute-unit
 * count, level and grid mix.  Call before loading states: it overwrites the
 * states with a lake at rest and resets every clock. */
int sme_batch_autotune(sme_batch *bt, const char *cache_path);
const char *sme_batch_last_error(const sme_batch *bt);
void sme_batch_destroy(sme_batch *bt);

/* ------------------------------------------------------------------------
 * Non-hydrostatic VAM channel (Sec. 3.3, the predictor-corrector splitting of
 * Sec. 2.1.2): the 1D vertically averaged momentum equations with linear u,
 * quadratic w and quadratic non-hydrostatic pressure, fields (h, h u0, h u1,
 * h w0, h w1) on nx uniform cells of [x0, x1] with extrapolation ends.  A step
 * is the explicit hydrostatic predictor (path-conservative Rusanov with the
 * model's flux and non-conservative product, the bed entering as g h b_x)
 * followed by the corrector: the pressure (p0, p1) for which the two
 * incompressibility constraints hold at the corrected state, found by one
 * linear solve (the constraints are affine in the pressure), then the
 * pressure source applied.  Spatial derivatives of the corrector are central
 * differences.  No friction (the paper's VAM case has none).
 *
 * Ownership as for sme_init: the caller owns the two state buffers, SoA
 * [5][field_stride] FP64 device memory, 256-byte aligned, field_stride from
 * sme_vam_layout; the library allocates sme_vam_workspace_size bytes (the
 * bathymetry, the pressure, the corrector's block system and its solution, the slots).
 * All work is queued on `stream`.  Errors: SME_EINVAL (size, pointer or
 * parameter), SME_ENOMEM, SME_EHIP, SME_ENONPHYS (h <= 0 or a non-finite value,
 * reported by the calls that synchronise); sme_vam_last_error gives the text.
 */
typedef struct sme_vam sme_vam;

int sme_vam_layout(int64_t nx, int64_t *field_stride);
int sme_vam_workspace_size(int64_t nx, size_t *bytes);
/* g > 0, cfl > 0, quad_points 1..8 (Gauss points of the path integral); b the
 * bathymetry [nx] on the host or (b_on_device) the device, NULL = flat. */
int sme_vam_init(sme_vam **out, int64_t nx, double x0, double x1, double g, double cfl, int quad_points,
                 double *const q_dev[2], const double *b, int b_on_device, void *stream);
/* state [5][nx] (host or device), or one of the two bound buffers in place;
 * resets the clock and reduces the CFL ratio of the state */
int sme_vam_set_state(sme_vam *v, const double *q, int on_device);
int sme_vam_get_state(sme_vam *v, double *q, int on_device);
/* (p0, p1) [2][nx] of the last corrector */
int sme_vam_pressure(sme_vam *v, double *p, int on_device);
/* one step: dt > 0 as given, else the CFL step (dt = cfl dx / max(|u0| +
 * sqrt(g h + u1^2))) computed on the device; dt_used may be NULL */
int sme_vam_step(sme_vam *v, double dt, double *dt_used);
/* n_steps CFL steps, the last one shortened to end at t_end if t_end > 0
 * (steps past t_end leave the state unchanged) */
int sme_vam_run(sme_vam *v, int64_t n_steps, double t_end, double *t_out, int64_t *steps_done);
int sme_vam_time(sme_vam *v, double *t, int64_t *steps);
int sme_vam_current(const sme_vam *v);   /* which bound buffer holds the state */
int64_t sme_vam_field_stride(const sme_vam *v);
const char *sme_vam_last_error(const sme_vam *v);
void sme_vam_destroy(sme_vam *v);

/* ------------------------------------------------------------------------
 * Learned closure: a small network (9 -> 64 -> 64 -> 2, tanh, FP32 training
 * and inference kernels) that corrects the level-1 step towards level 8.  The
 * paper has no learned closure; its level hierarchy (Eq. (1), Sec. 3.4) is
 * what the network shortcuts.  Features of a cell along a direction with
 * normal momenta (q_0, q_1): (h, q_0, q_1), their differences to the next and
 * the previous cell along that direction.  The network maps normalised
 * features x~ = (x - mu)/sigma to normalised rates y~; the rate of (q_0, q_1)
 * is y~ * out_scale and the level-1 step adds dt times it.  Parameters are one
 * FP32 array of 4930: W1[64][9], b1[64], W2[64][64], b2[64], W3[2][64], b3[2].
 */
typedef struct sme_mlp sme_mlp;

int sme_mlp_create(sme_mlp **out, void *stream);
/* Glorot-uniform initial weights, U(-a, a) with a = sqrt(6 / (fan_in +
 * fan_out)) drawn from a splitmix64 stream of `seed`, zero biases; resets Adam. */
int sme_mlp_init(sme_mlp *m, uint64_t seed);
int sme_mlp_set_params(sme_mlp *m, const float *params, int on_device);
int sme_mlp_get_params(sme_mlp *m, float *params, int on_device);
/* Normalisation (mu, sigma: 9 each), output scale (2) and the training box of
 * the raw features (box_lo, box_hi: 9 each, FP64); outside the box a cell
 * counts as out of range (sme_closure_out_of_range).  Any pointer may be NULL
 * (that part is kept).  Until set: mu 0, sigma 1, out_scale 1, no box. */
int sme_mlp_set_scaling(sme_mlp *m, const float *mu, const float *sigma, const float *out_scale,
                        const double *box_lo, const double *box_hi);
/* Scaling from n training samples (device arrays feat [n][9], targ [n][2],
 * raw): mu = column means, sigma = sample standard deviations (at least
 * 1e-6), out_scale = target standard deviations (at least 1e-12), box =
 * [min - margin*span, max + margin*span] per feature; FP64 two-pass sums in a
 * fixed order, so the result is deterministic.  Synchronises. */
int sme_mlp_fit_scaling(sme_mlp *m, const float *feat, const float *targ, int64_t n, double margin);
/* The current scaling (host arrays; any pointer may be NULL). */
int sme_mlp_get_scaling(const sme_mlp *m, float *mu, float *sigma, float *out_scale, double *box_lo,
                        double *box_hi);
/* Device arrays, raw features x [batch][9] -> normalised outputs y~ [batch][2];
 * the network normalises its inputs with its scaling. */
int sme_mlp_forward(sme_mlp *m, const float *x, int64_t batch, float *y);
/* MSE loss L = (1/batch) sum |y~ - t~|^2 (t~ = t / out_scale) and its
 * gradient (device, 4930; NULL skips the copy); loss into host memory (NULL:
 * no synchronisation).  x [.][9] and t [.][2] hold raw samples; the batch is
 * rows idx[0..batch-1] (device int64; NULL: rows 0..batch-1). */
int sme_mlp_loss_grad(sme_mlp *m, const float *x, const float *t, const int64_t *idx, int64_t batch, float *loss,
                      float *grad);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on a batch (as above). */
int sme_mlp_train_step(sme_mlp *m, const float *x, const float *t, const int64_t *idx, int64_t batch, float lr,
                       float *loss);
int sme_mlp_reset_optimizer(sme_mlp *m);
const char *sme_mlp_last_error(const sme_mlp *m);
void sme_mlp_destroy(sme_mlp *m);

/* Training samples on a periodic 1D row (device arrays, SoA with the given
 * field strides): raw features of cells[s] from the level-8 state q8 and
 * targets (q_k of q8_next - q_k of q1_step) / dt, k = 0, 1, where q1_step is
 * the level-1 step (same dt) of the first three fields of q8.
 * feat [nsamples][9], targ [nsamples][2] (FP32). */
int sme_closure_samples(const double *q8, int64_t stride8, const double *q8_next, int64_t stride8n,
                        const double *q1_step, int64_t stride1, int64_t ncells, double dt,
                        const int64_t *cells, int64_t nsamples, float *feat, float *targ, void *stream);
/* Attach the network (copied) to a level-1 1D or structured context; NULL
 * detaches.  Before every later step a rates pass evaluates the network on
 * the current state (every cell and direction); the step adds dt times the
 * rates.  sme_closure_attach evaluates it in FP32 (SME_CLOSURE_FP32).
 * sme_closure_attach_ex can instead choose SME_CLOSURE_FP16_MFMA: matrix-core
 * products with FP16 weights and activations and FP32 accumulation (feature
 * normalisation, activations and output scaling in FP32); its rates differ from
 * the FP32 ones by about 1e-3 relative.  SME_EINVAL for an unknown precision
 * or weights beyond the FP16 range. */
#define SME_CLOSURE_FP32 0
#define SME_CLOSURE_FP16_MFMA 1
int sme_closure_attach(sme_ctx *ctx, const sme_mlp *m);
int sme_closure_attach_ex(sme_ctx *ctx, const sme_mlp *m, int precision);
/* Cell-steps whose features left the training box since sme_set_state. */
int sme_closure_out_of_range(sme_ctx *ctx, int64_t *cells);

/* Train the network on n raw samples (device arrays feat [n][9], targ [n][2],
 * FP32): fit the scaling and the training box (sme_mlp_fit_scaling with
 * `margin`), reset Adam, then `epochs` passes over a seeded permutation of the
 * samples (splitmix64 stream of `seed`, Fisher-Yates) in max(1, n / batch)
 * batches of `batch` rows, one Adam step each (sme_mlp_train_step), with the
 * learning rate decaying geometrically from lr at the first step to lr_end at
 * the last.  loss_hist (host, `epochs` floats, NULL = none) receives the loss
 * of the last batch of every epoch.  Synchronises the network's stream. */
int sme_closure_train(sme_mlp *m, const float *feat, const float *targ, int64_t n, int epochs, int64_t batch,
                      float lr, float lr_end, uint64_t seed, double margin, float *loss_hist);

/* Level 1 + closure with a fallback.  c1 is a level-1 context with a network
 * attached and a state loaded, c8 a context of a higher level (normally 8) on
 * the same grid.  Advances c1 towards t_end (simulated time since its
 * sme_set_state) in chunks of `chunk` CFL steps, at most max_steps in all; the
 * state at the start of each chunk is kept on the device.  If more than
 * max_out_of_range * ncells * (steps of the chunk) cell-steps of a chunk left
 * the training box, the network is not trusted there: the chunk's starting
 * state is lifted into c8 (h, q_0, q_1 of each direction copied, higher
 * moments zero) and c8 runs from it to t_end instead.  Outputs (any may be
 * NULL): t_out the simulated time reached, steps_done the steps taken
 * (level-1 steps before the fallback plus c8's), fallback_at the time of the
 * lifted state, or -1 if c1 ran to the end (the final state is then c1's,
 * else c8's).  Synchronises both streams. */
int sme_closure_run(sme_ctx *c1, sme_ctx *c8, double t_end, int64_t chunk, int64_t max_steps,
                    double max_out_of_range, double *t_out, int64_t *steps_done, double *fallback_at);

/* Introspection, host only (no device work): the FP64 basis tensors the kernels
 * are compiled with (Eq. (1), Sec. 3.4): M[n], A[n*n*n], B[n*n*n], K[n*n] with
 * n = level + 1, A[(i*n + j)*n + k] = <phi_i phi_j, phi_k>,
 * B[(i*n + j)*n + k] = <phi_i Phi_j, phi_k'>, K[j*n + k] = <phi_j', phi_k'>.
 * Any pointer may be NULL. */
int sme_basis_tensors(int level, double *M, double *A, double *B, double *K);

const char *sme_strerror(int code);
const char *sme_last_error(const sme_ctx *ctx);
void sme_destroy(sme_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SME_H */
