/*
 * scfft — right-hand side and method-of-lines integrator of the FFT-based
 * bulk magnetization method of Prigozhin & Sokolovsky (arXiv:1803.01346,
 * "3D simulation of superconducting magnetic shields and lenses using the
 * Fast Fourier Transform"), for AMD Instinct MI355X (gfx950).
 *
 * The problem (paper Sec. 2): a superconductor Omega inside the box
 * D = {|x|<=Lx, |y|<=Ly, |z|<=Lz}, a uniform applied field h_e(t), the power
 * law e = rho(|j|) j (Eq. 1), the Biot-Savart law h = h_e + Phi[j] (Eq. 2),
 * Faraday's law mu0 dh/dt = -curl e (Eq. 3), Ampere's law j = curl h (Eq. 4),
 * the exterior fixed-point iteration (Eq. 5) and Phi evaluated in Fourier
 * space (Eq. 7, with 1/|k|^2 replaced by 0 at k = 0).  Derivatives are
 * spectral with Gaussian smoothing of width sigma = half the cell diagonal;
 * the node values of h obey an ODE system integrated in time (Sec. 2,
 * discretisation paragraph).  Internal units are those of Eq. 8.
 *
 * Conventions shared by every entry point
 *   Device arrays   caller-owned device memory (e.g. torch tensors).  A
 *                   vector field is dense, structure-of-arrays [3][Nz][Ny][Nx]
 *                   with x fastest and components (x, y, z), in the context's
 *                   precision: double for SCFFT_F64, float for SCFFT_F32.
 *                   Field values are dimensionless (h' = h/(jc l), Eq. 8).
 *                   A scalar mask is uint8 [Nz][Ny][Nx], nonzero = inside.
 *                   Vector fields must start on a multiple of 2 * element
 *                   size (16 bytes FP64, 8 bytes FP32): the transform passes
 *                   move the two nodes x = 2i, 2i+1 in one access.  A
 *                   misaligned field pointer is refused with SCFFT_ERR_ARG
 *                   (e.g. a view of a tensor at an odd element offset).
 *   Nodes           cell-centred: x_i = -L + (i + 1/2) 2L/N, i = 0..N-1.
 *   Streams         every call is ordered on the HIP stream given at create;
 *                   calls that return host values synchronise that stream.
 *   Workspace       device memory the caller provides (scfft_set_workspace)
 *                   and keeps alive while the context uses it; it holds the
 *                   spectrum, the warm start, masks, tables and ODE stages.
 *   Errors          every call returns an scfft_status; negative values are
 *                   errors (nothing was launched, or the context state is as
 *                   described per call), positive values are warnings.  The
 *                   message of the last failure is scfft_last_error(ctx).
 *   Threading       a context is not thread-safe; use one per host thread.
 */
#ifndef SCFFT_H
#define SCFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SCFFT_OK = 0,
  SCFFT_WARN_NOT_CONVERGED = 1, /* iteration (5) stopped at max_iter        */
  SCFFT_WARN_CLAMPED = 2,       /* power-law exponent clamped (overflow)    */
  SCFFT_WARN_TOPOLOGY = 3,      /* Omega not contourwise simply connected   */
  SCFFT_ERR_ARG = -1,           /* invalid argument (NULL, range, order)    */
  SCFFT_ERR_SHAPE = -2,         /* unsupported grid size                    */
  SCFFT_ERR_DEVICE = -3,        /* HIP runtime error or no device           */
  SCFFT_ERR_WORKSPACE = -4,     /* workspace missing, too small, misaligned */
  SCFFT_ERR_NAN = -5,           /* non-finite values met by the integrator  */
  SCFFT_ERR_STEP_UNDERFLOW = -6,/* step size fell below its floor           */
  SCFFT_ERR_GEOMETRY = -7,      /* mask not set, or empty where needed      */
  SCFFT_ERR_STATE = -8          /* checkpoint blob does not fit the context */
} scfft_status;

typedef enum { SCFFT_F64 = 0, SCFFT_F32 = 1 } scfft_precision;

/* Grid of the padded FFT box D.  n[a] = node counts (x, y, z): each a power
 * of two in [8, 512] or 3 * 2^k in [24, 192] (24, 48, 96, 192).
 * half_width_m[a] = L_a in metres.  Sec. 2. */
typedef struct {
  int32_t n[3];
  double half_width_m[3];
} scfft_grid;

/* Material and scaling (Eq. 1, Eq. 8).  n_power and jc (A/m^2) of the power
 * law, e0 (V/m; the paper's value is 1e-4), rho_out the dimensionless
 * fictitious exterior resistivity (Sec. 2; 20 and 100 in Sec. 3), l_char_m the
 * characteristic length l of Eq. 8 in metres. */
typedef struct {
  double n_power;
  double jc;
  double e0;
  double rho_out;
  double l_char_m;
} scfft_material;

/* Uniform applied field h_e(t) (Sec. 2), given as B = mu0 h in tesla.
 *   RAMP_HOLD  B(t) = dir * amp_T * min(t / t_ramp_s, 1)
 *   SINE       B(t) = dir * amp_T * sin(2 pi freq_hz t)
 *   PWL        B(t) linear between the n_pts points (t_s[k], b_T[3k..3k+2]),
 *              constant outside; points are copied at scfft_set_drive.
 * dir need not be normalised (it is).  Kinks are integrator breakpoints. */
enum { SCFFT_DRIVE_RAMP_HOLD = 0, SCFFT_DRIVE_SINE = 1, SCFFT_DRIVE_PWL = 2 };
typedef struct {
  int32_t kind;
  int32_t n_pts;
  double dir[3];
  double amp_T;
  double t_ramp_s;
  double freq_hz;
  const double* t_s;
  const double* b_T;
} scfft_drive;

/* Primitive of the voxelizer (the shape of Omega, Sec. 2).  Shapes apply in
 * order: ADD sets nodes strictly inside the primitive, SUB clears nodes inside
 * or on it; a node within 1e-9 * (smallest cell size) of a surface counts as
 * on it, so nodes on the boundary of Omega fall outside Omega.
 *   BOX       center_m, size_m = half-extents
 *   CYLINDER  center_m, axis (0, 1, 2), size_m = (radius, unused, half-height)
 *   SPHERE    center_m, size_m[0] = radius */
enum { SCFFT_SHAPE_BOX = 0, SCFFT_SHAPE_CYLINDER = 1, SCFFT_SHAPE_SPHERE = 2 };
enum { SCFFT_OP_ADD = 0, SCFFT_OP_SUB = 1 };
typedef struct {
  int32_t kind;
  int32_t op;
  int32_t axis;
  int32_t reserved;
  double center_m[3];
  double size_m[3];
} scfft_shape;

/* Options of the right-hand side (Sec. 2, iteration (5) and its stopping rule).
 *   delta_it     tolerance: stop when the mean over Omega_out nodes of
 *                |hdot^{i+1} - hdot^i| < delta_it * max(|dh_e/dt|, 1)
 *                (paper: 2e-5)
 *   min_iter     iterations always run (default 1)
 *   max_iter     stop with SCFFT_WARN_NOT_CONVERGED after this many (200)
 *   fixed_iter   if > 0, run exactly this many and skip the test
 *   smooth_phi   if nonzero, Phi's symbol is Gaussian-smoothed too (default 0)
 *   sigma_scale  smoothing width in units of half the cell diagonal (1)
 *   fuse_xy      per-component steps (warm start, masks, exterior update with
 *                fixed_iter) as one fused xy-plane pass instead of y inverse,
 *                x pass, y forward, where the plane fits on chip (Nx = Ny <=
 *                128): 0 never, 1 (default) where measured faster (Nx = Ny
 *                <= 64), 2 always.  Results agree to rounding.
 *   prune_box    1 (default): skip the parts of the transforms that only touch
 *                zeros or unused values outside the bounding box of Omega
 *                (fields masked to Omega, rates needed on Omega); 0: full
 *                transforms.  Results are identical.
 *   x_alt        0 (default) or 1: the per-component x passes (input, warm
 *                start, masks, exterior update with fixed_iter, store) hold
 *                the alternate number of elements per thread (8 instead of 4:
 *                other radices and rows per block).  Results agree to
 *                rounding; scfft_autotune picks it.
 *   y_alt, z_alt 0 (default) or 1: the y passes, and the z passes with the
 *                operator symbols, hold the alternate number of elements per
 *                thread (y: 8 instead of 4 in FP64, 4 instead of 8 in FP32;
 *                z: 8 instead of 4 in FP64, 4 instead of 8 in FP32), i.e.
 *                other radix sequences, column widths per block and register
 *                budgets.  Results agree to rounding; scfft_autotune picks
 *                them. */
typedef struct {
  double delta_it;
  int32_t min_iter;
  int32_t max_iter;
  int32_t fixed_iter;
  int32_t smooth_phi;
  double sigma_scale;
  int32_t fuse_xy;
  int32_t prune_box;
  int32_t x_alt;
  int32_t y_alt;
  int32_t z_alt;
} scfft_rhs_opts;

typedef struct {
  int32_t iters;        /* iterations (5) run                              */
  int32_t converged;    /* 1 if the stopping rule (or fixed_iter) ended it */
  double last_delta;    /* last mean |hdot^{i+1} - hdot^i| over Omega_out
                           (-1 with fixed_iter: not tracked)              */
  int64_t clamps;       /* power-law evaluations whose exponent was clamped */
} scfft_rhs_stats;

/* Options of the Bogacki-Shampine 3(2) integrator (the paper's ode23).
 *   rtol (2e-4), atol (1e-6, on dimensionless h); err = max_i |E_i| /
 *   max(|y_i|, |y_new,i|, atol/rtol), accept iff err <= rtol.
 *   dt0_s (0 = automatic), dt_max_s (0 = no cap), fixed_steps > 0 = that many
 *   equal steps, all accepted.  breakpoints_s: extra times never stepped over.
 *   max_steps bounds accepted + rejected steps (0 = 10^7).
 *   resume (0 = off): with adaptive steps, continue the step controller
 *   that the context keeps from its last adaptive integration (or from a
 *   state blob, scfft_set_state) when t0_s is the time where that
 *   integration stopped: the right-hand side value there (first same as
 *   last) and the next step size are reused instead of recomputed, so a run
 *   stopped by its observer and resumed from a checkpoint takes the steps
 *   the uninterrupted run takes.  The caller passes the state it stopped
 *   with.  Ignored (a fresh start) when t0_s differs or no continuation is
 *   held; every call that changes the mask, jc map, laws, drive, options,
 *   warm start or workspace drops the continuation. */
typedef struct {
  double rtol;
  double atol;
  double dt0_s;
  double dt_max_s;
  int32_t fixed_steps;
  int32_t n_bp;
  const double* breakpoints_s;
  int64_t max_steps;
  int32_t resume;
  int32_t reserved;
} scfft_ode_opts;

typedef struct {
  int64_t accepted;
  int64_t rejected;
  int64_t rhs_calls;
  int64_t iters_total;   /* sum of iterations (5) over all RHS calls  */
  int64_t not_converged; /* RHS calls that hit max_iter               */
  int64_t clamps;
  double t_s;            /* time reached                               */
  double dt_last_s;
  double err_last;
} scfft_ode_stats;

/* Called after every accepted step with the time (s) and the device state
 * (the integrator's own copy of h, valid during the call only; read it, do
 * not write it); it may call readout entry points on the same context, and
 * scfft_step_moment.  A nonzero return stops the integration
 * (scfft_integrate then returns SCFFT_OK). */
typedef int32_t (*scfft_observer)(void* user, double t_s, const void* h_dev);

/* Right-hand side on host arrays, for scfft_bs23_host. */
typedef int32_t (*scfft_host_rhs)(void* user, double t, const double* y, double* ydot);

typedef struct scfft_ctx scfft_ctx;

/* ---- host-only utilities (no device work) ---- */

/* Fill the defaults named above. */
void scfft_default_rhs_opts(scfft_rhs_opts* o);
void scfft_default_ode_opts(scfft_ode_opts* o);

/* Scaling of Eq. 8: t0 = mu0 jc l^2 / e0 (s) and h_scale = jc l (A/m). */
scfft_status scfft_units(const scfft_material* m, double* t0_s, double* h_scale);

/* Applied field of a drive at time t_s, dimensionless (h' and dh'/dt'). */
scfft_status scfft_drive_eval(const scfft_drive* d, const scfft_material* m, double t_s,
                              double he[3], double hedot[3]);

/* Voxelize shapes (coordinates in metres, scaled by m->l_char_m) on the grid
 * into a host uint8 mask [Nz][Ny][Nx] the caller owns. */
scfft_status scfft_voxelize_host(const scfft_grid* g, const scfft_material* m,
                                 const scfft_shape* shapes, int32_t n_shapes, uint8_t* mask);

/* Topology of a mask [Nz][Ny][Nx] (nonzero = Omega), taken as the union of
 * the closed voxels of its nodes in R^3: betti[0] components, betti[1]
 * independent closed contours that bound no surface inside Omega, betti[2]
 * enclosed cavities.  Sec. 2 restricts the method to contourwise simply
 * connected domains (every closed contour in Omega bounds a surface in
 * Omega), i.e. betti[1] = 0; otherwise the return is SCFFT_WARN_TOPOLOGY and
 * the exterior problem loses the circulation of h around the holes.
 * SCFFT_ERR_SHAPE for 2^31 - 1 nodes or more. */
scfft_status scfft_mask_betti_host(const int32_t n[3], const uint8_t* mask, int64_t betti[3]);

/* Bogacki-Shampine 3(2) with the step control of scfft_integrate, on host
 * arrays y[n] (in/out) with a host right-hand side; t in the caller's units.
 * The device integrator runs the same controller. */
scfft_status scfft_bs23_host(int64_t n, double* y, double t0, double t1, scfft_host_rhs f,
                             void* user, const scfft_ode_opts* o, scfft_ode_stats* st);

/* ---- context ---- */

/* Create a context on the current HIP device.  hip_stream is a hipStream_t
 * (NULL = the null stream).  Returns SCFFT_ERR_SHAPE for unsupported n,
 * SCFFT_ERR_DEVICE without a usable device. */
scfft_status scfft_create(scfft_ctx** out, const scfft_grid* g, const scfft_material* m,
                          scfft_precision prec, void* hip_stream);
void scfft_destroy(scfft_ctx* ctx);

/* Bytes of device workspace the context needs (256-byte aligned start). */
scfft_status scfft_workspace_size(const scfft_ctx* ctx, size_t* bytes);
/* Attach the workspace; uploads tables (synchronously); clears mask, jc map
 * and warm start. */
scfft_status scfft_set_workspace(scfft_ctx* ctx, void* dev_ptr, size_t bytes);

/* Voxelize Omega on the host and upload the mask (synchronous).  Returns
 * SCFFT_WARN_TOPOLOGY (the mask is still set) when Omega is not contourwise
 * simply connected (scfft_mask_betti_host). */
scfft_status scfft_voxelize(scfft_ctx* ctx, const scfft_shape* shapes, int32_t n_shapes);
/* Copy a caller's device mask uint8 [Nz][Ny][Nx] into the workspace; the
 * same topology warning. */
scfft_status scfft_set_mask(scfft_ctx* ctx, const uint8_t* dev_mask);
/* Betti numbers of the current mask, as scfft_mask_betti_host returns them;
 * SCFFT_ERR_GEOMETRY without a mask. */
scfft_status scfft_mask_betti(const scfft_ctx* ctx, int64_t betti[3]);
/* Optional local critical density kappa = jc(x)/jc [Nz][Ny][Nx] in the
 * context precision, all finite and > 0; NULL clears it (kappa = 1).
 * Copied, then checked on the device: SCFFT_ERR_ARG (and no map, kappa = 1)
 * if any value is not finite or not > 0, since Eq. 1 takes its logarithm.
 * Synchronous. */
scfft_status scfft_set_jc_map(scfft_ctx* ctx, const void* dev_kappa);
scfft_status scfft_set_drive(scfft_ctx* ctx, const scfft_drive* d);
/* Field-dependent critical density, the e(j, h) relation that Sec. 2 allows
 * after Eq. 1 (the paper fixes no form): a Kim-type law
 *   jc(x, B) = jc kappa(x) / (1 + |B| / b0_T)^alpha,  B = mu0 h the local field,
 * used in Eq. 1 in place of jc kappa(x).  b0_T = 0 switches it off (the
 * default); alpha >= 0.  The reverse mode rejects it (SCFFT_ERR_ARG). */
scfft_status scfft_set_field_law(scfft_ctx* ctx, double b0_T, double alpha);
/* Anisotropic current-voltage relation, another relation that Sec. 2 allows
 * in place of Eq. 1 (the paper fixes no form): in Omega
 *   e = e0 (|j|_A / jc_loc)^(n-1) A j / jc_loc,  A = diag(a[0], a[1], a[2]),
 *   |j|_A^2 = a[0] jx^2 + a[1] jy^2 + a[2] jz^2,
 * the gradient of the dissipation potential jc_loc e0/(n+1) (|j|_A/jc_loc)^(n+1),
 * with jc_loc = jc kappa(x) (and the field law's factor, if set); a current
 * along axis c alone meets e0 at jc_loc / sqrt(a[c])^((n+1)/n).  Weights in
 * x, y, z order, finite and > 0; NULL or (1, 1, 1) restores the isotropic
 * law (the default).  The reverse mode rejects it (SCFFT_ERR_ARG). */
scfft_status scfft_set_anisotropy(scfft_ctx* ctx, const double a[3]);
scfft_status scfft_set_rhs_opts(scfft_ctx* ctx, const scfft_rhs_opts* o);
/* The options in force (after scfft_autotune: its choice). */
scfft_status scfft_get_rhs_opts(const scfft_ctx* ctx, scfft_rhs_opts* o);
/* Forget the warm start of iteration (5): the next RHS starts from Ohm's law. */
scfft_status scfft_reset_warm(scfft_ctx* ctx);

/* Virgin state of Sec. 3: h = h_e(t0) everywhere (j = 0); clears the warm start. */
scfft_status scfft_init_state(scfft_ctx* ctx, double t0_s, void* h_dev);

/* The right-hand side hdot' = f(t, h) (Sec. 2): j = curl h, e from Eq. 1 in
 * Omega and rho_out j outside, hdot = -curl e in Omega, iteration (5) in
 * Omega_out from the warm start (hdot_out of the previous call; Ohm's law on
 * the first call).  h_dev and hdot_dev must not alias.  Updates the warm
 * start.  Requires workspace and mask.  stats may be NULL. */
scfft_status scfft_rhs_eval(scfft_ctx* ctx, double t_s, const void* h_dev, void* hdot_dev,
                            scfft_rhs_stats* stats);

/* Integrate h from t0_s to t1_s in place (method of lines, Sec. 2).  The
 * observer (may be NULL) sees every accepted step.  On SCFFT_ERR_NAN or
 * SCFFT_ERR_STEP_UNDERFLOW h holds the last accepted state.  The state is
 * advanced in a workspace buffer and copied back to h when the call ends;
 * the Runge-Kutta stage arguments y + c k are formed inside the first
 * transform pass of each evaluation.  With fixed_steps the next step is
 * enqueued before the host waits for the current one's error norm (the GPU
 * does not idle during the observer): when the observer stops the run, that
 * next step has already been evaluated and is dropped, and the context's
 * warm start is that of its evaluations. */
scfft_status scfft_integrate(scfft_ctx* ctx, double t0_s, double t1_s, void* h_dev,
                             const scfft_ode_opts* o, scfft_observer obs, void* user,
                             scfft_ode_stats* stats);

/* Autotuner: times one right-hand-side call (fixed_iter > 0) under each pass
 * schedule this grid supports on the caller's state h, calls times each after
 * a warm-up call, and keeps the fastest.  The schedules: row/column passes or
 * fused xy-plane passes where a z plane fits in LDS (rhs option fuse_xy 0 or
 * 2), crossed with the instantiated variants of the passes (x_alt for the
 * per-component x passes of the row/column schedule, y_alt, z_alt: other
 * elements per thread, radices and column widths).  The warm start is
 * restored afterwards.  fuse_xy and ms_per_call (may be NULL) receive the
 * schedule and its mean time per call; scfft_get_rhs_opts returns all
 * options.  Synchronous. */
scfft_status scfft_autotune(scfft_ctx* ctx, const void* h_dev, int32_t calls, int32_t* fuse_xy,
                            double* ms_per_call);

/* ---- graph-replayed fixed-step integration ----
 *
 * The fixed-step mode of scfft_integrate (equal steps (t1 - t0)/steps of the
 * Bogacki-Shampine pair, Sec. 2 method of lines) with each step captured once
 * as a HIP graph (two graphs: accepting a step swaps buffer roles) and
 * replayed, so a whole integration is enqueued without host round trips.
 * The applied-field rates at all stage times are tabulated on the host and
 * read on the device by step number; the error norm of every step is kept
 * on the device, and a non-finite one stops every later kernel.  Needs
 * fixed_iter > 0; no observer.  Asynchronous on the context stream:
 * scfft_integrate_graph enqueues and returns, scfft_integrate_wait
 * synchronises, writes the last accepted state to h and fills the stats
 * (SCFFT_ERR_NAN after a non-finite error norm).  In between, the context
 * accepts no other call (SCFFT_ERR_STATE), h and the graph workspace must
 * stay allocated, and contexts on different streams run concurrently (the
 * batched use).  graph_ws: device buffer of scfft_graph_workspace_size bytes,
 * 256-byte aligned, owned by the caller.  The captured graphs stay with the
 * context and are replayed by the next call with the same graph_ws, steps and
 * step size (a run continued chunk by chunk pays the capture once); any call
 * that changes the mask, jc map, field law, drive, options or workspace
 * forces a new capture. */
scfft_status scfft_graph_workspace_size(const scfft_ctx* ctx, int32_t steps, size_t* bytes);
scfft_status scfft_integrate_graph(scfft_ctx* ctx, double t0_s, double t1_s, int32_t steps,
                                   void* graph_ws, size_t graph_bytes, void* h_dev);
scfft_status scfft_integrate_wait(scfft_ctx* ctx, scfft_ode_stats* stats);
/* The magnetic moment (as scfft_moment: all nodes, or Omega only) of every
 * state accepted by the last graph integration, summed on the device by the
 * power-law pass of each step's last evaluation; valid after
 * scfft_integrate_wait while that integration's graph workspace is still
 * allocated.  Writes min(max_steps, accepted) rows m_Am2[3*k + c] (A m^2)
 * and the accepted count to *n_steps. */
scfft_status scfft_graph_moments(scfft_ctx* ctx, int32_t omega_only, int32_t max_steps, double* m_Am2,
                                 int32_t* n_steps);

/* ---- batches of same-size instances ----
 *
 * Many instances of the method (Sec. 2: each its own body, material and
 * applied field) on grids of one size, advanced together: every transform
 * pass is a single launch over all of them, so boxes too small to fill the
 * GPU alone do so as a batch.  The members are ordinary contexts, each set
 * up as usual (mask, drive, material n / jc / rho_out, optional jc map,
 * options), with
 *   - equal node counts, dimensionless half widths (box / l) and precision,
 *     one stream, equal right-hand-side options with fixed_iter > 0;
 *   - no field-dependent or anisotropic law; jc maps on all or on none;
 *   - workspaces that follow each other at one constant stride (member b's
 *     workspace = member 0's + b * stride bytes, stride >= the workspace
 *     size, a multiple of 256): one allocation carved in equal slices.
 * A batch holds no device memory of its own beyond those workspaces; the
 * members stay usable alone between batch calls.  Batched fields are
 * caller-owned device arrays with member b's field at base + b *
 * field_stride elements (field_stride >= 3 Nx Ny Nz, even).  Up to 512
 * members; every call runs on member 0's stream.  Errors of batch calls are
 * reported through member 0 (scfft_batch_last_error). */
typedef struct scfft_batch scfft_batch;
scfft_status scfft_batch_create(scfft_batch** out, scfft_ctx* const* members, int32_t count);
void scfft_batch_destroy(scfft_batch* batch);
/* One right-hand side of every member at time t_s (each in its own Eq. 8
 * units), as scfft_rhs_eval gives it, with batched launches; updates every
 * member's warm start (members must agree on having one). */
scfft_status scfft_batch_rhs_eval(scfft_batch* batch, double t_s, const void* h_dev, void* hdot_dev,
                                  int64_t field_stride);
/* The graph-replayed fixed-step integration of scfft_integrate_graph for
 * the whole batch: `steps` equal Bogacki-Shampine steps from t0_s to t1_s of
 * every member, one captured step of batched launches replayed `steps`
 * times; each member's step size, stage coefficients and applied-field rates
 * (tabulated on the host) follow its own time unit.  A non-finite error norm
 * of any member stops all.  scfft_batch_integrate_wait synchronises, writes
 * the last accepted states back to h (batched) and fills stats[count].
 * graph_ws: scfft_batch_graph_workspace_size bytes, 256-byte aligned. */
scfft_status scfft_batch_graph_workspace_size(const scfft_batch* batch, int32_t steps, size_t* bytes);
scfft_status scfft_batch_integrate_graph(scfft_batch* batch, double t0_s, double t1_s, int32_t steps,
                                         void* graph_ws, size_t graph_bytes, void* h_dev,
                                         int64_t field_stride);
scfft_status scfft_batch_integrate_wait(scfft_batch* batch, scfft_ode_stats* stats);
const char* scfft_batch_last_error(const scfft_batch* batch);

/* ---- reverse mode (gradients) ----
 *
 * Differentiating the discrete map is an extension of the paper (Sec. 2
 * gives the forward method only).  The map is made smooth by a fixed number
 * K = fixed_iter > 0 of exterior iterations (Eq. 5) and by carrying the warm
 * start as an explicit state: one right-hand-side call is
 *   (h, w) -> (hdot, w' = (1 - chi) hdot),   hdot^0 = chi g + (1 - chi) w,
 * g = -C_s e(C_s h) (Eqs. 1, 3, 4), a first call (no warm start) using
 * hdot^0 = g.  C_s and Phi have Hermitian symbols and the Jacobian of Eq. 1
 * is symmetric, so the reverse pass runs the forward passes in reverse order
 * at about the cost of one call.  All fields are dimensionless (Eq. 8),
 * layout [3][Nz][Ny][Nx], precision of the context; calls are synchronous.
 * SCFFT_ERR_ARG when fixed_iter is 0 or outputs alias inputs. */

/* Vector-Jacobian product of one call at state h: given lam = dL/dhdot and
 * mu = dL/dw' (may be NULL: zero), writes hbar = dL/dh (all nodes) and, if
 * wbar is non-NULL, wbar = dL/dw (zero in Omega); warm_used says whether the
 * forward call had a warm start.  kappa_bar (scalar field [Nz][Ny][Nx], may
 * be NULL) is ACCUMULATED with dL/dkappa, kappa = jc(x)/jc (1 where no map
 * is set).  n_bar = dL/dn and hedot_bar = dL/d(dh_e'/dt') (may be NULL). */
scfft_status scfft_rhs_vjp(scfft_ctx* ctx, const void* h_dev, int32_t warm_used,
                           const void* lam_dev, const void* mu_dev, void* hbar_dev, void* wbar_dev,
                           void* kappa_bar_dev, double* n_bar, double hedot_bar[3]);

/* Device workspace (bytes, 256-byte aligned start) for scfft_integrate_adjoint:
 * ceil(steps / checkpoint_every) checkpoints of 3 fields, a tape of
 * 6 * checkpoint_every + 1 fields and 10 work fields. */
scfft_status scfft_adjoint_workspace_size(const scfft_ctx* ctx, int32_t steps,
                                          int32_t checkpoint_every, size_t* bytes);

/* Gradient of a loss L(h(t1)) through `steps` equal Bogacki-Shampine steps
 * (the fixed-step mode of scfft_integrate) from h0 at t0_s, started with no
 * warm start (as after scfft_reset_warm).  The forward pass keeps
 * checkpoints every checkpoint_every steps; the reverse pass recomputes one
 * segment at a time and runs the adjoint steps backwards.  Given hT_bar =
 * dL/dh(t1) it writes hT (the forward result, may be NULL), h0_bar =
 * dL/dh0, n_bar (may be NULL) and p_bar = dL/dp (may be NULL) for the drive
 * vector p = amplitude x direction (dimensionless) of a drive h_e = p f(t)
 * (ramp-hold or sine; SCFFT_ERR_ARG for a PWL drive); kappa_bar (may be
 * NULL) is accumulated.  The context's warm start is cleared on return. */
scfft_status scfft_integrate_adjoint(scfft_ctx* ctx, double t0_s, double t1_s, int32_t steps,
                                     int32_t checkpoint_every, void* adj_ws, size_t adj_bytes,
                                     const void* h0_dev, const void* hT_bar_dev, void* hT_dev,
                                     void* h0_bar_dev, void* kappa_bar_dev, double* n_bar,
                                     double p_bar[3]);

/* ---- operators and readouts ---- */

/* out = C_s v, the smoothed spectral curl (derivatives of Eqs. 3, 4). */
scfft_status scfft_curl(scfft_ctx* ctx, const void* v_dev, void* out_dev);
/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): out =
 * C_s v exactly as scfft_curl computes it, but the half spectrum and the
 * axis tables live in a static device array of the library instead of the
 * context's workspace, which need not be attached.  The array holds 8 MiB
 * on each GPU the library runs on, kept until the process ends; grids whose
 * spectrum and tables need more (e.g. above 64^3 nodes in FP64, 64 x 64 x
 * 128 in FP32) are refused with SCFFT_ERR_WORKSPACE.  No allocating routine
 * is called.  Every call on one GPU reuses that GPU's array: calls ordered
 * on one stream are safe, calls that overlap in time on one GPU (other
 * streams or threads) race.  The current device must be the context's
 * (SCFFT_ERR_DEVICE otherwise).  Asynchronous on the context stream. */
scfft_status scfft_curl_noalloc(scfft_ctx* ctx, const void* v_dev, void* out_dev);
/* out = Phi[v], Eq. 7 with the k = 0 rule (smoothed iff smooth_phi). */
scfft_status scfft_phi(scfft_ctx* ctx, const void* v_dev, void* out_dev);
/* j' = C_s h (dimensionless current density, all nodes). */
scfft_status scfft_current(scfft_ctx* ctx, const void* h_dev, void* j_dev);
/* Magnetic moment m = 1/2 sum (r x j) dV in A m^2, r from the box centre,
 * over all nodes (omega_only = 0) or Omega nodes only. */
scfft_status scfft_moment(scfft_ctx* ctx, const void* h_dev, int32_t omega_only, double m_Am2[3]);
/* Inside an integrator observer: the moment (as scfft_moment) of the state
 * just accepted, summed from the current density j = C_s h that the
 * right-hand side already formed at that state (Eq. 4), so no transform runs.
 * SCFFT_ERR_STATE when called outside an observer callback. */
scfft_status scfft_step_moment(scfft_ctx* ctx, int32_t omega_only, double m_Am2[3]);
/* Mean of |B| = mu0 |h| (tesla) over the nodes of a device region mask. */
scfft_status scfft_region_mean_abs_b(scfft_ctx* ctx, const void* h_dev, const uint8_t* dev_region,
                                     double* b_T);
/* Stray-current fraction ||(1 - chi) j|| / ||chi j|| (Euclidean norms over
 * all nodes and components) of j = C_s h (Eq. 4): the current left in
 * Omega_out, which Sec. 2 suppresses through rho_out and iteration (5) rather
 * than removes exactly.  0 when j vanishes in Omega.  Requires the mask;
 * synchronous; overwrites the reverse-mode buffers of the workspace. */
scfft_status scfft_stray_fraction(scfft_ctx* ctx, const void* h_dev, double* frac);
/* B = mu0 h (tesla) at npts points (metres), trilinear between nodes with
 * periodic wrap; b_T[3*p + c]. */
scfft_status scfft_probe_b(scfft_ctx* ctx, const void* h_dev, const double* xyz_m, int32_t npts,
                           double* b_T);

/* ---- per-kernel timing ---- */

/* Kernel kinds of the pass schedule.  X passes (rows along x, fused pointwise
 * work) by operation, Y passes (columns along y) by direction, Z passes
 * (columns along z with the operator symbol) by symbol. */
enum {
  SCFFT_KERNEL_X_FWD = 0,    /* real field -> x spectrum                   */
  SCFFT_KERNEL_X_LAW,        /* -> j -> e of Eq. 1 -> spectrum             */
  SCFFT_KERNEL_X_HIN,        /* -> -curl e, warm start -> hdot, spectrum   */
  SCFFT_KERNEL_X_MASK,       /* -> jdot masked to Omega -> spectrum        */
  SCFFT_KERNEL_X_UPDATE,     /* -> Phi, exterior update (Eq. 5) -> spectrum */
  SCFFT_KERNEL_X_UPDATE_LAST,/* the same without the forward transform     */
  SCFFT_KERNEL_X_STORE,      /* -> real field                              */
  SCFFT_KERNEL_X_MOMENT,     /* -> j -> moment partial sums                */
  SCFFT_KERNEL_Y_FWD,
  SCFFT_KERNEL_Y_INV,
  SCFFT_KERNEL_Z_CURL,       /* z transform, smoothed i k x, inverse       */
  SCFFT_KERNEL_Z_PHI,        /* z transform, i k x / |k|^2, inverse        */
  SCFFT_KERNEL_XY_FWD,       /* fused xy-plane passes (one component, one  */
  SCFFT_KERNEL_XY_HIN,       /* z plane in LDS): y inverse, x inverse,     */
  SCFFT_KERNEL_XY_MASK,      /* pointwise step, x forward, y forward       */
  SCFFT_KERNEL_XY_UPDATE,
  SCFFT_KERNEL_XY_UPDATE_LAST,
  SCFFT_KERNEL_XY_STORE,
  SCFFT_KERNEL_X_ADJ_START,  /* reverse mode: cotangent in, masked -> spectrum */
  SCFFT_KERNEL_X_ADJ_ACC,    /* -> adjoint iterate, running sum -> spectrum  */
  SCFFT_KERNEL_X_ADJ_LAST,   /* -> last adjoint iterate, gbar -> spectrum    */
  SCFFT_KERNEL_X_ADJ_LAW,    /* -> ebar -> jbar (Eq. 1 transposed) -> spectrum */
  SCFFT_KERNEL_KINDS
};

/* enable != 0: start timing every pass launch (and reset the totals); 0: stop.
 * Each pass dispatch carries its own start/stop HIP event pair on the context
 * stream, so the durations are those of the kernel bodies. */
scfft_status scfft_profile(scfft_ctx* ctx, int32_t enable);
/* Launch counts, summed kernel durations (ms) and summed algorithmic bytes
 * (one read of each launch's inputs and one write of its outputs, for the
 * ranges it covered) per kind since enable; total_bytes may be NULL.
 * Synchronises with the recorded events. */
scfft_status scfft_profile_read(scfft_ctx* ctx, int64_t launches[SCFFT_KERNEL_KINDS],
                                double total_ms[SCFFT_KERNEL_KINDS],
                                double total_bytes[SCFFT_KERNEL_KINDS]);

/* ---- checkpoint ---- */

/* Serialise the context's evolving state (pass blob = NULL to query
 * bytes): the right-hand-side options, the warm start of iteration (5), the
 * iteration count the adaptive loop launches first, and the continuation of
 * the adaptive step controller (time, next step size, whether the last
 * step was rejected, and the first-same-as-last right-hand side k1 at that
 * time), so that scfft_set_state on a fresh context of the same grid and
 * precision followed by scfft_integrate with resume = 1 repeats what the
 * original context would have done.  Host blob, caller-owned; SCFFT_ERR_STATE
 * on a blob for another grid or precision, or cut short. */
scfft_status scfft_get_state(scfft_ctx* ctx, void* blob, size_t* bytes);
scfft_status scfft_set_state(scfft_ctx* ctx, const void* blob, size_t bytes);

const char* scfft_status_string(scfft_status s);
const char* scfft_last_error(const scfft_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SCFFT_H */
