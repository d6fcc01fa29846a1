/*
 * fcsph.h - C ABI of the MI355X (gfx950) FC(Gram)-based spectral ISPH step.
 *
 * The library implements the data-parallel hot path of the FC-based spectral
 * incompressible SPH scheme (Lin, Fourtakas & Rogers): Fourier continuation of
 * non-periodic fields across walls, kernel-weighted SPH gradient / divergence /
 * Laplacian evaluated in frequency space through the convolution theorem, a
 * spectral pressure-Poisson solve, and the first-order projection update.
 * Every stage runs in hand-written HIP kernels on the device.
 *
 * Conventions for every call
 *  - Field arrays are DEVICE pointers, contiguous, row-major with x fastest:
 *    2D [ny][nx], 3D [nz][ny][nx].  Physical arrays have exactly the physical
 *    shape; the output of fcsph_fc_extend has n+C points on each walled axis.
 *  - State arrays (velocity, pressure, forcing, wall data) are FP64.
 *    Derivative outputs and the PPE right-hand side are double in FCSPH_FP64
 *    plans and float in FCSPH_FP32_MIXED plans.
 *  - The caller owns every buffer, including the plan workspace; the library
 *    never allocates device memory.  A plan keeps pointers into its
 *    workspace, which must outlive the plan.
 *  - Calls are asynchronous on the context's HIP stream.  Argument errors are
 *    detected synchronously and returned as status codes; device faults
 *    surface as FCSPH_E_HIP at the next call or at fcsph_ctx_sync.  No call
 *    aborts or throws across the ABI.
 *  - A plan is immutable after creation.  Calls on one context must not run
 *    concurrently from several host threads.
 */
#ifndef FCSPH_H
#define FCSPH_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FCSPH_OK = 0,
  FCSPH_E_INVALID = -1,      /* bad argument (null pointer, shape, value)          */
  FCSPH_E_UNSUPPORTED = -2,  /* valid but not implemented (e.g. a BC combination) */
  FCSPH_E_WORKSPACE = -3,    /* workspace too small or misaligned                  */
  FCSPH_E_HIP = -4,          /* HIP runtime error (launch failure, device fault)   */
  FCSPH_E_NONFINITE = -5     /* reserved: non-finite values detected               */
} fcsph_status;

typedef enum { FCSPH_AXIS_PERIODIC = 0, FCSPH_AXIS_WALLED = 1 } fcsph_axis_kind;
typedef enum { FCSPH_BC_DIRICHLET = 0, FCSPH_BC_NEUMANN = 1 } fcsph_bc;
typedef enum { FCSPH_FIELD_VELOCITY = 0, FCSPH_FIELD_PRESSURE = 1 } fcsph_field_class;
typedef enum { FCSPH_FP64 = 0, FCSPH_FP32_MIXED = 1 } fcsph_precision;
typedef enum { FCSPH_PPE_PHYSICAL = 0, FCSPH_PPE_EXTENDED = 1 } fcsph_ppe_domain;
typedef enum { FCSPH_EIG_SPECTRAL = 0, FCSPH_EIG_FD2 = 1, FCSPH_EIG_SPH = 2 } fcsph_eig;
/* SPH kernels.  Wendland C2 (compact support 2h).  The Gaussian family of
 * the section on high-order Gaussian kernel functions and its appendix:
 * W_2n = (1/(pi h^2)) P_n(q^2) exp(-q^2) with P_n from the moment conditions
 * (G4 = 2 - q^2, G6 = 3 - 3q^2 + q^4/2, G8 = 4 - 6q^2 + 2q^4 - q^6/6; G10 as the
 * conditions give it, 5 - 10q^2 + 5q^4 - 5q^6/6 + q^8/24, where the printed
 * formula violates them); infinite support, sampled at the minimum-image
 * displacement over the whole extended lattice (an offset of exactly half a
 * period averages its two images).  The Gaussians are built for 2D lattices
 * on the whole-period route (FCSPH_OPS_FFT): the windowed and direct routes
 * rely on a compact support. */
typedef enum {
  FCSPH_KERNEL_WENDLAND_C2 = 0,
  FCSPH_KERNEL_GAUSSIAN_G2 = 2,
  FCSPH_KERNEL_GAUSSIAN_G4 = 4,
  FCSPH_KERNEL_GAUSSIAN_G6 = 6,
  FCSPH_KERNEL_GAUSSIAN_G8 = 8,
  FCSPH_KERNEL_GAUSSIAN_G10 = 10
} fcsph_kernel;
/* How the circular convolutions of the operators (period n + C on a walled
 * axis) are evaluated; all three give the same result up to rounding:
 *  FCSPH_OPS_FFT         DFT of the whole FC-extended line (length n + C,
 *                        Bluestein where n + C has a large prime factor),
 *                        symbol multiply, inverse DFT, restriction;
 *  FCSPH_OPS_DIRECT      direct tap sums over the compact kernel support;
 *  FCSPH_OPS_FFT_WINDOW  the convolution theorem on the window the physical
 *                        outputs see: the n physical values, the first R and
 *                        the last R continuation values (R = kernel reach in
 *                        lattice points), zero padded to a smooth length
 *                        L >= n + 2R.  A length-L cyclic convolution of that
 *                        window equals the period-(n + C) convolution at every
 *                        physical point, because no tap reaches farther. */
typedef enum { FCSPH_OPS_FFT = 0, FCSPH_OPS_DIRECT = 1, FCSPH_OPS_FFT_WINDOW = 2 } fcsph_op_eval;

/*
 * Problem descriptor.  Axes are indexed 0 = x, 1 = y, 2 = z.
 *  n[a]        physical points on axis a (n[2] ignored in 2D)
 *  dx          isotropic lattice spacing; a walled axis spans [0, (n-1) dx]
 *              with both walls on lattice points, a periodic axis has period
 *              n dx
 *  axis[a]     fcsph_axis_kind
 *  vel_bc, prs_bc [a][0|1]  wall types (fcsph_bc) of the low / high wall of a
 *              walled axis, for the velocity and the pressure field classes
 *              (wall conditions: eqs. BC_velocity and BC_pressure)
 *  fc_d, fc_C  FC matching / continuation points: 5 and 25 for FC(Gram);
 *              any 1 <= fc_d <= 16, 2 <= fc_C <= 4096 (the paper's own FC:
 *              d fit points, C = the extension length, e.g. 10 and n / 4)
 *  fc_M_dir, fc_M_neu  HOST pointers to the C x d row-major FP64 continuation
 *              maps of a Dirichlet / Neumann wall (row r - 1: the value r
 *              lattice steps beyond the wall from the d values nearest it,
 *              ordered inward to wall; the low wall uses the same map on its
 *              mirrored values, so a map must be of that symmetric form, as
 *              FC(Gram) and the paper's blended polynomial FC are); copied at
 *              plan creation
 *  kernel, h_over_dx   SPH kernel (fcsph_kernel) and smoothing length h / dx
 *              (1.3 for Wendland C2 in the configured workloads, 8 for the
 *              Gaussians as printed)
 *  prec        fcsph_precision
 *  ppe_domain  fcsph_ppe_domain.  FCSPH_PPE_PHYSICAL (the paper's solver): the
 *              PPE on the physical lattice by per-axis transforms (section on
 *              the spatial discretisation of pressure).  FCSPH_PPE_EXTENDED
 *              (the fully periodic alternative named at the end of the section
 *              integrating FC into the solver): the projection of u* on the
 *              extended periodic lattice in its spectrum, phi_hat = (rho/dt)
 *              sum_a S_a e_a / sum_a S_a^2 with e_a = DFT(FC(u*_a)) and S_a
 *              the gradient symbols (modes where the sum vanishes get zero),
 *              u <- IDFT(e_a - (dt/rho) S_a phi_hat) restricted, walls reset;
 *              there the corrected spectrum has zero SPH divergence.  Needs
 *              op_eval FCSPH_OPS_FFT and FP64 (else FCSPH_E_UNSUPPORTED); it
 *              changes fcsph_project_step only (fcsph_ppe_solve keeps the
 *              physical-domain PPE; fcsph_rk3_substep refuses such plans).
 *  eig         fcsph_eig, the eigenvalues of the PPE division (eq.
 *              division4PPE): SPECTRAL, the exact wavenumbers of each axis
 *              transform; FD2, second-order finite differences; SPH, sum_a
 *              sigma_a(k)^2 with S_a = i sigma_a the gradient symbols (then
 *              the PPE inverts div o grad of the method exactly), for 2D
 *              lattices periodic on every axis and the FFT routes only
 *  rho         fluid density
 *  op_eval     fcsph_op_eval
 *  window_len[a], lines_per_group   schedule hints (0 = the library's
 *              choice): the transform length of a walled axis under
 *              FCSPH_OPS_FFT_WINDOW (>= n + 2R, a product of radices 2, 3, 4,
 *              5, 7, 8 whose stages fit 512 threads per line), and the upper
 *              bound on lines per workgroup of the line kernels (1..16;
 *              default 1).  They change speed, never the result beyond
 *              rounding.
 *  batched     1: the plan will also run in batches (fcsph_batch_add_*).
 *              Its PPE transforms then never use the streamed radix stages
 *              (odd primes 11..31), which only the single-problem kernels
 *              carry; 0 (default): a PPE axis of few, long lines may use
 *              them, and the batch calls refuse such a plan
 *              (FCSPH_E_UNSUPPORTED).  Plain calls of a batched plan give
 *              bitwise the results of its batch items.
 *  radix_order schedule hint for the operator line transforms: 0 (default)
 *              keeps the library's stage order (radices 8, 4, 2, then odd
 *              ascending); k >= 1 runs each operator line plan's stages in
 *              the ((k - 1) mod m)-th of its m distinct radix orderings,
 *              counted in lexicographic order from the ascending one.  The
 *              PPE transforms keep their order.  Changes speed and rounding
 *              only; negative values are FCSPH_E_INVALID.
 */
typedef struct {
  int ndim;
  int n[3];
  double dx;
  int axis[3];
  int vel_bc[3][2];
  int prs_bc[3][2];
  int fc_d, fc_C;
  const double *fc_M_dir;
  const double *fc_M_neu;
  int kernel;
  double h_over_dx;
  int prec;
  int ppe_domain;
  int eig;
  double rho;
  int op_eval;
  int window_len[3];
  int lines_per_group;
  int batched;
  int radix_order;
} fcsph_desc;

typedef struct fcsph_ctx fcsph_ctx;
typedef struct fcsph_plan fcsph_plan;

/* Context: binds a device and a HIP stream (NULL = the default stream).
 * Returns FCSPH_E_INVALID for a bad device index. */
fcsph_status fcsph_ctx_create(int device, void *hip_stream, fcsph_ctx **out);
fcsph_status fcsph_ctx_destroy(fcsph_ctx *c);
/* Waits for all work on the context stream; reports device faults as FCSPH_E_HIP. */
fcsph_status fcsph_ctx_sync(fcsph_ctx *c);
const char *fcsph_status_string(fcsph_status s);
/* Text of the last error on this context (never NULL). */
const char *fcsph_ctx_last_error(fcsph_ctx *c);

/*
 * Kernel timing (a profiling aid, not part of the method).  While enabled,
 * every kernel the library launches on this context is bracketed by two HIP
 * events recorded on the context stream.  fcsph_ctx_read_timing waits for the
 * stream, aggregates the elapsed times by kernel kind since the last read and
 * clears the record: for up to `cap` kinds it writes a NUL-terminated name
 * (at most 31 characters) into names + 32 * i, the launch count and the total
 * milliseconds; *n receives the number of kinds written.
 */
fcsph_status fcsph_ctx_set_timing(fcsph_ctx *c, int enable);
fcsph_status fcsph_ctx_read_timing(fcsph_ctx *c, int cap, char *names, int *counts,
                                   double *total_ms, int *n);
/* Restrict timing to launches of one kernel kind (the name read_timing
 * reports, copied; at most 31 characters); NULL or "" times every kind.
 * Timing one kind brackets one launch per call with events instead of every
 * launch, which keeps the event overhead out of the other kernels.
 * FCSPH_E_INVALID for a longer name. */
fcsph_status fcsph_ctx_set_timing_only(fcsph_ctx *c, const char *name);

/* Bytes of device workspace a plan for *d needs (tables + scratch); the
 * workspace must be 256-byte aligned. */
fcsph_status fcsph_plan_workspace_bytes(const fcsph_desc *d, size_t *bytes);
/* Builds a plan: validates *d, computes every table on the host and copies
 * it into the workspace on the context stream.  Validation: ndim 2 or 3;
 * walled axes need n >= 2 fc_d; the kernel support 2h must be below half of
 * every extended period; FCSPH_E_UNSUPPORTED for combinations not built.
 * Every transform line runs in one workgroup of at most 512 threads.  An
 * operator line's thread holds two butterflies of radix <= 4 or one of radix
 * 5..8 per stage, a PPE line's up to six of radix 2 and two of radix 5..8; a
 * length whose stages need more threads uses Bluestein, with a work length
 * up to 4096 (operators) or 8192 (PPE), and a length beyond that is
 * FCSPH_E_UNSUPPORTED (in practice: lattice sides above about 2020 on the
 * whole-period and direct routes, whose plans hold whole-period transforms;
 * on the windowed route up to about 3050 with Neumann or Dirichlet pressure
 * walls in FP64 (the PPE at length n - 1), and up to 2049 where the
 * PPE needs a transform of length 2(n - 1) (the FP32 form, mixed walls),
 * depending on the factors). */
fcsph_status fcsph_plan_create(fcsph_ctx *c, const fcsph_desc *d, void *workspace,
                               size_t bytes, fcsph_plan **out);
fcsph_status fcsph_plan_destroy(fcsph_plan *p);
/* Operator transform length per axis (L[a] for a < ndim, 1 beyond): n + C on
 * a walled axis, or the window length under FCSPH_OPS_FFT_WINDOW; n on a
 * periodic axis.  For reporting; the layout of user buffers never depends on it. */
fcsph_status fcsph_plan_transform_lengths(const fcsph_plan *p, int L[3]);

/*
 * FC(Gram) extension (FC section, eq. eq:fc_extended and its 2D form
 * eq. eq:fc_2d; FC(Gram) paragraph).  On every walled axis each line
 * f_0..f_{n-1} is extended by C values
 *     e[n-1+i] = (M_hi f_hi)[i] + (M_lo f_lo_rev)[C+1-i],   i = 1..C,
 * with f_hi = (f_{n-d}..f_{n-1}), f_lo_rev = (f_{d-1}..f_0) and the map of each
 * wall's type for field class fc; axes are applied in order x, y, z to every
 * line of the current array.  f: physical FP64 array; f_ext: FP64 array of
 * the extended shape.  Physical values are copied bitwise.
 */
fcsph_status fcsph_fc_extend(fcsph_plan *p, int fc, const double *f, double *f_ext);

/*
 * Spectral SPH gradient (eq. final_dft_gradient evaluated as the circular
 * convolution of eq. circularConv on the FC-extended periodic lattice):
 *     g_a = restrict( IDFT( DFT(FC(f)) * DFT(dV d_a W sampled, corner-wrapped) ) )
 * f: physical FP64 array; g[a] (a < ndim): physical arrays of the plan's
 * output type.  fc selects the velocity or pressure wall maps.
 */
fcsph_status fcsph_spectral_grad(fcsph_plan *p, int fc, const double *f, void *const *g);
/* Spectral SPH divergence sum_a G_a u_a of a velocity (velocity wall maps). */
fcsph_status fcsph_spectral_div(fcsph_plan *p, const double *const *u, void *div);
/* Spectral SPH Laplacian: f convolved with dV lap W (kernel Laplacian). */
fcsph_status fcsph_spectral_lap(fcsph_plan *p, int fc, const double *f, void *lap);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * Laplacian as fcsph_spectral_lap, same kernels and launch sequence, same
 * arguments and output, but its intermediate spectra (x spectra, output
 * spectra, the y-extended spectra in 3D, the FP64 boundary rows of FP32
 * plans, the ghost values of the direct route) live in a fixed 64 MiB static
 * device array instead of the plan's workspace.  Allocates nothing and calls
 * no allocating routine.
 * Limit: lattices whose intermediates need more than 64 MiB (for example
 * 2D beyond about 1900^2 windowed FP64, 3D beyond about 128^3) return
 * FCSPH_E_UNSUPPORTED with the needed size in the context's message.
 * The array is one per GPU and shared by every call on that GPU: calls that
 * overlap on one GPU (other contexts, streams or host threads) race on it;
 * it keeps the last call's contents (every element a call reads it has
 * written first, so nothing needs clearing).  FCSPH_E_HIP if the array's
 * device address could not be obtained at context creation. */
fcsph_status fcsph_spectral_lap_noalloc(fcsph_plan *p, int fc, const double *f, void *lap);

/*
 * Spectral PPE on the physical lattice (pressure section, eqs. DCTI4PPE,
 * DCTDFT_PPE and division4PPE): per axis a DFT (periodic), DCT-I (Neumann
 * walls), DST-I (Dirichlet walls) or a quarter-wave transform (mixed walls);
 * phi_hat = -rhs_hat / sum_a mu_a with the plan's eigenvalue family, in FP64;
 * a vanishing eigenvalue sum (the constant mode) gives phi_hat = 0.
 * rhs: physical array of the plan's output type; phi: physical FP64 array,
 * 0 on Dirichlet pressure walls.
 */
fcsph_status fcsph_ppe_solve(fcsph_plan *p, const void *rhs, double *phi);

/*
 * Finiteness check of a device FP64 array of n values (a served request's
 * output, a state before the next step): counts the NaN and infinite values
 * on the device (a counter in the plan's workspace, cleared by a kernel), then
 * waits for the plan's context stream.  *count (host) receives the count;
 * returns FCSPH_E_NONFINITE when it is nonzero, FCSPH_OK otherwise.  The
 * paper states no such check; it is the error path of the served form.
 */
fcsph_status fcsph_check_finite(fcsph_plan *p, const double *x, size_t n, unsigned long long *count);

/*
 * One first-order projection step (eqs. uStarRK3 and rhsMomtem with
 * a = g = 1, z = 0; eqs. PPE and u^n+1):
 *   u*  = u - dt [ (u . grad) u - nu lap u - force ],  Dirichlet walls <- wall_vel
 *   lap phi = (rho/dt) div u*,   u <- u* - (dt/rho) grad phi,  walls <- wall_vel
 * u[a]: FP64 velocity components, updated in place; p_out: FP64 pressure phi
 * (may be NULL); force[a], wall_vel[a]: FP64 arrays or NULL (zero).  Only the
 * Dirichlet wall entries of wall_vel are read.
 */
fcsph_status fcsph_project_step(fcsph_plan *p, double *const *u, double *p_out,
                                const double *const *force, const double *const *wall_vel,
                                double dt, double nu);

/*
 * Linear advection of a scalar with inflow / outflow walls (the Gaussian
 * vortex convection section, eq. linearAdvection, read with C_y du/dy as the
 * second term): sub-step k (0, 1, 2) of the low-storage RK3 of the temporal
 * discretisation section,
 *   F = c[0] du/dx + c[1] du/dy,   u <- u - dt (g_k F + z_k F_prev),
 * with the spectral SPH gradient of the FC-extended u.  The scalar has no wall
 * condition of its own: every wall uses the plain continuation map (the
 * Dirichlet-wall map fc_M_dir, values only); inflow walls (c . n < 0, n the
 * outward normal) take `inflow` (physical array: the exact or imposed values
 * at the end of the sub-step; NULL: zero), outflow walls keep the computed
 * values.  u: physical FP64 device array, updated in place; F_store: physical
 * FP64 device array (caller-owned), holds F of sub-step k - 1 on entry (read
 * when k > 0) and F on exit; c: host array of the two velocity components
 * (x, y); dt: the whole RK3 step; inflow: physical FP64 device array or NULL.
 * A full step is the three calls k = 0, 1, 2 in order on the same F_store.
 * Errors: FCSPH_E_INVALID for a NULL u, F_store or c, k outside 0..2 or a
 * non-positive dt; FCSPH_E_UNSUPPORTED unless the plan is FP64, 2D and on an
 * FFT route (not FCSPH_OPS_DIRECT).
 */
fcsph_status fcsph_advect_rk3_substep(fcsph_plan *p, int k, double *u, double *F_store, const double *c, double dt,
                                      const double *inflow);

/*
 * Sub-step k (0, 1, 2) of the low-storage third-order Runge-Kutta scheme
 * (temporal discretisation section: eqs. uStarRK3, rhsMomtem, PPE and u^n+1
 * with the RK3 coefficients a = (8/15, 2/15, 1/3), g = (8/15, 5/12, 3/4),
 * z = (0, -17/60, -5/12)); signs and the dropped pressure term read as in
 * fcsph_project_step:
 *   F   = (u . grad) u - nu lap u
 *   u*  = u - dt [ g_k F + z_k F_prev - a_k force ],  Dirichlet walls <- wall_vel
 *   lap phi = rho / (a_k dt) div u*,   u <- u* - a_k (dt/rho) grad phi,  walls <- wall_vel
 * dt is the whole RK3 step; sub-step k spans a_k dt, so wall_vel holds the
 * wall data at the end of the sub-step and force its time average over it.
 * F_store[a]: caller-owned FP64 physical arrays, one per velocity component:
 * F_prev on entry (not read for k = 0) and this sub-step's F on exit.
 * u, p_out, force, wall_vel: as for fcsph_project_step.  A full RK3 step is
 * the three calls k = 0, 1, 2 in order on the same F_store.
 * Errors: FCSPH_E_INVALID for k outside 0..2 or a NULL F_store component,
 * otherwise as fcsph_project_step.
 */
fcsph_status fcsph_rk3_substep(fcsph_plan *p, int k, double *const *u, double *p_out,
                               const double *const *force, const double *const *wall_vel,
                               double *const *F_store, double dt, double nu);

/*
 * Batches: the projection steps and PPE solves of many independent plans
 * (different sizes, wall types, precisions and operator evaluations) issued
 * together.  Each added call is validated and its launch sequence recorded
 * (nothing runs); fcsph_batch_launch groups the items whose sequences have the
 * same kernels and launch shapes and issues every launch of a group once for
 * all its items (the group index is the third grid dimension), groups on
 * separate streams.  Results are bitwise those of the plain calls.
 * The argument arrays live in a caller-owned device workspace of
 * fcsph_batch_workspace_bytes(max_items) bytes (256-byte aligned); the batch
 * also holds a pinned host staging copy and its own HIP streams.
 * A plan may appear once per batch (items of one plan would share its
 * scratch); its buffers are read when the batch runs, not when added.
 * The batch stream waits for the context stream before it starts, and the
 * context stream waits for the batch to finish.
 */
typedef struct fcsph_batch fcsph_batch;
fcsph_status fcsph_batch_workspace_bytes(int max_items, size_t *bytes);
fcsph_status fcsph_batch_create(fcsph_ctx *c, int max_items, void *workspace, size_t bytes,
                                fcsph_batch **out);
fcsph_status fcsph_batch_destroy(fcsph_batch *b);
/* Removes every item (the captured graph, if any, stays valid until the next launch). */
fcsph_status fcsph_batch_clear(fcsph_batch *b);
/* Adds one fcsph_project_step / fcsph_ppe_solve call (same arguments). */
fcsph_status fcsph_batch_add_step(fcsph_batch *b, fcsph_plan *p, double *const *u, double *p_out,
                                  const double *const *force, const double *const *wall_vel,
                                  double dt, double nu);
/* Adds one fcsph_rk3_substep call (same arguments).  A replayed graph repeats
 * the recorded sub-step index; the three sub-steps of an RK3 step are three
 * batches. */
fcsph_status fcsph_batch_add_rk3_substep(fcsph_batch *b, fcsph_plan *p, int k, double *const *u,
                                         double *p_out, const double *const *force,
                                         const double *const *wall_vel, double *const *F_store,
                                         double dt, double nu);
fcsph_status fcsph_batch_add_ppe(fcsph_batch *b, fcsph_plan *p, const void *rhs, double *phi);
/* Uploads the argument arrays and issues the grouped launches (asynchronous). */
fcsph_status fcsph_batch_launch(fcsph_batch *b);
/* Captures the launches of the last fcsph_batch_launch (without the upload)
 * into a HIP graph; fcsph_batch_replay runs it again on the same buffers
 * (for steps: the next step of every item). */
fcsph_status fcsph_batch_capture(fcsph_batch *b);
fcsph_status fcsph_batch_replay(fcsph_batch *b);
/* Items, groups and grouped launches of the last launch. */
fcsph_status fcsph_batch_info(const fcsph_batch *b, int *items, int *groups, int *launches);

#ifdef __cplusplus
}
#endif
#endif /* FCSPH_H */
