/*
 * sph.h -- C ABI of the MI355X DFSPH time step (libsph.so).
 *
 * The library advances a particle fluid by one Divergence-Free SPH step as
 * arXiv 2403.11156 ("Journey into SPH Simulation") states the problem:
 * particles carry mass, position and velocity (Sec. 3.2); fluid and rigid
 * particle sets with radius r, support radius h, rest density rho0, a
 * viscosity model and a domain are configured up front (Sec. 4.1); one call
 * runs one simulation iteration in the order of Algorithm 1 and Sec. 4.2
 * (gravity, viscosity, pressure, then rigid and fluid update), with the
 * pressure found by the iterative scheme of Algorithm 2 applied to the
 * velocity-source (Eq. 10) and density-source (Eqs. 8-9) problems.
 *
 * Conventions for every call:
 *   - Status codes: SPH_OK (0) or a negative SPH_ERR_*.  No C++ exception
 *     crosses this boundary.  sph_last_error() returns the message of the
 *     most recent failure on a context (thread-local for sph_create).
 *   - Host arrays passed in are copied; the caller keeps ownership.  Host
 *     arrays passed out are caller-owned and filled by the call.
 *   - Arrays of 3-vectors are array-of-structures float32 [n][3].  Particle
 *     arrays exchanged with the host are in ORIGINAL order (the index the
 *     particle had in the scene), whatever order the device keeps them in.
 *   - "Device pointer" means memory from hipMalloc (or a torch tensor on
 *     the same device); the library never frees memory it did not allocate.
 *   - All device work is queued on the stream given to sph_create (NULL =
 *     the legacy default stream).  Calls that return host data synchronise
 *     that stream.  One context per stream; a context is not thread-safe.
 */
#ifndef SPH_H_
#define SPH_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPH_ABI_VERSION 1

/* status codes */
#define SPH_OK 0
#define SPH_ERR_INVALID -1  /* bad argument or parameter */
#define SPH_ERR_OOM -2      /* device or host allocation failed */
#define SPH_ERR_DEVICE -3   /* a HIP call failed */
#define SPH_ERR_CAPACITY -4 /* a neighbour list exceeded its capacity */
#define SPH_ERR_STATE -5    /* call out of order (e.g. step without fresh neighbours) */
#define SPH_ERR_NUMERIC -6  /* non-finite state after a step */

/* viscosity models (Sec. 3.6) */
#define SPH_VISC_NONE 0
#define SPH_VISC_XSPH 1      /* v* += eps sum_j (m/rho_j)(v_j - v_i) W_ij */
#define SPH_VISC_LAPLACIAN 2 /* explicit Laplacian, Eq. (15), nu in m^2/s */
#define SPH_VISC_IMPLICIT 3  /* implicit solve (I - dt A) v* = v~, Eqs. (16)-(19), CG */

/* initial stiffness of the two pressure solves (Algorithm 2, "initialize p^l") */
#define SPH_WARM_ZERO 0
#define SPH_WARM_PREVIOUS 1 /* warm_factor * the previous step's accumulated stiffness */
#define SPH_WARM_LEARNED 2  /* density solve: per-particle MLP prediction (sph_set_warm_start) */

/* pressure solver (Sec. 3.4: the EOS solver of Sec. 3.4.1, or the PPE solvers
 * of Sec. 3.4.2) */
#define SPH_SOLVER_DFSPH 0  /* divergence-free and constant-density Jacobi solves (Algorithm 2) */
#define SPH_SOLVER_WCSPH 1  /* equation of state p = k ((rho/rho0)^gamma - 1), one pressure pass */
#define SPH_SOLVER_PCISPH 2 /* constant-density solve with PCISPH's prototype stiffness factor */

typedef struct sph_ctx sph_ctx;
typedef struct sph_mlp sph_mlp;

/*
 * Simulation parameters (Sec. 4.1).  All lengths in metres, SI units.
 *   r, h            particle radius and kernel support radius (Sec. 3.2);
 *                   the fluid mass is m = rho0 (2r)^3.
 *   rho0            rest density (Sec. 5: 1000 kg/m^3).
 *   gravity         body acceleration (Eq. 3, f_ext / rho).
 *   domain_min/max  fluid container interior; the uniform grid covers it
 *                   with one cell of margin, particles outside are clamped
 *                   into the border cells (neighbour sets stay exact).
 *   eta_density     stop threshold of the density solve: mean over fluid
 *                   particles of max(rho* - rho0, 0) / rho0 (Algorithm 2).
 *   eta_divergence  stop threshold of the divergence solve: dt/rho0 times
 *                   the mean of max(D rho / Dt, 0).
 *   max_iters       iteration cap of each solve (non-convergence is flagged
 *                   in the stats, it is not an error).
 *   dt_max          the time step when cfl_lambda == 0, else its upper bound.
 *   cfl_lambda      > 0: dt = fl32(min(dt_max, cfl_lambda * 2r / max|v|)).
 *   visc_model/visc SPH_VISC_*; visc is the XSPH epsilon or the kinematic
 *                   viscosity nu [m^2/s] (mu = nu rho0).
 *   cg_tol/cg_max_iters  implicit viscosity: relative residual and cap.
 *   cg_warm_factor  implicit viscosity: the CG starts from x0 = v~ + cg_warm_factor
 *                   times the previous step's correction v* - v~ (0: x0 = v~;
 *                   [0, 4]; the correction is SPH_FIELD_DVISC).
 *   warm_start      SPH_WARM_*; warm_factor scales the previous stiffness
 *                   (the density solve starts from warm_factor K_prev; the
 *                   divergence solve from stiffness over density
 *                   warm_factor Kv_prev / rho_prev, i.e. Kv0 = that times the
 *                   step's density).
 *   max_neighbors, max_boundary_neighbors  list capacities per particle.
 *   auto_rebuild    1: sph_step rebuilds stale neighbour lists itself: it
 *                   queues the next step's sort and neighbour build at its
 *                   end (the device runs them while the host is away) and
 *                   reads their status during the next step.  Read-back
 *                   between steps is unaffected (every field of the step
 *                   just taken, in original particle order); a
 *                   sph_write_state makes the next step sort again.
 *   solver          SPH_SOLVER_*.  WCSPH (Sec. 3.4.1): p_i = wcsph_k
 *                   ((rho_i/rho0)^wcsph_gamma - 1), clamped at zero, applied
 *                   in one pressure pass after gravity and viscosity; dt_max
 *                   must respect the acoustic limit ~0.4 h / c with
 *                   c = sqrt(wcsph_k wcsph_gamma / rho0).  PCISPH (Sec. 3.4.2,
 *                   Algorithm 2): no divergence-free solve; the
 *                   constant-density solve runs with kappa_i = (rho*_i -
 *                   rho0) c / (rho_i dt^2), c = rho0^2 / (2 sum_j |m gradW_j|^2)
 *                   over a prototype particle in a filled lattice of spacing
 *                   2r (PCISPH's delta), and reports c / rho_i as alpha.
 *                   eta_divergence applies to DFSPH only, eta_density and
 *                   warm_start to DFSPH and PCISPH; SPH_WARM_LEARNED needs
 *                   DFSPH (SPH_ERR_INVALID otherwise).
 *   separate_div_check  0 (default): with explicit viscosity, when the
 *                   last two steps' divergence-free solves needed no
 *                   iteration, the non-pressure pass also computes that
 *                   solve's first error (both read the same velocities);
 *                   if the error then calls for iterations they run and the
 *                   non-pressure pass is repeated, so the step computes the
 *                   same thing either way.  1: always run the check as a
 *                   pass of its own.
 *   alpha_max_factor  > 0: the DFSPH factor alpha_i = rho_i / D_i (Eq. 12's
 *                   density over the squared neighbour-gradient sums) is
 *                   capped at alpha_max_factor times the bulk-lattice factor
 *                   alpha_ref = 2.35376 (2r)^2 / rho0; a particle whose few
 *                   neighbours sit at the edge of the support otherwise gets
 *                   an unbounded factor, and the stiffness it accumulates is
 *                   carried into the next step.  0: no cap.  alpha = 0 when
 *                   D_i <= 1e-12 of a bulk particle's D (a vanishing
 *                   gradient, e.g. a neighbour within rounding of the
 *                   support's edge).  [0, 1e6].
 *   eta_density_max > 0: the density solve also iterates while the largest
 *                   predicted compression max_i max(rho*_i - rho0, 0) / rho0
 *                   exceeds it (the mean of eta_density alone lets a few
 *                   hundred particles of a million stay compressed by 10%
 *                   where a wave hits a wall).  0: the mean only.
 *   rigid_coupling  0 (weak, Sec. 3.5): the bodies keep their velocity during
 *                   the fluid solve and take the step's total reaction
 *                   (Eq. 14) afterwards.  1 (strong, the interlinked
 *                   coupling of the paper's outlook, Sec. 6): every pressure
 *                   pass of both solves (warm starts included) advances the
 *                   bodies' velocities by its own reaction at once (FP64 on
 *                   the device), so the next pass sees their new boundary
 *                   velocities; gravity and the gyroscopic term reach the
 *                   bodies between the two solves; the pose moves at the
 *                   step's end.  The reported force and torque are the
 *                   step's summed reaction either way.
 *   rigid_contact   0: the bodies meet only the tank, through a stand-in
 *                   that pushes a body back inside the interior shrunk by r
 *                   and drops its velocity into the wall.  1: frictionless
 *                   contact without restitution between bodies and with the
 *                   tank (the paper takes contact from a physics engine,
 *                   Sec. 4.2).  The bodies' sample points are the contact
 *                   geometry: a point within s = 2r of the shrunk interior's
 *                   planes, or within 2s of another body's point, is a
 *                   contact whose gap (distance to the plane; distance minus
 *                   s) may close by at most itself in one step.  Normal
 *                   impulses by projected Gauss-Seidel, 30 sweeps in a fixed
 *                   order, on the host in FP64 at the step's end, before
 *                   the pose moves.  Host cost grows with the number of
 *                   point pairs of bodies within reach of each other.
 */
typedef struct sph_params {
    double r, h, rho0;
    double gravity[3];
    double domain_min[3], domain_max[3];
    double eta_density, eta_divergence;
    int32_t max_iters;
    double dt_max, cfl_lambda;
    int32_t visc_model;
    double visc;
    double cg_tol;
    int32_t cg_max_iters;
    int32_t warm_start;
    double warm_factor;
    int32_t max_neighbors, max_boundary_neighbors;
    int32_t auto_rebuild;
    int32_t solver;
    double wcsph_k, wcsph_gamma;
    double cg_warm_factor;
    int32_t separate_div_check;
    double alpha_max_factor;
    double eta_density_max;
    int32_t rigid_coupling;
    int32_t rigid_contact;
} sph_params;

/* A rigid body (Sec. 3.5): mass, principal moments of inertia (body frame,
 * diagonal), centre of mass, orientation quaternion (w, x, y, z), linear and
 * angular velocity (world frame).  FP64. */
typedef struct sph_rigid_desc {
    double mass;
    double inertia[3];
    double com[3];
    double quat[4];
    double vel[3];
    double omega[3];
} sph_rigid_desc;

/* Initial scene (Sec. 4.1: fluid blocks and rigid bodies sampled as Akinci
 * boundary particles).  body_of_boundary[k] = -1 for the static tank, else
 * the index of the rigid body particle k samples; rigid particles move with
 * their body.
 *
 * device_arena (optional): device memory the caller lends the context, e.g.
 * a tensor its framework allocated, of device_arena_bytes bytes on the
 * current device, at least sph_required_bytes() of them, starting at a
 * 256-byte aligned address (SPH_ERR_INVALID otherwise; a smaller arena is
 * SPH_ERR_OOM).  The context then carves every device buffer it needs from
 * it (256-byte aligned pieces) and calls no hipMalloc; it never frees the
 * arena, which must stay valid and otherwise untouched until sph_destroy.
 * NULL: the context allocates and frees its own buffers. */
typedef struct sph_scene {
    int64_t n_fluid, n_boundary;
    int32_t n_rigid;
    const float *x_fluid;            /* [n_fluid][3] */
    const float *v_fluid;            /* [n_fluid][3], NULL = zero */
    const float *x_boundary;         /* [n_boundary][3] */
    const int32_t *body_of_boundary; /* [n_boundary], NULL = all static */
    const sph_rigid_desc *rigid;     /* [n_rigid] */
    void *device_arena;              /* device pointer, borrowed; NULL = allocate */
    int64_t device_arena_bytes;
} sph_scene;

/* Host statistics of one sph_step. */
typedef struct sph_step_stats {
    double dt;
    int32_t iters_div, iters_dens;         /* Jacobi iterations of the two solves */
    int32_t converged_div, converged_dens; /* err <= eta at exit */
    double err_div, err_dens;              /* final errors (FP64 reductions) */
    int32_t cg_iters;                      /* implicit viscosity */
    double cg_resid;                       /* final |r| / |b| */
    int32_t nbr_min, nbr_max;              /* fluid + boundary neighbours per fluid particle */
    double nbr_mean;
    int32_t warm_fallback;                 /* learned warm start fell back to PREVIOUS */
    int64_t step_index;                    /* steps completed, including this one */
    double err_dens_max;                   /* largest predicted compression / rho0 after the
                                              density solve (0 unless eta_density_max > 0) */
} sph_step_stats;

/* field mask for sph_read_state / sph_write_state */
#define SPH_FIELD_X (1u << 0)        /* fluid positions (read, write) */
#define SPH_FIELD_V (1u << 1)        /* fluid velocities (read, write) */
#define SPH_FIELD_RHO (1u << 2)      /* density of the last step, Eq. (12) (read, write: the next
                                        step's divergence warm start divides by it) */
#define SPH_FIELD_ALPHA (1u << 3)    /* DFSPH factor of the last step */
#define SPH_FIELD_K (1u << 4)        /* accumulated density stiffness (read, write) */
#define SPH_FIELD_KV (1u << 5)       /* accumulated divergence stiffness (read, write) */
#define SPH_FIELD_KAPPA (1u << 6)    /* stiffness applied in the last density iteration */
#define SPH_FIELD_ACCEL (1u << 7)    /* (v_new - v_old) / dt of the last step */
#define SPH_FIELD_NBR (1u << 8)      /* fluid and boundary neighbour counts */
#define SPH_FIELD_PSI (1u << 9)      /* Akinci boundary mass Psi, Eq. (11) */
#define SPH_FIELD_BOUNDARY (1u << 10)/* boundary positions and velocities (read, write) */
#define SPH_FIELD_RIGID (1u << 11)   /* rigid states (read, write), force and torque (read) */
#define SPH_FIELD_DVISC (1u << 12)   /* implicit-viscosity correction v* - v~ of the last step (read, write) */

/* Host buffers for sph_read_state / sph_write_state; NULL members are
 * skipped.  Fluid arrays have n_fluid entries, boundary arrays n_boundary,
 * rigid arrays n_rigid; all in original order. */
typedef struct sph_host_view {
    float *x, *v;
    float *rho, *alpha, *K, *Kv, *kappa, *accel;
    int32_t *n_fluid_nbrs, *n_boundary_nbrs;
    float *psi;
    float *x_boundary, *v_boundary;
    sph_rigid_desc *rigid;
    double *rigid_force, *rigid_torque; /* [n_rigid][3], Eq. (14) summed per body */
    float *dvisc;                       /* [n_fluid][3] */
} sph_host_view;

/* Static facts about a context. */
typedef struct sph_info {
    int64_t n_fluid, n_boundary;
    int32_t n_rigid;
    int32_t grid_n[3];       /* cells per axis */
    float cell, inv_cell;    /* cell edge fl32(h (1 + 2^-10)) and fl32(1/cell) */
    float origin[3];         /* fl32(domain_min - cell) */
    float h2;                /* fl32(h)^2, the neighbour predicate d^2 < h2 */
    int32_t max_neighbors, max_boundary_neighbors;
    int64_t device_bytes;    /* device memory the context holds */
} sph_info;

/* ---- life cycle -------------------------------------------------------- */

/* Create a context: validate, allocate device buffers, upload the scene.
 * hip_stream is a hipStream_t (borrowed) or NULL.  On failure *out stays
 * NULL and a negative status is returned. */
int sph_create(const sph_params *params, const sph_scene *scene, void *hip_stream, sph_ctx **out);

/* Device bytes sph_create needs for these parameters and scene sizes (the
 * arrays and the arena of the scene are not read), the size of a
 * scene->device_arena.  Validates like sph_create; SPH_ERR_INVALID on
 * invalid input.  A too-small arena makes sph_create fail with
 * SPH_ERR_OOM. */
int sph_required_bytes(const sph_params *params, const sph_scene *scene, int64_t *bytes);

void sph_destroy(sph_ctx *ctx);

/* ---- the time step ----------------------------------------------------- */

/* Uniform-grid neighbour search (Sec. 5.6, prefix sums): cell keys of the
 * current positions, counting sort by (cell key, particle id), reordering of
 * the particle state, fluid and boundary neighbour lists (d^2 < h^2 in FP32,
 * ascending sorted index), and the boundary mass Psi of Eq. (11) when the
 * boundary moved.  Queued on the stream; synchronises once to read the
 * capacity flag.  SPH_ERR_CAPACITY: a list overflowed; the lists are left
 * stale and the state unchanged apart from its order. */
int sph_build_neighbors(sph_ctx *ctx);

/* One DFSPH step (Algorithm 1 with Algorithm 2): time step, density and
 * factor alpha (Eq. 12), divergence-free solve (Eq. 10), non-pressure
 * accelerations (gravity and viscosity, Sec. 3.6), warm start, constant-
 * density solve (Eqs. 8-9, pressure acceleration Eq. 7 and boundary term
 * Eq. 13), reaction on rigid bodies (Eq. 14) and their FP64 update,
 * symplectic Euler.  Needs fresh neighbours (else SPH_ERR_STATE unless
 * auto_rebuild).  stats may be NULL.  SPH_ERR_NUMERIC if the new state is not
 * finite (the state is kept for inspection). */
int sph_step(sph_ctx *ctx, sph_step_stats *stats);

/* ---- state exchange ---------------------------------------------------- */

/* Blocking copy of the fields in field_mask into dst (original order). */
int sph_read_state(sph_ctx *ctx, uint32_t field_mask, const sph_host_view *dst);

/* Overwrite x, v, rho, K, Kv, the implicit-viscosity correction, boundary and
 * rigid state from host buffers (original order); marks the neighbour lists
 * stale.  Used to resume from a checkpoint or to re-anchor a test on given
 * inputs: a fresh context given the fields read from a running one (x, v,
 * rho, K, Kv, dvisc, boundary, rigid) continues it bit for bit when
 * separate_div_check = 1 (with 0, whether the next divergence check runs
 * inside the non-pressure pass depends on the solves of the last two steps,
 * which a fresh context has not seen; both give the same result up to
 * rounding).  SPH_ERR_INVALID on non-finite positions or a density <= 0. */
int sph_write_state(sph_ctx *ctx, uint32_t field_mask, const sph_host_view *src);

int sph_get_info(const sph_ctx *ctx, sph_info *info);

/* ---- diagnostics ------------------------------------------------------- */

/* Neighbour structure of the last build, for bit-exact comparison, all in
 * sorted-index space.  Fluid: keys_f[n_fluid] (cell key of the particle at
 * each sorted position), perm_f[n_fluid] (its original index), start_f
 * [ncell+1] (first sorted position of each cell), counts_f[n_fluid] and
 * lists_f (CSR concatenation, capacity cap_f entries) of fluid neighbours,
 * counts_b/lists_b (capacity cap_b) of boundary neighbours (indices into the
 * sorted boundary set); keys_b, perm_b, start_b for the boundary set.  NULL
 * pointers are skipped.  SPH_ERR_CAPACITY if a CSR capacity is too small,
 * SPH_ERR_STATE if no build happened since the last change of state. */
typedef struct sph_nbr_view {
    uint32_t *keys_f, *perm_f, *start_f, *counts_f, *lists_f;
    uint32_t *keys_b, *perm_b, *start_b, *counts_b, *lists_b;
    int64_t cap_f, cap_b;
} sph_nbr_view;
int sph_read_neighbors(sph_ctx *ctx, const sph_nbr_view *dst);

/* Run exactly div / dens iterations in the next steps regardless of the
 * error (-1 restores the stop rule).  For parity runs against a reference
 * whose stop decision falls within rounding of eta. */
int sph_set_forced_iters(sph_ctx *ctx, int32_t div, int32_t dens);

/* Per-kernel timing with HIP events recorded on the context's stream around
 * every launch of the named kernels while enabled.  sph_profile_read returns
 * the launch count and the summed event time [ms] of one kernel name, and the
 * algorithmic bytes those launches moved: each fluid particle's own fields
 * read and written once, as 3-vectors and scalars without padding (per
 * particle: integrate and cell key 44 B, sort and reorder 88, neighbour
 * build 16, density and alpha 36 (+16 with the divergence warm start),
 * divergence predict 32, density predict 36, pressure update 52,
 * non-pressure 40 (+44 with the warm start's pressure, +32 with the folded
 * divergence check)), plus 4 bytes per neighbour-list entry walked or
 * written.  Names:
 * "nbr_build", "density_alpha", "pressure_update", "predict", "xsph", "visc",
 * "sort", "warm_features", "mlp", "integrate", "eos".  sph_profile_only
 * restricts the recording to one name (NULL: all), so that a timed run pays
 * for the events of that kernel only; it applies from the next
 * sph_profile_enable on. */
int sph_profile_enable(sph_ctx *ctx, int32_t enable);
int sph_profile_only(sph_ctx *ctx, const char *kernel);
int sph_profile_read(sph_ctx *ctx, const char *kernel, int64_t *launches, double *total_ms, double *bytes);

/* ---- learned warm start ---------------------------------------------------- */
/*
 * A per-particle MLP predicts the initial stiffness of the constant-density
 * solve (Algorithm 2, "initialize p^l"); the solve still iterates to the same
 * eta, so the prediction only changes how many iterations are needed.
 * Network: 5 features -> 64 -> 64 -> 1, ReLU, bf16 weights and activations,
 * FP32 accumulation on the matrix cores, FP32 biases.  Packed FP32 parameters
 * (SPH_MLP_PARAMS floats): W1[64][5] b1[64] W2[64][64] b2[64] w3[64] b3
 * in_shift[5] in_scale[5] out_scale; output y = out_scale * z with
 * z = h2 . w3 + b3 and inputs normalised as (f - in_shift) * in_scale.
 * Features of particle i, all dimensionless: (rho_i - rho0)/rho0,
 * dt d_i/rho0 (d the density change rate, Eq. 9 in the DFSPH form, of the
 * step's input velocity, before any pressure of the step), n_i/26 (fluid +
 * boundary neighbours), K_prev dt^2/(alpha_i rho0),
 * alpha_i/alpha_ref (alpha_ref = 2.35376 (2r)^2/rho0).  Prediction y is the
 * step's final density stiffness in the same units: K0 = max(0, y alpha rho0
 * / dt^2).
 */
#define SPH_MLP_PARAMS 4620

/* Create an MLP from host parameters (copied); its work runs on hip_stream. */
int sph_mlp_create(const float *params, void *hip_stream, sph_mlp **out);
void sph_mlp_destroy(sph_mlp *mlp);
int sph_mlp_get_params(sph_mlp *mlp, float *params);
int sph_mlp_set_params(sph_mlp *mlp, const float *params);
/* y[i] = MLP(features[i]) for device arrays features[n][5], y[n]. */
int sph_mlp_forward(sph_mlp *mlp, const float *features, float *y, int64_t n);
/* Gradient of mean((z - t / out_scale)^2) over n samples (device features
 * [n][5], targets [n]), copied to host grad[SPH_MLP_PARAMS] (zeros for the
 * fixed normalisation entries); *loss gets the mean.  Deterministic. */
int sph_mlp_grad(sph_mlp *mlp, const float *features, const float *targets, int64_t n, float *grad, double *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the same loss; the
 * step counter lives in the MLP object.  *loss (may be NULL) gets the loss
 * before the update. */
int sph_mlp_train_step(sph_mlp *mlp, const float *features, const float *targets, int64_t n, float lr, double *loss);

/* Allocation-free variant of sph_mlp_grad, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight training loops, hosts
 * that forbid hipMalloc).  No sph_mlp object is needed: params (device,
 * SPH_MLP_PARAMS FP32 masters, layout above), features (device [n][5]) and
 * targets (device [n]) are read; grad (device, SPH_MLP_PARAMS floats) gets the
 * same gradient as sph_mlp_grad, and loss_sum (device, one double) the SUM of
 * the n squared residuals (sph_mlp_grad reports that sum over n).  Queued on
 * hip_stream (NULL = the legacy default stream) and returns without
 * synchronising; it calls no allocating routine.  The per-workgroup partial
 * sums live in a library-owned device array of 4,732,928 bytes (256 partial
 * gradients of 4620 floats and 256 FP64 loss partials), one copy per device,
 * held until the process ends; every call rewrites all of it, so its contents
 * never need clearing.  Calls that overlap on one device (two streams, two
 * threads) share that array and race.  SPH_ERR_INVALID: a NULL pointer, n < 1,
 * or n > SPH_MLP_NOALLOC_MAX_ROWS (the kernel scales each residual by 2/n with
 * n in FP32, exact up to 2^24 rows). */
#define SPH_MLP_NOALLOC_MAX_ROWS (1LL << 24)
int sph_mlp_grad_noalloc(const float *params, const float *features, const float *targets, int64_t n, float *grad,
                         double *loss_sum, void *hip_stream);

/* Select the warm start of the density solve: SPH_WARM_ZERO, _PREVIOUS, or
 * _LEARNED with mlp (borrowed; must outlive its use).  Non-finite MLP
 * parameters make the context fall back to PREVIOUS with
 * stats.warm_fallback = 1. */
int sph_set_warm_start(sph_ctx *ctx, int32_t mode, sph_mlp *mlp);

/* Trace capture for training: every following sph_step appends n_fluid rows
 * of features (device float [capacity][5]) and targets (device float
 * [capacity], the final stiffness K dt^2 / (alpha rho0)) until capacity rows
 * are used.  features == NULL stops capturing.  *rows (sph_trace_rows) is the
 * number of rows written so far. */
int sph_enable_trace(sph_ctx *ctx, float *features, float *targets, int64_t capacity);
int sph_trace_rows(const sph_ctx *ctx, int64_t *rows);

/* ---- errors -------------------------------------------------------------- */
const char *sph_last_error(const sph_ctx *ctx);
const char *sph_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* SPH_H_ */
