/*
 * sclbm — two-component Shan-Chen lattice Boltzmann droplet solver for MI355X
 * (gfx950), after Milan, Biferale, Sbragaglia and Toschi, "Sub-Kolmogorov
 * droplet dynamics in isotropic turbulence using a multiscale Lattice Boltzmann
 * scheme", arXiv 2112.09972.
 *
 * The library time-steps one or more independent cubic boxes (Sec. 3, Fig. 1):
 * a droplet of component A at the centre of a box of component B, D3Q19
 * populations for both components, the pair interaction force of Sec. 2 Eq. 7,
 * single-rate collision (Sec. 2 Eqs. 9-10) and ghost nodes on the faces that hold
 * the equilibrium (Sec. 2 Eq. 8) of a constant density and the linear velocity
 * u = A(t) (x - x_c) (Sec. 3 Eq. 14), where A(t) is the velocity-gradient history
 * that drives the box.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Lattice node (x, y, z), 0 <= x < nx etc.; x_c = ((nx-1)/2, (ny-1)/2, (nz-1)/2)
 *    is the box centre, the droplet's fixed centre of mass (Sec. 3).
 *  - Scalar fields are FP64 arrays of nx*ny*nz values, x fastest:
 *    index = (z*ny + y)*nx + x.  Vector fields are [3][nx*ny*nz].
 *  - A velocity gradient is 9 doubles, row-major, A[3*i + j] = d u_i / d x_j
 *    (the paper's G_ij = d_j v_i, Sec. 2 Eq. 2).
 *  - Time: the state after n steps is "time n".  Step n -> n+1 streams the
 *    ghost populations built from gradient-table row n.  Observables describe
 *    the populations after streaming at time n.
 *  - Pointers named dev_* or documented as device pointers must be device
 *    memory of the GPU the context runs on; all others are host memory.
 *  - Every call that launches work enqueues it on the context's stream and
 *    returns without waiting, except the calls documented to synchronise
 *    (they return host values).  A context is not thread-safe.
 *  - Errors: every call returns an sclbm_status; on failure sclbm_last_error()
 *    returns a thread-local message.  No exception crosses this interface.  A
 *    call that fails leaves the state as it was unless stated otherwise.
 *
 * Ownership: the caller owns the device workspace and every buffer it passes.
 * The library allocates no device memory; sclbm_destroy frees only the host
 * context.
 */
#ifndef SCLBM_H
#define SCLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SCLBM_OK = 0,
    SCLBM_EINVAL = -1,    /* bad argument */
    SCLBM_ESIZE = -2,     /* workspace or buffer too small */
    SCLBM_EHIP = -3,      /* HIP runtime error */
    SCLBM_EUNSTABLE = -4, /* NaN/Inf or non-positive density found */
    SCLBM_ESTATE = -5     /* call not valid in the current state (e.g. stepping past the gradient table) */
} sclbm_status;

typedef enum {
    SCLBM_BC_PERIODIC = 0, /* periodic box (test fixture; no ghost nodes) */
    SCLBM_BC_GHOST = 1     /* ghost nodes with density rho_b and velocity A(t)(x - x_c), Sec. 2 Eq. 8 */
} sclbm_bc;

typedef enum {
    SCLBM_F64 = 0,     /* FP64 populations, FP64 arithmetic */
    SCLBM_F32 = 1,     /* FP32 populations, FP32 arithmetic (force-stencil densities summed in FP64) */
    SCLBM_F16DEV = 2,  /* FP16 relative deviations f_i / (w_i rho_ref) - 1, FP32 arithmetic;
                          both components of a population share a 32-bit word */
    SCLBM_BF16DEV = 3, /* BF16 relative deviations f_i / (w_i rho_ref) - 1, FP32 arithmetic;
                          both components of a population share a 32-bit word */
    SCLBM_F32D = 4     /* FP32 populations, FP64 arithmetic: only the storage rounds (slower) */
} sclbm_prec;

typedef struct {
    int32_t nx, ny, nz;  /* nodes per box along x, y, z (each >= 3; nx <= 4096) */
    int32_t nbox;        /* independent boxes stepped together (>= 1) */
    int32_t bc;          /* sclbm_bc */
    int32_t prec;        /* sclbm_prec */
    int64_t table_len;   /* capacity, in rows, of each box's gradient table (>= 1 in ghost mode) */
    double tau[2];       /* relaxation times of A and B, each > 1/2 (Sec. 2 Eq. 10) */
    double g_ab;         /* coupling G_AB = G_BA of Sec. 2 Eq. 7 (G_AA = G_BB = 0) */
    double rho_b[2];     /* ghost densities of A and B (> 0); in the deviation
                            precisions also the reference densities rho_ref */
    double mach_max;     /* if > 0, gradient rows whose ghost speed exceeds
                            mach_max * c_s (c_s = 1/sqrt 3) are rejected */
} sclbm_config;

typedef struct {
    int64_t step;        /* time n of the state measured */
    double volume;       /* S0: nodes with rho_A > rho_B */
    double com[3];       /* centre of mass of those nodes */
    double cov[6];       /* covariance xx, xy, xz, yy, yz, zz about com */
    double semi_axes[3]; /* a_k = sqrt(5 lambda_k), descending (uniform-ellipsoid relation) */
    double deformation;  /* D = (a_1 - a_3)/(a_1 + a_3), Sec. 2 Eq. 4 */
    double r_eq;         /* (3 S0 / 4 pi)^(1/3) */
} sclbm_droplet_stats;

typedef struct sclbm_ctx sclbm_ctx;

/* Library infrastructure (not an operation of the paper): bytes of device
 * workspace a context with this configuration needs.
 * Errors: EINVAL for an invalid configuration. */
sclbm_status sclbm_workspace_bytes(const sclbm_config *cfg, size_t *bytes);

/* Library infrastructure: create a context on the current HIP device.  dev_workspace: device memory of
 * at least sclbm_workspace_bytes bytes, 256-byte aligned, owned by the caller and
 * kept alive until sclbm_destroy.  hip_stream: the hipStream_t every call
 * enqueues on (NULL = the null stream).  The populations are undefined until an
 * init call.  Errors: EINVAL (config), ESIZE (workspace too small or misaligned). */
sclbm_status sclbm_create(const sclbm_config *cfg, void *dev_workspace, size_t bytes, void *hip_stream,
                          sclbm_ctx **out);

/* Library infrastructure: free the host context.  Does not touch device memory. */
sclbm_status sclbm_destroy(sclbm_ctx *ctx);

/* Initial state of one box (box = -1: every box): a spherical droplet of A of
 * radius `radius` centred at center[3], density
 *   rho_A = (rho_in + rho_out)/2 - (rho_in - rho_out)/2 tanh((r - radius)/width),
 *   rho_B = rho_in + rho_out - rho_A,
 * velocity u = A0 (x - x_c) (A0 may be NULL for rest), and populations at
 * equilibrium g_eq(rho_sigma, u) (Sec. 2 Eq. 8).  Resets the time to 0.
 * The paper places the droplet at the box centre (Sec. 3, Fig. 1) and gives no
 * profile; the tanh profile is this library's choice. */
sclbm_status sclbm_init_droplet(sclbm_ctx *ctx, int32_t box, const double center[3], double radius,
                                double width, double rho_in, double rho_out, const double A0[9]);

/* Initial state of one box from FP64 device fields rho_a[N], rho_b[N], u[3][N]
 * (u may be NULL for rest): populations at the equilibrium of Sec. 2 Eq. 8 of
 * each node's densities and velocity (the densities and velocity of Eq. 6
 * then reproduce the fields).  Resets the time to 0.  Errors: EINVAL (box,
 * NULL density field).  The fields are read before the call returns. */
sclbm_status sclbm_init_fields(sclbm_ctx *ctx, int32_t box, const double *rho_a, const double *rho_b,
                               const double *u);

/* Initial state of one box (box = -1: every box): uniform densities rho_a,
 * rho_b (> 0) moving with u0[3] (NULL: at rest), populations at the equilibrium
 * of Sec. 2 Eq. 8.  A uniform bulk state is a fixed point of the update (the
 * stationarity check of the method).  Resets the time to 0.  Errors: EINVAL. */
sclbm_status sclbm_init_uniform(sclbm_ctx *ctx, int32_t box, double rho_a, double rho_b, const double u0[3]);

/* Copy n rows of a box's velocity-gradient table from host memory: row t drives
 * step first_step + t (Sec. 3 Eq. 14; Sec. 4 holds each sample of the turbulent
 * gradient for a number of steps, the caller expands it into per-step rows).
 * n <= table_len.  With mach_max > 0 every row is checked on every ghost node
 * (|A (x_g - x_c)| <= mach_max c_s) and the call fails with EINVAL naming the
 * first offending row; the previous table then stays in force. */
sclbm_status sclbm_set_gradient_table(sclbm_ctx *ctx, int32_t box, const double *A_rows, int64_t first_step,
                                      int64_t n);

/* A constant velocity gradient A[9] for one box (box = -1: every box), as in the
 * steady simple shear of the validation of Sec. 4 (u = A (x - x_c), Sec. 3
 * Eq. 14): fills the box's whole table, table_len rows, starting at the
 * current time n, so the next table_len steps use A.  Same checks as
 * sclbm_set_gradient_table (ESTATE in periodic mode, EINVAL for a non-finite
 * entry or a ghost speed above mach_max c_s).  Synchronises. */
sclbm_status sclbm_set_gradient(sclbm_ctx *ctx, int32_t box, const double A[9]);

/* Advance every box by nsteps time steps of the method (Sec. 2 Eqs. 6-9: moments,
 * pair force of Eq. 7, velocity shift, single-rate collision, streaming; ghost
 * populations of Sec. 2 Eq. 8 at the faces with u = A(t)(x - x_c), Sec. 3
 * Eq. 14), one fused kernel launch per step.  In ghost mode every box's table
 * must cover steps n..n+nsteps-1, else ESTATE and nothing is launched.  With
 * the health check on (sclbm_set_health_check), every time that is a multiple
 * of its interval is checked, which synchronises; EUNSTABLE then stops the
 * call at that time (the steps before it are done). */
sclbm_status sclbm_step(sclbm_ctx *ctx, int64_t nsteps);

/* The step of sclbm_step (Sec. 2 Eqs. 6-9, ghost nodes of Sec. 2 Eq. 8 and
 * Sec. 3 Eq. 14): advance every box by nsteps through a captured hipGraph of
 * nsteps fused launches (nsteps even and >= 2).  The graph is captured on first use for this
 * nsteps, launch shape and buffer parity, then replayed; the kernels read the
 * time from a device counter, so a replay continues where the last one ended.
 * Same table rules as sclbm_step.  The graph is rebuilt after sclbm_set_launch
 * or when an odd number of eager steps changed the buffer parity. */
sclbm_status sclbm_step_graph(sclbm_ctx *ctx, int64_t nsteps);

/* A guard the paper does not have (library infrastructure): health check of
 * the step calls, every `every` steps (0: off, the default)
 * sclbm_step computes every box's FP64 mass and counts the nodes with a NaN/Inf
 * or non-positive density (the same reduction as sclbm_totals) and returns
 * EUNSTABLE naming the first bad box; sclbm_step_graph checks once after each
 * replay.  Each check costs one read of every population.  Errors: EINVAL
 * (every < 0). */
sclbm_status sclbm_set_health_check(sclbm_ctx *ctx, int64_t every);

/* Library infrastructure: the current time n (steps taken since the last init or load). */
sclbm_status sclbm_get_step(const sclbm_ctx *ctx, int64_t *step);

/* Observables of one box at time n into FP64 device arrays: densities rho_a[N],
 * rho_b[N] (Sec. 2 Eq. 6, per component) and, if u != NULL, the barycentric
 * velocity u[3][N] = (j_A + j_B + (F_A + F_B)/2)/(rho_A + rho_B) (Sec. 2 Eq. 6
 * with the half-force term of the Shan-Chen model; F from Sec. 2 Eq. 7).
 * rho_a and rho_b must not be NULL. */
sclbm_status sclbm_fields(sclbm_ctx *ctx, int32_t box, double *rho_a, double *rho_b, double *u);

/* FP64 totals of one box at time n: mass[2] = sum rho_A, sum rho_B and
 * momentum[3] = sum (j_A + j_B), with rho and j the moments of Sec. 2 Eq. 6
 * summed over the box's nodes (the ghost boundary does not conserve them, which
 * is why Sec. 2 puts mass back into the droplet).  Accumulated in FP64 whatever
 * the storage format; deterministic fixed-order reduction.  Synchronises the
 * stream.  EUNSTABLE if a NaN/Inf or non-positive density is found (the totals
 * are still returned). */
sclbm_status sclbm_totals(sclbm_ctx *ctx, int32_t box, double mass[2], double momentum[3]);

/* Indicator moments of one box at time n, phi = [rho_A > rho_B], about x_c,
 * written as 10 FP64 values to device memory: S0, S1x, S1y, S1z, S2xx, S2xy,
 * S2xz, S2yy, S2yz, S2zz.  They give the droplet's inertia tensor, whose
 * eigenvalues set the ellipsoid semi-axes and the deformation D of Sec. 2
 * Eq. 4 (sclbm_droplet_from_moments); the paper names the tensor but not how
 * it is measured, the sharp indicator is this library's choice.  Does not
 * synchronise (for time series: collect many, copy once).  Errors: EINVAL. */
sclbm_status sclbm_droplet_moments(sclbm_ctx *ctx, int32_t box, double *dev_out10);

/* The same 10 moments (droplet inertia tensor for Sec. 2 Eq. 4) for every box
 * in one pass, dev_out[nbox][10] (device).  Does not synchronise. */
sclbm_status sclbm_droplet_moments_all(sclbm_ctx *ctx, double *dev_out);

/* sclbm_droplet_moments_all without the workspace's reduction area, for callers
 * that cannot allocate device memory or size a workspace for it (code under HIP
 * graph capture, tight serving loops).  The partial sums and per-box results live
 * in a static device array of 2 MiB that the library holds on every GPU it runs
 * on until the process ends; a context of nbox boxes needs
 * nbox * (blocks per box + 1) * 16 doubles of it (blocks per box: about one per
 * 2048 nodes, at least 1024 / nbox, at most 1024), else ESIZE and nothing is
 * launched (64 boxes of 64^3 use 1.0 MiB).  Same kernels and results as
 * sclbm_droplet_moments_all, bit for bit.  Allocates nothing.  Calls that overlap
 * on one GPU (several streams or host threads) share the array and race; each
 * call overwrites what it reads before reading it.  Does not synchronise. */
sclbm_status sclbm_droplet_moments_all_static(sclbm_ctx *ctx, double *dev_out);

/* Droplet statistics from 10 indicator moments about `center` (host only, no
 * GPU work): covariance, its eigenvalues by the closed-form trigonometric
 * method for symmetric 3x3 matrices, semi-axes, deformation (Sec. 2 Eq. 4). */
sclbm_status sclbm_droplet_from_moments(const double moments[10], const double center[3], int64_t step,
                                        sclbm_droplet_stats *out);

/* Droplet semi-axes and deformation of Sec. 2 Eq. 4 for one box at time n:
 * sclbm_droplet_moments + copy + sclbm_droplet_from_moments.  Synchronises. */
sclbm_status sclbm_droplet(sclbm_ctx *ctx, int32_t box, sclbm_droplet_stats *out);

/* Global velocity error E0 of Sec. 4 Eq. 16 for one box at time n against the
 * linear flow A (x - x_c): sqrt(<|u - A(x - x_c)|^2>) / sqrt(<|A(x - x_c)|^2>),
 * averages over the box's nodes, u as in sclbm_fields.  Synchronises. */
sclbm_status sclbm_velocity_error(sclbm_ctx *ctx, int32_t box, const double A[9], double *e0);

/* Droplet surface, for the deformation measure D_LBM = sqrt(1 - Omega_0 / Omega)
 * of Sec. 5 Eq. 17 (Omega the droplet's surface area, Omega_0 that of the sphere
 * of equal volume).  For every box: the area of the level set rho_A = rho_B
 * and the volume of rho_A > rho_B, with phi = rho_A - rho_B taken linear inside
 * the six tetrahedra of every lattice cell (each cell split along its main
 * diagonal; the paper does not say how it measures the area).  dev_out:
 * [nbox][2] = {area, volume}, FP64 sums in a fixed order.  Enqueued. */
sclbm_status sclbm_droplet_surface_all(sclbm_ctx *ctx, double *dev_out);

/* D_LBM of Sec. 5 Eq. 17 from an area and a volume (host arithmetic; area > 0, volume >= 0);
 * Omega_0 = (36 pi V^2)^(1/3).  0 when the area does not exceed Omega_0. */
sclbm_status sclbm_deformation_lbm(double area, double volume, double *d_lbm);

/* Droplet mass of every box, the quantity the reinjection of Sec. 2 restores:
 * the sum of rho_A over the nodes with rho_A > rho_B.  dev_out: [nbox] FP64.  Enqueued. */
sclbm_status sclbm_droplet_mass_all(sclbm_ctx *ctx, double *dev_out);

/* Mass reinjection (Sec. 2: the ghost-node boundary does not conserve mass,
 * and mass is put back into the droplet so that its density stays fixed).
 * For box `box` (or every box, box = -1): measure the droplet mass M as in
 * sclbm_droplet_mass_all and multiply component A at every droplet node by
 * target / M — every population in the FP64/FP32 formats, the node's reference
 * density in the deviation formats (rounded to FP16 there).  Component A's
 * velocity is unchanged.  target_mass: host, one value per selected box (> 0).
 * A scale above 1 reaches the target exactly; below 1, interface nodes may
 * leave the droplet and the mass lands slightly under it.  Synchronises. */
sclbm_status sclbm_reinject(sclbm_ctx *ctx, int32_t box, const double *target_mass);

/* Library infrastructure, checkpoint: bytes needed, save the state (populations of every box, time)
 * into host memory, restore it.  Save synchronises; load is bitwise exact. */
sclbm_status sclbm_state_bytes(const sclbm_ctx *ctx, size_t *bytes);
sclbm_status sclbm_save(sclbm_ctx *ctx, void *host_buf, size_t bytes);
sclbm_status sclbm_load(sclbm_ctx *ctx, const void *host_buf, size_t bytes);

/* Library infrastructure (how the step is launched; no operation of the
 * paper).  Launch shape of the step kernel: a tile of tile_rows rows of
 * tile_waves 64-node columns, (tile_rows, tile_waves) one of (4, 1), (8, 1),
 * (4, 2), and for the 16-bit deviation formats also (4, 4) (256 nodes wide, 16
 * wavefronts; EINVAL for the other formats); and planes per z-chunk (>= 1).  A
 * tile as wide as the box's rows lets every x-shifted store write whole cache
 * lines; the default is (4, 2) for nx > 64, else (8, 1), and (8, 1) also where
 * the last 128-wide tile of a row would be at most half full (nx mod 128 in
 * 1..64); the 16-bit formats take (4, 4) where the row's last 256-wide tile is
 * full or holds more than 160 nodes.  The default z-chunk minimises (rounds of
 * resident workgroups) x (planes per chunk + 2), at most 64 planes for the
 * 16-bit formats.  The shape only
 * changes speed, never results.  Pointers of get_launch may be NULL. */
sclbm_status sclbm_set_launch(sclbm_ctx *ctx, int32_t tile_rows, int32_t zchunk, int32_t tile_waves);
sclbm_status sclbm_get_launch(const sclbm_ctx *ctx, int32_t *tile_rows, int32_t *zchunk, int32_t *tile_waves);

/* The launch shape a context with this configuration starts with (the
 * defaults above), computed on the host without a device.  Pointers may be
 * NULL.  Errors: EINVAL for an invalid configuration. */
sclbm_status sclbm_default_launch(const sclbm_config *cfg, int32_t *tile_rows, int32_t *zchunk, int32_t *tile_waves);

/* Library infrastructure, autotuner: time trial_steps steps (after one warm-up
 * step) for every tile shape ((4, 1), (8, 1), (4, 2) when nx > 64, (4, 4) for
 * the 16-bit formats when nx > 128) and z-chunk (2, 4, 8, 16, 32, 64, capped at nz, the
 * tile's default z-chunk, so the default launch is one of the candidates, and
 * the chunk that puts all workgroups in one round of resident ones, if any),
 * keep the fastest and set it.  The output pointers
 * (may be NULL) receive its shape and the best average step time in ms.
 * The trials overwrite the populations (call it before an init call, or
 * re-initialise after) but restore the time.  In ghost mode every box's table
 * must cover steps n .. n + trial_steps.  Synchronises. */
sclbm_status sclbm_autotune(sclbm_ctx *ctx, int32_t trial_steps, int32_t *tile_rows, int32_t *zchunk,
                            int32_t *tile_waves, float *best_ms);

/* Semi-axes over the reference radius of n Maffettone-Minale tensors M[n][9]
 * (host memory, Sec. 2 Eqs. 1-2: M = I is the sphere, an ellipsoid has the
 * squared semi-axes as eigenvalues): axes[n][3] = sqrt of the eigenvalues of
 * the symmetric part of M, descending (closed-form 3x3 eigenvalues, as in
 * sclbm_droplet_from_moments; a negative eigenvalue from rounding gives 0).
 * Host only, no GPU work.  Errors: EINVAL (NULL pointer, n < 0). */
sclbm_status sclbm_mm_semi_axes(const double *M, int64_t n, double *axes);

/* Maffettone-Minale morphology tensor (Sec. 2 Eqs. 1, 2, 5) for ntraj
 * trajectories on the GPU, one thread each, FP64 classical RK4 with `substeps`
 * steps per table row and A(t) linear between rows; M = I is the sphere of the
 * reference radius.  dev_A: [ntraj][nrows][9] velocity gradients in table time
 * units; tau_d = eta_s R / sigma in the same units; chi the viscosity ratio;
 * dev_M0: [ntraj][9] initial tensors or NULL for I; dev_M: [ntraj][nrec][9] with
 * nrec = 1 + (nrows - 1) / record_every, record r at time r * record_every.
 * Needs no context; enqueues on hip_stream (NULL = null stream). */
sclbm_status sclbm_mm_integrate(const double *dev_A, int64_t ntraj, int64_t nrows, double tau_d, double chi,
                                int32_t substeps, int32_t record_every, const double *dev_M0, double *dev_M,
                                void *hip_stream);

/* Message of the last failed call on this thread ("" if none). */
const char *sclbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SCLBM_H */
