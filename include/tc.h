/*
 * tc.h -- C ABI of libtc.so: one RK3 / implicit-viscous time step of the
 * Taylor--Couette DNS of Pirro & Quadrio ("Direct Numerical Simulation of
 * turbulent Taylor--Couette flow"), on one AMD MI355X (gfx950) GPU.
 *
 * The calls follow the paper's problem statement: set the geometry (radius
 * ratio, gap, Reynolds number, resolution; Sec. 2 and Fig. 1, Sec. 3.1,
 * Sec. 4), load the radial velocity and radial vorticity fields (Appendix),
 * advance them by full 3-substep Runge--Kutta steps (Sec. 2.1, Sec. 3.1) and
 * return the statistics the paper reports (torque, eq. (torque) and Table 2;
 * wall shear and Re_tau, Sec. 5).
 *
 * Conventions shared by every call
 * --------------------------------
 * Units: lengths in units of the gap d = R_o - R_i (scaled by `gap`),
 *   velocities in units of the inner-wall speed W_i, nu = gap / Re, time in
 *   units of d / W_i.  R_i = gap zeta / (1 - zeta), R_o = gap / (1 - zeta).
 * Spectral layout: a spectral field is complex128, interleaved (re, im),
 *   row-major [r][j][l + K_z] with r = 0..N_r-1 (both walls included),
 *   j = 0..K_theta (azimuthal index, m_j = 2 pi j / Theta) and
 *   l = -K_z..K_z (axial index, alpha_l = 2 pi l / L_z), where
 *   K = floor((N - 1) / 3) for N physical points (3/2-rule dealiasing).
 *   Negative j follow from f[-j][-l] = conj(f[j][l]).  The (j, l) = (0, 0)
 *   slot is the mean flow and is carried separately as real profiles.
 * Ownership: the caller owns every host buffer and keeps it valid for the
 *   duration of the call; the context owns all device memory.  Calls that
 *   move data synchronise the context's stream before returning.
 * Errors: every call returns TC_OK or a negative code; nothing is thrown
 *   across the ABI.  On error the context stays valid and unchanged, except
 *   that tc_step / tc_substep returning TC_ENONFINITE leave the failing state
 *   in place for inspection.  tc_last_error() returns the message of the last
 *   failing call on that context.
 * Threading: one context is used by one host thread at a time.
 */
#ifndef TC_H
#define TC_H

#ifdef __cplusplus
extern "C" {
#endif

#define TC_ABI_VERSION 1

typedef struct tc_ctx tc_ctx;

enum {
    TC_OK = 0,
    TC_EINVAL = -1,      /* bad argument or geometry                       */
    TC_ENOMEM = -2,      /* device allocation failed                       */
    TC_EDEVICE = -3,     /* HIP runtime error, or no usable gfx950 device  */
    TC_ENONFINITE = -4,  /* NaN or Inf in loaded or stepped fields         */
    TC_ESHAPE = -5       /* loaded fields violate boundary/symmetry rules  */
};

enum { TC_PREC_FP64 = 0, TC_PREC_MIXED = 1 };

enum {
    TC_FLAG_LINEAR = 1,      /* nonlinear terms off: the six products are zero, so
                                the step integrates the linear (Stokes) equations
                                of Sec. 2 about the current mean profiles, with
                                every explicit viscous term kept (a test mode) */
    TC_FLAG_DRYRUN = 2,      /* validate and size only; allocate no device memory  */
    TC_FLAG_GENERIC_FFT = 4  /* use the run-time-length FFT kernels for every size
                                (the compiled lengths 8..768 otherwise take the
                                fixed-length kernels); results agree to rounding */
};

/* Geometry and resolution of one instance (Sec. 2, Fig. 1; Sec. 4).
 * radius_ratio  zeta = R_i / R_o, in (0, 1).
 * gap           length unit d > 0 (1 for the paper's non-dimensionalisation).
 * re            W_i d / nu > 0 (Sec. 2 defines Re with the full gap).
 * re_outer      W_o d / nu of the outer wall (0: at rest, the paper's set-up).
 * nr            radial points including both walls, >= 7.
 * ntheta, nz    physical (3/2-padded) points in theta and z: >= 4, of the
 *               form 2^a 3^b (b <= 1), nz even, ntheta <= 1536, nz <= 1536.
 * theta_period  Theta in radians; 0 selects min(2 pi, 5 pi d / r_c) with
 *               r_c = (R_i + R_o)/2, the paper's L_theta = 10 pi h at mid-gap.
 * lz            axial period; 0 selects 2.5 d (the paper's L_z = 5 h).
 * stretch       tanh clustering s of the radial grid (0: uniform):
 *               r_n = R_i + d (1 + tanh(s xi_n)/tanh(s)) / 2,
 *               xi_n = -1 + 2 n / (N_r - 1).
 * dt            time step (d / W_i units), > 0.
 * precision     TC_PREC_FP64, or TC_PREC_MIXED (transforms and products in
 *               FP32; recovery, radial solves, mean flow and statistics FP64).
 * flags         bitwise OR of TC_FLAG_*. */
typedef struct {
    double radius_ratio;
    double gap;
    double re;
    double re_outer;
    int nr, ntheta, nz;
    double theta_period;
    double lz;
    double stretch;
    double dt;
    int precision;
    int flags;
} tc_geometry;

/* Statistics of one instance (Sec. 3 eq. (torque) and Table 2; Sec. 5).
 * torque_in/out  T = 2 pi R_i g_i and 2 pi R_o^2 g_o / R_i with
 *                g = |dw/dr - w/r| of the mean azimuthal velocity at the
 *                wall (torque per unit length over mu W_i R_i).
 * tau_in/out     wall shear nu g;  retau = sqrt(tau) (d/2) / nu.
 * energy         volume-averaged kinetic energy, mean flow included;
 * energy_pert    the same without the (0,0) mode.
 * nonfinite      1 if any stored value is NaN or Inf. */
typedef struct {
    double time;
    double torque_in, torque_out;
    double tau_in, tau_out;
    double retau_in, retau_out;
    double energy, energy_pert;
    long long steps;
    int nonfinite;
} tc_stats_t;

/* Returns TC_ABI_VERSION. */
int tc_abi_version(void);

/* Create a context for n_instances independent instances g[0..n_instances-1]
 * (n_instances >= 1; all instances must share `precision`).  Builds the
 * radial grid, the compact-scheme coefficients and the FFT tables on the
 * host in extended precision, allocates device memory on the current HIP
 * device and zeroes the fields.  Errors: TC_EINVAL (bad geometry, null
 * pointers), TC_ENOMEM, TC_EDEVICE (no gfx950 device).  *out is set only on
 * success; with TC_FLAG_DRYRUN the context is host-only and only the
 * shape/grid queries work on it. */
int tc_create(const tc_geometry* g, int n_instances, tc_ctx** out);

/* Free every resource of the context (NULL is accepted). */
int tc_destroy(tc_ctx* ctx);

/* Use the given hipStream_t for all later work (NULL: the context's own
 * stream).  The caller keeps the stream alive while the context uses it. */
int tc_set_stream(tc_ctx* ctx, void* hip_stream);

/* Shape of instance `inst`: *nr, *nj = K_theta + 1, *nl = 2 K_z + 1. */
int tc_mode_shape(const tc_ctx* ctx, int inst, int* nr, int* nj, int* nl);

/* Copy the radial grid r_0..r_{N_r-1} of instance `inst` into r[nr]. */
int tc_grid(const tc_ctx* ctx, int inst, double* r);

/* Load v_hat and eta_hat ([nr][nj][nl] complex128, host) and the mean
 * axial/azimuthal velocity u_mean, w_mean ([nr] float64, host) of instance
 * `inst` (Appendix: the state is v and eta on every mode plus the mean flow,
 * Sec. 4).  Resets the Runge--Kutta registers.  Checks (TC_ESHAPE): wall rows
 * of v, eta zero; (0,0) slots of v, eta zero; the j = 0 column Hermitian
 * (f[0][-l] == conj f[0][l]); u_mean zero and w_mean equal to 1 and W_o at the
 * walls.  Non-finite input gives TC_ENONFINITE.  The device state is only
 * changed on success. */
int tc_load_fields(tc_ctx* ctx, int inst, const double* v_hat, const double* eta_hat,
                   const double* u_mean, const double* w_mean);

/* Copy the current fields of instance `inst` to host buffers of the layout
 * tc_load_fields takes.  Any pointer may be NULL to skip that field. */
int tc_get_fields(tc_ctx* ctx, int inst, double* v_hat, double* eta_hat,
                  double* u_mean, double* w_mean);

/* Advance every instance by nsteps >= 0 full steps of the 3-substep
 * Runge--Kutta / Crank--Nicolson scheme (Sec. 2.1, Sec. 3.1).  Work is
 * queued on the stream and synchronised once at the end, after a device
 * check for non-finite values (TC_ENONFINITE). */
int tc_step(tc_ctx* ctx, int nsteps);

/* Run only substep k in {1, 2, 3} of the scheme on every instance (a full
 * step is substeps 1, 2, 3 in order; this call lets a caller check one
 * substep in isolation).  Does not advance the step counter or the time. */
int tc_substep(tc_ctx* ctx, int k);

/* Velocity recovery (Appendix, continuity substitution): spectral axial and
 * azimuthal velocity u_hat, w_hat of instance `inst` on the host layout
 * above, with the mean profiles in the (0,0) slot (imaginary part 0).
 * Either pointer may be NULL. */
int tc_velocity(tc_ctx* ctx, int inst, double* u_hat, double* w_hat);

/* Dealiased Fourier coefficients of the six velocity products uu, uv, uw,
 * vv, vw, ww of the current state (Appendix, nonlinear terms of
 * eq. (final-v) and eq. (final-eta)), written to prod[6][nr][nj][nl]
 * complex128 in that order. */
int tc_products(tc_ctx* ctx, int inst, double* prod);

/* Radial profiles of the statistics Sec. 5 reports across the gap: at each
 * radial node r_n, averages over theta and z of the current state, written
 * to out[6][nr] (host memory, caller-owned): the mean axial and azimuthal
 * velocities u_mean, w_mean, the variances <u'u'>, <v'v'>, <w'w'> of the
 * fluctuations about the plane mean and the covariance <v'w'>, in units of
 * W_i (squared).  Computed in FP64 by Parseval over the stored half
 * spectrum; synchronous.  Time averages are the caller's (sum calls). */
int tc_profiles(tc_ctx* ctx, int inst, double* out);

/* Statistics of instance `inst` (FP64 device reductions, fixed order). */
int tc_stats(tc_ctx* ctx, int inst, tc_stats_t* out);

/* Replay whole steps from a captured HIP graph (enable = 1, the default) or
 * launch every kernel eagerly (0).  The graph holds one full step of every
 * instance and is captured on the first tc_step call on a stream; it is
 * dropped when the stream changes.  Steps taken while per-kernel timing is on
 * are always launched eagerly. */
int tc_use_graphs(tc_ctx* ctx, int enable);

/* Where the forward elimination of the Crank--Nicolson solves runs (Sec. 2.1;
 * Appendix, boundary conditions).  enable = 1 (the default): for a context of
 * one instance whose explicit-term kernel takes each column whole (tc_tuning's
 * rhs_rows = N_r - 4), N_r <= 256 and a segmented solve, the explicit-term
 * kernel eliminates each column as its right-hand-side rows complete and the
 * solve only substitutes back; otherwise, and with enable = 0, the solve does
 * both.  The two forms solve the same systems (results equal to rounding).
 * The step graph is recaptured on the next tc_step.  TC_EINVAL for a
 * host-only context. */
int tc_set_rhs_elimination(tc_ctx* ctx, int enable);

/* tc_stats for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same statistics, from the same kernels in the same order (bit-identical
 * results), with the reduction partials, flags and results in a static
 * device array of the library (about 25 KB per GPU, held until the process
 * ends; its address is looked up once per device by tc_create) instead of
 * context-owned memory.  Makes no device allocation.  Limit: 1024 reduction
 * blocks, which every grid fits (the reductions never use more); a larger
 * need returns TC_EINVAL.  The context's device must be the current HIP
 * device (else TC_EINVAL).  Every call on a GPU shares that GPU's array and
 * overwrites what it reads: calls that overlap on one GPU (several threads or
 * streams) race and must be serialised by the caller. */
int tc_stats_noalloc(tc_ctx* ctx, int inst, tc_stats_t* out);

/* Pick, by timing on the device, the launch parameters that do not change the
 * method: the rows per chunk of the explicit-term kernel (the columns split
 * into 1, 2, 3, 4, 5, 6, 8 or 10 chunks, each instance's rows divided evenly,
 * or 21, 16, 11 or 6 rows for every instance), the segment shape of the
 * radial solve (8 x 4, 8 x 8 or 16 x 8 rows, each with one lane per mode or
 * with the two signs of l of a wavenumber pair in the two halves of a
 * wavefront) and the tile shapes of the fixed-length transform kernels (z
 * kernels at half, the default or twice the columns per block; theta kernel
 * at 1, 2 or 4 wavefronts per block; see tc_tiles), per launch group.  Runs one substep to fill the intermediates, times `repeats`
 * launches (1..1000) of each candidate and restores the state, the N
 * registers and the time exactly, so the fields are unchanged on return.
 * Allocates a temporary copy of the state (freed before returning).  The
 * step graph is recaptured on the next tc_step. */
int tc_autotune(tc_ctx* ctx, int repeats);

/* Set the rows per chunk of the explicit-term kernel for instance `inst`
 * (1 <= rows <= nr - 4, else TC_EINVAL and nothing changes): each radial
 * column is walked in ceil((nr - 4) / rows) chunks.  Every row's terms are
 * summed in the same order whatever the chunking, so the results are
 * bit-identical for every value; only the speed changes.  Lets a caller
 * reuse a tuning found earlier.  The step graph is recaptured on the next
 * tc_step. */
int tc_set_rhs_rows(tc_ctx* ctx, int inst, int rows);

/* The launch parameters in use for instance `inst` (after tc_create, or
 * after tc_autotune): rows per chunk of the explicit-term kernel, and the
 * solve's segment shape as 100 * segments + rows per segment, plus 10000
 * when the two signs of l of a pair share a wavefront (0: one lane walks
 * every row).  Either pointer may be NULL. */
int tc_tuning(const tc_ctx* ctx, int inst, int* rhs_rows, int* solve_shape);

/* Set the segment shape of the radial solve (a code as tc_tuning reports:
 * 804, 808 or 1608, plus 10000 for the paired lane layout) for every instance
 * that shares instance `inst`'s solve launch.  TC_EINVAL if the shape does not
 * cover one of them or the solve is not segmented.  The two layouts and the
 * segmentations solve the same systems (results equal to rounding).  The step
 * graph is recaptured on the next tc_step. */
int tc_set_solve_shape(tc_ctx* ctx, int inst, int code);

/* Set the tile shapes of the transform stages (codes as tc_tiles reports)
 * for every instance that shares instance `inst`'s launch of each stage.
 * TC_EINVAL if a shape is not compiled for the stage's transform length and
 * precision.  Results are bit-identical for every tile shape (theta codes 4
 * and 5 select other transforms: equal to rounding).  The step graph is
 * recaptured on the next tc_step. */
int tc_set_tiles(tc_ctx* ctx, int inst, int zinv, int theta, int zfwd);

/* The tile shapes of the transform stages in use for instance `inst` (after
 * tc_create: 0 everywhere, the defaults; after tc_autotune: the choice of the
 * instance's launch group).  z kernels (inverse and forward): 0 the default
 * columns per block, 1 half of them, 2 twice; theta kernel: 0 the default
 * wavefronts per block, 1, 2 or 3 for 1, 2 or 4.  At N_theta = 768, where
 * the default theta transform swaps lane digits (two of them through LDS,
 * one in registers), theta code 4 selects the Stockham transform through LDS
 * and code 5 the transform with every exchange in registers, both at the
 * default wavefronts per block; these two give the default's products to
 * rounding, not bit for bit, and the autotuner does not pick them.  Code 6
 * keeps the lane-digit transform and fetches the third velocity field the
 * other way (at this length FP64 loads it into registers by default and FP32
 * has the memory unit copy it into LDS while the first two are transformed;
 * code 6 swaps the two, at 2 wavefronts per block for the LDS form in FP64
 * and the default for the register form in FP32): the same arithmetic in
 * another order of instructions, equal to rounding (the compiler may fuse
 * multiply-adds differently), an autotuner candidate.  Any pointer may be
 * NULL. */
int tc_tiles(const tc_ctx* ctx, int inst, int* zinv, int* theta, int* zfwd);

/* Per-kernel timing with HIP events on the context's stream.
 * enable = 1 starts recording (and clears the totals), 0 stops.  While on,
 * every launch is bracketed by events; tc_kernel_times fills ms[i] with the
 * summed milliseconds and calls[i] with the launch count of kernel i for
 * i < min(n, tc_kernel_count()).  Names come from tc_kernel_name(i). */
int tc_timing(tc_ctx* ctx, int enable);
int tc_kernel_times(tc_ctx* ctx, double* ms, long long* calls, int n);
int tc_kernel_count(void);
const char* tc_kernel_name(int id);

/* Algorithmic HBM bytes one launch of kernel `id` moves for instance `inst`
 * (the per-kernel traffic model: every array the kernel must read or write,
 * counted once).  Returns 0 for unknown ids. */
double tc_kernel_bytes(const tc_ctx* ctx, int inst, int id);

/* Compact-scheme tables of instance `inst` (Sec. 2.1 and Appendix): coef
 * receives [5][nr][5] doubles for the families d0 (shared denominator), d1
 * (D), d2 (D D), d2s (D D_*) and d4s (D D_* D D_*), row n acting on the
 * points sigma[n] .. sigma[n] + 4; sigma receives [nr] ints.  Either pointer
 * may be NULL.  Works on TC_FLAG_DRYRUN contexts. */
int tc_coefficients(const tc_ctx* ctx, int inst, double* coef, int* sigma);

/* Message of the last failing call on ctx (or of the last failing
 * tc_create when ctx is NULL).  Valid until the next call on ctx. */
const char* tc_last_error(const tc_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* TC_H */
