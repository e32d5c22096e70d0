/*
 * sscn.h -- C ABI of the MI355X (gfx950) split-step Crank-Nicolson solver
 * for the rotating Gross-Pitaevskii equation.
 *
 * Method: Kumar, Loncar, Muruganandam, Adhikari, Balaz, "C and Fortran
 * OpenMP programs for rotating Bose-Einstein condensates" (arXiv:1906.06327),
 * Sec. 2.  One time step is the Lie splitting H1 -> H2 -> H3 (-> z part in
 * 3D) of Eqs. (eq1)-(eq3) and (split): the pointwise potential/nonlinear
 * factor, then Crank-Nicolson line solves along x (Eqs. (eqD.9:kn1),
 * (eqD.11), (eq5)), along y ("similarly", rotation coefficient y_j -> -x_i)
 * and, in 3D, along z (no rotation term).  Imaginary time replaces Delta by
 * -i Delta everywhere and renormalises after every step.
 *
 * Grid: each axis stores n points x_i = -n*h/2 + i*h, i = 0..n-1; index 0 is
 * a Dirichlet wall (psi = 0) and the wall at i = n is implied.  The paper's
 * (N+1)-point grid is this grid plus its always-zero last row.
 *
 * Data: psi is a caller-owned DEVICE buffer, contiguous, x fastest:
 * psi[(k*ny + j)*nx + i].  Elements are interleaved (re, im) pairs of double
 * (precision SSCN_C128, 16 bytes) or float (SSCN_C64, 8 bytes) -- the layout
 * of torch.complex128 / torch.complex64.  The library borrows the buffer
 * from sscn_init until sscn_destroy; it owns only a second state-sized work
 * buffer and small reduction buffers.
 *
 * Streams: every call enqueues its work on the hipStream_t given to
 * sscn_init (pass the caller's stream; NULL means the null stream).  Calls
 * that return data to the host synchronise that stream.  A handle is not
 * thread safe: use one handle per host thread.
 *
 * Errors: every int-returning call returns 0 on success or a negative
 * SSCN_E* code; sscn_last_error() describes the most recent failure of the
 * calling thread.  On error no state is modified unless stated.
 */
#ifndef SSCN_H
#define SSCN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SSCN_OK = 0,
    SSCN_EINVAL = -1,     /* bad sizes, non-positive steps, null pointers     */
    SSCN_EOMEGA = -2,     /* Omega >= min(gamma, nu): no rotating ground state */
    SSCN_EUNSTABLE = -3,  /* line systems not diagonally dominant (see init)  */
    SSCN_ENONFINITE = -4, /* a NaN or Inf appeared in the state               */
    SSCN_EHIP = -5,       /* a HIP runtime call failed                        */
    SSCN_ENOMEM = -6      /* device allocation failed                         */
};

enum { SSCN_IMAG = 0, SSCN_REAL = 1 };      /* propagation mode              */
enum { SSCN_PLAN_AUTO = 0, SSCN_PLAN_SWEEPS = 1, SSCN_PLAN_FUSED = 2 }; /* kernels */
enum { SSCN_C128 = 0, SSCN_C64 = 1 };       /* storage/arithmetic precision  */

typedef struct sscn_params {
    int dim;                  /* 2 or 3                                        */
    int nx, ny, nz;           /* stored points per axis, each >= 3 (nz ignored
                                 when dim == 2)                                */
    double hx, hy, hz;        /* space steps, > 0                              */
    double gamma, nu, lambda; /* trap anisotropies of Eq. (3d) / Eq. (2d)      */
    double g;                 /* g_2D (dim 2) or g_3D (dim 3)                   */
    double omega;             /* rotation frequency, |omega| < min(gamma, nu)  */
    double dt;                /* time step Delta, > 0                          */
    int mode;                 /* SSCN_IMAG or SSCN_REAL                        */
    int precision;            /* SSCN_C128, or SSCN_C64 (complex64 sweeps with
                                 FP64 reductions)                              */
} sscn_params;

/* Observables of the current state (paper Sec. 2: Eqs. (e2dr)/(e3dr) for mu
 * and energy with alpha = 1 and 1/2, the kinetic term entering with +1/2;
 * Eqs. (e2d)/(e3d) for the full functional; rms sizes sqrt(<x^2>) etc.).
 * Integrals are h^d times plain sums; derivatives are forward differences
 * in the kinetic terms and central differences in the rotation terms. */
typedef struct sscn_obs {
    double norm;          /* h^d sum |psi|^2                                  */
    double mu, energy;    /* real-part form                                   */
    double mu_full, energy_full; /* full functional, divided by the norm      */
    double mu_4th, energy_4th;   /* the same with fourth-order central
                                    differences: the continuum values to
                                    O(h^4), the form Table 1 prints           */
    double rms_x, rms_y, rms_z, rms_r;
    double max_density;   /* max |psi|^2                                      */
    int64_t step;         /* steps taken since sscn_init                      */
    double sums[16];      /* the raw reductions (see sscn_observables)        */
} sscn_obs;

typedef struct sscn_handle sscn_handle;

/* Create a solver on the current HIP device for the state buffer psi_dev
 * (layout above, precision params->precision).  Validates the parameters:
 * SSCN_EOMEGA when |omega| >= min(gamma, nu) (the rotating-frame energy is
 * unbounded below, Sec. 2); SSCN_EUNSTABLE when a line system is not
 * strictly diagonally dominant, which in real time means
 * dt*|omega|*max|coordinate| / (2h) >= 1 on an axis.  psi is not touched;
 * the caller fills it with sscn_init_state or sscn_set_state (or writes it
 * directly and then calls sscn_set_state_device).  On success *out is set. */
int sscn_init(const sscn_params *params, void *psi_dev, void *hip_stream,
              sscn_handle **out);

/* Initial state of Eq. (fun): kind 1 = one vortex (x + i y) at the centre,
 * kind 0 = Gaussian ((x + i y) -> 1), width d_xy; in 3D times the z Gaussian
 * of width d_z (d_z <= 0 selects 1/sqrt(lambda), the ansatz of Eq. (anz)).
 * phase_host: NULL for no random phase, else ny*nx host doubles R(x, y)
 * (row-major, x fastest) entering as exp(2 pi i R), constant along z.  Walls
 * are zeroed and the state is normalised to 1.  Synchronises the stream. */
int sscn_init_state(sscn_handle *h, int kind, const double *phase_host,
                    double d_xy, double d_z);

/* The same initial state of Eq. (fun) with the random number R(x, y) drawn
 * on the device from a counter-based generator (no host array): with
 * random_phase != 0, R at point (i, j) is u = 2^-53 (h(seed XOR (j nx + i))
 * >> 11), uniform in [0, 1), where h is the output function of the
 * SplitMix64 generator (Steele, Lea and Flood, 2014: add
 * 0x9E3779B97F4A7C15, then z = (z ^ z >> 30) * 0xBF58476D1CE4E5B9, z = (z ^
 * z >> 27) * 0x94D049BB133111EB, z ^ z >> 31, all modulo 2^64); constant
 * along z.  The paper leaves the generator of R unspecified (Sec. 2, after
 * Eq. (fun)); integer arithmetic makes u the same bits on every platform
 * (sscn_phase_field_seed returns them).  Synchronises the stream. */
int sscn_init_state_seed(sscn_handle *h, int kind, int random_phase, uint64_t seed,
                         double d_xy, double d_z);

/* The random numbers sscn_init_state_seed uses: out_dev[j nx + i] = u(seed,
 * j nx + i) for an ny x nx plane (caller-owned device buffer of nx*ny
 * doubles).  Asynchronous on hip_stream.  SSCN_EINVAL for a null buffer or
 * non-positive sizes. */
int sscn_phase_field_seed(uint64_t seed, int nx, int ny, double *out_dev, void *hip_stream);

/* Enqueue nsteps >= 0 SSCN steps (paper's NPAS loop body).  Asynchronous:
 * no host synchronisation.  In imaginary time the state left in psi after
 * the call is normalised.  A call of n >= 2 steps replays captured HIP
 * graphs: n = q G + r with G = min(n, 64), q launches of the G-step graph,
 * then an r-step graph (r >= 2) or one directly launched step; graphs are
 * captured on first use and kept per handle (the four most recent step
 * counts).  The first call of an SSCN_PLAN_AUTO handle also picks the plan
 * (sscn_set_plan). */
int sscn_step(sscn_handle *h, int64_t nsteps);

/* Do, without advancing the state, the one-time work of a later
 * sscn_step(h, nsteps): pick the plan (timed on a saved copy of the state,
 * which is restored) and capture the graphs that call replays, so that its
 * duration is the steps alone.  Synchronises the stream.  SSCN_EINVAL for a
 * null handle or nsteps < 0. */
int sscn_prepare_steps(sscn_handle *h, int64_t nsteps);

/* Observables of the current state; synchronises the stream.  Returns
 * SSCN_ENONFINITE (and still fills *out) when any reduction is NaN/Inf.
 * sums[]: 0 |psi|^2, 1 psi_R^2, 2 kinetic(psi_R), 3 V psi_R^2,
 * 4 g|psi|^2 psi_R^2, 5 rotation(psi_R, psi_I), 6 kinetic(psi), 7 V|psi|^2,
 * 8 g|psi|^4, 9 Omega Im[psi^*(y d/dx - x d/dy)psi], 10-12 x^2,y^2,z^2
 * |psi|^2 (all times h^d), 13 max |psi|^2, 14 1/2 |grad psi|^2 and 15
 * Omega Im[psi^*(y d/dx - x d/dy)psi] with fourth-order central differences
 * (-f[i+2] + 8 f[i+1] - 8 f[i-1] + f[i-2]) / (12 h) (times h^d): mu_4th and
 * energy_4th.  The discrete-operator forms (mu, energy, mu_full,
 * energy_full) are what the iteration converges; they differ from the
 * continuum values by O(h^2) terms that grow with the phase gradients of
 * fast rotation. */
int sscn_observables(sscn_handle *h, sscn_obs *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the raw
 * sums of sscn_observables (sums[0..15] of sscn_obs, integrals already times
 * h^d, sums_dev[13] the max density) of the state psi_dev, described by
 * params (layout and precision as for sscn_init; the parameters are
 * validated as there), written to the caller-owned device buffer sums_dev
 * (16 doubles).  No handle; asynchronous on hip_stream (NULL: the null
 * stream); it calls no allocating routine.  The per-block partial sums go
 * to a static scratch array of the library (1024 rows of 16 doubles, 128
 * KiB per GPU, held until the process ends), so concurrent calls on one GPU
 * race: serialise them (one stream, or events).  The kernels and the
 * reduction order are those of sscn_observables, so the sums are the same
 * bits.  SSCN_EINVAL for null pointers or invalid parameters, SSCN_EOMEGA as
 * sscn_init, SSCN_EHIP if the scratch address cannot be obtained or a launch
 * fails. */
int sscn_observables_noalloc(const sscn_params *params, const void *psi_dev, void *hip_stream,
                             double *sums_dev);

/* Copy a host state (same layout and precision as psi) into psi, zeroing
 * the walls (paper's NSTP = 0 restart).  Synchronises the stream. */
int sscn_set_state(sscn_handle *h, const void *host_psi);

/* Tell the handle psi was written by the caller on the device: zeroes the
 * walls.  Asynchronous. */
int sscn_set_state_device(sscn_handle *h);

/* Continuation start (Sec. 3): a converged state of smaller nonlinearity
 * or rotation seeds the run for larger ones, on a larger grid of the same
 * spacing to hold the larger condensate.  Centred embedding:
 * dst[k][j][i] = src[k - oz][j - oy][i - ox] with o = (n - n_src) / 2 per
 * axis, so the grids' centres x = 0 coincide; zero where that index lies
 * outside src (a smaller dst crops) and on the walls of dst (index 0).
 * src: device buffer nz_src x ny_src x nx_src, dst: device buffer
 * nz x ny x nx, x fastest, both in `precision` (SSCN_C128 or SSCN_C64),
 * caller-owned, not overlapping; 2D: nz_src = nz = 1.  n - n_src must be
 * even on every axis, else SSCN_EINVAL (likewise for null or non-positive
 * arguments and overlap).  Enqueued on `stream` (hipStream_t, NULL for the
 * null stream), asynchronous; no normalisation (an enlarged normalised
 * state stays normalised).  Independent of any handle: fill a handle's
 * buffer and call sscn_set_state_device, or embed into a scratch buffer. */
int sscn_embed_state(const void *src, int nx_src, int ny_src, int nz_src, void *dst, int nx, int ny, int nz,
                     int precision, void *stream);

/* Product start of the 3D form of Eq. (fun) (Sec. 2): the z dependence is
 * a Gaussian of width d_z, so a 2D field xy(x, y) becomes
 * dst[k][j][i] = xy[j][i] exp(-z_k^2 / (2 d_z^2)) / sqrt(hz S), with
 * z_k = -nz hz / 2 + k hz (the grid convention above) and
 * S = sum_{k=1}^{nz-1} exp(-z_k^2 / d_z^2): a 2D field normalised on its
 * grid gives a 3D state normalised over the interior.  The wall plane k = 0
 * is written too; call sscn_set_state_device on the 3D handle to zero it.
 * xy: device buffer ny x nx, dst: device buffer nz x ny x nx, x fastest,
 * both in `precision` (SSCN_C128 or SSCN_C64), caller-owned, not
 * overlapping.  SSCN_EINVAL for null or overlapping buffers, sizes below 2,
 * or hz, d_z not positive and finite.  Enqueued on `stream` (hipStream_t,
 * NULL for the null stream), asynchronous. */
int sscn_extend_z(const void *xy, int nx, int ny, void *dst, int nz, double hz, double d_z, int precision,
                  void *stream);

/* Interpolation between 2D grids of different spacing and extent, for the
 * learned initial state (a network working in coordinates scaled to each
 * condensate's size, whose output seeds a run on the instance's own grid;
 * the paper moves states between grids only by the centred embedding of
 * sscn_embed_state).  Both grids are centred as the solver's (x_i =
 * -n h / 2 + i h); the destination point (x, y) takes the value at
 * (cos(angle) x - sin(angle) y, sin(angle) x + cos(angle) y) of Keys' cubic
 * convolution interpolant of src (kernel parameter a = -1/2, separable, 4 x 4
 * samples; third order; quadratics reproduced exactly), src samples beyond
 * its grid taken as zero; the destination walls (index 0) are zero.  No
 * normalisation (sscn_set_state_device or sscn_batch_set_state_device
 * normalises a state written into a handle's buffer).  src: device buffer
 * ny_src x nx_src, dst: device buffer ny x nx, x fastest, both in
 * `precision` (SSCN_C128 or SSCN_C64; FP64 arithmetic in both), caller-owned,
 * not overlapping.  SSCN_EINVAL for null or overlapping buffers, sizes below
 * 2, spacings not positive and finite, or a non-finite angle.  Enqueued on
 * `stream` (hipStream_t, NULL for the null stream), asynchronous. */
int sscn_resample(const void *src, int nx_src, int ny_src, double hx_src, double hy_src, void *dst, int nx, int ny,
                  double hx, double hy, double angle, int precision, void *stream);

/* Angular Fourier components of a 2D state's density about the grid centre,
 * M_k = hx hy sum |psi|^2 exp(i k phi), phi = atan2(y, x), k = 0..kmax
 * (kmax <= 8), into out_dev[2k] (real part) and out_dev[2k + 1] (imaginary
 * part), FP64, caller-owned device buffer of 2 kmax + 2 doubles; a point at
 * the origin enters M_0 only.  The orientation arg(M_k) / k of a k-fold
 * pattern fixes the canonical rotation of learned-start targets where the
 * trap leaves the lattice orientation free.  psi: ny x nx device buffer in
 * `precision`.  SSCN_EINVAL for bad arguments.  Asynchronous on `stream`. */
int sscn_angular_moments(const void *psi, int nx, int ny, double hx, double hy, int kmax, int precision,
                         double *out_dev, void *stream);

/* Copy psi to a host buffer of the same layout.  Synchronises the stream. */
int sscn_get_state(sscn_handle *h, void *host_psi);

/* Switch propagation mode (imaginary -> real hand-off of the paper's
 * workflow) and/or precision.  A precision change converts the state into
 * new_psi_dev (caller-owned, the new precision's layout), which the handle
 * borrows from then on; pass NULL when the precision is unchanged.  New
 * parameters are validated as in sscn_init; on error nothing changes. */
int sscn_set_mode(sscn_handle *h, int mode, int precision, void *new_psi_dev);

/* Density profiles, the paper's density outputs (Sec. 3: full density,
 * densities integrated over the other dimensions, cross-sections), written
 * as FP64 into the caller-owned device buffer out_dev:
 *   SSCN_DEN_FULL   |psi|^2 at every point (layout of psi);
 *   SSCN_DEN_XY     integral over z of |psi|^2, ny x nx (2D: |psi|^2);
 *   SSCN_DEN_X / _Y / _Z  integral over the two other axes, nx / ny / nz
 *                   values (2D: over the one other axis);
 *   SSCN_DEN_CUT_X / _Y / _Z  |psi|^2 along one axis through the centre
 *                   indices ny/2, nx/2 (and nz/2) of the others.
 * Integrals are h times plain sums in a fixed order (reading R4).  The z
 * profiles need a 3D handle (else SSCN_EINVAL, as for a bad kind or a null
 * pointer).  Enqueued on the handle's stream; asynchronous. */
enum { SSCN_DEN_FULL = 0, SSCN_DEN_XY = 1, SSCN_DEN_X = 2, SSCN_DEN_Y = 3, SSCN_DEN_Z = 4,
       SSCN_DEN_CUT_X = 5, SSCN_DEN_CUT_Y = 6, SSCN_DEN_CUT_Z = 7 };
int sscn_density(sscn_handle *h, int kind, double *out_dev);

/* Vortex count on the z = 0 plane (k = nz/2 in 3D; the only plane in 2D):
 * plaquettes whose counter-clockwise sum of wrapped phase differences is
 * 2 pi w, w > 0, counted w times, when the largest density within `box`
 * points of the plaquette is >= density_frac * max density of the plane;
 * plaquettes with a corner of exactly zero amplitude are skipped.  The
 * paper counts by eye (Sec. 4).  Synchronises the stream. */
int sscn_vortex_count(sscn_handle *h, double density_frac, int box, int *count);

/* Current parameters of the handle (mode and precision change with
 * sscn_set_mode and sscn_converge). */
int sscn_get_params(sscn_handle *h, sscn_params *out);

/* Imaginary-time run to a converged lattice.  Every check_every steps mu
 * (real-part form) is evaluated; the state is converged when |mu - mu_prev| <
 * tol at two consecutive checks with the vortex count (density_frac 0.05,
 * box 3) unchanged between them.  The paper runs a fixed number of steps;
 * this criterion is the library's.  In complex64 mode the bulk runs in FP32
 * until its plateau (|dmu| < switch_tol, or, once |dmu| < 10 switch_tol, no
 * new minimum of |dmu| for 5 checks), then the state is upcast into
 * fp64_psi_dev (caller-owned complex128 buffer, borrowed from then on as by
 * sscn_set_mode) and the run continues in FP64 to tol.  *steps_out = steps taken, *converged = 1 if the
 * criterion was met within max_steps, *switch_out (may be NULL) = the step
 * of the upcast, or -1 if the run stayed in one precision.  Synchronises at
 * every check. */
int sscn_converge(sscn_handle *h, int64_t max_steps, int check_every, double tol, double switch_tol,
                  void *fp64_psi_dev, int64_t *steps_out, int *converged, int64_t *switch_out);

/* Advance nsteps >= 1 steps with a HIP event recorded on the handle's
 * stream before and after every sweep kernel, and return in ms_out[0..3] the
 * average duration (milliseconds) of the x-sweep (with the fused H1), the
 * y-sweep, the z-sweep (0 in 2D) and of a whole step.  For measurement: it
 * launches each kernel on its own, without graphs.  Synchronises the stream. */
int sscn_profile_step(sscn_handle *h, int64_t nsteps, double *ms_out);

/* Choose the kernels of a step.  SSCN_PLAN_SWEEPS: one launch per axis
 * (x with H1 and the pending rescale fused in front; y; z).
 * SSCN_PLAN_FUSED (2D only): one launch per step over 32 x 32 tiles with
 * halos, H1 + x + y fused.  SSCN_PLAN_AUTO (default): on the first step the
 * library times the available plans from a saved copy of the state and
 * keeps the fastest (cached per process).  All plans compute the same step
 * to rounding.  SSCN_EINVAL if the fused plan is not available (3D, or a
 * window above 20 rows in complex128 / 32 in complex64). */
int sscn_set_plan(sscn_handle *h, int plan);

/* Average duration (ms) of one kernel of the step, from nlaunch >= 1
 * back-to-back launches between two HIP events on the handle's stream:
 * which = 0 the fused 2D step or the x-sweep (with H1 and the pending
 * rescale), 1 the y-sweep, 2 the z-sweep.  The launches read the current
 * state and write the library's work buffer and scratch partials, so the
 * state is unchanged.  SSCN_EINVAL if the resolved plan has no such kernel
 * (the fused plan has only kernel 0; 2D has no z-sweep) or the handle uses
 * the exact whole-line path.  Resolves the plan first (as sscn_step).
 * Synchronises the stream. */
int sscn_profile_kernel(sscn_handle *h, int which, int nlaunch, double *avg_ms);

/* Window (rows of look-ahead) used by the truncated line solves per axis
 * (0 means the exact whole-line solve), segment length per axis, the plan
 * in use (SSCN_PLAN_AUTO until the first step resolves it) and the lines
 * per block of the x-sweep staging.  Any output pointer may be NULL.  For
 * diagnostics and tests.  The first step of an SSCN_PLAN_AUTO handle picks
 * the plan and the x-sweep lines per block by timing the candidates; with
 * the environment variable SSCN_TUNE_CACHE naming a file, the choices are
 * also kept there (JSON, keyed by architecture, shape, precision, mode and
 * window). */
int sscn_solver_info(sscn_handle *h, int *window_xyz, int *segment_xyz, int *plan, int *x_lines);

/* Output tile (rows along y, columns along x) of the fused 2D step (Sec. 2's
 * x- and y-direction Crank-Nicolson solves with H1 in one launch, one block
 * per tile): 32 x 32, 32 x 16 or 16 x 16 (more, smaller tiles for grids
 * whose wide tiles leave most compute units idle).  The first step of an
 * SSCN_PLAN_AUTO handle times every shape along with the sweep plans; the
 * environment variable SSCN_FUSED_TILE=0 (32 x 32), 1 (32 x 16) or 2
 * (16 x 16), read at sscn_init, fixes the shape.  The shapes give the same
 * steps to rounding (the norm partials are summed per tile).  SSCN_EINVAL
 * for a NULL argument. */
int sscn_fused_tile(sscn_handle *h, int *rows, int *cols);

void sscn_destroy(sscn_handle *h);

/* ---------------------------------------------------------------------------
 * Batched instances: n problems of different grid sizes and parameters
 * advanced together, HIP-graph replayed, with the convergence test done on
 * the device and converged instances dropped from the work lists.  2D
 * batches step with one fused launch over all instances' 32 x 32 tiles
 * (SSCN_PLAN_FUSED) or with one launch per axis over work lists of line
 * blocks and tiles (SSCN_PLAN_SWEEPS).  3D batches (the identical
 * prescription of Sec. 2 for the third axis) take the sweep plan: x, y and
 * z launches per step over every instance.  Every params[k] must have the
 * same dim (2 or 3), precision and mode; the window (rows of look-ahead) is
 * the largest any instance needs (the z window separately).  psi_devs[k] is
 * instance k's caller-owned state buffer (layout as above), borrowed until
 * sscn_batch_destroy; the library owns one work buffer per instance.  All
 * work goes to hip_stream. */
typedef struct sscn_batch sscn_batch;

int sscn_batch_init(const sscn_params *params, int n, void *const *psi_devs, void *hip_stream,
                    sscn_batch **out);

/* Initial state of Eq. (fun) for instance k (as sscn_init_state; in 3D
 * the z Gaussian has width 1/sqrt(lambda), Eq. (anz)).  Synchronises the
 * stream. */
int sscn_batch_init_state(sscn_batch *b, int k, int kind, const double *phase_host, double d_xy);

/* Enqueue nsteps steps of every active instance; each state is left
 * normalised (imaginary time) in its buffer.  Asynchronous.  A call of
 * n >= 2 steps replays captured HIP graphs: n = q G + r with G = min(n, 256),
 * q launches of the G-step graph, then an r-step graph (r >= 2) or one
 * directly launched step (graphs captured on first use, the four most recent
 * step counts kept).  The first stepping call of an SSCN_PLAN_AUTO batch also
 * picks the plan (sscn_batch_set_plan). */
int sscn_batch_step(sscn_batch *b, int64_t nsteps);

/* The one-time work of a later sscn_batch_step(b, nsteps) without advancing
 * the states: plan choice (timed on saved copies, restored) and graph
 * capture.  Synchronises the stream.  SSCN_EINVAL for a null batch or
 * nsteps < 0. */
int sscn_batch_prepare_steps(sscn_batch *b, int64_t nsteps);

/* Advance nsteps (1..100000) steps launched one by one (no graph), with a HIP
 * event recorded on the batch's stream around every kernel, and return the
 * average durations in milliseconds: sweep plan ms_out[0] the batched
 * x-sweep (with H1 and the pending rescale, which it forms from the norm
 * partials itself), [1] the batched y-sweep, [2] the batched z-sweep (3D
 * batches; 0 in 2D); fused plan ms_out[0] the fused step, [1] = [2] = 0;
 * ms_out[3] a whole step (the finish pass at the end of the call is not
 * timed).  For measurement: the kernels run in the order and on the
 * data of ordinary steps.  Synchronises the stream. */
int sscn_batch_profile_step(sscn_batch *b, int64_t nsteps, double *ms_out);

/* Observables of all n instances into out[0..n-1] (out[k].step: the step at
 * which instance k converged, else the batch step count).  Synchronises. */
int sscn_batch_observables(sscn_batch *b, sscn_obs *out);

/* Imaginary-time run to convergence with the criterion of sscn_converge,
 * evaluated per instance on the device: replay check_every (rounded up to
 * even) steps, compute mu (real-part form) of every active instance, and
 * when |mu - mu_prev| < tol_dmu also its vortex count (density_frac 0.05,
 * box 3, as sscn_vortex_count); an instance is converged at two consecutive
 * checks with |mu - mu_prev| < tol_dmu and an unchanged vortex count.
 * Converged instances leave the work list.  Stops when all have converged or
 * max_steps steps were taken.  steps_out[k] (may be NULL): the batch step
 * count at instance k's convergence, or -1.  Synchronises at every check. */
int sscn_batch_run(sscn_batch *b, int64_t max_steps, int check_every, double tol_dmu, int64_t *steps_out);

/* Make every instance active again and clear the convergence state. */
int sscn_batch_reset(sscn_batch *b);

/* Copy instance k's state to a host buffer.  Synchronises the stream. */
int sscn_batch_get_state(sscn_batch *b, int k, void *host_psi);

/* The caller has written a state into instance k's buffer (psi_devs[k] of
 * sscn_batch_init, e.g. a learned initial state): zero its walls and
 * normalise it to h_x h_y sum |psi|^2 = 1, the finishing steps of the
 * initial state of Eq. (fun) (Sec. 2).  Synchronises the stream. */
int sscn_batch_set_state_device(sscn_batch *b, int k);

/* Vortex count of instance k as sscn_vortex_count (phase winding of each
 * plaquette, density mask).  Synchronises the stream. */
int sscn_batch_vortex_count(sscn_batch *b, int k, double density_frac, int box, int *count);

/* Plan of the batch's steps: SSCN_PLAN_FUSED (one fused 2D step kernel over
 * every instance's tiles), SSCN_PLAN_SWEEPS (an x-sweep kernel and a
 * y-sweep kernel over every instance's line blocks and y tiles, with a
 * per-instance rescale), or SSCN_PLAN_AUTO (default: the first stepping
 * call times both from a saved copy of the states and keeps the faster).
 * Both plans give the same steps within rounding.  The first stepping call
 * under the sweep plan (chosen or forced) also times the x-sweep's two
 * lines-per-block options (sscn_batch_x_lines), which give the same bits.
 * SSCN_EINVAL for the sweep plan when an instance's lines are too long to
 * stage. */
int sscn_batch_set_plan(sscn_batch *b, int plan);

/* The plan in use (SSCN_PLAN_AUTO until the first stepping call resolves
 * it) and the common window W of the batch.  Either pointer may be NULL. */
int sscn_batch_info(sscn_batch *b, int *plan, int *window);

/* Lines per block of the batched x-sweep (sweep plan, Sec. 3's x-direction
 * Crank-Nicolson solves, one block per group of whole x-lines of an
 * instance): *option = 0 for the most lines the segment count and staging
 * allow, 1 for that number halved until a block's LDS is at most 40 KiB
 * (four blocks per CU; the launch reserves the largest instance's LDS for
 * every block).  Option 1 until the autotuner (first stepping call under the
 * sweep plan) keeps the faster; the environment variable
 * SSCN_BATCH_XLINES=0 or 1, read at sscn_batch_init, fixes it instead.
 * tune_ms (2 floats, may be NULL) receives the autotuner's times of 8 steps
 * under each option (0 if not timed). */
int sscn_batch_x_lines(sscn_batch *b, int *option, float *tune_ms);

void sscn_batch_destroy(sscn_batch *b);

const char *sscn_strerror(int code);
const char *sscn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SSCN_H */
