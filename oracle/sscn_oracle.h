/*
 * Oracle for the split-step Crank-Nicolson (SSCN) solver of the rotating
 * Gross-Pitaevskii equation (Kumar, Loncar, Muruganandam, Adhikari, Balaz,
 * "C and Fortran OpenMP programs for rotating Bose-Einstein condensates").
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU implementation
 * written straight from the paper so that the GPU library can be checked
 * against it.  It shares no code with the GPU library and must never be
 * linked into, imported by, or called from the product path.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark use it.
 *
 * Grid convention (paper, Sec. 2 after Eq. (eqD.9:kn1), and Sec. 3 on the
 * (N+1)-point grids): each axis stores n points x_i = -n*h/2 + i*h,
 * i = 0..n-1.  Index 0 is the Dirichlet wall (psi = 0); the paper's last
 * index n (x = +n*h/2) is also a wall and is implied, never stored.
 * Unknowns are i = 1..n-1.  Layout psi[(k*ny + j)*nx + i] (x fastest).
 */
#ifndef SSCN_ORACLE_H
#define SSCN_ORACLE_H

#include <complex.h>

typedef struct {
    int dim;                 /* 2 or 3 */
    int nx, ny, nz;          /* stored points per axis (nz = 1 when dim = 2) */
    double hx, hy, hz;       /* space steps */
    double gamma, nu, lambda;/* trap anisotropies, Eq. (3d) / Eq. (2d) */
    double g;                /* g_2D (dim 2) or g_3D (dim 3) */
    double omega;            /* rotation frequency */
    double dt;               /* time step Delta */
    int mode;                /* 0 = imaginary time (renormalise), 1 = real time */
} orc_params;

typedef struct {
    double norm;             /* h^d sum |psi|^2 */
    double mu, energy;       /* real-part form, Eq. (e2dr)/(e3dr), alpha = 1 and 1/2 */
    double mu_full, energy_full; /* full functional, Eq. (e2d)/(e3d) */
    double mu_4th, energy_4th;   /* the same functional with fourth-order central differences */
    double rms_x, rms_y, rms_z, rms_r;
    double max_density;
    /* the raw sums, each already multiplied by the volume element */
    double sums[16];
} orc_obs;

/* Thomas algorithm (Gaussian elimination without pivoting) for
 * a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = d[i], i = 0..n-1. */
void orc_thomas(int n, const double complex *a, const double complex *b,
                const double complex *c, const double complex *d,
                double complex *x);

/* Pointwise H1 sub-step (Eq. (eq1) propagated over Delta). */
void orc_h1(const orc_params *p, double complex *psi);

/* One Crank-Nicolson sweep along axis 0 (x), 1 (y) or 2 (z). */
void orc_sweep(const orc_params *p, int axis, double complex *psi);

/* psi <- psi / sqrt(h^d sum |psi|^2); returns the norm before scaling. */
double orc_normalize(const orc_params *p, double complex *psi);

/* nsteps full SSCN steps: H1, x, y, [z], then renormalise in imaginary time. */
void orc_step(const orc_params *p, double complex *psi, long nsteps);

/* Initial state of Eq. (fun): kind 1 = one vortex, kind 0 = Gaussian.
 * phase: ny*nx values of the random number R(x,y), or NULL for no random
 * phase.  d_z is only used when dim = 3.  The result is normalised. */
void orc_init_state(const orc_params *p, int kind, const double *phase,
                    double d_xy, double d_z, double complex *psi);

/* Observables of Eqs. (e2dr)/(e3dr), (e2d)/(e3d) and the rms sizes. */
void orc_observables(const orc_params *p, const double complex *psi, orc_obs *out);

/* Vortex count by plaquette phase winding on the z = 0 plane. */
int orc_vortex_count(const orc_params *p, const double complex *psi,
                     double density_frac, int box);

#endif
