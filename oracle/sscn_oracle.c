/*
 * Oracle for the SSCN solver of the rotating Gross-Pitaevskii equation.
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, obviously-correct FP64 CPU
 * implementation of what the GPU path computes.  It shares no code with the
 * GPU library; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it.
 *
 * Every function follows the paper step by step (sections and equations
 * cited below).  Readings of places where the paper is silent are marked
 * "Reading:".  OpenMP is used only over independent lines and points; every
 * reduction is a serial loop in a fixed order, so the results do not depend
 * on the thread count.
 */
#include "sscn_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Grid point i of an axis with n stored points and step h (Sec. 2, the
 * definition x_i = -N_x h_x / 2 + i h_x below Eq. (eqD.9:kn1)). */
static double coord(int n, double h, int i) { return -0.5 * n * h + i * h; }

/* Complex time step.  Real time: tau = Delta.  Imaginary time: the paper
 * obtains it by the transformation Delta -> -i Delta (Sec. 2, the paragraph
 * after Eq. (eq5)).  Reading: the substitution is applied to every Delta, so
 * one formula with complex tau serves both modes. */
static double complex tau_of(const orc_params *p)
{
    return p->mode == 1 ? (double complex)p->dt : -I * p->dt;
}

static long npoints(const orc_params *p)
{
    return (long)p->nx * p->ny * (p->dim == 3 ? p->nz : 1);
}

static double volume_element(const orc_params *p)
{
    return p->hx * p->hy * (p->dim == 3 ? p->hz : 1.0);
}

/* Harmonic trap of Eq. (3d) (dim 3) or Eq. (2d) (dim 2). */
static double potential(const orc_params *p, double x, double y, double z)
{
    double v = p->gamma * p->gamma * x * x + p->nu * p->nu * y * y;
    if (p->dim == 3)
        v += p->lambda * p->lambda * z * z;
    return 0.5 * v;
}

void orc_thomas(int n, const double complex *a, const double complex *b,
                const double complex *c, const double complex *d,
                double complex *x)
{
    /* Textbook forward elimination and back substitution, no pivoting. */
    double complex *cp = malloc(sizeof(double complex) * (size_t)n);
    double complex *dp = malloc(sizeof(double complex) * (size_t)n);
    cp[0] = (n > 1) ? c[0] / b[0] : 0.0;
    dp[0] = d[0] / b[0];
    for (int i = 1; i < n; i++) {
        double complex den = b[i] - a[i] * cp[i - 1];
        cp[i] = (i < n - 1) ? c[i] / den : 0.0;
        dp[i] = (d[i] - a[i] * dp[i - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; i--)
        x[i] = dp[i] - cp[i] * x[i + 1];
    free(cp);
    free(dp);
}

void orc_h1(const orc_params *p, double complex *psi)
{
    /* Sub-step with H1 = V + g|psi|^2 (Eq. (eq1)), "analytic solution"
     * (Sec. 2).  Reading: the density is taken from the input of the
     * sub-step, psi <- exp(-i tau (V + g|psi|^2)) psi.  In real time this is
     * the exact solution because |psi| is invariant. */
    const double complex tau = tau_of(p);
    const int nz = (p->dim == 3) ? p->nz : 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < p->ny; j++) {
            double y = coord(p->ny, p->hy, j);
            double z = (p->dim == 3) ? coord(p->nz, p->hz, k) : 0.0;
            for (int i = 0; i < p->nx; i++) {
                double x = coord(p->nx, p->hx, i);
                long idx = ((long)k * p->ny + j) * p->nx + i;
                double complex v = psi[idx];
                double dens = creal(v) * creal(v) + cimag(v) * cimag(v);
                double w = potential(p, x, y, z) + p->g * dens;
                psi[idx] = cexp(-I * tau * w) * v;
            }
        }
}

/* Crank-Nicolson propagation of one grid line under
 *   H = -1/2 d^2/ds^2 + (rotation term),
 * following Eq. (eqD.9:kn1) -> Eqs. (eqD.11), (eq5).  `v` holds the n stored
 * values of the line (v[0] is the wall); the implied wall v[n] is 0.
 * `rot` is Omega * y_j for x-lines (Eq. (eq2)), -Omega * x_i for y-lines
 * (Eq. (eq3): "similarly" with y_j -> -x_i) and 0 for z-lines. */
static void cn_line(int n, double h, double rot, double complex tau,
                    double complex *v)
{
    int m = n - 1; /* unknowns 1..n-1 */
    if (m <= 0)
        return;
    double complex *a = malloc(sizeof(double complex) * (size_t)m);
    double complex *b = malloc(sizeof(double complex) * (size_t)m);
    double complex *c = malloc(sizeof(double complex) * (size_t)m);
    double complex *d = malloc(sizeof(double complex) * (size_t)m);
    double complex *x = malloc(sizeof(double complex) * (size_t)m);

    const double complex A0 = 1.0 + I * tau / (2.0 * h * h);
    const double complex Am = -(I * tau / (4.0 * h)) * (1.0 / h - I * rot);
    const double complex Ap = -(I * tau / (4.0 * h)) * (1.0 / h + I * rot);
    for (int r = 0; r < m; r++) {
        int i = r + 1;
        double complex vm = v[i - 1];
        double complex v0 = v[i];
        double complex vp = (i + 1 < n) ? v[i + 1] : 0.0;
        a[r] = Am;
        b[r] = A0;
        c[r] = Ap;
        d[r] = (I * tau / (4.0 * h * h)) * (vp - 2.0 * v0 + vm)
             - (tau * rot / (4.0 * h)) * (vp - vm) + v0;
    }
    orc_thomas(m, a, b, c, d, x);
    v[0] = 0.0;
    for (int r = 0; r < m; r++)
        v[r + 1] = x[r];
    free(a);
    free(b);
    free(c);
    free(d);
    free(x);
}

void orc_sweep(const orc_params *p, int axis, double complex *psi)
{
    const double complex tau = tau_of(p);
    const int nx = p->nx, ny = p->ny, nz = (p->dim == 3) ? p->nz : 1;
    const long sx = 1, sy = nx, sz = (long)nx * ny;
    int n, nlines;
    double h;
    if (axis == 0) {
        n = nx; h = p->hx; nlines = ny * nz;
    } else if (axis == 1) {
        n = ny; h = p->hy; nlines = nx * nz;
    } else {
        n = nz; h = p->hz; nlines = nx * ny;
    }
#pragma omp parallel for schedule(static)
    for (int line = 0; line < nlines; line++) {
        long base, stride;
        double rot;
        if (axis == 0) {          /* x-line at (j, k) */
            int j = line % ny, k = line / ny;
            base = (long)k * sz + (long)j * sy;
            stride = sx;
            rot = p->omega * coord(ny, p->hy, j);
        } else if (axis == 1) {   /* y-line at (i, k) */
            int i = line % nx, k = line / nx;
            base = (long)k * sz + i;
            stride = sy;
            rot = -p->omega * coord(nx, p->hx, i);
        } else {                  /* z-line at (i, j), no rotation term */
            int i = line % nx, j = line / nx;
            base = (long)j * sy + i;
            stride = sz;
            rot = 0.0;
        }
        double complex *v = malloc(sizeof(double complex) * (size_t)n);
        for (int t = 0; t < n; t++)
            v[t] = psi[base + t * stride];
        cn_line(n, h, rot, tau, v);
        for (int t = 0; t < n; t++)
            psi[base + t * stride] = v[t];
        free(v);
    }
}

double orc_normalize(const orc_params *p, double complex *psi)
{
    /* Normalisation condition of Eq. (2d)/(3d): integral |psi|^2 = 1.
     * Reading: the integral is the plain sum times the volume element (equal
     * to the trapezoid rule because the walls are zero). */
    long np = npoints(p);
    double s = 0.0;
    for (long t = 0; t < np; t++)
        s += creal(psi[t]) * creal(psi[t]) + cimag(psi[t]) * cimag(psi[t]);
    double norm = s * volume_element(p);
    double scale = 1.0 / sqrt(norm);
    for (long t = 0; t < np; t++)
        psi[t] *= scale;
    return norm;
}

void orc_step(const orc_params *p, double complex *psi, long nsteps)
{
    /* Lie splitting: H1, then H2 (x), then H3 (y), in that order (Sec. 2,
     * Eq. (split)); in 3D the z part follows ("identical prescription").
     * Imaginary time renormalises after every step. */
    for (long s = 0; s < nsteps; s++) {
        orc_h1(p, psi);
        orc_sweep(p, 0, psi);
        orc_sweep(p, 1, psi);
        if (p->dim == 3)
            orc_sweep(p, 2, psi);
        if (p->mode == 0)
            orc_normalize(p, psi);
    }
}

void orc_init_state(const orc_params *p, int kind, const double *phase,
                    double d_xy, double d_z, double complex *psi)
{
    /* Eq. (fun).  kind 1: (x + i y) one-vortex factor; kind 0: the Gaussian
     * obtained by setting (x + i y) = 1.  R(x, y) depends on (x, y) only. */
    const int nz = (p->dim == 3) ? p->nz : 1;
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < p->ny; j++)
            for (int i = 0; i < p->nx; i++) {
                long idx = ((long)k * p->ny + j) * p->nx + i;
                if (i == 0 || j == 0 || (p->dim == 3 && k == 0)) {
                    psi[idx] = 0.0;
                    continue;
                }
                double x = coord(p->nx, p->hx, i);
                double y = coord(p->ny, p->hy, j);
                double complex f = kind ? (x + I * y) : 1.0;
                double complex v = f / sqrt(M_PI * d_xy * d_xy)
                                 * exp(-(x * x + y * y) / (2.0 * d_xy * d_xy));
                if (phase)
                    v *= cexp(2.0 * M_PI * I * phase[(long)j * p->nx + i]);
                if (p->dim == 3) {
                    double z = coord(p->nz, p->hz, k);
                    v *= pow(M_PI * d_z * d_z, -0.25)
                       * exp(-z * z / (2.0 * d_z * d_z));
                }
                psi[idx] = v;
            }
    orc_normalize(p, psi);
}

/* psi at (i, j, k), zero outside the stored grid (walls). */
static double complex at(const orc_params *p, const double complex *psi,
                         int i, int j, int k)
{
    int nz = (p->dim == 3) ? p->nz : 1;
    if (i < 0 || j < 0 || k < 0 || i >= p->nx || j >= p->ny || k >= nz)
        return 0.0;
    return psi[((long)k * p->ny + j) * p->nx + i];
}

void orc_observables(const orc_params *p, const double complex *psi, orc_obs *out)
{
    /* Sums, in a fixed serial order:
     *  [0] |psi|^2          [1] psi_R^2
     *  [2] 1/2 (grad psi_R)^2 (forward differences)
     *  [3] V psi_R^2        [4] g |psi|^2 psi_R^2
     *  [5] Omega psi_R (y d/dx - x d/dy) psi_I (central differences)
     *  [6] 1/2 |grad psi|^2 [7] V |psi|^2   [8] g |psi|^4
     *  [9] Omega Im[psi^* (y d/dx - x d/dy) psi]  (= -Omega <L_z> density)
     *  [10..12] x^2, y^2, z^2 times |psi|^2       [13] max |psi|^2
     *  [14] 1/2 |grad psi|^2 and [15] Omega Im[psi^* (y d/dx - x d/dy) psi]
     *       with fourth-order central differences
     *       (-f[i+2] + 8 f[i+1] - 8 f[i-1] + f[i-2]) / (12 h)
     * Reading of Eq. (e2dr)/(e3dr): the kinetic term enters with +1/2, as
     * integrating psi_R times Eq. (real) by parts gives. */
    const int nz = (p->dim == 3) ? p->nz : 1;
    double s[16];
    memset(s, 0, sizeof s);
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < p->ny; j++)
            for (int i = 0; i < p->nx; i++) {
                double x = coord(p->nx, p->hx, i);
                double y = coord(p->ny, p->hy, j);
                double z = (p->dim == 3) ? coord(p->nz, p->hz, k) : 0.0;
                double complex v = at(p, psi, i, j, k);
                double vr = creal(v), vi = cimag(v);
                double dens = vr * vr + vi * vi;
                double V = potential(p, x, y, z);

                /* forward differences for the kinetic terms */
                double complex fx = (at(p, psi, i + 1, j, k) - v) / p->hx;
                double complex fy = (at(p, psi, i, j + 1, k) - v) / p->hy;
                double complex fz = 0.0;
                if (p->dim == 3)
                    fz = (at(p, psi, i, j, k + 1) - v) / p->hz;
                double kin_r = creal(fx) * creal(fx) + creal(fy) * creal(fy)
                             + creal(fz) * creal(fz);
                double kin = cabs(fx) * cabs(fx) + cabs(fy) * cabs(fy)
                           + cabs(fz) * cabs(fz);

                /* central differences for the rotation terms */
                double complex cx = (at(p, psi, i + 1, j, k) - at(p, psi, i - 1, j, k))
                                  / (2.0 * p->hx);
                double complex cy = (at(p, psi, i, j + 1, k) - at(p, psi, i, j - 1, k))
                                  / (2.0 * p->hy);
                double complex lz = y * cx - x * cy; /* (y d/dx - x d/dy) psi */

                /* fourth-order central differences */
                double complex qx = (-at(p, psi, i + 2, j, k) + 8.0 * at(p, psi, i + 1, j, k)
                                     - 8.0 * at(p, psi, i - 1, j, k) + at(p, psi, i - 2, j, k))
                                    / (12.0 * p->hx);
                double complex qy = (-at(p, psi, i, j + 2, k) + 8.0 * at(p, psi, i, j + 1, k)
                                     - 8.0 * at(p, psi, i, j - 1, k) + at(p, psi, i, j - 2, k))
                                    / (12.0 * p->hy);
                double complex qz = 0.0;
                if (p->dim == 3)
                    qz = (-at(p, psi, i, j, k + 2) + 8.0 * at(p, psi, i, j, k + 1)
                          - 8.0 * at(p, psi, i, j, k - 1) + at(p, psi, i, j, k - 2))
                         / (12.0 * p->hz);
                double kin4 = cabs(qx) * cabs(qx) + cabs(qy) * cabs(qy) + cabs(qz) * cabs(qz);
                double complex lz4 = y * qx - x * qy;

                s[0] += dens;
                s[1] += vr * vr;
                s[2] += 0.5 * kin_r;
                s[3] += V * vr * vr;
                s[4] += p->g * dens * vr * vr;
                s[5] += p->omega * vr * cimag(lz);
                s[6] += 0.5 * kin;
                s[7] += V * dens;
                s[8] += p->g * dens * dens;
                s[9] += p->omega * cimag(conj(v) * lz);
                s[10] += x * x * dens;
                s[11] += y * y * dens;
                s[12] += z * z * dens;
                if (dens > s[13])
                    s[13] = dens;
                s[14] += 0.5 * kin4;
                s[15] += p->omega * cimag(conj(v) * lz4);
            }
    double dv = volume_element(p);
    for (int t = 0; t < 16; t++)
        if (t != 13)
            s[t] *= dv;
    memcpy(out->sums, s, sizeof s);
    out->norm = s[0];
    out->mu = (s[2] + s[3] + s[4] + s[5]) / s[1];
    out->energy = (s[2] + s[3] + 0.5 * s[4] + s[5]) / s[1];
    out->mu_full = (s[6] + s[7] + s[8] + s[9]) / s[0];
    out->energy_full = (s[6] + s[7] + 0.5 * s[8] + s[9]) / s[0];
    out->mu_4th = (s[14] + s[7] + s[8] + s[15]) / s[0];
    out->energy_4th = (s[14] + s[7] + 0.5 * s[8] + s[15]) / s[0];
    out->rms_x = sqrt(s[10] / s[0]);
    out->rms_y = sqrt(s[11] / s[0]);
    out->rms_z = sqrt(s[12] / s[0]);
    out->rms_r = sqrt((s[10] + s[11] + s[12]) / s[0]);
    out->max_density = s[13];
}

int orc_vortex_count(const orc_params *p, const double complex *psi,
                     double density_frac, int box)
{
    /* The paper counts vortices by eye from density plots (Sec. 4).
     * Reading: a plaquette (i,j)-(i+1,j)-(i+1,j+1)-(i,j+1) holds a vortex of
     * charge w = round(sum of wrapped phase differences / 2 pi) taken
     * counter-clockwise; it is counted (w times, w > 0) when the largest
     * density within `box` points of the plaquette reaches density_frac of
     * the plane's maximum, which excludes phase defects in the empty outer
     * region.  Plaquettes with a corner of exactly zero amplitude (the walls)
     * are skipped.  In 3D the plane is z = 0, k = nz / 2. */
    const int k0 = (p->dim == 3) ? p->nz / 2 : 0;
    const int nx = p->nx, ny = p->ny;
    double dmax = 0.0;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            double complex v = at(p, psi, i, j, k0);
            double d = creal(v) * creal(v) + cimag(v) * cimag(v);
            if (d > dmax)
                dmax = d;
        }
    int count = 0;
    for (int j = 0; j + 1 < ny; j++)
        for (int i = 0; i + 1 < nx; i++) {
            double complex c00 = at(p, psi, i, j, k0);
            double complex c10 = at(p, psi, i + 1, j, k0);
            double complex c11 = at(p, psi, i + 1, j + 1, k0);
            double complex c01 = at(p, psi, i, j + 1, k0);
            /* a corner of exactly zero amplitude has no phase: no winding */
            if (c00 == 0.0 || c10 == 0.0 || c11 == 0.0 || c01 == 0.0)
                continue;
            double sum = carg(c10 * conj(c00)) + carg(c11 * conj(c10))
                       + carg(c01 * conj(c11)) + carg(c00 * conj(c01));
            int w = (int)lround(sum / (2.0 * M_PI));
            if (w <= 0)
                continue;
            double local = 0.0;
            for (int jj = j - box; jj <= j + 1 + box; jj++)
                for (int ii = i - box; ii <= i + 1 + box; ii++) {
                    double complex v = at(p, psi, ii, jj, k0);
                    double d = creal(v) * creal(v) + cimag(v) * cimag(v);
                    if (d > local)
                        local = d;
                }
            if (local >= density_frac * dmax)
                count += w;
        }
    return count;
}
