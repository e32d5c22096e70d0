/* Drives the FP64 oracle through every entry point on small 2D and 3D grids
 * in both propagation modes, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  Exits 0 when every
 * result is finite and the norm checks hold. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "sscn_oracle.h"

static int check(int ok, const char *what)
{
    if (!ok)
        fprintf(stderr, "oracle driver: %s failed\n", what);
    return ok ? 0 : 1;
}

static int run(int dim, int mode, int nx, int ny, int nz)
{
    orc_params p = {dim, nx, ny, dim == 3 ? nz : 1, 0.2, 0.17, 0.25, 1.0, 1.1, 2.0, 40.0, 0.45, 2e-3, mode};
    const long n = (long)nx * ny * p.nz;
    double complex *psi = malloc(sizeof(double complex) * n);
    double *phase = malloc(sizeof(double) * nx * ny);
    int bad = 0;
    for (int e = 0; e < nx * ny; ++e)
        phase[e] = fmod(0.6180339887 * (e + 1), 1.0);
    orc_init_state(&p, 1, phase, 1.0, 0.7, psi);
    orc_step(&p, psi, 7);
    orc_h1(&p, psi);
    for (int ax = 0; ax < dim; ++ax)
        orc_sweep(&p, ax, psi);
    const double nrm = orc_normalize(&p, psi);
    orc_obs o;
    orc_observables(&p, psi, &o);
    const int count = orc_vortex_count(&p, psi, 0.05, 3);
    bad += check(isfinite(nrm) && nrm > 0, "norm before normalisation");
    bad += check(fabs(o.norm - 1.0) < 1e-12, "normalised norm");
    bad += check(isfinite(o.mu) && isfinite(o.energy) && isfinite(o.mu_4th) && isfinite(o.rms_r), "observables");
    bad += check(count >= 0, "vortex count");
    free(psi);
    free(phase);
    return bad;
}

int main(void)
{
    int bad = 0;
    double complex a[9], b[9], c[9], d[9], x[9];
    for (int i = 0; i < 9; ++i) {
        a[i] = -0.2 + 0.1 * I;
        b[i] = 1.5 + 0.05 * i * I;
        c[i] = -0.3 - 0.1 * I;
        d[i] = 1.0 + i * I;
    }
    orc_thomas(9, a, b, c, d, x);
    for (int i = 0; i < 9; ++i)
        bad += check(isfinite(creal(x[i])) && isfinite(cimag(x[i])), "thomas");
    for (int mode = 0; mode < 2; ++mode) {
        bad += run(2, mode, 13, 11, 1);
        bad += run(3, mode, 9, 8, 7);
    }
    printf("oracle driver: %s\n", bad ? "FAILED" : "ok");
    return bad ? 1 : 0;
}
