// Host-side setup of the solver, plain C++ without HIP: parameter
// validation, the per-axis Crank-Nicolson coefficients and window sizes,
// the grid geometry, and the pivot tables of the windowed line solves.
// Compiled into libsscn.so, and on its own with the sanitizers by the tests.
#include "sscn_setup.hpp"

#include <algorithm>
#include <cmath>
#include <string>

namespace sscn {

namespace {
thread_local std::string g_err;
}  // namespace

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

const char *last_error() { return g_err.c_str(); }

// Bound on the truncation error of a windowed line solve (relative to the
// largest |rhs| on the line) for a strictly diagonally dominant tridiagonal
// Toeplitz system with |A-| <= ab, |A0| = bb, |A+| <= cb:
//  - Thomas factors satisfy |c'_k| <= mu = cb / (bb - ab);
//  - the forward sweep damps by lam = ab / (bb - ab mu) per row;
//  - the exact solution just outside a window is at most 1/(bb - ab - cb)
//    times max|rhs| (Varah's bound), and enters the window through one
//    off-diagonal coefficient at each end;
//  - so at W rows from both window ends the error of y is at most
//    yb kappa (ab lam^W / (1 - mu lam) + cb mu^W), kappa = 1/(bb - ab mu),
//    and the Cayley output 2y - v doubles it.
// Returns the smallest W meeting tol, or -1 if not diagonally dominant.
int window_rows(double ab, double bb, double cb, double tol)
{
    if (!(ab + cb < bb))
        return -1;
    const double mu = cb / (bb - ab);
    const double lam = ab / (bb - ab * mu);
    const double kappa = 1.0 / (bb - ab * mu);
    const double yb = 1.0 / (bb - ab - cb);
    for (int w = 0; w <= 4096; ++w) {
        const double err = 2.0 * yb * kappa * (ab * std::pow(lam, w) / (1.0 - mu * lam) + cb * std::pow(mu, w));
        if (err <= tol)
            return w;
    }
    return 4097;
}

int validate(const sscn_params &p)
{
    if (p.dim != 2 && p.dim != 3)
        return fail(SSCN_EINVAL, "dim must be 2 or 3");
    if (p.nx < 3 || p.ny < 3 || (p.dim == 3 && p.nz < 3))
        return fail(SSCN_EINVAL, "every axis needs at least 3 stored points");
    if ((int64_t)p.nx * p.ny * (p.dim == 3 ? p.nz : 1) > ((int64_t)1 << 40))
        return fail(SSCN_EINVAL, "grid too large");
    if (!(p.hx > 0) || !(p.hy > 0) || (p.dim == 3 && !(p.hz > 0)) || !(p.dt > 0))
        return fail(SSCN_EINVAL, "space and time steps must be positive");
    if (p.mode != SSCN_IMAG && p.mode != SSCN_REAL)
        return fail(SSCN_EINVAL, "mode must be SSCN_IMAG or SSCN_REAL");
    if (p.precision != SSCN_C128 && p.precision != SSCN_C64)
        return fail(SSCN_EINVAL, "precision must be SSCN_C128 or SSCN_C64");
    if (!std::isfinite(p.g) || !std::isfinite(p.omega) || !std::isfinite(p.gamma) || !std::isfinite(p.nu) ||
        (p.dim == 3 && !std::isfinite(p.lambda)))
        return fail(SSCN_EINVAL, "non-finite physical parameter");
    if (!(std::fabs(p.omega) < std::min(p.gamma, p.nu)))
        return fail(SSCN_EOMEGA, "|omega| must be below min(gamma, nu)");
    return 0;
}

// Crank-Nicolson coefficients of one axis and its window size.
int axis_setup(const sscn_params &p, int axis, AxisCoef &c, int &W)
{
    using cd = std::complex<double>;
    const cd I(0.0, 1.0);
    const cd tau = p.mode == SSCN_REAL ? cd(p.dt, 0.0) : cd(0.0, -p.dt);
    const double h = axis == 0 ? p.hx : axis == 1 ? p.hy : p.hz;
    const int n = axis == 0 ? p.nx : axis == 1 ? p.ny : p.nz;
    const cd k0 = I * tau / (2.0 * h * h);
    const cd A0 = 1.0 + k0;
    const cd u = -I * tau / (4.0 * h * h);
    const cd q = tau / (4.0 * h);
    c = AxisCoef{A0.real(), A0.imag(), k0.real(), k0.imag(), u.real(), u.imag(), q.real(), q.imag()};
    // the largest rotation coefficient on this axis's lines
    double rmax = 0.0;
    if (axis == 0)
        rmax = std::fabs(p.omega) * 0.5 * p.ny * p.hy;
    else if (axis == 1)
        rmax = std::fabs(p.omega) * 0.5 * p.nx * p.hx;
    const double amax = std::max(std::abs(u + q * rmax), std::abs(u - q * rmax));
    const double tol = p.precision == SSCN_C128 ? std::ldexp(1.0, -56) : std::ldexp(1.0, -27);
    const int w = window_rows(amax, std::abs(A0), amax, tol);
    if (w < 0)
        return fail(SSCN_EUNSTABLE, "line system of axis " + std::to_string(axis) +
                                        " is not strictly diagonally dominant (dt*|omega|*max|coord|/(2h) too large)");
    W = 0;
    for (int cand : kWindows)
        if (cand >= w) {
            W = cand;
            break;
        }
    (void)n;
    return 0;
}

// Grid geometry and physical constants of the step and observables kernels
// (everything of StepArgs but the per-axis line coefficients).
void fill_args(const sscn_params &p, StepArgs &a)
{
    a.dim = p.dim;
    a.nx = p.nx;
    a.ny = p.ny;
    a.nz = p.dim == 3 ? p.nz : 1;
    a.hx = p.hx;
    a.hy = p.hy;
    a.hz = p.dim == 3 ? p.hz : 1.0;
    a.x0 = -0.5 * p.nx * p.hx;
    a.y0 = -0.5 * p.ny * p.hy;
    a.z0 = p.dim == 3 ? -0.5 * p.nz * p.hz : 0.0;
    a.vx = 0.5 * p.gamma * p.gamma;
    a.vy = 0.5 * p.nu * p.nu;
    a.vz = p.dim == 3 ? 0.5 * p.lambda * p.lambda : 0.0;
    a.g = p.g;
    a.omega = p.omega;
    a.dt = p.dt;
    a.dV = p.hx * p.hy * (p.dim == 3 ? p.hz : 1.0);
}

// The fixed point c* = A+ / (A0 - A- c*) of the Thomas recurrence of a
// diagonally dominant line: the root of A- c^2 - A0 c + A+ = 0 of smaller
// modulus, c* = 2 A+ / (A0 + s) with s = sqrt(A0^2 - 4 A- A+) taken with
// Re(conj(A0) s) >= 0 (no cancellation in A0 + s), then polished by the
// recurrence itself.  Each iteration multiplies the error by
// |A- c* r*| < 1/2 (r* = 1/(A0 - A- c*)), so it stops after a few, when the
// change is within 4 ulps (at most 16 iterations).
std::complex<double> pivot_fixed_point(std::complex<double> A0, std::complex<double> Am, std::complex<double> Ap)
{
    using cd = std::complex<double>;
    cd sq = std::sqrt(A0 * A0 - 4.0 * Am * Ap);
    if ((std::conj(A0) * sq).real() < 0.0)
        sq = -sq;
    cd c = 2.0 * Ap / (A0 + sq);
    for (int it = 0; it < 16; ++it) {
        const cd nc = Ap / (A0 - Am * c);
        const bool done = std::abs(nc - c) <= 4.0 * 2.220446049250313e-16 * std::abs(nc);
        c = nc;
        if (done)
            break;
    }
    return c;
}

// The pivot table of axis ax (rows of stride W + 2, one per distinct line:
// y-lines by i, x-lines by j, one for z), as build_tables uploads it: the
// fixed point c*, r* of the Thomas recurrence c' = A+ r, r = 1/(A0 - A- c'),
// then the wall correction zeta_u = 2 gamma z_u (u = 1..W) with
// z = T_abs^{-1} e_1 over the whole line and gamma = A- c* / (1 + A- c* z_1)
// (Sherman-Morrison for the one diagonal entry in which the line matrix
// differs from T_abs).  FP64.
void pivot_table(const sscn_params &p, const StepArgs &a, int ax, int W, std::vector<std::complex<double>> &t)
{
    using cd = std::complex<double>;
    const AxisCoef &c = a.ax[ax];
    const cd A0(c.a0r, c.a0i), u(c.ur, c.ui), q(c.qr, c.qi);
    const int ntypes = ax == 0 ? p.ny : ax == 1 ? p.nx : 1;
    const int m = (ax == 0 ? p.nx : ax == 1 ? p.ny : p.nz) - 1;  // unknowns per line
    const int stride = W + 2;
    t.assign((size_t)ntypes * stride, cd(0.0));
    std::vector<cd> z((size_t)m + 2);
    for (int ty = 0; ty < ntypes; ++ty) {
        double rot = 0.0;
        if (ax == 0)
            rot = p.omega * (a.y0 + ty * p.hy);
        else if (ax == 1)
            rot = -p.omega * (a.x0 + ty * p.hx);
        const cd Ap = u + q * rot, Am = u - q * rot;
        const cd cs = pivot_fixed_point(A0, Am, Ap);
        const cd rs = 1.0 / (A0 - Am * cs);
        // z = T_abs^{-1} e_1: forward d'_1 = r*, d'_k = -A- r* d'_{k-1};
        // back z_m = d'_m, z_k = d'_k - c* z_{k+1}
        cd d = rs;
        z[1] = d;
        for (int k = 2; k <= m; ++k) {
            d = -Am * rs * d;
            z[k] = d;
        }
        for (int k = m - 1; k >= 1; --k)
            z[k] = z[k] - cs * z[k + 1];
        const cd gam = Am * cs / (1.0 + Am * cs * z[1]);
        cd *row = &t[(size_t)ty * stride];
        row[0] = cs;
        row[1] = rs;
        for (int k = 1; k <= W; ++k)
            row[1 + k] = k <= m ? 2.0 * gam * z[k] : cd(0.0);
    }
}

}  // namespace sscn
