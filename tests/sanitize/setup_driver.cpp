// Drives the library's host-side setup (paper_1906_06327_amd/csrc/
// sscn_setup.cpp: validation, coefficients, windows, pivot tables) over valid
// and invalid parameter sets, for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  Exits 0 when every
// invalid set is rejected with the documented code and every table is
// finite with its pivot at the fixed point.
#include <cmath>
#include <complex>
#include <cstdio>
#include <vector>

#include "sscn_setup.hpp"

using namespace sscn;

static int bad = 0;

static void check(bool ok, const char *what)
{
    if (!ok) {
        std::fprintf(stderr, "setup driver: %s failed (%s)\n", what, last_error());
        ++bad;
    }
}

static sscn_params base(int dim)
{
    sscn_params p{};
    p.dim = dim;
    p.nx = 40;
    p.ny = 36;
    p.nz = dim == 3 ? 20 : 1;
    p.hx = 0.1;
    p.hy = 0.12;
    p.hz = 0.2;
    p.gamma = 1.0;
    p.nu = 1.05;
    p.lambda = 4.0;
    p.g = 500.0;
    p.omega = 0.9;
    p.dt = 1e-3;
    p.mode = SSCN_IMAG;
    p.precision = SSCN_C128;
    return p;
}

int main()
{
    // invalid sets and their codes
    struct Case {
        const char *name;
        void (*edit)(sscn_params &);
        int code;
    };
    const Case cases[] = {
        {"dim 4", [](sscn_params &p) { p.dim = 4; }, SSCN_EINVAL},
        {"nx 2", [](sscn_params &p) { p.nx = 2; }, SSCN_EINVAL},
        {"hx 0", [](sscn_params &p) { p.hx = 0.0; }, SSCN_EINVAL},
        {"dt negative", [](sscn_params &p) { p.dt = -1e-3; }, SSCN_EINVAL},
        {"mode 7", [](sscn_params &p) { p.mode = 7; }, SSCN_EINVAL},
        {"precision 3", [](sscn_params &p) { p.precision = 3; }, SSCN_EINVAL},
        {"g NaN", [](sscn_params &p) { p.g = std::nan(""); }, SSCN_EINVAL},
        {"omega 1", [](sscn_params &p) { p.omega = 1.0; }, SSCN_EOMEGA},
        {"omega above nu", [](sscn_params &p) { p.gamma = 2.0; p.omega = 1.06; }, SSCN_EOMEGA},
        {"grid beyond 2^40", [](sscn_params &p) { p.dim = 3; p.nx = p.ny = 1 << 14; p.nz = 1 << 14; }, SSCN_EINVAL},
    };
    for (const Case &c : cases) {
        sscn_params p = base(2);
        c.edit(p);
        check(validate(p) == c.code, c.name);
    }
    // real time with a large rotation step: not diagonally dominant
    {
        sscn_params p = base(2);
        p.mode = SSCN_REAL;
        p.dt = 0.5;
        p.nx = p.ny = 400;
        AxisCoef ac;
        int W = -1;
        check(validate(p) == 0, "valid real-time set");
        check(axis_setup(p, 0, ac, W) == SSCN_EUNSTABLE, "unstable real time");
    }
    // valid sets: every axis, both modes and precisions; tables at the fixed point
    for (int dim = 2; dim <= 3; ++dim)
        for (int mode = 0; mode < 2; ++mode)
            for (int prec = 0; prec < 2; ++prec) {
                sscn_params p = base(dim);
                p.mode = mode;
                p.precision = prec;
                check(validate(p) == 0, "valid set");
                StepArgs a{};
                fill_args(p, a);
                check(std::fabs(a.dV - p.hx * p.hy * (dim == 3 ? p.hz : 1.0)) < 1e-18, "volume element");
                for (int ax = 0; ax < dim; ++ax) {
                    int W = -1;
                    check(axis_setup(p, ax, a.ax[ax], W) == 0, "axis setup");
                    check(W > 0 && W <= 32, "window in range");
                    std::vector<std::complex<double>> t;
                    pivot_table(p, a, ax, W, t);
                    const int types = ax == 0 ? p.ny : ax == 1 ? p.nx : 1;
                    check((int)t.size() == types * (W + 2), "table size");
                    const std::complex<double> A0(a.ax[ax].a0r, a.ax[ax].a0i), u(a.ax[ax].ur, a.ax[ax].ui),
                        q(a.ax[ax].qr, a.ax[ax].qi);
                    for (int ty = 0; ty < types; ++ty) {
                        const double rot = ax == 0 ? p.omega * (a.y0 + ty * p.hy)
                                           : ax == 1 ? -p.omega * (a.x0 + ty * p.hx) : 0.0;
                        const std::complex<double> Ap = u + q * rot, Am = u - q * rot;
                        const std::complex<double> cs = t[(size_t)ty * (W + 2)];
                        check(std::abs(cs - Ap / (A0 - Am * cs)) <= 1e-14 * std::abs(cs) + 1e-300, "fixed point");
                        check(std::abs(cs) < 1.0, "pivot below one");
                        for (int k = 0; k < W + 2; ++k)
                            check(std::isfinite(t[(size_t)ty * (W + 2) + k].real()) &&
                                      std::isfinite(t[(size_t)ty * (W + 2) + k].imag()),
                                  "finite table");
                    }
                }
            }
    check(window_rows(0.3, 1.0, 0.8, 1e-16) == -1, "window of a dominance-free system");
    std::printf("setup driver: %s\n", bad ? "FAILED" : "ok");
    return bad ? 1 : 0;
}
