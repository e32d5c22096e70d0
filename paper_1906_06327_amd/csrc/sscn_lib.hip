// Host side of the SSCN C ABI (include/sscn.h): parameter validation, the
// per-axis Crank-Nicolson coefficients, window selection, kernel dispatch,
// step sequencing with HIP graphs, observables and vortex counting.
#include "sscn.h"
#include "sscn_device.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace sscn;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIPCHECK(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(SSCN_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

constexpr int kSeg = 8;             // outputs per thread segment (all axes)
constexpr int kGraphSteps = 64;     // steps per captured graph
constexpr int kRedBlocks = 1024;    // blocks of the grid-stride reductions
constexpr int kTile = 32;           // fused 2D step: output tile side
constexpr size_t kXLdsCap = 64 * 1024;

// Supported window sizes (template instantiations).
const int kWindows[] = {4, 6, 8, 10, 12, 16, 20, 24, 32};

}  // namespace

struct sscn_handle {
    sscn_params p;
    void *psi = nullptr;    // caller-owned state
    void *work = nullptr;   // second state-sized buffer (strided sweeps)
    void *ws = nullptr;     // exact-path workspace
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    int64_t npts = 0;
    size_t esize = 0;
    StepArgs args{};
    int W[3] = {0, 0, 0};   // window per axis; 0 = exact whole-line path
    bool exact = false;
    int xL = 1;             // lines per block of the x-sweep
    size_t xlds = 0;
    int nemit = 0;          // partials written by the last sweep
    double *partials = nullptr;  // norm partials between steps
    double *obs_part = nullptr;  // observables / vortex partials
    double *obs_buf = nullptr;   // finished reductions (device)
    double *phase = nullptr;
    void *tab[3] = {nullptr, nullptr, nullptr};  // per-axis pivot tables
    int ygrid[3] = {0, 0, 0};  // strided-sweep logical grids (gx, gy, gz)
    int zgrid[2] = {0, 0};
    bool pending = false;   // partials hold the norm of an unnormalised state
    int64_t steps = 0;
    // fused 2D step (one launch per step over a work list of tiles)
    int plan = SSCN_PLAN_AUTO;   // requested plan
    int active_plan = SSCN_PLAN_SWEEPS;
    bool fused_ok = false;
    Inst2D *d_inst = nullptr;
    int2 *d_work = nullptr;
    int *d_nwork = nullptr;
    int ntiles = 0;
    double *partials2 = nullptr;
    int fparity = 0;        // buffer (0 = psi, 1 = work) holding the state
    int pbuf = 0;           // partial buffer holding the pending norm
    float tune_ms[3] = {0, 0, 0};
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
};

namespace {

int64_t npoints(const sscn_params &p)
{
    return (int64_t)p.nx * p.ny * (p.dim == 3 ? p.nz : 1);
}

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

int setup(sscn_handle *h)
{
    const sscn_params &p = h->p;
    StepArgs &a = h->args;
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
    h->exact = false;
    for (int ax = 0; ax < p.dim; ++ax) {
        int r = axis_setup(p, ax, a.ax[ax], h->W[ax]);
        if (r)
            return r;
        if (h->W[ax] == 0)
            h->exact = true;
    }
    if (p.dim == 2) {
        a.ax[2] = a.ax[1];
        h->W[2] = 0;
        // one window for both axes (the fused step needs a common table stride)
        h->W[0] = h->W[1] = std::max(h->W[0], h->W[1]);
    }
    h->npts = npoints(p);
    h->esize = p.precision == SSCN_C128 ? 16 : 8;
    // x-sweep staging: L lines per block, one (line, segment) per thread
    const int nseg = (p.nx - 2) / kSeg + 1;
    const size_t LS = (size_t)p.nx + p.nx / kSeg + 1;
    const int L = std::max(1, std::min({256 / nseg, 256 * kXLoad / p.nx, 512 / (h->W[0] + 2)}));
    h->xL = L;
    h->xlds = (L * LS + (size_t)L * (h->W[0] + 2) + L) * h->esize;
    if (nseg > 256 || p.nx > 256 * kXLoad || h->xlds > kXLdsCap)
        h->exact = true;  // lines too long to stage; whole-line path
    // strided sweeps: logical grids and the partials written by the last one
    h->ygrid[0] = (p.nx + 63) / 64;
    h->ygrid[1] = ((p.ny - 2) / kSeg + 1 + kSegBlock - 1) / kSegBlock;
    h->ygrid[2] = p.dim == 3 ? p.nz : 1;
    h->zgrid[0] = (int)(((int64_t)p.nx * p.ny + 63) / 64);
    h->zgrid[1] = p.dim == 3 ? ((p.nz - 2) / kSeg + 1 + kSegBlock - 1) / kSegBlock : 1;
    if (p.dim == 2)
        h->nemit = h->ygrid[0] * h->ygrid[1];
    else
        h->nemit = h->zgrid[0] * h->zgrid[1];
    if (h->exact) {
        h->W[0] = h->W[1] = h->W[2] = 0;
        h->nemit = kRedBlocks;
    }
    h->fused_ok = p.dim == 2 && !h->exact && h->W[0] > 0 &&
                  h->W[0] <= (p.precision == SSCN_C128 ? 20 : 32);
    h->ntiles = ((p.nx - 2) / kTile + 1) * ((p.ny - 2) / kTile + 1);
    return 0;
}

// Pivot tables of the windowed solves, one row per distinct line of an axis
// (x-lines by j, y-lines by i, one for z), stride W + 2: the fixed point c*,
// r* of the Thomas recurrence c' = A+ r, r = 1/(A0 - A- c'), then the wall
// correction zeta_u = 2 gamma z_u (u = 1..W) with z = T_abs^{-1} e_1 over the
// whole line and gamma = A- c* / (1 + A- c* z_1) (Sherman-Morrison for the
// one diagonal entry in which the line matrix differs from T_abs).  FP64.
int build_tables(sscn_handle *h)
{
    using cd = std::complex<double>;
    const sscn_params &p = h->p;
    for (int ax = 0; ax < 3; ++ax) {
        if (h->tab[ax])
            (void)hipFree(h->tab[ax]);
        h->tab[ax] = nullptr;
    }
    if (h->exact)
        return 0;
    for (int ax = 0; ax < p.dim; ++ax) {
        const int W = h->W[ax];
        const AxisCoef &c = h->args.ax[ax];
        const cd A0(c.a0r, c.a0i), u(c.ur, c.ui), q(c.qr, c.qi);
        const int ntypes = ax == 0 ? p.ny : ax == 1 ? p.nx : 1;
        const int m = (ax == 0 ? p.nx : ax == 1 ? p.ny : p.nz) - 1;  // unknowns per line
        const int stride = W + 2;
        std::vector<cd> t((size_t)ntypes * stride);
        std::vector<cd> z((size_t)m + 2);
        for (int ty = 0; ty < ntypes; ++ty) {
            double rot = 0.0;
            if (ax == 0)
                rot = p.omega * (h->args.y0 + ty * p.hy);
            else if (ax == 1)
                rot = -p.omega * (h->args.x0 + ty * p.hx);
            const cd Ap = u + q * rot, Am = u - q * rot;
            cd cs = 0.0;
            for (int it = 0; it < 100000; ++it) {
                const cd nc = Ap / (A0 - Am * cs);
                const bool done = std::abs(nc - cs) <= 1e-18 * std::abs(nc);
                cs = nc;
                if (done)
                    break;
            }
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
        const size_t n = t.size();
        if (p.precision == SSCN_C128) {
            if (hipMalloc(&h->tab[ax], n * sizeof(Cx<double>)) != hipSuccess)
                return fail(SSCN_ENOMEM, "hipMalloc of a pivot table failed");
            HIPCHECK(hipMemcpy(h->tab[ax], t.data(), n * sizeof(Cx<double>), hipMemcpyHostToDevice));
        } else {
            std::vector<Cx<float>> f(n);
            for (size_t e = 0; e < n; ++e)
                f[e] = Cx<float>{(float)t[e].real(), (float)t[e].imag()};
            if (hipMalloc(&h->tab[ax], n * sizeof(Cx<float>)) != hipSuccess)
                return fail(SSCN_ENOMEM, "hipMalloc of a pivot table failed");
            HIPCHECK(hipMemcpy(h->tab[ax], f.data(), n * sizeof(Cx<float>), hipMemcpyHostToDevice));
        }
    }
    return 0;
}

int red_blocks(int64_t n) { return (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (n + 255) / 256)); }

// ---------------------------------------------------------------------------
// Kernel dispatch.

template <class R> using V = typename Vec<R>::T;

// Dispatch on the window size W (a template parameter of the sweeps).
#define SSCN_W_SWITCH(Wv, CALL)                                                                             \
    switch (Wv) {                                                                                            \
    case 4: CALL(4); break;                                                                                  \
    case 6: CALL(6); break;                                                                                  \
    case 8: CALL(8); break;                                                                                  \
    case 10: CALL(10); break;                                                                                \
    case 12: CALL(12); break;                                                                                \
    case 16: CALL(16); break;                                                                                \
    case 20: CALL(20); break;                                                                                \
    case 24: CALL(24); break;                                                                                \
    default: CALL(32); break;                                                                                \
    }

unsigned round8(int64_t n) { return (unsigned)((n + 7) / 8 * 8); }

template <class R, int W, bool RT>
void go_x(const sscn_handle *h, const void *src, void *dst, int npart, hipStream_t st)
{
    const int nlines = h->p.ny * (h->p.dim == 3 ? h->p.nz : 1);
    const int blocks = (nlines + h->xL - 1) / h->xL;
    hipLaunchKernelGGL((k_xsweep<R, kSeg, W, RT>), dim3(blocks), dim3(256), h->xlds, st, (const V<R> *)src,
                       (V<R> *)dst, h->args, h->xL, h->partials, npart, (const Cx<R> *)h->tab[0]);
}

template <class R, bool RT>
void launch_x(const sscn_handle *h, const void *src, void *dst, int npart, hipStream_t st)
{
#define SSCN_CALL_X(Wc) go_x<R, Wc, RT>(h, src, dst, npart, st)
    SSCN_W_SWITCH(h->W[0], SSCN_CALL_X)
#undef SSCN_CALL_X
}

template <class R, int W, bool EMIT>
void go_y(const sscn_handle *h, const void *src, void *dst, hipStream_t st)
{
    const int *g = h->ygrid;
    hipLaunchKernelGGL((k_ysweep<R, kSeg, W, EMIT>), dim3(round8((int64_t)g[0] * g[1] * g[2])), dim3(64, 4), 0,
                       st, (const V<R> *)src, (V<R> *)dst, h->args, h->partials, g[0], g[1], g[2],
                       (const Cx<R> *)h->tab[1]);
}

template <class R, bool EMIT>
void launch_y(const sscn_handle *h, const void *src, void *dst, hipStream_t st)
{
#define SSCN_CALL_Y(Wc) go_y<R, Wc, EMIT>(h, src, dst, st)
    SSCN_W_SWITCH(h->W[1], SSCN_CALL_Y)
#undef SSCN_CALL_Y
}

template <class R, int W, bool EMIT>
void go_z(const sscn_handle *h, const void *src, void *dst, hipStream_t st)
{
    const int *g = h->zgrid;
    hipLaunchKernelGGL((k_zsweep<R, kSeg, W, EMIT>), dim3(round8((int64_t)g[0] * g[1])), dim3(64, 4), 0, st,
                       (const V<R> *)src, (V<R> *)dst, h->args, h->partials, g[0], g[1],
                       (const Cx<R> *)h->tab[2]);
}

template <class R, bool EMIT>
void launch_z(const sscn_handle *h, const void *src, void *dst, hipStream_t st)
{
#define SSCN_CALL_Z(Wc) go_z<R, Wc, EMIT>(h, src, dst, st)
    SSCN_W_SWITCH(h->W[2], SSCN_CALL_Z)
#undef SSCN_CALL_Z
}

template <class R>
void launch_rescale(sscn_handle *h, hipStream_t st)
{
    hipLaunchKernelGGL((k_rescale<R>), dim3(red_blocks(h->npts)), dim3(256), 0, st, (const V<R> *)h->psi,
                       (V<R> *)h->psi, h->npts, h->args.dV, h->partials, h->nemit);
}

template <class R>
void launch_norm(sscn_handle *h, hipStream_t st)
{
    hipLaunchKernelGGL((k_norm_partials<R>), dim3(kRedBlocks), dim3(256), 0, st, (const V<R> *)h->psi, h->npts,
                       h->partials);
}

#define SSCN_W_SWITCH_FUSED(R, Wv, CALL)                                                                   \
    switch (Wv) {                                                                                            \
    case 4: CALL(4); break;                                                                                  \
    case 6: CALL(6); break;                                                                                  \
    case 8: CALL(8); break;                                                                                  \
    case 10: CALL(10); break;                                                                                \
    case 12: CALL(12); break;                                                                                \
    case 16: CALL(16); break;                                                                                \
    default: CALL(20); break;                                                                                \
    }

template <class R, int W, bool RT>
void go_fused(const sscn_handle *h, int parity, const double *pin, double *pout, int use_pin, hipStream_t st)
{
    constexpr size_t lds = step2d_lds_bytes<R, kSeg, W, kTile, kTile>();
    hipLaunchKernelGGL((k_step2d<R, kSeg, W, kTile, kTile, RT>), dim3(h->ntiles), dim3(256), lds, st, h->d_inst,
                       h->d_work, h->d_nwork, parity, pin, pout, use_pin);
}

template <class R, bool RT>
void launch_fused(const sscn_handle *h, int parity, const double *pin, double *pout, int use_pin, hipStream_t st)
{
#define SSCN_CALL_F(Wc) go_fused<R, Wc, RT>(h, parity, pin, pout, use_pin, st)
    if constexpr (std::is_same<R, float>::value) {
        if (h->W[0] > 20) {
            if (h->W[0] <= 24)
                go_fused<R, 24, RT>(h, parity, pin, pout, use_pin, st);
            else
                go_fused<R, 32, RT>(h, parity, pin, pout, use_pin, st);
            return;
        }
    }
    SSCN_W_SWITCH_FUSED(R, h->W[0], SSCN_CALL_F)
#undef SSCN_CALL_F
}

template <class R, int W, bool RT>
hipError_t allow_fused_lds()
{
    constexpr size_t lds = step2d_lds_bytes<R, kSeg, W, kTile, kTile>();
    return hipFuncSetAttribute((const void *)k_step2d<R, kSeg, W, kTile, kTile, RT>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <class R>
hipError_t allow_fused_lds_all(int W)
{
    hipError_t e = hipSuccess;
#define SSCN_ALLOW(Wc)                                         \
    do {                                                       \
        e = allow_fused_lds<R, Wc, false>();                   \
        if (e == hipSuccess)                                   \
            e = allow_fused_lds<R, Wc, true>();                \
    } while (0)
    if constexpr (std::is_same<R, float>::value) {
        if (W > 20) {
            if (W <= 24)
                SSCN_ALLOW(24);
            else
                SSCN_ALLOW(32);
            return e;
        }
    }
    SSCN_W_SWITCH_FUSED(R, W, SSCN_ALLOW)
#undef SSCN_ALLOW
    return e;
}

// n fused steps (state ping-pongs between psi and work), ending with the
// state in psi, normalised in imaginary time.
template <class R>
void enqueue_fused(sscn_handle *h, int64_t n, hipStream_t st, hipEvent_t *ev = nullptr)
{
    const bool imag = h->p.mode == SSCN_IMAG;
    double *fp[2] = {h->partials, h->partials2};
    for (int64_t s = 0; s < n; ++s) {
        if (ev)
            (void)hipEventRecord(ev[4 * s], st);
        if (imag)
            launch_fused<R, false>(h, h->fparity, fp[h->pbuf], fp[h->pbuf ^ 1], h->pending ? 1 : 0, st);
        else
            launch_fused<R, true>(h, h->fparity, nullptr, nullptr, 0, st);
        if (ev)
            for (int t = 1; t < 4; ++t)
                (void)hipEventRecord(ev[4 * s + t], st);
        h->fparity ^= 1;
        if (imag) {
            h->pbuf ^= 1;
            h->pending = true;
        }
    }
    void *bufs[2] = {h->psi, h->work};
    const int nb = red_blocks(h->npts);
    if (imag && h->pending) {
        hipLaunchKernelGGL((k_rescale<R>), dim3(nb), dim3(256), 0, st, (const V<R> *)bufs[h->fparity],
                           (V<R> *)h->psi, h->npts, h->args.dV, fp[h->pbuf], h->ntiles);
        h->pending = false;
    } else if (h->fparity == 1) {
        hipLaunchKernelGGL((k_copy<R>), dim3(nb), dim3(256), 0, st, (const V<R> *)h->work, (V<R> *)h->psi,
                           h->npts);
    }
    h->fparity = 0;
}

int setup_fused(sscn_handle *h)
{
    if (!h->fused_ok)
        return 0;
    const sscn_params &p = h->p;
    Inst2D in{};
    in.nx = p.nx;
    in.ny = p.ny;
    in.tiles_x = (p.nx - 2) / kTile + 1;
    in.tiles_y = (p.ny - 2) / kTile + 1;
    in.poff = 0;
    in.active = 1;
    in.hx = p.hx;
    in.hy = p.hy;
    in.x0 = h->args.x0;
    in.y0 = h->args.y0;
    in.vx = h->args.vx;
    in.vy = h->args.vy;
    in.g = p.g;
    in.omega = p.omega;
    in.dt = p.dt;
    in.dV = h->args.dV;
    in.ax[0] = h->args.ax[0];
    in.ax[1] = h->args.ax[1];
    in.buf[0] = h->psi;
    in.buf[1] = h->work;
    in.tab[0] = h->tab[0];
    in.tab[1] = h->tab[1];
    std::vector<int2> wl(h->ntiles);
    for (int t = 0; t < h->ntiles; ++t)
        wl[t] = int2{0, t};
    if (!h->d_inst && (hipMalloc(&h->d_inst, sizeof(Inst2D)) != hipSuccess ||
                       hipMalloc(&h->d_nwork, sizeof(int)) != hipSuccess))
        return fail(SSCN_ENOMEM, "hipMalloc of the fused-step descriptors failed");
    if (h->d_work)
        (void)hipFree(h->d_work);
    if (h->partials2)
        (void)hipFree(h->partials2);
    h->d_work = nullptr;
    h->partials2 = nullptr;
    if (hipMalloc(&h->d_work, sizeof(int2) * wl.size()) != hipSuccess ||
        hipMalloc(&h->partials2, sizeof(double) * std::max(h->ntiles, kRedBlocks)) != hipSuccess)
        return fail(SSCN_ENOMEM, "hipMalloc of the fused-step work list failed");
    HIPCHECK(hipMemcpy(h->d_inst, &in, sizeof in, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(h->d_work, wl.data(), sizeof(int2) * wl.size(), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(h->d_nwork, &h->ntiles, sizeof(int), hipMemcpyHostToDevice));
    hipError_t e = p.precision == SSCN_C128 ? allow_fused_lds_all<double>(h->W[0])
                                            : allow_fused_lds_all<float>(h->W[0]);
    if (e != hipSuccess)
        return fail(SSCN_EHIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
    return 0;
}

// One SSCN step on stream st.  npart > 0: the partials hold the norm of the
// (unnormalised) state and the rescale is folded into H1.  ev (optional, 4
// events) is recorded before the x-, y-, z-sweeps and after the step.
template <class R>
void enqueue_one(sscn_handle *h, int npart, hipStream_t st, hipEvent_t *ev = nullptr)
{
    auto mark = [&](int t) {
        if (ev)
            (void)hipEventRecord(ev[t], st);
    };
    const bool imag = h->p.mode == SSCN_IMAG;
    void *A = h->psi, *B = h->work;
    mark(0);
    if (h->exact) {
        const int nb = red_blocks(h->npts);
        if (imag)
            hipLaunchKernelGGL((k_h1<R, false>), dim3(nb), dim3(256), 0, st, (const V<R> *)A, (V<R> *)A, h->args,
                               h->partials, npart);
        else
            hipLaunchKernelGGL((k_h1<R, true>), dim3(nb), dim3(256), 0, st, (const V<R> *)A, (V<R> *)A, h->args,
                               h->partials, 0);
        const sscn_params &p = h->p;
        const int nz = p.dim == 3 ? p.nz : 1;
        auto line = [&](int axis, void *s, void *d) {
            const int nl = axis == 0 ? p.ny * nz : axis == 1 ? p.nx * nz : p.nx * p.ny;
            hipLaunchKernelGGL((k_line_exact<R>), dim3((nl + 255) / 256), dim3(256), 0, st, (const V<R> *)s,
                               (V<R> *)d, h->args, axis, (Cx<R> *)h->ws);
        };
        line(0, A, B);
        mark(1);
        line(1, B, A);
        mark(2);
        if (p.dim == 3) {
            line(2, A, B);
            hipLaunchKernelGGL((k_copy<R>), dim3(nb), dim3(256), 0, st, (const V<R> *)B, (V<R> *)A, h->npts);
        }
        if (imag)
            launch_norm<R>(h, st);
        mark(3);
        return;
    }
    if (h->p.dim == 2) {
        if (imag) {
            launch_x<R, false>(h, A, B, npart, st);
            mark(1);
            launch_y<R, true>(h, B, A, st);
        } else {
            launch_x<R, true>(h, A, B, 0, st);
            mark(1);
            launch_y<R, false>(h, B, A, st);
        }
        mark(2);
    } else {
        if (imag) {
            launch_x<R, false>(h, A, A, npart, st);
            mark(1);
            launch_y<R, false>(h, A, B, st);
            mark(2);
            launch_z<R, true>(h, B, A, st);
        } else {
            launch_x<R, true>(h, A, A, 0, st);
            mark(1);
            launch_y<R, false>(h, A, B, st);
            mark(2);
            launch_z<R, false>(h, B, A, st);
        }
    }
    mark(3);
}

// n steps launched one by one, ending with a normalised state in imaginary
// time.
template <class R>
void enqueue_direct(sscn_handle *h, int64_t n, hipStream_t st)
{
    if (h->active_plan == SSCN_PLAN_FUSED) {
        enqueue_fused<R>(h, n, st);
        return;
    }
    const bool imag = h->p.mode == SSCN_IMAG;
    for (int64_t s = 0; s < n; ++s) {
        enqueue_one<R>(h, (imag && h->pending) ? h->nemit : 0, st);
        if (imag)
            h->pending = true;
    }
    if (imag && h->pending) {
        launch_rescale<R>(h, st);
        h->pending = false;
    }
}

int build_graph(sscn_handle *h)
{
    if (h->gexec)
        return 0;
    HIPCHECK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    const bool was = h->pending;
    h->pending = false;
    if (h->p.precision == SSCN_C128)
        enqueue_direct<double>(h, kGraphSteps, h->cap);
    else
        enqueue_direct<float>(h, kGraphSteps, h->cap);
    h->pending = was;
    hipError_t e = hipStreamEndCapture(h->cap, &h->graph);
    if (e != hipSuccess)
        return fail(SSCN_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(h->graph);
        h->graph = nullptr;
        h->gexec = nullptr;
        return fail(SSCN_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    return 0;
}

void drop_graph(sscn_handle *h)
{
    if (h->gexec)
        (void)hipGraphExecDestroy(h->gexec);
    if (h->graph)
        (void)hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
}

// Autotuner: on the first step of a handle whose plan is SSCN_PLAN_AUTO,
// time every plan available for the problem (separate sweeps; fused 2D
// step) over a few steps from a saved copy of the state, restore the state,
// and keep the fastest.  Results are cached per process, keyed by the shape,
// precision, mode and window.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int, int, int>, int> g_tune_cache;

template <class R>
float time_plan(sscn_handle *h, int plan, const void *saved, int nsteps)
{
    const size_t bytes = (size_t)h->npts * h->esize;
    h->active_plan = plan;
    enqueue_direct<R>(h, 2, h->stream);
    (void)hipMemcpyAsync(h->psi, saved, bytes, hipMemcpyDeviceToDevice, h->stream);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventRecord(e0, h->stream);
    enqueue_direct<R>(h, nsteps, h->stream);
    (void)hipEventRecord(e1, h->stream);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipMemcpyAsync(h->psi, saved, bytes, hipMemcpyDeviceToDevice, h->stream);
    return ms;
}

int autotune(sscn_handle *h)
{
    if (h->plan != SSCN_PLAN_AUTO)
        return 0;
    h->plan = SSCN_PLAN_SWEEPS;  // resolved below
    if (!h->fused_ok) {
        h->active_plan = SSCN_PLAN_SWEEPS;
        return 0;
    }
    const sscn_params &p = h->p;
    const auto key = std::make_tuple(p.dim, p.nx, p.ny, p.nz, p.precision, p.mode, h->W[0]);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            h->active_plan = h->plan = it->second;
            return 0;
        }
    }
    void *saved = nullptr;
    const size_t bytes = (size_t)h->npts * h->esize;
    if (hipMalloc(&saved, bytes) != hipSuccess)
        return fail(SSCN_ENOMEM, "hipMalloc of the autotune copy failed");
    HIPCHECK(hipMemcpyAsync(saved, h->psi, bytes, hipMemcpyDeviceToDevice, h->stream));
    const int plans[2] = {SSCN_PLAN_SWEEPS, SSCN_PLAN_FUSED};
    int best = SSCN_PLAN_SWEEPS;
    float best_ms = 0.f;
    for (int k = 0; k < 2; ++k) {
        const float ms = p.precision == SSCN_C128 ? time_plan<double>(h, plans[k], saved, 16)
                                                  : time_plan<float>(h, plans[k], saved, 16);
        h->tune_ms[plans[k]] = ms;
        if (k == 0 || ms < best_ms) {
            best = plans[k];
            best_ms = ms;
        }
    }
    HIPCHECK(hipStreamSynchronize(h->stream));
    (void)hipFree(saved);
    h->pending = false;
    h->fparity = 0;
    h->active_plan = h->plan = best;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache[key] = best;
    return 0;
}

int alloc_buffers(sscn_handle *h)
{
    const size_t bytes = (size_t)h->npts * h->esize;
    if (hipMalloc(&h->work, bytes) != hipSuccess)
        return fail(SSCN_ENOMEM, "hipMalloc of the work buffer failed");
    HIPCHECK(hipMemsetAsync(h->work, 0, bytes, h->stream));
    if (h->exact) {
        const sscn_params &p = h->p;
        const int nz = p.dim == 3 ? p.nz : 1;
        const int64_t lines_pts = std::max({(int64_t)p.ny * nz * p.nx, (int64_t)p.nx * nz * p.ny,
                                            (int64_t)p.nx * p.ny * nz});
        if (hipMalloc(&h->ws, (size_t)lines_pts * 2 * h->esize) != hipSuccess)
            return fail(SSCN_ENOMEM, "hipMalloc of the exact-path workspace failed");
    }
    return 0;
}

void free_buffers(sscn_handle *h)
{
    if (h->work)
        (void)hipFree(h->work);
    if (h->ws)
        (void)hipFree(h->ws);
    h->work = nullptr;
    h->ws = nullptr;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI.

extern "C" {

const char *sscn_last_error(void) { return g_err.c_str(); }

const char *sscn_strerror(int code)
{
    switch (code) {
    case SSCN_OK: return "ok";
    case SSCN_EINVAL: return "invalid argument";
    case SSCN_EOMEGA: return "omega >= min(gamma, nu)";
    case SSCN_EUNSTABLE: return "line systems not diagonally dominant";
    case SSCN_ENONFINITE: return "non-finite value in the state";
    case SSCN_EHIP: return "HIP runtime error";
    case SSCN_ENOMEM: return "device allocation failed";
    default: return "unknown error";
    }
}

int sscn_init(const sscn_params *params, void *psi_dev, void *hip_stream, sscn_handle **out)
{
    if (!params || !psi_dev || !out)
        return fail(SSCN_EINVAL, "null argument");
    *out = nullptr;
    int r = validate(*params);
    if (r)
        return r;
    sscn_handle *h = new sscn_handle();
    h->p = *params;
    if (h->p.dim == 2)
        h->p.nz = 1;
    h->psi = psi_dev;
    h->stream = (hipStream_t)hip_stream;
    r = setup(h);
    if (r) {
        delete h;
        return r;
    }
    auto bail = [&](int code) {
        sscn_destroy(h);
        return code;
    };
    if (hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(SSCN_EHIP, "hipStreamCreateWithFlags failed"));
    r = alloc_buffers(h);
    if (r)
        return bail(r);
    r = build_tables(h);
    if (r)
        return bail(r);
    const size_t npart = std::max({(size_t)h->nemit, (size_t)kRedBlocks, (size_t)h->ntiles});
    if (hipMalloc(&h->partials, npart * sizeof(double)) != hipSuccess ||
        hipMalloc(&h->obs_part, (size_t)kRedBlocks * 14 * sizeof(double)) != hipSuccess ||
        hipMalloc(&h->obs_buf, 64 * sizeof(double)) != hipSuccess)
        return bail(fail(SSCN_ENOMEM, "hipMalloc of reduction buffers failed"));
    if (hipMemsetAsync(h->partials, 0, npart * sizeof(double), h->stream) != hipSuccess)
        return bail(fail(SSCN_EHIP, "hipMemsetAsync failed"));
    r = setup_fused(h);
    if (r)
        return bail(r);
    if (const char *env = std::getenv("SSCN_PLAN")) {
        if (!std::strcmp(env, "sweeps"))
            h->plan = SSCN_PLAN_SWEEPS;
        else if (!std::strcmp(env, "fused") && h->fused_ok)
            h->plan = SSCN_PLAN_FUSED;
    }
    h->active_plan = h->plan == SSCN_PLAN_FUSED ? SSCN_PLAN_FUSED : SSCN_PLAN_SWEEPS;
    *out = h;
    return 0;
}

void sscn_destroy(sscn_handle *h)
{
    if (!h)
        return;
    (void)hipStreamSynchronize(h->stream);
    drop_graph(h);
    free_buffers(h);
    for (int ax = 0; ax < 3; ++ax)
        if (h->tab[ax])
            (void)hipFree(h->tab[ax]);
    if (h->d_inst)
        (void)hipFree(h->d_inst);
    if (h->d_work)
        (void)hipFree(h->d_work);
    if (h->d_nwork)
        (void)hipFree(h->d_nwork);
    if (h->partials2)
        (void)hipFree(h->partials2);
    if (h->partials)
        (void)hipFree(h->partials);
    if (h->obs_part)
        (void)hipFree(h->obs_part);
    if (h->obs_buf)
        (void)hipFree(h->obs_buf);
    if (h->phase)
        (void)hipFree(h->phase);
    if (h->cap)
        (void)hipStreamDestroy(h->cap);
    delete h;
}

int sscn_init_state(sscn_handle *h, int kind, const double *phase_host, double d_xy, double d_z)
{
    if (!h || (kind != 0 && kind != 1) || !(d_xy > 0))
        return fail(SSCN_EINVAL, "bad init_state arguments");
    const sscn_params &p = h->p;
    if (p.dim == 3 && !(d_z > 0))
        d_z = 1.0 / std::sqrt(p.lambda);
    const double *ph = nullptr;
    if (phase_host) {
        const size_t bytes = (size_t)p.nx * p.ny * sizeof(double);
        if (!h->phase && hipMalloc(&h->phase, bytes) != hipSuccess)
            return fail(SSCN_ENOMEM, "hipMalloc of the phase buffer failed");
        HIPCHECK(hipMemcpyAsync(h->phase, phase_host, bytes, hipMemcpyHostToDevice, h->stream));
        ph = h->phase;
    }
    const int nb = red_blocks(h->npts);
    if (p.precision == SSCN_C128) {
        hipLaunchKernelGGL((k_init<double>), dim3(nb), dim3(256), 0, h->stream, (V<double> *)h->psi, h->args, kind,
                           ph, d_xy, d_z);
        launch_norm<double>(h, h->stream);
    } else {
        hipLaunchKernelGGL((k_init<float>), dim3(nb), dim3(256), 0, h->stream, (V<float> *)h->psi, h->args, kind,
                           ph, d_xy, d_z);
        launch_norm<float>(h, h->stream);
    }
    // normalise: the norm partials use kRedBlocks blocks
    const int saved = h->nemit;
    h->nemit = kRedBlocks;
    if (p.precision == SSCN_C128)
        launch_rescale<double>(h, h->stream);
    else
        launch_rescale<float>(h, h->stream);
    h->nemit = saved;
    h->pending = false;
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(h->stream));
    return 0;
}

int sscn_step(sscn_handle *h, int64_t nsteps)
{
    if (!h || nsteps < 0)
        return fail(SSCN_EINVAL, "bad step arguments");
    if (nsteps == 0)
        return 0;
    int r0 = autotune(h);
    if (r0)
        return r0;
    int64_t rem = nsteps;
    if (nsteps >= kGraphSteps && !h->pending) {
        int r = build_graph(h);
        if (r)
            return r;
        while (rem >= kGraphSteps) {
            HIPCHECK(hipGraphLaunch(h->gexec, h->stream));
            rem -= kGraphSteps;
        }
    }
    if (h->p.precision == SSCN_C128)
        enqueue_direct<double>(h, rem, h->stream);
    else
        enqueue_direct<float>(h, rem, h->stream);
    HIPCHECK(hipGetLastError());
    h->steps += nsteps;
    return 0;
}

int sscn_observables(sscn_handle *h, sscn_obs *out)
{
    if (!h || !out)
        return fail(SSCN_EINVAL, "null argument");
    const int nb = red_blocks(h->npts);
    if (h->p.precision == SSCN_C128)
        hipLaunchKernelGGL((k_observables<double>), dim3(nb), dim3(256), 0, h->stream, (const V<double> *)h->psi,
                           h->args, h->obs_part);
    else
        hipLaunchKernelGGL((k_observables<float>), dim3(nb), dim3(256), 0, h->stream, (const V<float> *)h->psi,
                           h->args, h->obs_part);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, h->stream, h->obs_part, nb, 14, 1u << 13, h->obs_buf);
    double s[14];
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(s, h->obs_buf, sizeof s, hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    const double dV = h->args.dV;
    for (int t = 0; t < 13; ++t)
        s[t] *= dV;
    std::memset(out, 0, sizeof *out);
    std::memcpy(out->sums, s, sizeof s);
    out->norm = s[0];
    out->mu = (s[2] + s[3] + s[4] + s[5]) / s[1];
    out->energy = (s[2] + s[3] + 0.5 * s[4] + s[5]) / s[1];
    out->mu_full = (s[6] + s[7] + s[8] + s[9]) / s[0];
    out->energy_full = (s[6] + s[7] + 0.5 * s[8] + s[9]) / s[0];
    out->rms_x = std::sqrt(s[10] / s[0]);
    out->rms_y = std::sqrt(s[11] / s[0]);
    out->rms_z = std::sqrt(s[12] / s[0]);
    out->rms_r = std::sqrt((s[10] + s[11] + s[12]) / s[0]);
    out->max_density = s[13];
    out->step = h->steps;
    for (int t = 0; t < 14; ++t)
        if (!std::isfinite(s[t]))
            return fail(SSCN_ENONFINITE, "non-finite reduction in the observables");
    return 0;
}

int sscn_set_state(sscn_handle *h, const void *host_psi)
{
    if (!h || !host_psi)
        return fail(SSCN_EINVAL, "null argument");
    HIPCHECK(hipMemcpyAsync(h->psi, host_psi, (size_t)h->npts * h->esize, hipMemcpyHostToDevice, h->stream));
    int r = sscn_set_state_device(h);
    if (r)
        return r;
    HIPCHECK(hipStreamSynchronize(h->stream));
    return 0;
}

int sscn_set_state_device(sscn_handle *h)
{
    if (!h)
        return fail(SSCN_EINVAL, "null argument");
    const int nb = red_blocks(h->npts);
    if (h->p.precision == SSCN_C128)
        hipLaunchKernelGGL((k_zero_walls<double>), dim3(nb), dim3(256), 0, h->stream, (V<double> *)h->psi, h->args);
    else
        hipLaunchKernelGGL((k_zero_walls<float>), dim3(nb), dim3(256), 0, h->stream, (V<float> *)h->psi, h->args);
    HIPCHECK(hipGetLastError());
    h->pending = false;
    return 0;
}

int sscn_get_state(sscn_handle *h, void *host_psi)
{
    if (!h || !host_psi)
        return fail(SSCN_EINVAL, "null argument");
    HIPCHECK(hipMemcpyAsync(host_psi, h->psi, (size_t)h->npts * h->esize, hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    return 0;
}

int sscn_set_mode(sscn_handle *h, int mode, int precision, void *new_psi_dev)
{
    if (!h)
        return fail(SSCN_EINVAL, "null argument");
    sscn_params np = h->p;
    np.mode = mode;
    np.precision = precision;
    int r = validate(np);
    if (r)
        return r;
    const bool conv = precision != h->p.precision;
    if (conv && !new_psi_dev)
        return fail(SSCN_EINVAL, "a precision change needs the new state buffer");
    sscn_handle tmp;
    tmp.p = np;
    r = setup(&tmp);
    if (r)
        return r;
    HIPCHECK(hipStreamSynchronize(h->stream));
    drop_graph(h);
    if (conv) {
        const int nb = red_blocks(h->npts);
        if (h->p.precision == SSCN_C64)
            hipLaunchKernelGGL((k_convert<float, double>), dim3(nb), dim3(256), 0, h->stream,
                               (const V<float> *)h->psi, (V<double> *)new_psi_dev, h->npts);
        else
            hipLaunchKernelGGL((k_convert<double, float>), dim3(nb), dim3(256), 0, h->stream,
                               (const V<double> *)h->psi, (V<float> *)new_psi_dev, h->npts);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipStreamSynchronize(h->stream));
        h->psi = new_psi_dev;
    }
    free_buffers(h);
    const int64_t steps = h->steps;
    h->p = np;
    r = setup(h);
    if (r)
        return r;
    r = alloc_buffers(h);
    if (r)
        return r;
    r = build_tables(h);
    if (r)
        return r;
    // the partials buffer must hold the new emit count
    (void)hipFree(h->partials);
    const size_t npart = std::max({(size_t)h->nemit, (size_t)kRedBlocks, (size_t)h->ntiles});
    if (hipMalloc(&h->partials, npart * sizeof(double)) != hipSuccess)
        return fail(SSCN_ENOMEM, "hipMalloc of the partials failed");
    r = setup_fused(h);
    if (r)
        return r;
    if (h->plan == SSCN_PLAN_FUSED && !h->fused_ok)
        h->plan = SSCN_PLAN_AUTO;
    h->active_plan = h->plan == SSCN_PLAN_FUSED ? SSCN_PLAN_FUSED : SSCN_PLAN_SWEEPS;
    h->fparity = 0;
    h->steps = steps;
    h->pending = false;
    HIPCHECK(hipStreamSynchronize(h->stream));
    return 0;
}

int sscn_vortex_count(sscn_handle *h, double density_frac, int box, int *count)
{
    if (!h || !count || box < 0 || !(density_frac >= 0))
        return fail(SSCN_EINVAL, "bad vortex_count arguments");
    const sscn_params &p = h->p;
    const int k0 = p.dim == 3 ? p.nz / 2 : 0;
    const int64_t plane = (int64_t)p.nx * p.ny;
    const int nb = red_blocks(plane);
    if (p.precision == SSCN_C128) {
        hipLaunchKernelGGL((k_plane_max<double>), dim3(nb), dim3(256), 0, h->stream, (const V<double> *)h->psi,
                           h->args, k0, h->obs_part);
    } else {
        hipLaunchKernelGGL((k_plane_max<float>), dim3(nb), dim3(256), 0, h->stream, (const V<float> *)h->psi,
                           h->args, k0, h->obs_part);
    }
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, h->stream, h->obs_part, nb, 1, 1u, h->obs_buf + 16);
    const int nbv = red_blocks((int64_t)(p.nx - 1) * (p.ny - 1));
    if (p.precision == SSCN_C128) {
        hipLaunchKernelGGL((k_vortex<double>), dim3(nbv), dim3(256), 0, h->stream, (const V<double> *)h->psi,
                           h->args, k0, density_frac, box, h->obs_buf + 16, h->obs_part);
    } else {
        hipLaunchKernelGGL((k_vortex<float>), dim3(nbv), dim3(256), 0, h->stream, (const V<float> *)h->psi,
                           h->args, k0, density_frac, box, h->obs_buf + 16, h->obs_part);
    }
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, h->stream, h->obs_part, nbv, 1, 0u, h->obs_buf + 17);
    double c = 0.0;
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(&c, h->obs_buf + 17, sizeof c, hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    *count = (int)c;
    return 0;
}

int sscn_profile_step(sscn_handle *h, int64_t nsteps, double *ms_out)
{
    if (!h || !ms_out || nsteps < 1 || nsteps > 100000)
        return fail(SSCN_EINVAL, "bad profile_step arguments");
    int rt = autotune(h);
    if (rt)
        return rt;
    const bool imag = h->p.mode == SSCN_IMAG;
    std::vector<hipEvent_t> ev((size_t)nsteps * 4, nullptr);
    int rc = 0;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            rc = fail(SSCN_EHIP, "hipEventCreate failed");
            break;
        }
    if (!rc && h->active_plan == SSCN_PLAN_FUSED) {
        if (h->p.precision == SSCN_C128)
            enqueue_fused<double>(h, nsteps, h->stream, ev.data());
        else
            enqueue_fused<float>(h, nsteps, h->stream, ev.data());
        h->steps += nsteps;
        if (hipStreamSynchronize(h->stream) != hipSuccess)
            rc = fail(SSCN_EHIP, "hipStreamSynchronize failed");
    } else if (!rc) {
        for (int64_t s = 0; s < nsteps; ++s) {
            const int npart = (imag && h->pending) ? h->nemit : 0;
            if (h->p.precision == SSCN_C128)
                enqueue_one<double>(h, npart, h->stream, &ev[(size_t)s * 4]);
            else
                enqueue_one<float>(h, npart, h->stream, &ev[(size_t)s * 4]);
            if (imag)
                h->pending = true;
        }
        if (imag) {
            if (h->p.precision == SSCN_C128)
                launch_rescale<double>(h, h->stream);
            else
                launch_rescale<float>(h, h->stream);
            h->pending = false;
        }
        h->steps += nsteps;
        if (hipStreamSynchronize(h->stream) != hipSuccess)
            rc = fail(SSCN_EHIP, "hipStreamSynchronize failed");
    }
    if (!rc) {
        double acc[4] = {0, 0, 0, 0};
        for (int64_t s = 0; s < nsteps && !rc; ++s) {
            hipEvent_t *e = &ev[(size_t)s * 4];
            float t01 = 0, t12 = 0, t23 = 0, t03 = 0;
            if (hipEventElapsedTime(&t01, e[0], e[1]) != hipSuccess ||
                hipEventElapsedTime(&t12, e[1], e[2]) != hipSuccess ||
                hipEventElapsedTime(&t23, e[2], e[3]) != hipSuccess ||
                hipEventElapsedTime(&t03, e[0], e[3]) != hipSuccess)
                rc = fail(SSCN_EHIP, "hipEventElapsedTime failed");
            acc[0] += t01;
            acc[1] += t12;
            acc[2] += t23;
            acc[3] += t03;
        }
        for (int t = 0; t < 4; ++t)
            ms_out[t] = acc[t] / (double)nsteps;
        if (h->p.dim == 2 && !h->exact)
            ms_out[2] = 0.0;
        if (h->active_plan == SSCN_PLAN_FUSED)
            ms_out[1] = ms_out[2] = 0.0;
    }
    for (auto &e : ev)
        if (e)
            (void)hipEventDestroy(e);
    return rc;
}

int sscn_set_plan(sscn_handle *h, int plan)
{
    if (!h || plan < SSCN_PLAN_AUTO || plan > SSCN_PLAN_FUSED)
        return fail(SSCN_EINVAL, "bad plan");
    if (plan == SSCN_PLAN_FUSED && !h->fused_ok)
        return fail(SSCN_EINVAL, "the fused 2D step is not available for this problem");
    HIPCHECK(hipStreamSynchronize(h->stream));
    drop_graph(h);
    h->plan = plan;
    h->active_plan = plan == SSCN_PLAN_FUSED ? SSCN_PLAN_FUSED : SSCN_PLAN_SWEEPS;
    return 0;
}

int sscn_solver_info(sscn_handle *h, int *window_xyz, int *segment_xyz, int *plan)
{
    if (!h)
        return fail(SSCN_EINVAL, "null argument");
    if (plan)
        *plan = h->plan == SSCN_PLAN_AUTO ? SSCN_PLAN_AUTO : h->active_plan;
    for (int a = 0; a < 3; ++a) {
        if (window_xyz)
            window_xyz[a] = h->exact ? 0 : h->W[a];
        if (segment_xyz)
            segment_xyz[a] = h->exact ? 0 : kSeg;
    }
    return 0;
}

}  // extern "C"
