// Host side of the SSCN C ABI (include/sscn.h): parameter validation, the
// per-axis Crank-Nicolson coefficients, window selection, kernel dispatch,
// step sequencing with HIP graphs, observables and vortex counting.
#include "sscn_host.hpp"
#include "sscn_setup.hpp"

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

// Vortex count of the convergence criterion (sscn_converge, sscn_batch_run):
// density fraction and box of sscn_vortex_count.
constexpr double kConvDensityFrac = 0.05;
constexpr int kConvBox = 3;

#define HIPCHECK(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(SSCN_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

// Events that time kernels between them: without the system-scope fence of
// a default event, whose cache write-back and invalidation at every record
// would slow the kernel that follows and add to the measured durations.  The
// host reads them only after synchronising with the stream or the event.
hipError_t timing_event(hipEvent_t *e)
{
    return hipEventCreateWithFlags(e, hipEventDisableSystemFence);
}

// Output rows and columns of the fused step's tile shape t
// (FusedLaunch::tile).
int fused_tile_rows(int t) { return kFusedTileR[t]; }
int fused_tile_cols(int t) { return kFusedTileC[t]; }

// The most tiles of any of the fused step's shapes (partial buffers).
size_t max_fused_tiles(const sscn_handle *h)
{
    size_t m = 0;
    for (int t = 0; t < kFusedTiles; ++t)
        m = std::max(m, (size_t)h->ntiles_t[t]);
    return m;
}

int64_t npoints(const sscn_params &p)
{
    return (int64_t)p.nx * p.ny * (p.dim == 3 ? p.nz : 1);
}

// Lines per block of the x-sweep and the LDS it stages: L padded lines
// (x_row_len entries), the pivot-table rows and the wall terms.
void set_x_lines(sscn_handle *h, int L)
{
    const size_t LS = (size_t)x_row_len(h->p.nx, kSegX, h->W[0]);
    h->xL = L;
    h->xlds = (L * LS + (size_t)L * (h->W[0] + 2) + L) * h->esize;
}

int setup(sscn_handle *h)
{
    const sscn_params &p = h->p;
    StepArgs &a = h->args;
    fill_args(p, a);
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
    const int nseg = (p.nx - 2) / kSegX + 1;
    int L = std::max(1, std::min({256 / nseg, 256 * kXLoad / p.nx, 512 / (h->W[0] + 2)}));
    while (L & (L - 1))  // a power of two: 256 / L threads stage each line
        L &= L - 1;
    h->xLmax = L;
    set_x_lines(h, L);
    if (nseg > 256 || p.nx > 256 * kXLoad || h->xlds > kXLdsCap)
        h->exact = true;  // lines too long to stage; whole-line path
    // strided sweeps: logical grids and the partials written by the last one
    h->ygrid[0] = (p.nx + kYLines - 1) / kYLines;
    h->ygrid[1] = ((p.ny - 2) / kSeg + 1 + kSegBlock - 1) / kSegBlock;
    h->ygrid[2] = p.dim == 3 ? p.nz : 1;
    h->zgrid[0] = (int)(((int64_t)p.nx * p.ny + kYLines - 1) / kYLines);
    h->zgrid[1] = p.dim == 3 ? ((p.nz - 2) / kSeg + 1 + kSegBlock - 1) / kSegBlock : 1;
    if (p.dim == 2)
        h->nemit = h->ygrid[0] * h->ygrid[1];
    else
        h->nemit = h->zgrid[0] * h->zgrid[1];
    if (h->exact) {
        h->W[0] = h->W[1] = h->W[2] = 0;
        h->nemit = kRedBlocks;
    }
    int any = -1;
    for (int t = 0; t < kFusedTiles; ++t) {
        const int tr = fused_tile_rows(t), tc = fused_tile_cols(t);
        const size_t flds = step2d_lds_elems(kSeg, h->W[0], tr, tc) * h->esize;
        h->fused_ok_t[t] = p.dim == 2 && !h->exact && h->W[0] > 0 &&
                           h->W[0] <= (p.precision == SSCN_C128 ? 20 : 32) && flds <= 150 * 1024 &&
                           (h->tile_force < 0 || h->tile_force == t);
        h->ntiles_t[t] = ((p.nx - 2) / tc + 1) * ((p.ny - 2) / tr + 1);
        if (h->fused_ok_t[t] && any < 0)
            any = t;
    }
    if (!h->fused_ok_t[h->tile] && any >= 0)
        h->tile = any;
    h->fused_ok = any >= 0;
    h->ntiles = h->ntiles_t[h->tile];
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
        std::vector<std::complex<double>> t;
        pivot_table(p, h->args, ax, W, t);
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
// Kernel dispatch (the sweep and fused-step launchers are in
// sscn_kernels.hip).

// folded: the renormalisation that ends a run of steps (k_rescale); false
// for a given state of arbitrary norm.
template <class R>
void launch_rescale(sscn_handle *h, hipStream_t st, bool folded = true)
{
    hipLaunchKernelGGL((k_rescale<R>), dim3(red_blocks(h->npts)), dim3(256), 0, st, (const V<R> *)h->psi,
                       (V<R> *)h->psi, h->npts, h->args.dV, h->partials, h->nemit, folded ? 1 : 0);
}

template <class R>
void launch_norm(sscn_handle *h, hipStream_t st)
{
    hipLaunchKernelGGL((k_norm_partials<R>), dim3(kRedBlocks), dim3(256), 0, st, (const V<R> *)h->psi, h->npts,
                       h->partials);
}



// n fused steps (state ping-pongs between psi and work), ending with the
// state in psi, normalised in imaginary time.
template <class R>
void enqueue_fused(sscn_handle *h, int64_t n, hipStream_t st, hipEvent_t *ev = nullptr)
{
    const bool imag = h->p.mode == SSCN_IMAG;
    double *fp[2] = {h->partials, h->partials2};
    const FusedLaunch f{h->d_inst, h->d_work, h->d_nwork, h->ntiles, h->W[0], &h->inst_host, h->tile};
    for (int64_t s = 0; s < n; ++s) {
        if (ev)
            (void)hipEventRecord(ev[4 * s], st);
        if (imag)
            launch_fused<R, false>(f, h->fparity, fp[h->pbuf], fp[h->pbuf ^ 1], h->pending ? 1 : 0, st);
        else
            launch_fused<R, true>(f, h->fparity, nullptr, nullptr, 0, st);
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
                           (V<R> *)h->psi, h->npts, h->args.dV, fp[h->pbuf], h->ntiles, 1);
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
    in.tiles_x = (p.nx - 2) / fused_tile_cols(h->tile) + 1;
    in.tiles_y = (p.ny - 2) / fused_tile_rows(h->tile) + 1;
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
        hipMalloc(&h->partials2, sizeof(double) * std::max(max_fused_tiles(h), (size_t)kRedBlocks)) != hipSuccess)
        return fail(SSCN_ENOMEM, "hipMalloc of the fused-step work list failed");
    h->inst_host = in;
    HIPCHECK(hipMemcpy(h->d_inst, &in, sizeof in, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(h->d_work, wl.data(), sizeof(int2) * wl.size(), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(h->d_nwork, &h->ntiles, sizeof(int), hipMemcpyHostToDevice));
    hipError_t e = p.precision == SSCN_C128 ? allow_fused_lds_all<double>(h->W[0])
                                            : allow_fused_lds_all<float>(h->W[0]);
    if (e != hipSuccess)
        return fail(SSCN_EHIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
    return 0;
}

void drop_graph(sscn_handle *h);

// Put the fused step's tile shape t in force: the tile count, the
// descriptor and work list on the device (setup_fused); the captured step
// graphs carry the old grid and are dropped.
int set_fused_tile(sscn_handle *h, int t)
{
    if (!h->fused_ok_t[t])
        return fail(SSCN_EINVAL, "this fused tile shape is not available for the problem");
    if (h->tile == t && h->d_work)
        return 0;
    drop_graph(h);
    h->tile = t;
    h->ntiles = h->ntiles_t[t];
    return setup_fused(h);
}

// Dynamic-LDS limit of the handle's x-sweep kernels (lines longer than the
// default 64 KiB allow).
int allow_x_lds(sscn_handle *h)
{
    if (h->exact)
        return 0;
    const hipError_t e = h->p.precision == SSCN_C128 ? allow_x_lds_all<double>(h->W[0])
                                                     : allow_x_lds_all<float>(h->W[0]);
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

// Find, or capture and instantiate, the graph of k steps in `cache` (at most
// kGraphCache entries: the oldest is destroyed first).  enqueue(k, stream)
// records the k steps; `capture` is the handle's capture stream.
template <class Enq>
int cached_graph(std::vector<std::pair<int64_t, hipGraphExec_t>> &cache, hipStream_t capture, int64_t k, Enq enqueue,
                 hipGraphExec_t *out)
{
    for (const auto &e : cache)
        if (e.first == k) {
            *out = e.second;
            return 0;
        }
    HIPCHECK(hipStreamBeginCapture(capture, hipStreamCaptureModeThreadLocal));
    enqueue(k, capture);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(capture, &g);
    if (e != hipSuccess)
        return fail(SSCN_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess)
        return fail(SSCN_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    if (cache.size() >= kGraphCache) {
        (void)hipGraphExecDestroy(cache.front().second);
        cache.erase(cache.begin());
    }
    cache.emplace_back(k, x);
    *out = x;
    return 0;
}

void drop_graphs(std::vector<std::pair<int64_t, hipGraphExec_t>> &cache)
{
    for (auto &e : cache)
        (void)hipGraphExecDestroy(e.second);
    cache.clear();
}

// The graph of k steps of a single instance.  A stepping call leaves the
// state normalised with no pending rescale, so every graph is captured from
// that state; the host-side step bookkeeping is restored after the capture.
int step_graph(sscn_handle *h, int64_t k, hipGraphExec_t *out)
{
    auto enq = [h](int64_t n, hipStream_t st) {
        const bool pending = h->pending;
        const int fparity = h->fparity, pbuf = h->pbuf;
        h->pending = false;
        if (h->p.precision == SSCN_C128)
            enqueue_direct<double>(h, n, st);
        else
            enqueue_direct<float>(h, n, st);
        h->pending = pending;
        h->fparity = fparity;
        h->pbuf = pbuf;
    };
    return cached_graph(h->graphs, h->cap, k, enq, out);
}

void drop_graph(sscn_handle *h) { drop_graphs(h->graphs); }

// The graphs a call of nsteps steps replays: nsteps = q G + r with G =
// min(nsteps, kGraphSteps): q launches of the G-step graph, then the r-step
// graph (r >= 2) or one direct step (r = 1).  launch = false only captures
// them.
int run_step_graphs(sscn_handle *h, int64_t nsteps, bool launch)
{
    const int64_t G = std::min<int64_t>(nsteps, kGraphSteps);
    const int64_t q = nsteps / G, r = nsteps % G;
    hipGraphExec_t x = nullptr;
    int rc = step_graph(h, G, &x);
    if (rc)
        return rc;
    for (int64_t t = 0; launch && t < q; ++t)
        HIPCHECK(hipGraphLaunch(x, h->stream));
    if (r >= 2) {
        rc = step_graph(h, r, &x);
        if (rc)
            return rc;
        if (launch)
            HIPCHECK(hipGraphLaunch(x, h->stream));
    } else if (r == 1 && launch) {
        if (h->p.precision == SSCN_C128)
            enqueue_direct<double>(h, 1, h->stream);
        else
            enqueue_direct<float>(h, 1, h->stream);
    }
    return 0;
}

// Autotuner: on the first step of a handle whose plan is SSCN_PLAN_AUTO,
// time every candidate configuration over a few steps from a saved copy of
// the state, restore the state, and keep the fastest.  Candidates: the three
// sweep kernels with the x-sweep staging L, L/2 or L/4 lines per block (L
// the largest that fits), and the fused 2D step where it is admissible.  The
// window W is not a candidate: the accuracy bound fixes it.  Results are
// cached per process, keyed by architecture, shape, precision, mode and
// window; with SSCN_TUNE_CACHE=<file> the cache is also read from and
// written to that JSON file.
struct TuneChoice {
    int plan = SSCN_PLAN_SWEEPS;
    int xl = 0;
    int tile = 0;  // the fused step's tile shape (plan SSCN_PLAN_FUSED)
    float ms = 0.f;
};
std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune_cache;
std::string g_tune_path;  // the SSCN_TUNE_CACHE file merged into the cache last

std::string device_arch()
{
    static std::string arch;
    if (arch.empty()) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            arch = prop.gcnArchName;
            const size_t c = arch.find(':');
            if (c != std::string::npos)
                arch.resize(c);
        }
        if (arch.empty())
            arch = "unknown";
    }
    return arch;
}

std::string tune_key(const sscn_handle *h)
{
    const sscn_params &p = h->p;
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s|%dd|%dx%dx%d|%s|%s|W%d", device_arch().c_str(), p.dim, p.nx, p.ny,
                  p.dim == 3 ? p.nz : 1, p.precision == SSCN_C128 ? "c128" : "c64",
                  p.mode == SSCN_IMAG ? "imag" : "real", h->W[0]);
    return buf;
}

// Entries are lines of the form
//   "<key>": {"plan": 1|2, "x_lines": L, "tile": 0|1, "ms_per_step": t},
// ("tile" may be absent: 0).
void tune_cache_load()
{
    const char *path = std::getenv("SSCN_TUNE_CACHE");
    if (!path || !*path || g_tune_path == path)
        return;
    g_tune_path = path;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        const char *q0 = std::strchr(line, '"');
        const char *q1 = q0 ? std::strchr(q0 + 1, '"') : nullptr;
        const char *pl = std::strstr(line, "\"plan\":");
        const char *xl = std::strstr(line, "\"x_lines\":");
        const char *ms = std::strstr(line, "\"ms_per_step\":");
        const char *tl = std::strstr(line, "\"tile\":");
        if (!q1 || !pl || !xl)
            continue;
        TuneChoice c;
        c.plan = std::atoi(pl + 7);
        c.xl = std::atoi(xl + 10);
        c.tile = tl ? std::atoi(tl + 7) : 0;
        c.ms = ms ? (float)std::atof(ms + 14) : 0.f;
        if ((c.plan == SSCN_PLAN_SWEEPS || c.plan == SSCN_PLAN_FUSED) && c.xl >= 1 && c.tile >= 0 && c.tile < kFusedTiles)
            g_tune_cache[std::string(q0 + 1, q1)] = c;
    }
    std::fclose(f);
}

void tune_cache_save()
{
    const char *path = std::getenv("SSCN_TUNE_CACHE");
    if (!path || !*path)
        return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f)
        return;
    std::fprintf(f, "{\n");
    size_t k = 0;
    for (const auto &e : g_tune_cache)
        std::fprintf(f, "  \"%s\": {\"plan\": %d, \"x_lines\": %d, \"tile\": %d, \"ms_per_step\": %.6f}%s\n",
                     e.first.c_str(), e.second.plan, e.second.xl, e.second.tile, e.second.ms,
                     ++k < g_tune_cache.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

template <class R>
float time_plan(sscn_handle *h, int plan, const void *saved, int nsteps)
{
    const size_t bytes = (size_t)h->npts * h->esize;
    h->active_plan = plan;
    h->pending = false;
    enqueue_direct<R>(h, 2, h->stream);
    (void)hipMemcpyAsync(h->psi, saved, bytes, hipMemcpyDeviceToDevice, h->stream);
    h->pending = false;
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
    h->active_plan = SSCN_PLAN_SWEEPS;
    if (h->exact)
        return 0;
    const std::string key = tune_key(h);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        tune_cache_load();
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end() && it->second.xl <= h->xLmax && !(it->second.xl & (it->second.xl - 1)) &&
            (it->second.plan == SSCN_PLAN_SWEEPS || h->fused_ok_t[it->second.tile])) {
            set_x_lines(h, it->second.xl);
            if (it->second.plan == SSCN_PLAN_FUSED) {
                const int r = set_fused_tile(h, it->second.tile);
                if (r)
                    return r;
            }
            h->active_plan = h->plan = it->second.plan;
            return 0;
        }
    }
    std::vector<TuneChoice> cand;
    for (int d : {1, 2, 4}) {
        const int xl = std::max(1, h->xLmax / d);
        if (cand.empty() || cand.back().xl != xl) {
            TuneChoice c;
            c.plan = SSCN_PLAN_SWEEPS;
            c.xl = xl;
            cand.push_back(c);
        }
    }
    for (int t = 0; t < kFusedTiles; ++t)
        if (h->fused_ok_t[t]) {
            TuneChoice c;
            c.plan = SSCN_PLAN_FUSED;
            c.xl = h->xLmax;
            c.tile = t;
            cand.push_back(c);
        }
    void *saved = nullptr;
    const size_t bytes = (size_t)h->npts * h->esize;
    if (hipMalloc(&saved, bytes) != hipSuccess)
        return fail(SSCN_ENOMEM, "hipMalloc of the autotune copy failed");
    HIPCHECK(hipMemcpyAsync(saved, h->psi, bytes, hipMemcpyDeviceToDevice, h->stream));
    const int nsteps = 16;
    size_t best = 0;
    for (size_t k = 0; k < cand.size(); ++k) {
        set_x_lines(h, cand[k].xl);
        if (cand[k].plan == SSCN_PLAN_FUSED) {
            const int r = set_fused_tile(h, cand[k].tile);
            if (r) {
                (void)hipFree(saved);
                return r;
            }
        }
        const float ms = h->p.precision == SSCN_C128 ? time_plan<double>(h, cand[k].plan, saved, nsteps)
                                                     : time_plan<float>(h, cand[k].plan, saved, nsteps);
        cand[k].ms = ms / nsteps;
        float &tm = h->tune_ms[cand[k].plan];
        tm = (tm == 0.f || ms < tm) ? ms : tm;
        if (cand[k].ms < cand[best].ms)
            best = k;
    }
    HIPCHECK(hipStreamSynchronize(h->stream));
    (void)hipFree(saved);
    h->pending = false;
    h->fparity = 0;
    set_x_lines(h, cand[best].xl);
    if (cand[best].plan == SSCN_PLAN_FUSED) {
        const int r = set_fused_tile(h, cand[best].tile);
        if (r)
            return r;
    }
    h->active_plan = h->plan = cand[best].plan;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache[key] = cand[best];
    tune_cache_save();
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

// Free the device buffers that depend on the grid and parameters (work,
// exact-path workspace, pivot tables, norm partials and the fused-step
// descriptors), leaving the handle's observables buffers, phase buffer and
// capture stream.
void release_step_buffers(sscn_handle *h)
{
    free_buffers(h);
    for (int ax = 0; ax < 3; ++ax) {
        if (h->tab[ax])
            (void)hipFree(h->tab[ax]);
        h->tab[ax] = nullptr;
    }
    void **bufs[] = {(void **)&h->partials, (void **)&h->d_inst, (void **)&h->d_work, (void **)&h->d_nwork,
                     (void **)&h->partials2};
    for (void **q : bufs) {
        if (*q)
            (void)hipFree(*q);
        *q = nullptr;
    }
}

// ---------------------------------------------------------------------------
// Batched 2D instances (one fused launch per step over all their tiles).

void batch_group_offsets(sscn_batch *b);
int batch_lists(sscn_batch *b, bool all_for_obs = false);
void batch_drop_graph(sscn_batch *b);

// Groups of the sweep plan (sscn_batch::group): G = ceil(bytes / budget)
// groups, where bytes counts both state buffers of every instance, filled
// largest instance first into the group with the fewest bytes so far.  Each
// group's regions of the x and y work lists follow the previous group's.
void batch_groups(sscn_batch *b, size_t esize)
{
    int64_t mb = kBatchGroupMB;
    if (const char *e = std::getenv("SSCN_BATCH_GROUP_MB"))
        mb = std::max(0L, std::strtol(e, nullptr, 10));
    if (b->dim3)
        mb = 0;  // the z-sweep's list is not split into groups
    std::vector<int64_t> bytes(b->n);
    int64_t total = 0;
    for (int k = 0; k < b->n; ++k) {
        bytes[k] = 2 * (int64_t)b->p[k].nx * b->p[k].ny * (int64_t)esize;
        total += bytes[k];
    }
    const int64_t budget = mb * (1 << 20);
    int G = budget > 0 ? (int)((total + budget - 1) / budget) : 1;
    G = std::max(1, std::min(G, b->n));
    std::vector<int> order(b->n);
    for (int k = 0; k < b->n; ++k)
        order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return bytes[x] > bytes[y]; });
    std::vector<int64_t> load(G, 0);
    b->group.assign(b->n, 0);
    for (int k : order) {
        const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        b->group[k] = g;
        load[g] += bytes[k];
    }
    b->ngroups = G;
    batch_group_offsets(b);
}

// Each group's region of the x and y work lists from the instances' item
// counts.
void batch_group_offsets(sscn_batch *b)
{
    const int G = b->ngroups;
    b->gx_tot.assign(G, 0);
    b->gy_tot.assign(G, 0);
    for (int k = 0; k < b->n; ++k) {
        b->gx_tot[b->group[k]] += b->xitems[k];
        b->gy_tot[b->group[k]] += b->yitems[k];
    }
    b->gx_off.assign(G, 0);
    b->gy_off.assign(G, 0);
    for (int g = 1; g < G; ++g) {
        b->gx_off[g] = b->gx_off[g - 1] + b->gx_tot[g - 1];
        b->gy_off[g] = b->gy_off[g - 1] + b->gy_tot[g - 1];
    }
    b->gx_cnt = b->gx_tot;
    b->gy_cnt = b->gy_tot;
}

// Dynamic LDS of a batched x-sweep block of instance k with L lines: the
// padded lines, their pivot-table rows and wall terms.
size_t batch_x_lds(const sscn_batch *b, int k, int L)
{
    const size_t esize = b->precision == SSCN_C128 ? 16 : 8;
    const size_t LS = (size_t)x_row_len(b->p[k].nx, kSegX, b->W);
    return ((size_t)L * LS + (size_t)L * (b->W + 2) + L) * esize;
}

// x-sweep work items (line blocks) of instance k with L lines per block.
int batch_x_items(const sscn_batch *b, int k, int L)
{
    const int lines = b->p[k].ny * (b->dim3 ? b->p[k].nz : 1);
    return (lines + L - 1) / L;
}

// Put the x-sweep's lines-per-block option sel in force: every instance's
// L, the x work items and group regions, the launch's LDS and staging width
// (before the device buffers exist, host state only; after, also the
// instance descriptors and work lists on the device, and the captured
// graphs, whose launches carry the old grid and LDS, are dropped).
int batch_xlines(sscn_batch *b, int sel)
{
    b->xsel = sel;
    b->xlds = 0;
    b->xshort = true;
    b->total_x = 0;
    for (int k = 0; k < b->n; ++k) {
        const int L = b->xl_opt[sel][k];
        b->hinst[k].xl = L;
        b->xitems[k] = batch_x_items(b, k, L);
        b->total_x += b->xitems[k];
        b->xlds = std::max(b->xlds, batch_x_lds(b, k, L));
        if ((int64_t)b->p[k].nx * L > 256 * 8)
            b->xshort = false;
    }
    batch_group_offsets(b);
    if (!b->d_inst)
        return 0;
    batch_drop_graph(b);
    HIPCHECK(hipMemcpy(b->d_inst, b->hinst.data(), sizeof(Inst2D) * b->n, hipMemcpyHostToDevice));
    return batch_lists(b);
}

// Upload the work lists of the active instances: tiles (largest instances
// first), finish chunks and observable chunks with each instance's range.
int batch_lists(sscn_batch *b, bool all_for_obs)
{
    std::vector<int> order(b->n);
    for (int k = 0; k < b->n; ++k)
        order[k] = k;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->ntiles[x] > b->ntiles[y]; });
    std::vector<int2> wl, fl, ol;
    std::vector<int2> xl(std::max(b->total_x, 1)), yl(std::max(b->total_y, 1)), zl;
    std::vector<int> obase(b->n, 0), ocount(b->n, 0), kl;
    b->gx_cnt.assign(b->ngroups, 0);
    b->gy_cnt.assign(b->ngroups, 0);
    for (int k : order)
        if (b->active[k]) {
            for (int t = 0; t < b->ntiles[k]; ++t)
                wl.push_back(int2{k, t});
            kl.push_back(k);
            if (b->sweeps_ok) {
                // within the region of the instance's group, active instances first
                const int g = b->group[k];
                for (int t = 0; t < b->xitems[k]; ++t)
                    xl[b->gx_off[g] + b->gx_cnt[g]++] = int2{k, t * b->hinst[k].xl};
                for (int t = 0; t < b->yitems[k]; ++t)
                    yl[b->gy_off[g] + b->gy_cnt[g]++] = int2{k, t};
                for (int t = 0; t < b->zitems[k]; ++t)
                    zl.push_back(int2{k, t});
            }
        }
    for (int k = 0; k < b->n; ++k) {
        if (b->active[k])
            for (int c = 0; c < b->nchunk[k]; ++c)
                fl.push_back(int2{k, c});
        if (b->active[k] || all_for_obs) {
            obase[k] = (int)ol.size();
            ocount[k] = b->nchunk[k];
            for (int c = 0; c < b->nchunk[k]; ++c)
                ol.push_back(int2{k, c});
        }
    }
    const int nw = (int)wl.size(), nfl = (int)fl.size(), nol = (int)ol.size();
    const int nkl = (int)kl.size();
    int nxl = 0, nyl = 0;
    for (int g = 0; g < b->ngroups; ++g) {
        nxl += b->gx_cnt[g];
        nyl += b->gy_cnt[g];
    }
    if (b->sweeps_ok) {
        HIPCHECK(hipMemcpy(b->d_xwork, xl.data(), sizeof(int2) * b->total_x, hipMemcpyHostToDevice));
        HIPCHECK(hipMemcpy(b->d_ywork, yl.data(), sizeof(int2) * b->total_y, hipMemcpyHostToDevice));
    }
    if (nkl)
        HIPCHECK(hipMemcpy(b->d_klist, kl.data(), sizeof(int) * nkl, hipMemcpyHostToDevice));
    const int nzl = (int)zl.size();
    if (nzl)
        HIPCHECK(hipMemcpy(b->d_zwork, zl.data(), sizeof(int2) * nzl, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(b->d_nzl, &nzl, sizeof(int), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(b->d_nx, b->gx_cnt.data(), sizeof(int) * b->ngroups, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(b->d_ny, b->gy_cnt.data(), sizeof(int) * b->ngroups, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(b->d_nk, &nkl, sizeof(int), hipMemcpyHostToDevice));
    if (nw)
        HIPCHECK(hipMemcpy(b->d_work, wl.data(), sizeof(int2) * nw, hipMemcpyHostToDevice));
    if (nfl)
        HIPCHECK(hipMemcpy(b->d_fwork, fl.data(), sizeof(int2) * nfl, hipMemcpyHostToDevice));
    if (nol)
        HIPCHECK(hipMemcpy(b->d_owork, ol.data(), sizeof(int2) * nol, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(b->d_nwork, &nw, sizeof(int), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(b->d_nf, &nfl, sizeof(int), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(b->d_no, &nol, sizeof(int), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(b->d_obase, obase.data(), sizeof(int) * b->n, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(b->d_ocount, ocount.data(), sizeof(int) * b->n, hipMemcpyHostToDevice));
    if (!all_for_obs) {
        b->grid_tiles = nw;
        b->grid_chunks = nfl;
        b->grid_x = nxl;
        b->grid_y = nyl;
        b->grid_z = nzl;
        b->grid_k = nkl;
    }
    return 0;
}


// nsteps fused steps of every listed instance, then the finish pass that
// leaves each state normalised (imaginary time) in its caller buffer.
// ev (optional, 4 events per step): the sweep plan records them around its
// kernels (batch_sweep_step); the fused plan records ev[4s] before step s's
// launch and the other three after it.
template <class R>
void batch_enqueue(sscn_batch *b, int64_t nsteps, hipStream_t st, int grid_tiles, int grid_chunks, bool all,
                   hipEvent_t *ev = nullptr)
{
    const bool imag = b->mode == SSCN_IMAG;
    if (b->active_plan == SSCN_PLAN_SWEEPS) {
        // group by group (sscn_batch::group): all the steps of one group run
        // before the next group's, so a group's two state buffers stay in the
        // Infinity Cache between its sweeps
        const bool pending = b->pending;
        for (int g = 0; g < b->ngroups; ++g) {
            b->pending = pending;
            for (int64_t s = 0; s < nsteps; ++s)
                batch_sweep_step<R>(b, st, g, all, ev ? ev + 4 * (g * nsteps + s) : nullptr);
        }
        const int grid_k = all ? b->n : b->grid_k;
        if (imag && b->pending) {
            hipLaunchKernelGGL(k_batch_scale, dim3(std::max(grid_k, 1)), dim3(256), 0, st, b->d_inst, b->d_klist,
                               b->d_nk, b->ypart, b->d_scale);
            hipLaunchKernelGGL((k_batch_finish<R>), dim3(std::max(grid_chunks, 1)), dim3(256), 0, st, b->d_inst,
                               b->d_fwork, b->d_nf, 0, b->ypart, 1, (const double *)b->d_scale);
        }
        b->pending = false;
        b->fparity = 0;
        return;
    }
    const FusedLaunch f{b->d_inst, b->d_work, b->d_nwork, std::max(grid_tiles, 1), b->W, nullptr};
    for (int64_t s = 0; s < nsteps; ++s) {
        if (ev)
            (void)hipEventRecord(ev[4 * s], st);
        if (imag)
            launch_fused<R, false>(f, b->fparity, b->part[b->pbuf], b->part[b->pbuf ^ 1], b->pending ? 1 : 0, st);
        else
            launch_fused<R, true>(f, b->fparity, nullptr, nullptr, 0, st);
        if (ev)
            for (int t = 1; t < 4; ++t)
                (void)hipEventRecord(ev[4 * s + t], st);
        b->fparity ^= 1;
        if (imag) {
            b->pbuf ^= 1;
            b->pending = true;
        }
    }
    if ((imag && b->pending) || b->fparity == 1)
        hipLaunchKernelGGL((k_batch_finish<R>), dim3(std::max(grid_chunks, 1)), dim3(256), 0, st, b->d_inst,
                           b->d_fwork, b->d_nf, b->fparity, b->part[b->pbuf], (imag && b->pending) ? 1 : 0,
                           (const double *)nullptr);
    b->pending = false;
    b->fparity = 0;
}

void batch_drop_graph(sscn_batch *b)
{
    if (b->gexec)
        (void)hipGraphExecDestroy(b->gexec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->graph_k = 0;
    drop_graphs(b->step_graphs);
}

// Record k steps of every listed instance on stream st for a graph: the
// launch grids cover every instance (the kernels read the current list
// lengths on the device, so the graph stays valid when converged instances
// leave the lists); the host-side step bookkeeping is restored after.
void batch_capture_steps(sscn_batch *b, int64_t k, hipStream_t st)
{
    const int fparity = b->fparity, pbuf = b->pbuf;
    const bool pending = b->pending;
    if (b->precision == SSCN_C128)
        batch_enqueue<double>(b, k, st, b->total_tiles, b->total_chunks, true);
    else
        batch_enqueue<float>(b, k, st, b->total_tiles, b->total_chunks, true);
    b->fparity = fparity;
    b->pbuf = pbuf;
    b->pending = pending;
}

int batch_graph(sscn_batch *b, int k)
{
    if (b->gexec && b->graph_k == k)
        return 0;
    if (b->gexec)
        (void)hipGraphExecDestroy(b->gexec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    HIPCHECK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    batch_capture_steps(b, k, b->cap);
    hipError_t e = hipStreamEndCapture(b->cap, &b->graph);
    if (e != hipSuccess)
        return fail(SSCN_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess)
        return fail(SSCN_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    b->graph_k = k;
    return 0;
}

// The graphs a sscn_batch_step call of nsteps steps replays: nsteps = q G +
// r, G = min(nsteps, kBatchGraphSteps); q launches of the G-step graph, then
// the r-step graph (r >= 2) or one direct step.  launch = false only
// captures them.
int batch_run_step_graphs(sscn_batch *b, int64_t nsteps, bool launch)
{
    const int64_t G = std::min<int64_t>(nsteps, kBatchGraphSteps);
    const int64_t q = nsteps / G, r = nsteps % G;
    auto enq = [b](int64_t n, hipStream_t st) { batch_capture_steps(b, n, st); };
    hipGraphExec_t x = nullptr;
    int rc = cached_graph(b->step_graphs, b->cap, G, enq, &x);
    if (rc)
        return rc;
    for (int64_t t = 0; launch && t < q; ++t)
        HIPCHECK(hipGraphLaunch(x, b->stream));
    if (r >= 2) {
        rc = cached_graph(b->step_graphs, b->cap, r, enq, &x);
        if (rc)
            return rc;
        if (launch)
            HIPCHECK(hipGraphLaunch(x, b->stream));
    } else if (r == 1 && launch) {
        if (b->precision == SSCN_C128)
            batch_enqueue<double>(b, 1, b->stream, b->grid_tiles, b->grid_chunks, false);
        else
            batch_enqueue<float>(b, 1, b->stream, b->grid_tiles, b->grid_chunks, false);
    }
    return 0;
}

// Observables of the listed instances into d_sums; with tol > 0 also a
// convergence check: the vortex count of every listed instance and the
// criterion of sscn_converge (k_batch_conv).
template <class R>
void batch_obs_launch(sscn_batch *b, int nchunks, double tol)
{
    hipLaunchKernelGGL((k_batch_obs<R>), dim3(std::max(nchunks, 1)), dim3(256), 0, b->stream, b->d_inst, b->d_owork,
                       b->d_no, b->opart);
    hipLaunchKernelGGL(k_batch_obs_final, dim3(b->n), dim3(256), 0, b->stream, b->n, b->d_obase, b->d_ocount,
                       b->opart, b->d_sums);
    if (tol > 0.0) {
        hipLaunchKernelGGL((k_batch_vortex<R>), dim3(std::max(nchunks, 1)), dim3(256), 0, b->stream, b->d_inst,
                           b->d_owork, b->d_no, (const double *)b->d_sums, kConvDensityFrac, kConvBox, b->vpart);
        hipLaunchKernelGGL(k_batch_conv, dim3((b->n + 255) / 256), dim3(256), 0, b->stream, b->n, b->d_obase,
                           b->d_ocount, (const double *)b->vpart, (const double *)b->d_sums, b->d_mu_prev, b->d_hits,
                           b->d_count_prev, b->d_counts, b->d_conv, tol, (long long)b->steps);
    }
}

// Time 8 steps of the batch as it stands (plan, x option) for the
// autotuner: one untimed step first (the first launch of a kernel also
// loads its code object), then the states restored from saved, the timed
// steps, and the states restored again.
int batch_time_steps(sscn_batch *b, const char *saved, const std::vector<size_t> &off, float *ms)
{
    auto restore = [&]() -> int {
        for (int k = 0; k < b->n; ++k)
            HIPCHECK(hipMemcpyAsync(b->psi[k], saved + off[k], off[k + 1] - off[k], hipMemcpyDeviceToDevice,
                                    b->stream));
        return 0;
    };
    b->pending = false;
    b->fparity = 0;
    b->pbuf = 0;
    if (b->precision == SSCN_C128)
        batch_enqueue<double>(b, 1, b->stream, b->grid_tiles, b->grid_chunks, false);
    else
        batch_enqueue<float>(b, 1, b->stream, b->grid_tiles, b->grid_chunks, false);
    int rc = restore();
    if (rc)
        return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timing_event(&e0) != hipSuccess || timing_event(&e1) != hipSuccess)
        rc = fail(SSCN_EHIP, "hipEventCreate failed");
    if (!rc) {
        (void)hipEventRecord(e0, b->stream);
        if (b->precision == SSCN_C128)
            batch_enqueue<double>(b, 8, b->stream, b->grid_tiles, b->grid_chunks, false);
        else
            batch_enqueue<float>(b, 8, b->stream, b->grid_tiles, b->grid_chunks, false);
        (void)hipEventRecord(e1, b->stream);
        *ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(ms, e0, e1) != hipSuccess)
            rc = fail(SSCN_EHIP, "event timing failed");
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    return rc ? rc : restore();
}

// The first stepping call of a batch times its candidates from a saved copy
// of every state, restores the states and keeps the fastest.  The
// candidates: with SSCN_PLAN_AUTO the fused step and the sweep plan; with
// the sweep plan (chosen or forced) its two x-sweep lines-per-block options
// (sscn_batch::xl_opt), unless they coincide or SSCN_BATCH_XLINES fixes
// one.  Every candidate is timed twice, in turn, and keeps its faster time,
// so that a clock still rising during the first round does not favour the
// later candidates.
int batch_autotune(sscn_batch *b)
{
    const bool plan_auto = b->plan == SSCN_PLAN_AUTO;
    if (plan_auto)
        b->plan = b->active_plan = SSCN_PLAN_FUSED;
    if (!b->sweeps_ok)
        return 0;
    const bool tune_x = !b->xtuned && b->xforce < 0 && b->xl_opt[0] != b->xl_opt[1];
    if (!plan_auto && !(tune_x && b->plan == SSCN_PLAN_SWEEPS))
        return 0;
    struct Cand {
        int plan, xsel;
    };
    std::vector<Cand> cand;
    if (plan_auto)
        cand.push_back({SSCN_PLAN_FUSED, b->xsel});
    if (tune_x) {
        cand.push_back({SSCN_PLAN_SWEEPS, 0});
        cand.push_back({SSCN_PLAN_SWEEPS, 1});
    } else {
        cand.push_back({SSCN_PLAN_SWEEPS, b->xsel});
    }
    const size_t esize = b->precision == SSCN_C128 ? 16 : 8;
    std::vector<size_t> off(b->n + 1, 0);
    for (int k = 0; k < b->n; ++k)
        off[k + 1] = off[k] + (size_t)b->p[k].nx * b->p[k].ny * (b->dim3 ? b->p[k].nz : 1) * esize;
    char *saved = nullptr;
    if (hipMalloc(&saved, off[b->n]) != hipSuccess)
        return fail(SSCN_ENOMEM, "hipMalloc of the batch autotune copy failed");
    int rc = 0;
    for (int k = 0; k < b->n && !rc; ++k)
        if (hipMemcpyAsync(saved + off[k], b->psi[k], off[k + 1] - off[k], hipMemcpyDeviceToDevice, b->stream) !=
            hipSuccess)
            rc = fail(SSCN_EHIP, "hipMemcpyAsync of the batch autotune copy failed");
    std::vector<float> best(cand.size(), INFINITY);
    for (int rep = 0; rep < 2 && !rc; ++rep)
        for (size_t c = 0; c < cand.size() && !rc; ++c) {
            b->active_plan = cand[c].plan;
            if (cand[c].plan == SSCN_PLAN_SWEEPS && b->xsel != cand[c].xsel)
                rc = batch_xlines(b, cand[c].xsel);
            float ms = 0.f;
            if (!rc)
                rc = batch_time_steps(b, saved, off, &ms);
            best[c] = std::min(best[c], ms);
        }
    if (!rc && hipStreamSynchronize(b->stream) != hipSuccess)
        rc = fail(SSCN_EHIP, "the batch autotune steps failed");
    (void)hipFree(saved);
    if (rc)
        return rc;
    size_t win = 0, xwin = 0;
    bool have_x = false;
    b->tune_ms[SSCN_PLAN_FUSED] = b->tune_ms[SSCN_PLAN_SWEEPS] = 0.f;
    for (size_t c = 0; c < cand.size(); ++c) {
        if (best[c] < best[win])
            win = c;
        if (cand[c].plan == SSCN_PLAN_SWEEPS) {
            b->tune_x_ms[cand[c].xsel] = best[c];
            if (!have_x || best[c] < best[xwin])
                xwin = c;
            have_x = true;
        }
        float &tm = b->tune_ms[cand[c].plan];
        tm = tm > 0.f ? std::min(tm, best[c]) : best[c];
    }
    if (tune_x)
        b->xtuned = true;
    // the faster x option stays in force, also when the fused plan wins (for
    // a later sscn_batch_set_plan)
    if (have_x && b->xsel != cand[xwin].xsel) {
        rc = batch_xlines(b, cand[xwin].xsel);
        if (rc)
            return rc;
    }
    if (plan_auto)
        b->plan = cand[win].plan;
    b->active_plan = b->plan;
    b->pending = false;
    b->fparity = 0;
    b->pbuf = 0;
    HIPCHECK(hipGetLastError());
    return 0;
}

void batch_free(sscn_batch *b)
{
    batch_drop_graph(b);
    for (auto *v : {&b->work, &b->tabx, &b->taby, &b->tabz})
        for (void *q : *v)
            if (q)
                (void)hipFree(q);
    void *bufs[] = {b->d_inst, b->d_work, b->d_fwork, b->d_owork, b->d_nwork, b->d_nf, b->d_no, b->d_obase,
                    b->d_ocount, b->part[0], b->part[1], b->opart, b->d_sums, b->d_mu_prev, b->d_hits, b->d_conv,
                    b->d_count_prev, b->d_counts, b->vpart,
                    b->phase, b->d_xwork, b->d_ywork, b->d_nx, b->d_ny, b->d_klist, b->d_nk, b->ypart,
                    b->d_scale, b->d_zwork, b->d_nzl};
    for (void *q : bufs)
        if (q)
            (void)hipFree(q);
    if (b->cap)
        (void)hipStreamDestroy(b->cap);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI.

extern "C" {

const char *sscn_last_error(void) { return last_error(); }

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
    if (const char *env = std::getenv("SSCN_FUSED_TILE"))
        h->tile_force = (env[0] >= '0' && env[0] < '0' + kFusedTiles && env[1] == 0) ? env[0] - '0' : -1;
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
    const size_t npart = std::max({(size_t)h->nemit, (size_t)kRedBlocks, max_fused_tiles(h)});
    if (hipMalloc(&h->partials, npart * sizeof(double)) != hipSuccess ||
        hipMalloc(&h->obs_part, (size_t)kRedBlocks * kObsN * sizeof(double)) != hipSuccess ||
        hipMalloc(&h->obs_buf, 64 * sizeof(double)) != hipSuccess)
        return bail(fail(SSCN_ENOMEM, "hipMalloc of reduction buffers failed"));
    if (hipMemsetAsync(h->partials, 0, npart * sizeof(double), h->stream) != hipSuccess)
        return bail(fail(SSCN_EHIP, "hipMemsetAsync failed"));
    r = setup_fused(h);
    if (r)
        return bail(r);
    r = allow_x_lds(h);
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

// The initial state of Eq. (fun) with the random phase from a host array
// (phase_host), from the counter-based generator (seeded), or none.
static int init_state_impl(sscn_handle *h, int kind, const double *phase_host, int seeded, uint64_t seed, double d_xy,
                           double d_z)
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
                           ph, d_xy, d_z, seeded, seed);
        launch_norm<double>(h, h->stream);
    } else {
        hipLaunchKernelGGL((k_init<float>), dim3(nb), dim3(256), 0, h->stream, (V<float> *)h->psi, h->args, kind,
                           ph, d_xy, d_z, seeded, seed);
        launch_norm<float>(h, h->stream);
    }
    // normalise: the norm partials use kRedBlocks blocks
    const int saved = h->nemit;
    h->nemit = kRedBlocks;
    if (p.precision == SSCN_C128)
        launch_rescale<double>(h, h->stream, false);
    else
        launch_rescale<float>(h, h->stream, false);
    h->nemit = saved;
    h->pending = false;
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(h->stream));
    return 0;
}

int sscn_init_state(sscn_handle *h, int kind, const double *phase_host, double d_xy, double d_z)
{
    return init_state_impl(h, kind, phase_host, 0, 0, d_xy, d_z);
}

int sscn_init_state_seed(sscn_handle *h, int kind, int random_phase, uint64_t seed, double d_xy, double d_z)
{
    return init_state_impl(h, kind, nullptr, random_phase ? 1 : 0, seed, d_xy, d_z);
}

int sscn_phase_field_seed(uint64_t seed, int nx, int ny, double *out_dev, void *hip_stream)
{
    if (!out_dev || nx < 1 || ny < 1)
        return fail(SSCN_EINVAL, "bad phase_field_seed arguments");
    const int64_t n = (int64_t)nx * ny;
    const int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(k_phase_seed, dim3(nb), dim3(256), 0, (hipStream_t)hip_stream, out_dev, nx, ny, seed);
    HIPCHECK(hipGetLastError());
    return 0;
}

int sscn_prepare_steps(sscn_handle *h, int64_t nsteps)
{
    if (!h || nsteps < 0)
        return fail(SSCN_EINVAL, "bad prepare_steps arguments");
    int r = autotune(h);
    if (!r && nsteps >= 2)
        r = run_step_graphs(h, nsteps, false);
    if (r)
        return r;
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
    if (nsteps >= 2 && !h->pending) {
        int r = run_step_graphs(h, nsteps, true);
        if (r)
            return r;
    } else if (h->p.precision == SSCN_C128) {
        enqueue_direct<double>(h, nsteps, h->stream);
    } else {
        enqueue_direct<float>(h, nsteps, h->stream);
    }
    HIPCHECK(hipGetLastError());
    h->steps += nsteps;
    return 0;
}

}  // extern "C"

namespace {

// Scratch of sscn_observables_noalloc: the per-block partial sums of the
// observables kernel (at most kRedBlocks rows of kObsN doubles, 128 KiB),
// in device memory that exists from the library's load on, one copy per
// GPU.  Host code must not use the name as an address: every call takes the
// device address of the current GPU's copy from noalloc_scratch().
constexpr int kNoallocRows = kRedBlocks;
static __device__ __align__(256) double scratch[kNoallocRows * kObsN];

std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_ptr;  // device ordinal -> address of its scratch

// The current device's scratch address, looked up once per device with
// hipGetSymbolAddress (no allocation).
int noalloc_scratch(double **out)
{
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *ptr = nullptr;
        HIPCHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        it = g_scratch_ptr.emplace(dev, (double *)ptr).first;
    }
    *out = it->second;
    return 0;
}

// sums[t] *= dV for every sum but the maximum density (t = 13), as the host
// does for sscn_observables.
__global__ __launch_bounds__(64) void k_scale_obs_sums(double *sums, double dV)
{
    const int t = threadIdx.x;
    if (t < kObsN && t != 13)
        sums[t] *= dV;
}

}  // namespace

extern "C" {

int sscn_observables_noalloc(const sscn_params *params, const void *psi_dev, void *hip_stream, double *sums_dev)
{
    if (!params || !psi_dev || !sums_dev)
        return fail(SSCN_EINVAL, "null argument");
    sscn_params p = *params;
    if (p.dim == 2)
        p.nz = 1;
    int r = validate(p);
    if (r)
        return r;
    StepArgs a{};
    fill_args(p, a);
    const int64_t n = npoints(p);
    const int nb = red_blocks(n);
    if (nb > kNoallocRows)  // red_blocks never exceeds kRedBlocks; kept as the stated limit
        return fail(SSCN_EINVAL, "more partial rows than the static scratch holds");
    double *part = nullptr;
    r = noalloc_scratch(&part);
    if (r)
        return r;
    hipStream_t st = (hipStream_t)hip_stream;
    if (p.precision == SSCN_C128)
        hipLaunchKernelGGL((k_observables<double>), dim3(nb), dim3(256), 0, st, (const V<double> *)psi_dev, a, part);
    else
        hipLaunchKernelGGL((k_observables<float>), dim3(nb), dim3(256), 0, st, (const V<float> *)psi_dev, a, part);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, st, (const double *)part, nb, kObsN, 1u << 13,
                       sums_dev);
    hipLaunchKernelGGL(k_scale_obs_sums, dim3(1), dim3(64), 0, st, sums_dev, a.dV);
    HIPCHECK(hipGetLastError());
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
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, h->stream, h->obs_part, nb, kObsN, 1u << 13,
                       h->obs_buf);
    double s[kObsN];
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(s, h->obs_buf, sizeof s, hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    const double dV = h->args.dV;
    for (int t = 0; t < kObsN; ++t)
        if (t != 13)
            s[t] *= dV;
    std::memset(out, 0, sizeof *out);
    std::memcpy(out->sums, s, sizeof s);
    out->norm = s[0];
    out->mu = (s[2] + s[3] + s[4] + s[5]) / s[1];
    out->energy = (s[2] + s[3] + 0.5 * s[4] + s[5]) / s[1];
    out->mu_full = (s[6] + s[7] + s[8] + s[9]) / s[0];
    out->energy_full = (s[6] + s[7] + 0.5 * s[8] + s[9]) / s[0];
    out->mu_4th = (s[14] + s[7] + s[8] + s[15]) / s[0];
    out->energy_4th = (s[14] + s[7] + 0.5 * s[8] + s[15]) / s[0];
    out->rms_x = std::sqrt(s[10] / s[0]);
    out->rms_y = std::sqrt(s[11] / s[0]);
    out->rms_z = std::sqrt(s[12] / s[0]);
    out->rms_r = std::sqrt((s[10] + s[11] + s[12]) / s[0]);
    out->max_density = s[13];
    out->step = h->steps;
    for (int t = 0; t < kObsN; ++t)
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

int sscn_embed_state(const void *src, int nx_src, int ny_src, int nz_src, void *dst, int nx, int ny, int nz,
                     int precision, void *stream)
{
    if (!src || !dst || nx_src < 1 || ny_src < 1 || nz_src < 1 || nx < 1 || ny < 1 || nz < 1)
        return fail(SSCN_EINVAL, "bad embed arguments");
    if (precision != SSCN_C128 && precision != SSCN_C64)
        return fail(SSCN_EINVAL, "precision must be SSCN_C128 or SSCN_C64");
    if ((nx - nx_src) % 2 || (ny - ny_src) % 2 || (nz - nz_src) % 2)
        return fail(SSCN_EINVAL, "grid sizes must differ by an even number of points on every axis");
    const int dim = (nz == 1 && nz_src == 1) ? 2 : 3;
    const size_t es = precision == SSCN_C128 ? 16 : 8;
    const char *s0 = (const char *)src, *s1 = s0 + (size_t)nx_src * ny_src * nz_src * es;
    const char *d0 = (const char *)dst, *d1 = d0 + (size_t)nx * ny * nz * es;
    if (s0 < d1 && d0 < s1)
        return fail(SSCN_EINVAL, "src and dst overlap");
    const int ox = (nx - nx_src) / 2, oy = (ny - ny_src) / 2, oz = (nz - nz_src) / 2;
    const int nb = red_blocks((int64_t)nx * ny * nz);
    if (precision == SSCN_C128)
        hipLaunchKernelGGL((k_embed<double>), dim3(nb), dim3(256), 0, (hipStream_t)stream, (const V<double> *)src,
                           nx_src, ny_src, nz_src, (V<double> *)dst, nx, ny, nz, ox, oy, oz, dim);
    else
        hipLaunchKernelGGL((k_embed<float>), dim3(nb), dim3(256), 0, (hipStream_t)stream, (const V<float> *)src,
                           nx_src, ny_src, nz_src, (V<float> *)dst, nx, ny, nz, ox, oy, oz, dim);
    HIPCHECK(hipGetLastError());
    return 0;
}

int sscn_extend_z(const void *xy, int nx, int ny, void *dst, int nz, double hz, double d_z, int precision,
                  void *stream)
{
    if (!xy || !dst || nx < 2 || ny < 2 || nz < 2)
        return fail(SSCN_EINVAL, "bad extend_z arguments");
    if (!(hz > 0.0) || !(d_z > 0.0) || !std::isfinite(hz) || !std::isfinite(d_z))
        return fail(SSCN_EINVAL, "hz and d_z must be positive and finite");
    if (precision != SSCN_C128 && precision != SSCN_C64)
        return fail(SSCN_EINVAL, "precision must be SSCN_C128 or SSCN_C64");
    const size_t es = precision == SSCN_C128 ? 16 : 8;
    const char *s0 = (const char *)xy, *s1 = s0 + (size_t)nx * ny * es;
    const char *d0 = (const char *)dst, *d1 = d0 + (size_t)nx * ny * nz * es;
    if (s0 < d1 && d0 < s1)
        return fail(SSCN_EINVAL, "xy and dst overlap");
    // z_k = -nz hz / 2 + k hz; the Gaussian normalised over the interior
    // points k = 1 .. nz - 1 (the wall k = 0 is zeroed by the caller)
    const double z0 = -0.5 * nz * hz;
    double sum = 0.0;
    for (int k = 1; k < nz; ++k) {
        const double t = (z0 + k * hz) / d_z;
        sum += std::exp(-t * t);
    }
    const double c = 1.0 / std::sqrt(hz * sum);
    const int nb = red_blocks((int64_t)nx * ny * nz);
    if (precision == SSCN_C128)
        hipLaunchKernelGGL((k_extend_z<double>), dim3(nb), dim3(256), 0, (hipStream_t)stream,
                           (const V<double> *)xy, nx, ny, (V<double> *)dst, nz, z0, hz, d_z, c);
    else
        hipLaunchKernelGGL((k_extend_z<float>), dim3(nb), dim3(256), 0, (hipStream_t)stream,
                           (const V<float> *)xy, nx, ny, (V<float> *)dst, nz, z0, hz, d_z, c);
    HIPCHECK(hipGetLastError());
    return 0;
}

int sscn_resample(const void *src, int nx_src, int ny_src, double hx_src, double hy_src, void *dst, int nx, int ny,
                  double hx, double hy, double angle, int precision, void *stream)
{
    if (!src || !dst || nx_src < 2 || ny_src < 2 || nx < 2 || ny < 2)
        return fail(SSCN_EINVAL, "bad resample arguments");
    if (!(hx_src > 0) || !(hy_src > 0) || !(hx > 0) || !(hy > 0) || !std::isfinite(hx_src) ||
        !std::isfinite(hy_src) || !std::isfinite(hx) || !std::isfinite(hy) || !std::isfinite(angle))
        return fail(SSCN_EINVAL, "spacings must be positive and finite, the angle finite");
    if (precision != SSCN_C128 && precision != SSCN_C64)
        return fail(SSCN_EINVAL, "precision must be SSCN_C128 or SSCN_C64");
    const size_t es = precision == SSCN_C128 ? 16 : 8;
    const char *s0 = (const char *)src, *s1 = s0 + (size_t)nx_src * ny_src * es;
    const char *d0 = (const char *)dst, *d1 = d0 + (size_t)nx * ny * es;
    if (s0 < d1 && d0 < s1)
        return fail(SSCN_EINVAL, "src and dst overlap");
    const double ca = std::cos(angle), sa = std::sin(angle);
    const int nb = red_blocks((int64_t)nx * ny);
    if (precision == SSCN_C128)
        hipLaunchKernelGGL((k_resample<double>), dim3(nb), dim3(256), 0, (hipStream_t)stream, (const V<double> *)src,
                           nx_src, ny_src, hx_src, hy_src, (V<double> *)dst, nx, ny, hx, hy, ca, sa);
    else
        hipLaunchKernelGGL((k_resample<float>), dim3(nb), dim3(256), 0, (hipStream_t)stream, (const V<float> *)src,
                           nx_src, ny_src, hx_src, hy_src, (V<float> *)dst, nx, ny, hx, hy, ca, sa);
    HIPCHECK(hipGetLastError());
    return 0;
}

int sscn_angular_moments(const void *psi, int nx, int ny, double hx, double hy, int kmax, int precision,
                         double *out_dev, void *stream)
{
    if (!psi || !out_dev || nx < 1 || ny < 1 || kmax < 0 || kmax > 8 || !(hx > 0) || !(hy > 0))
        return fail(SSCN_EINVAL, "bad angular_moments arguments");
    if (precision != SSCN_C128 && precision != SSCN_C64)
        return fail(SSCN_EINVAL, "precision must be SSCN_C128 or SSCN_C64");
    if (precision == SSCN_C128)
        hipLaunchKernelGGL((k_angular_moments<double>), dim3(1), dim3(1024), 0, (hipStream_t)stream,
                           (const V<double> *)psi, nx, ny, hx, hy, kmax, out_dev);
    else
        hipLaunchKernelGGL((k_angular_moments<float>), dim3(1), dim3(1024), 0, (hipStream_t)stream,
                           (const V<float> *)psi, nx, ny, hx, hy, kmax, out_dev);
    HIPCHECK(hipGetLastError());
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
    HIPCHECK(hipStreamSynchronize(h->stream));
    // The new configuration is built completely in a second handle (every
    // device allocation included) before anything of h changes, so that an
    // error leaves h as it was.
    sscn_handle *t = new sscn_handle();
    t->p = np;
    t->psi = conv ? new_psi_dev : h->psi;
    t->stream = h->stream;
    t->tile = h->tile;  // the fused tile shape carries over where it still fits
    t->tile_force = h->tile_force;
    auto drop_t = [&](int code) {
        release_step_buffers(t);
        delete t;
        return code;
    };
    r = setup(t);
    if (!r)
        r = alloc_buffers(t);
    if (!r)
        r = build_tables(t);
    if (!r) {
        const size_t npart = std::max({(size_t)t->nemit, (size_t)kRedBlocks, max_fused_tiles(t)});
        if (hipMalloc(&t->partials, npart * sizeof(double)) != hipSuccess)
            r = fail(SSCN_ENOMEM, "hipMalloc of the partials failed");
    }
    if (!r)
        r = setup_fused(t);
    if (!r)
        r = allow_x_lds(t);
    if (!r && conv) {
        const int nb = red_blocks(h->npts);
        if (h->p.precision == SSCN_C64)
            hipLaunchKernelGGL((k_convert<float, double>), dim3(nb), dim3(256), 0, h->stream,
                               (const V<float> *)h->psi, (V<double> *)new_psi_dev, h->npts);
        else
            hipLaunchKernelGGL((k_convert<double, float>), dim3(nb), dim3(256), 0, h->stream,
                               (const V<double> *)h->psi, (V<float> *)new_psi_dev, h->npts);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess)
            r = fail(SSCN_EHIP, "the precision conversion failed");
    }
    if (r)
        return drop_t(r);
    // commit: h takes t's configuration and buffers, t takes h's old buffers
    drop_graph(h);
    release_step_buffers(h);
    const int64_t steps = h->steps;
    const int plan = h->plan;
    h->p = np;
    h->psi = t->psi;
    r = setup(h);  // host-side geometry; cannot fail (it succeeded for t)
    (void)r;
    h->work = t->work;
    h->ws = t->ws;
    for (int ax = 0; ax < 3; ++ax)
        h->tab[ax] = t->tab[ax];
    h->partials = t->partials;
    h->d_inst = t->d_inst;
    h->d_work = t->d_work;
    h->d_nwork = t->d_nwork;
    h->partials2 = t->partials2;
    h->inst_host = t->inst_host;
    h->tile = t->tile;
    h->ntiles = t->ntiles;
    delete t;  // owns nothing now
    h->plan = (plan == SSCN_PLAN_FUSED && !h->fused_ok) ? SSCN_PLAN_AUTO : plan;
    h->active_plan = h->plan == SSCN_PLAN_FUSED ? SSCN_PLAN_FUSED : SSCN_PLAN_SWEEPS;
    h->fparity = 0;
    h->pbuf = 0;
    h->steps = steps;
    h->pending = false;
    return 0;
}

int sscn_density(sscn_handle *h, int kind, double *out_dev)
{
    if (!h || !out_dev || kind < SSCN_DEN_FULL || kind > SSCN_DEN_CUT_Z)
        return fail(SSCN_EINVAL, "bad density arguments");
    const sscn_params &p = h->p;
    const int nz = p.dim == 3 ? p.nz : 1;
    if (p.dim == 2 && (kind == SSCN_DEN_Z || kind == SSCN_DEN_CUT_Z))
        return fail(SSCN_EINVAL, "z profiles need a 3D handle");
    const int64_t nout = kind == SSCN_DEN_FULL ? h->npts
                         : kind == SSCN_DEN_XY ? (int64_t)p.nx * p.ny
                         : (kind == SSCN_DEN_X || kind == SSCN_DEN_CUT_X) ? p.nx
                         : (kind == SSCN_DEN_Y || kind == SSCN_DEN_CUT_Y) ? p.ny
                                                                           : nz;
    const int nb = red_blocks(nout);
    if (p.precision == SSCN_C128)
        hipLaunchKernelGGL((k_density<double>), dim3(nb), dim3(256), 0, h->stream, (const V<double> *)h->psi, p.nx,
                           p.ny, nz, p.hx, p.hy, p.hz, kind, nout, out_dev);
    else
        hipLaunchKernelGGL((k_density<float>), dim3(nb), dim3(256), 0, h->stream, (const V<float> *)h->psi, p.nx,
                           p.ny, nz, p.hx, p.hy, p.hz, kind, nout, out_dev);
    HIPCHECK(hipGetLastError());
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
        if (timing_event(&e) != hipSuccess) {
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

}  // extern "C"

namespace {

// Launch kernel `which` of the step (0: the fused step or the x-sweep, 1:
// y-sweep, 2: z-sweep) nlaunch times back to back from psi into the work
// buffer, between two events on the handle's stream.
template <class R>
int profile_kernel(sscn_handle *h, int which, int nlaunch, double *avg_ms)
{
    const bool imag = h->p.mode == SSCN_IMAG;
    const bool fused = h->active_plan == SSCN_PLAN_FUSED;
    const int npk = std::max({h->nemit, h->ntiles, kRedBlocks});
    double *prof_part = nullptr;
    if (hipMalloc(&prof_part, sizeof(double) * 2 * npk) != hipSuccess)
        return fail(SSCN_ENOMEM, "hipMalloc of the profiling partials failed");
    HIPCHECK(hipMemsetAsync(prof_part, 0, sizeof(double) * 2 * npk, h->stream));
    sscn_handle t = *h;  // the same kernels with partials into the prof_part
    t.partials = prof_part;
    const FusedLaunch f{h->d_inst, h->d_work, h->d_nwork, h->ntiles, h->W[0], &h->inst_host, h->tile};
    auto launch = [&](bool first) {
        if (fused) {
            if (imag)
                launch_fused<R, false>(f, 0, prof_part, prof_part + npk, first ? 0 : 1, h->stream);
            else
                launch_fused<R, true>(f, 0, nullptr, nullptr, 0, h->stream);
            if (imag && first)  // the partials of this state are the next launches' input
                (void)hipMemcpyAsync(prof_part, prof_part + npk, sizeof(double) * npk, hipMemcpyDeviceToDevice,
                                     h->stream);
        } else if (which == 0) {
            if (imag)
                launch_x<R, false>(&t, h->psi, h->work, first ? 0 : h->nemit, h->stream, false);
            else
                launch_x<R, true>(&t, h->psi, h->work, 0, h->stream, false);
        } else if (which == 1) {
            if (imag && h->p.dim == 2)
                launch_y<R, true>(&t, h->psi, h->work, h->stream);
            else
                launch_y<R, false>(&t, h->psi, h->work, h->stream);
        } else {
            if (imag)
                launch_z<R, true>(&t, h->psi, h->work, h->stream);
            else
                launch_z<R, false>(&t, h->psi, h->work, h->stream);
        }
    };
    if (!fused && which == 0 && imag) {  // partials of the state, and s - 1 from them
        launch_y<R, false>(&t, h->psi, h->work, h->stream);
        if (h->p.dim == 2)
            launch_y<R, true>(&t, h->psi, h->work, h->stream);
        else
            launch_z<R, true>(&t, h->psi, h->work, h->stream);
        hipLaunchKernelGGL(k_norm_scale, dim3(1), dim3(256), 0, h->stream, prof_part, h->nemit, h->args.dV,
                           h->obs_buf + kScaleSlot);
    }
    launch(true);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    if (timing_event(&e0) != hipSuccess || timing_event(&e1) != hipSuccess)
        rc = fail(SSCN_EHIP, "hipEventCreate failed");
    if (!rc) {
        (void)hipEventRecord(e0, h->stream);
        for (int k = 0; k < nlaunch; ++k)
            launch(false);
        (void)hipEventRecord(e1, h->stream);
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            rc = fail(SSCN_EHIP, "event timing failed");
        else if (hipGetLastError() != hipSuccess)
            rc = fail(SSCN_EHIP, "kernel launch failed");
        *avg_ms = ms / nlaunch;
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(prof_part);
    return rc;
}

}  // namespace

extern "C" {

int sscn_profile_kernel(sscn_handle *h, int which, int nlaunch, double *avg_ms)
{
    if (!h || !avg_ms || nlaunch < 1 || nlaunch > 100000 || which < 0 || which > 2)
        return fail(SSCN_EINVAL, "bad profile_kernel arguments");
    int rt = autotune(h);
    if (rt)
        return rt;
    if (h->exact)
        return fail(SSCN_EINVAL, "the exact whole-line path has no kernel to profile this way");
    if ((h->active_plan == SSCN_PLAN_FUSED && which != 0) || (h->p.dim == 2 && which == 2))
        return fail(SSCN_EINVAL, "this plan has no such kernel");
    HIPCHECK(hipStreamSynchronize(h->stream));
    return h->p.precision == SSCN_C128 ? profile_kernel<double>(h, which, nlaunch, avg_ms)
                                       : profile_kernel<float>(h, which, nlaunch, avg_ms);
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

int sscn_solver_info(sscn_handle *h, int *window_xyz, int *segment_xyz, int *plan, int *x_lines)
{
    if (!h)
        return fail(SSCN_EINVAL, "null argument");
    if (x_lines)
        *x_lines = h->xL;
    if (plan)
        *plan = h->plan == SSCN_PLAN_AUTO ? SSCN_PLAN_AUTO : h->active_plan;
    for (int a = 0; a < 3; ++a) {
        if (window_xyz)
            window_xyz[a] = h->exact ? 0 : h->W[a];
        if (segment_xyz)
            segment_xyz[a] = h->exact ? 0 : (a == 0 && h->active_plan != SSCN_PLAN_FUSED ? kSegX : kSeg);
    }
    return 0;
}

int sscn_fused_tile(sscn_handle *h, int *rows, int *cols)
{
    if (!h || !rows || !cols)
        return fail(SSCN_EINVAL, "null argument");
    *rows = fused_tile_rows(h->tile);
    *cols = fused_tile_cols(h->tile);
    return 0;
}

int sscn_get_params(sscn_handle *h, sscn_params *out)
{
    if (!h || !out)
        return fail(SSCN_EINVAL, "null argument");
    *out = h->p;
    return 0;
}

int sscn_converge(sscn_handle *h, int64_t max_steps, int check_every, double tol, double switch_tol,
                  void *fp64_psi_dev, int64_t *steps_out, int *converged, int64_t *switch_out)
{
    if (switch_out)
        *switch_out = -1;
    if (!h || max_steps < 0 || check_every < 1 || !(tol > 0))
        return fail(SSCN_EINVAL, "bad converge arguments");
    if (h->p.mode != SSCN_IMAG)
        return fail(SSCN_EINVAL, "convergence runs are imaginary-time runs");
    if (h->p.precision == SSCN_C64 && !fp64_psi_dev)
        return fail(SSCN_EINVAL, "a complex64 run needs the complex128 buffer for the refinement");
    int64_t done = 0;
    double prev = std::nan(""), best = INFINITY;
    int hits = 0, stall = 0, count_prev = -1;
    bool ok = false;
    sscn_obs o;
    while (done < max_steps) {
        const int64_t k = std::min<int64_t>(check_every, max_steps - done);
        int r = sscn_step(h, k);
        if (r)
            return r;
        done += k;
        r = sscn_observables(h, &o);
        if (r)
            return r;
        const double d = std::fabs(o.mu - prev);
        prev = o.mu;
        if (h->p.precision == SSCN_C64) {
            // FP32 plateau: |dmu| under switch_tol, or, once within a decade
            // of it, no new minimum for 5 checks (rounding noise floor)
            if (d < best) {
                best = d;
                stall = 0;
            } else if (d < 10.0 * switch_tol) {
                ++stall;
            }
            if (d < switch_tol || stall >= 5) {
                r = sscn_set_mode(h, SSCN_IMAG, SSCN_C128, fp64_psi_dev);
                if (r)
                    return r;
                if (switch_out)
                    *switch_out = done;
                prev = std::nan("");
                hits = 0;
                count_prev = -1;
            }
            continue;
        }
        if (d < tol) {
            int c = 0;
            r = sscn_vortex_count(h, kConvDensityFrac, kConvBox, &c);
            if (r)
                return r;
            hits = (count_prev < 0 || c == count_prev) ? hits + 1 : 1;
            count_prev = c;
            if (hits >= 2) {
                ok = true;
                break;
            }
        } else {
            hits = 0;
            count_prev = -1;
        }
    }
    if (steps_out)
        *steps_out = done;
    if (converged)
        *converged = ok ? 1 : 0;
    return 0;
}

int sscn_batch_init(const sscn_params *params, int n, void *const *psi_devs, void *hip_stream, sscn_batch **out)
{
    if (!params || !psi_devs || !out || n < 1)
        return fail(SSCN_EINVAL, "bad batch_init arguments");
    *out = nullptr;
    sscn_batch *b = new sscn_batch();
    b->n = n;
    b->stream = (hipStream_t)hip_stream;
    b->precision = params[0].precision;
    b->mode = params[0].mode;
    auto bail = [&](int code) {
        batch_free(b);
        delete b;
        return code;
    };
    std::vector<sscn_handle> tmp(n);
    for (int k = 0; k < n; ++k) {
        if (!psi_devs[k])
            return bail(fail(SSCN_EINVAL, "null state buffer in the batch"));
        int r = validate(params[k]);
        if (r)
            return bail(r);
        if (params[k].dim != params[0].dim || params[k].precision != b->precision || params[k].mode != b->mode)
            return bail(fail(SSCN_EINVAL, "batch instances must have a common dim, precision and mode"));
        tmp[k].p = params[k];
        if (params[k].dim == 2)
            tmp[k].p.nz = 1;
        r = setup(&tmp[k]);
        if (r)
            return bail(r);
        if (tmp[k].exact)
            return bail(fail(SSCN_EINVAL, "a batch instance needs the exact whole-line path"));
        b->W = std::max(b->W, tmp[k].W[0]);
        if (params[k].dim == 3)
            b->Wz = std::max(b->Wz, tmp[k].W[2]);
    }
    b->dim3 = params[0].dim == 3;
    const size_t esize = b->precision == SSCN_C128 ? 16 : 8;
    const size_t flds = step2d_lds_elems(kSeg, b->W, kTileR, kTileC) * esize;
    if (!b->dim3 && (b->W > (b->precision == SSCN_C128 ? 20 : 32) || flds > 150 * 1024))
        return bail(fail(SSCN_EINVAL, "the common window of the batch is too large for the fused step"));
    if (b->dim3)
        b->plan = b->active_plan = SSCN_PLAN_SWEEPS;  // the fused step is 2D
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(SSCN_EHIP, "hipStreamCreateWithFlags failed"));
    int poff = 0, ypoff = 0, zoff = 0;
    for (int k = 0; k < n; ++k) {
        sscn_handle &h = tmp[k];
        h.W[0] = h.W[1] = b->W;
        if (b->dim3)
            h.W[2] = b->Wz;
        h.fused_ok = !b->dim3;
        int r = build_tables(&h);
        if (r)
            return bail(r);
        b->p.push_back(h.p);
        b->args.push_back(h.args);
        b->psi.push_back(psi_devs[k]);
        b->tabx.push_back(h.tab[0]);
        b->taby.push_back(h.tab[1]);
        b->tabz.push_back(b->dim3 ? h.tab[2] : nullptr);
        h.tab[0] = h.tab[1] = nullptr;  // owned by the batch now
        if (b->dim3)
            h.tab[2] = nullptr;
        void *w = nullptr;
        const size_t bytes = (size_t)h.npts * esize;
        if (hipMalloc(&w, bytes) != hipSuccess)
            return bail(fail(SSCN_ENOMEM, "hipMalloc of a batch work buffer failed"));
        b->work.push_back(w);
        HIPCHECK(hipMemset(w, 0, bytes));
        const int tx = (h.p.nx - 2) / kTileC + 1, ty = (h.p.ny - 2) / kTileR + 1;
        b->ntiles.push_back(tx * ty);
        b->nchunk.push_back((int)((h.npts + kChunk - 1) / kChunk));
        Inst2D in{};
        in.nx = h.p.nx;
        in.ny = h.p.ny;
        in.tiles_x = tx;
        in.tiles_y = ty;
        in.poff = poff;
        in.active = 1;
        in.hx = h.p.hx;
        in.hy = h.p.hy;
        in.x0 = h.args.x0;
        in.y0 = h.args.y0;
        in.vx = h.args.vx;
        in.vy = h.args.vy;
        in.g = h.p.g;
        in.omega = h.p.omega;
        in.dt = h.p.dt;
        in.dV = h.args.dV;
        in.ax[0] = h.args.ax[0];
        in.ax[1] = h.args.ax[1];
        in.ax[2] = h.args.ax[2];
        in.nz = b->dim3 ? h.p.nz : 1;
        in.hz = h.p.hz;
        in.z0 = h.args.z0;
        in.vz = h.args.vz;
        in.buf[0] = psi_devs[k];
        in.buf[1] = w;
        in.tab[0] = b->tabx.back();
        in.tab[1] = b->taby.back();
        in.tab[2] = b->tabz.back();
        // sweep plan: x-sweep staging as for a single instance (L a power of
        // two), the y tile grid and the offset of this instance's y partials
        const int nseg = (h.p.nx - 2) / kSegX + 1;
        int L = std::max(1, std::min({256 / nseg, 256 * kXLoad / h.p.nx, 512 / (b->W + 2)}));
        while (L & (L - 1))
            L &= L - 1;
        int Lc = L;  // the capped option
        while (Lc > 1 && batch_x_lds(b, k, Lc) > kBatchXLds)
            Lc >>= 1;
        if (nseg > 256 || h.p.nx > 256 * kXLoad || batch_x_lds(b, k, Lc) > kXLdsCap)
            b->sweeps_ok = false;
        if (batch_x_lds(b, k, L) > kXLdsCap)
            L = Lc;
        b->xl_opt[0].push_back(L);
        b->xl_opt[1].push_back(Lc);
        in.xl = Lc;  // set with the work lists by batch_xlines
        in.ygx = (h.p.nx + kYLines - 1) / kYLines;
        in.ygy = ((h.p.ny - 2) / kSeg + 1 + kSegBlock - 1) / kSegBlock;
        in.ypoff = ypoff;
        // 3D: y tiles in every plane, z tiles over the plane's columns; the
        // z-sweep emits the norm partials (offsets shifted past the y ones
        // below), in 2D the y-sweep
        const int planes = b->dim3 ? h.p.nz : 1;
        b->xitems.push_back(0);
        b->yitems.push_back(in.ygx * in.ygy * planes);
        ypoff += in.ygx * in.ygy * planes;
        in.zgx = in.zgy = 0;
        in.zpoff = 0;
        in.eoff = in.ypoff;
        in.ecount = in.ygx * in.ygy;
        if (b->dim3) {
            in.zgx = (int)(((int64_t)h.p.nx * h.p.ny + kYLines - 1) / kYLines);
            in.zgy = ((h.p.nz - 2) / kSeg + 1 + kSegBlock - 1) / kSegBlock;
            in.zpoff = zoff;
            in.eoff = zoff;
            in.ecount = in.zgx * in.zgy;
            zoff += in.zgx * in.zgy;
        }
        b->zitems.push_back(in.zgx * in.zgy);
        b->total_y += b->yitems.back();
        b->total_z += b->zitems.back();
        b->hinst.push_back(in);
        poff += tx * ty;
        b->total_chunks += b->nchunk.back();
    }
    b->total_tiles = poff;
    b->active.assign(n, 1);
    b->conv.assign(n, -1);
    if (b->dim3 && !b->sweeps_ok)
        return bail(fail(SSCN_EINVAL, "the lines of a 3D batch instance are too long to stage"));
    if (b->dim3)
        for (auto &in : b->hinst) {  // the z partials follow all the y ones
            in.zpoff += ypoff;
            in.eoff = in.zpoff;
        }
    for (const auto &in : b->hinst)
        if (in.ecount > kBatchPrescale)
            b->prescale = true;
    if (const char *e = std::getenv("SSCN_BATCH_XLINES"))
        b->xforce = (e[0] == '0') ? 0 : (e[0] == '1') ? 1 : -1;
    for (int o = 0; o < 2; ++o) {
        int64_t items = 0;
        for (int k = 0; k < n; ++k)
            items += batch_x_items(b, k, b->xl_opt[o][k]);
        b->xwork_cap = (int)std::max<int64_t>(b->xwork_cap, items);
    }
    batch_groups(b, esize);
    batch_xlines(b, b->xforce >= 0 ? b->xforce : 1);
    const size_t nopart = std::max((size_t)b->total_chunks * kObsN, (size_t)kRedBlocks);
    if (hipMalloc(&b->d_inst, sizeof(Inst2D) * n) != hipSuccess ||
        hipMalloc(&b->d_work, sizeof(int2) * b->total_tiles) != hipSuccess ||
        hipMalloc(&b->d_fwork, sizeof(int2) * b->total_chunks) != hipSuccess ||
        hipMalloc(&b->d_owork, sizeof(int2) * b->total_chunks) != hipSuccess ||
        hipMalloc(&b->d_nwork, sizeof(int)) != hipSuccess || hipMalloc(&b->d_nf, sizeof(int)) != hipSuccess ||
        hipMalloc(&b->d_no, sizeof(int)) != hipSuccess || hipMalloc(&b->d_obase, sizeof(int) * n) != hipSuccess ||
        hipMalloc(&b->d_ocount, sizeof(int) * n) != hipSuccess ||
        hipMalloc(&b->part[0], sizeof(double) * std::max(b->total_tiles, kRedBlocks)) != hipSuccess ||
        hipMalloc(&b->part[1], sizeof(double) * std::max(b->total_tiles, kRedBlocks)) != hipSuccess ||
        hipMalloc(&b->opart, sizeof(double) * nopart) != hipSuccess ||
        hipMalloc(&b->d_sums, sizeof(double) * (kObsN * n + 2)) != hipSuccess ||
        hipMalloc(&b->d_mu_prev, sizeof(double) * n) != hipSuccess ||
        hipMalloc(&b->d_hits, sizeof(int) * n) != hipSuccess ||
        hipMalloc(&b->d_count_prev, sizeof(int) * n) != hipSuccess ||
        hipMalloc(&b->d_counts, sizeof(int) * n) != hipSuccess ||
        hipMalloc(&b->vpart, sizeof(double) * std::max(b->total_chunks, 1)) != hipSuccess ||
        hipMalloc(&b->d_conv, sizeof(long long) * n) != hipSuccess ||
        hipMalloc(&b->d_xwork, sizeof(int2) * std::max(b->xwork_cap, 1)) != hipSuccess ||
        hipMalloc(&b->d_ywork, sizeof(int2) * std::max(b->total_y, 1)) != hipSuccess ||
        hipMalloc(&b->d_nx, sizeof(int) * b->ngroups) != hipSuccess ||
        hipMalloc(&b->d_ny, sizeof(int) * b->ngroups) != hipSuccess ||
        hipMalloc(&b->d_klist, sizeof(int) * n) != hipSuccess || hipMalloc(&b->d_nk, sizeof(int)) != hipSuccess ||
        hipMalloc(&b->ypart, sizeof(double) * std::max(b->total_y + b->total_z, 1)) != hipSuccess ||
        hipMalloc(&b->d_zwork, sizeof(int2) * std::max(b->total_z, 1)) != hipSuccess ||
        hipMalloc(&b->d_nzl, sizeof(int)) != hipSuccess ||
        hipMalloc(&b->d_scale, sizeof(double) * n) != hipSuccess)
        return bail(fail(SSCN_ENOMEM, "hipMalloc of the batch buffers failed"));
    HIPCHECK(hipMemcpy(b->d_inst, b->hinst.data(), sizeof(Inst2D) * n, hipMemcpyHostToDevice));
    int r = sscn_batch_reset(b);
    if (r)
        return bail(r);
    hipError_t e = b->precision == SSCN_C128 ? allow_fused_lds_all<double>(b->W) : allow_fused_lds_all<float>(b->W);
    if (e == hipSuccess && b->sweeps_ok)
        e = b->precision == SSCN_C128 ? batch_allow_x_lds_all<double>(b->W) : batch_allow_x_lds_all<float>(b->W);
    if (e != hipSuccess)
        return bail(fail(SSCN_EHIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e)));
    *out = b;
    return 0;
}

int sscn_batch_reset(sscn_batch *b)
{
    if (!b)
        return fail(SSCN_EINVAL, "null argument");
    b->active.assign(b->n, 1);
    b->conv.assign(b->n, -1);
    std::vector<double> nan(b->n, std::nan(""));
    std::vector<int> zero(b->n, 0);
    std::vector<long long> neg(b->n, -1);
    HIPCHECK(hipMemcpy(b->d_mu_prev, nan.data(), sizeof(double) * b->n, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(b->d_hits, zero.data(), sizeof(int) * b->n, hipMemcpyHostToDevice));
    std::vector<int> none(b->n, -1);
    HIPCHECK(hipMemcpy(b->d_count_prev, none.data(), sizeof(int) * b->n, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(b->d_counts, none.data(), sizeof(int) * b->n, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(b->d_conv, neg.data(), sizeof(long long) * b->n, hipMemcpyHostToDevice));
    return batch_lists(b);
}

int sscn_batch_init_state(sscn_batch *b, int k, int kind, const double *phase_host, double d_xy)
{
    if (!b || k < 0 || k >= b->n || (kind != 0 && kind != 1) || !(d_xy > 0))
        return fail(SSCN_EINVAL, "bad batch_init_state arguments");
    const sscn_params &p = b->p[k];
    const StepArgs &a = b->args[k];
    const int64_t plane = (int64_t)p.nx * p.ny;
    const int64_t npts = plane * (p.dim == 3 ? p.nz : 1);
    const double d_z = p.dim == 3 ? 1.0 / std::sqrt(p.lambda) : 0.0;
    const double *ph = nullptr;
    if (phase_host) {
        if (b->phase)
            (void)hipFree(b->phase);
        b->phase = nullptr;
        if (hipMalloc(&b->phase, sizeof(double) * plane) != hipSuccess)
            return fail(SSCN_ENOMEM, "hipMalloc of the phase buffer failed");
        HIPCHECK(hipMemcpy(b->phase, phase_host, sizeof(double) * plane, hipMemcpyHostToDevice));
        ph = b->phase;
    }
    const int nb = red_blocks(npts);
    if (b->precision == SSCN_C128) {
        hipLaunchKernelGGL((k_init<double>), dim3(nb), dim3(256), 0, b->stream, (V<double> *)b->psi[k], a, kind, ph,
                           d_xy, d_z, 0, (uint64_t)0);
        hipLaunchKernelGGL((k_norm_partials<double>), dim3(kRedBlocks), dim3(256), 0, b->stream,
                           (const V<double> *)b->psi[k], npts, b->opart);
        hipLaunchKernelGGL((k_rescale<double>), dim3(nb), dim3(256), 0, b->stream, (const V<double> *)b->psi[k],
                           (V<double> *)b->psi[k], npts, a.dV, b->opart, kRedBlocks, 0);
    } else {
        hipLaunchKernelGGL((k_init<float>), dim3(nb), dim3(256), 0, b->stream, (V<float> *)b->psi[k], a, kind, ph,
                           d_xy, d_z, 0, (uint64_t)0);
        hipLaunchKernelGGL((k_norm_partials<float>), dim3(kRedBlocks), dim3(256), 0, b->stream,
                           (const V<float> *)b->psi[k], npts, b->opart);
        hipLaunchKernelGGL((k_rescale<float>), dim3(nb), dim3(256), 0, b->stream, (const V<float> *)b->psi[k],
                           (V<float> *)b->psi[k], npts, a.dV, b->opart, kRedBlocks, 0);
    }
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(b->stream));
    return 0;
}

int sscn_batch_prepare_steps(sscn_batch *b, int64_t nsteps)
{
    if (!b || nsteps < 0)
        return fail(SSCN_EINVAL, "bad batch_prepare_steps arguments");
    int r = batch_autotune(b);
    if (!r && nsteps >= 2)
        r = batch_run_step_graphs(b, nsteps, false);
    if (r)
        return r;
    HIPCHECK(hipStreamSynchronize(b->stream));
    return 0;
}

int sscn_batch_step(sscn_batch *b, int64_t nsteps)
{
    if (!b || nsteps < 0)
        return fail(SSCN_EINVAL, "bad batch_step arguments");
    if (nsteps == 0)
        return 0;
    int r = batch_autotune(b);
    if (r)
        return r;
    if (nsteps >= 2) {
        r = batch_run_step_graphs(b, nsteps, true);
        if (r)
            return r;
    } else if (b->precision == SSCN_C128) {
        batch_enqueue<double>(b, nsteps, b->stream, b->grid_tiles, b->grid_chunks, false);
    } else {
        batch_enqueue<float>(b, nsteps, b->stream, b->grid_tiles, b->grid_chunks, false);
    }
    HIPCHECK(hipGetLastError());
    b->steps += nsteps;
    return 0;
}

int sscn_batch_profile_step(sscn_batch *b, int64_t nsteps, double *ms_out)
{
    if (!b || !ms_out || nsteps < 1 || nsteps > 100000)
        return fail(SSCN_EINVAL, "bad batch_profile_step arguments");
    int r = batch_autotune(b);
    if (r)
        return r;
    // the sweep plan runs the steps group by group: 4 events per step and group
    const int64_t nrec = nsteps * (b->active_plan == SSCN_PLAN_SWEEPS ? b->ngroups : 1);
    std::vector<hipEvent_t> ev((size_t)nrec * 4, nullptr);
    int rc = 0;
    for (auto &e : ev)
        if (timing_event(&e) != hipSuccess) {
            rc = fail(SSCN_EHIP, "hipEventCreate failed");
            break;
        }
    if (!rc) {
        if (b->precision == SSCN_C128)
            batch_enqueue<double>(b, nsteps, b->stream, b->grid_tiles, b->grid_chunks, false, ev.data());
        else
            batch_enqueue<float>(b, nsteps, b->stream, b->grid_tiles, b->grid_chunks, false, ev.data());
        b->steps += nsteps;
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(b->stream) != hipSuccess)
            rc = fail(SSCN_EHIP, "the profiled batch steps failed");
    }
    double acc[4] = {0, 0, 0, 0};
    for (int64_t s = 0; s < nrec && !rc; ++s) {
        const hipEvent_t *e = &ev[(size_t)s * 4];
        float t01 = 0, t12 = 0, t23 = 0, t03 = 0;
        if (hipEventElapsedTime(&t01, e[0], e[1]) != hipSuccess || hipEventElapsedTime(&t12, e[1], e[2]) != hipSuccess ||
            hipEventElapsedTime(&t23, e[2], e[3]) != hipSuccess || hipEventElapsedTime(&t03, e[0], e[3]) != hipSuccess)
            rc = fail(SSCN_EHIP, "hipEventElapsedTime failed");
        acc[0] += t01;
        acc[1] += t12;
        acc[2] += t23;
        acc[3] += t03;
    }
    if (!rc) {
        const double n = (double)nsteps;
        if (b->active_plan == SSCN_PLAN_SWEEPS) {
            ms_out[0] = acc[0] / n;  // x-sweep
            ms_out[1] = acc[1] / n;  // y-sweep
            ms_out[2] = acc[2] / n;  // z-sweep (3D; 0 in 2D)
        } else {
            ms_out[0] = acc[0] / n;  // fused step
            ms_out[1] = ms_out[2] = 0.0;
        }
        ms_out[3] = acc[3] / n;
    }
    for (auto &e : ev)
        if (e)
            (void)hipEventDestroy(e);
    return rc;
}

int sscn_batch_observables(sscn_batch *b, sscn_obs *out)
{
    if (!b || !out)
        return fail(SSCN_EINVAL, "null argument");
    int r = batch_lists(b, true);
    if (r)
        return r;
    if (b->precision == SSCN_C128)
        batch_obs_launch<double>(b, b->total_chunks, 0.0);
    else
        batch_obs_launch<float>(b, b->total_chunks, 0.0);
    std::vector<double> sums((size_t)kObsN * b->n);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(sums.data(), b->d_sums, sizeof(double) * kObsN * b->n, hipMemcpyDeviceToHost,
                            b->stream));
    HIPCHECK(hipStreamSynchronize(b->stream));
    r = batch_lists(b);
    if (r)
        return r;
    int rc = 0;
    for (int k = 0; k < b->n; ++k) {
        double s[kObsN];
        std::memcpy(s, &sums[(size_t)kObsN * k], sizeof s);
        const double dV = b->args[k].dV;
        for (int t = 0; t < kObsN; ++t)
            if (t != 13)
                s[t] *= dV;
        sscn_obs &o = out[k];
        std::memset(&o, 0, sizeof o);
        std::memcpy(o.sums, s, sizeof s);
        o.norm = s[0];
        o.mu = (s[2] + s[3] + s[4] + s[5]) / s[1];
        o.energy = (s[2] + s[3] + 0.5 * s[4] + s[5]) / s[1];
        o.mu_full = (s[6] + s[7] + s[8] + s[9]) / s[0];
        o.energy_full = (s[6] + s[7] + 0.5 * s[8] + s[9]) / s[0];
        o.mu_4th = (s[14] + s[7] + s[8] + s[15]) / s[0];
        o.energy_4th = (s[14] + s[7] + 0.5 * s[8] + s[15]) / s[0];
        o.rms_x = std::sqrt(s[10] / s[0]);
        o.rms_y = std::sqrt(s[11] / s[0]);
        o.rms_z = std::sqrt(s[12] / s[0]);  // 0 in 2D (z = 0)
        o.rms_r = std::sqrt((s[10] + s[11] + s[12]) / s[0]);
        o.max_density = s[13];
        o.step = b->conv[k] >= 0 ? b->conv[k] : b->steps;
        for (int t = 0; t < kObsN; ++t)
            if (!std::isfinite(s[t]))
                rc = fail(SSCN_ENONFINITE, "non-finite reduction in the batch observables");
    }
    return rc;
}

int sscn_batch_run(sscn_batch *b, int64_t max_steps, int check_every, double tol_dmu, int64_t *steps_out)
{
    if (!b || max_steps < 0 || check_every < 2 || !(tol_dmu > 0))
        return fail(SSCN_EINVAL, "bad batch_run arguments");
    const int K = check_every + (check_every & 1);
    int r = batch_autotune(b);
    if (r)
        return r;
    r = batch_graph(b, K);
    if (r)
        return r;
    int64_t done = 0;
    std::vector<long long> cv(b->n);
    while (done < max_steps) {
        int nact = 0;
        for (char a : b->active)
            nact += a;
        if (!nact)
            break;
        HIPCHECK(hipGraphLaunch(b->gexec, b->stream));
        b->steps += K;
        done += K;
        if (b->precision == SSCN_C128)
            batch_obs_launch<double>(b, b->total_chunks, tol_dmu);
        else
            batch_obs_launch<float>(b, b->total_chunks, tol_dmu);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipMemcpyAsync(cv.data(), b->d_conv, sizeof(long long) * b->n, hipMemcpyDeviceToHost, b->stream));
        HIPCHECK(hipStreamSynchronize(b->stream));
        bool changed = false;
        for (int k = 0; k < b->n; ++k)
            if (b->active[k] && cv[k] >= 0) {
                b->active[k] = 0;
                b->conv[k] = cv[k];
                changed = true;
            }
        if (changed) {
            r = batch_lists(b);
            if (r)
                return r;
        }
    }
    if (steps_out)
        for (int k = 0; k < b->n; ++k)
            steps_out[k] = b->conv[k];
    return 0;
}

int sscn_batch_get_state(sscn_batch *b, int k, void *host_psi)
{
    if (!b || k < 0 || k >= b->n || !host_psi)
        return fail(SSCN_EINVAL, "bad batch_get_state arguments");
    const size_t bytes = (size_t)npoints(b->p[k]) * (b->precision == SSCN_C128 ? 16 : 8);
    HIPCHECK(hipMemcpyAsync(host_psi, b->psi[k], bytes, hipMemcpyDeviceToHost, b->stream));
    HIPCHECK(hipStreamSynchronize(b->stream));
    return 0;
}

int sscn_batch_set_state_device(sscn_batch *b, int k)
{
    if (!b || k < 0 || k >= b->n)
        return fail(SSCN_EINVAL, "bad batch_set_state_device arguments");
    const StepArgs &a = b->args[k];
    const int64_t npts = npoints(b->p[k]);
    const int nb = red_blocks(npts);
    if (b->precision == SSCN_C128) {
        V<double> *psi = (V<double> *)b->psi[k];
        hipLaunchKernelGGL((k_zero_walls<double>), dim3(nb), dim3(256), 0, b->stream, psi, a);
        hipLaunchKernelGGL((k_norm_partials<double>), dim3(kRedBlocks), dim3(256), 0, b->stream,
                           (const V<double> *)psi, npts, b->opart);
        hipLaunchKernelGGL((k_rescale<double>), dim3(nb), dim3(256), 0, b->stream, (const V<double> *)psi, psi, npts,
                           a.dV, b->opart, kRedBlocks, 0);
    } else {
        V<float> *psi = (V<float> *)b->psi[k];
        hipLaunchKernelGGL((k_zero_walls<float>), dim3(nb), dim3(256), 0, b->stream, psi, a);
        hipLaunchKernelGGL((k_norm_partials<float>), dim3(kRedBlocks), dim3(256), 0, b->stream,
                           (const V<float> *)psi, npts, b->opart);
        hipLaunchKernelGGL((k_rescale<float>), dim3(nb), dim3(256), 0, b->stream, (const V<float> *)psi, psi, npts,
                           a.dV, b->opart, kRedBlocks, 0);
    }
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(b->stream));
    return 0;
}

int sscn_batch_vortex_count(sscn_batch *b, int k, double density_frac, int box, int *count)
{
    if (!b || k < 0 || k >= b->n || !count || box < 0 || !(density_frac >= 0))
        return fail(SSCN_EINVAL, "bad batch_vortex_count arguments");
    const sscn_params &p = b->p[k];
    const StepArgs &a = b->args[k];
    double *out = b->d_sums + (size_t)kObsN * b->n;  // two doubles past the observable sums
    const int k0 = p.dim == 3 ? p.nz / 2 : 0;           // 3D: the z = 0 plane, as sscn_vortex_count
    const int nb = red_blocks((int64_t)p.nx * p.ny);
    const int nbv = red_blocks((int64_t)(p.nx - 1) * (p.ny - 1));
    if (b->precision == SSCN_C128) {
        hipLaunchKernelGGL((k_plane_max<double>), dim3(nb), dim3(256), 0, b->stream, (const V<double> *)b->psi[k], a,
                           k0, b->opart);
        hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, b->stream, b->opart, nb, 1, 1u, out);
        hipLaunchKernelGGL((k_vortex<double>), dim3(nbv), dim3(256), 0, b->stream, (const V<double> *)b->psi[k], a, k0,
                           density_frac, box, out, b->opart);
    } else {
        hipLaunchKernelGGL((k_plane_max<float>), dim3(nb), dim3(256), 0, b->stream, (const V<float> *)b->psi[k], a,
                           k0, b->opart);
        hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, b->stream, b->opart, nb, 1, 1u, out);
        hipLaunchKernelGGL((k_vortex<float>), dim3(nbv), dim3(256), 0, b->stream, (const V<float> *)b->psi[k], a, k0,
                           density_frac, box, out, b->opart);
    }
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, b->stream, b->opart, nbv, 1, 0u, out + 1);
    double c = 0.0;
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(&c, out + 1, sizeof c, hipMemcpyDeviceToHost, b->stream));
    HIPCHECK(hipStreamSynchronize(b->stream));
    *count = (int)c;
    return 0;
}

int sscn_batch_set_plan(sscn_batch *b, int plan)
{
    if (!b || plan < SSCN_PLAN_AUTO || plan > SSCN_PLAN_FUSED)
        return fail(SSCN_EINVAL, "bad plan");
    if (plan == SSCN_PLAN_SWEEPS && !b->sweeps_ok)
        return fail(SSCN_EINVAL, "the batched sweep plan is not available for these instances");
    if (b->dim3 && plan == SSCN_PLAN_FUSED)
        return fail(SSCN_EINVAL, "a 3D batch steps with the sweep plan only");
    HIPCHECK(hipStreamSynchronize(b->stream));
    batch_drop_graph(b);
    if (b->dim3)
        plan = SSCN_PLAN_SWEEPS;
    b->plan = plan;
    b->active_plan = plan == SSCN_PLAN_SWEEPS ? SSCN_PLAN_SWEEPS : SSCN_PLAN_FUSED;
    return 0;
}

int sscn_batch_x_lines(sscn_batch *b, int *option, float *tune_ms)
{
    if (!b || !option)
        return fail(SSCN_EINVAL, "null argument");
    *option = b->xsel;
    if (tune_ms) {
        tune_ms[0] = b->tune_x_ms[0];
        tune_ms[1] = b->tune_x_ms[1];
    }
    return 0;
}

int sscn_batch_info(sscn_batch *b, int *plan, int *window)
{
    if (!b)
        return fail(SSCN_EINVAL, "null argument");
    if (plan)
        *plan = b->plan == SSCN_PLAN_AUTO ? SSCN_PLAN_AUTO : b->active_plan;
    if (window)
        *window = b->W;
    return 0;
}

void sscn_batch_destroy(sscn_batch *b)
{
    if (!b)
        return;
    (void)hipStreamSynchronize(b->stream);
    batch_free(b);
    delete b;
}

}  // extern "C"
