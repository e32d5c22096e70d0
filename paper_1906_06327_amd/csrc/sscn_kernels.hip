// Kernel launchers of the solver, compiled once per (part, precision):
// SSCN_PART 1 = the x-, y- and z-sweeps, 2, 4 and 5 = the fused 2D step
// with tile shapes 0, 1 and 2 (kFusedTileR x kFusedTileC), 3 = the batched
// sweeps; SSCN_REAL_T = double or float.  Each compilation
// explicitly instantiates its part's launchers (declared in sscn_host.hpp)
// for one precision.
#include "sscn_host.hpp"

#if !defined(SSCN_PART) || !defined(SSCN_REAL_T)
#error "compile with -DSSCN_PART=1|2|3|4|5 -DSSCN_REAL_T=double|float"
#endif

namespace sscn {

// Raise the dynamic-LDS limit of an x-sweep kernel to kXLdsCap (the default
// limit is 64 KiB).
inline hipError_t allow_x_lds(const void *kernel)
{
    return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kXLdsCap);
}

#if SSCN_PART == 1

template <class R, int W, bool RT>
void go_x(const sscn_handle *h, const void *src, void *dst, int npart, hipStream_t st, bool reduce)
{
    const int nlines = h->p.ny * (h->p.dim == 3 ? h->p.nz : 1);
    const int groups = (nlines + h->xL - 1) / h->xL;
    double *sm1 = nullptr;
    if (!RT && npart > 0) {
        sm1 = h->obs_buf + kScaleSlot;
        if (reduce)
            hipLaunchKernelGGL(k_norm_scale, dim3(1), dim3(256), 0, st, h->partials, npart, h->args.dV, sm1);
    }
    if ((int64_t)h->p.nx * h->xL <= 256 * 8)
        hipLaunchKernelGGL((k_xsweep<R, kSegX, W, RT, 8>), dim3(groups), dim3(256), h->xlds, st, (const V<R> *)src,
                           (V<R> *)dst, h->args, h->xL, (const double *)sm1, (const Cx<R> *)h->tab[0]);
    else
        hipLaunchKernelGGL((k_xsweep<R, kSegX, W, RT, kXLoad>), dim3(groups), dim3(256), h->xlds, st,
                           (const V<R> *)src, (V<R> *)dst, h->args, h->xL, (const double *)sm1,
                           (const Cx<R> *)h->tab[0]);
}

template <class R, bool RT>
void launch_x(const sscn_handle *h, const void *src, void *dst, int npart, hipStream_t st, bool reduce)
{
#define SSCN_CALL_X(Wc) go_x<R, Wc, RT>(h, src, dst, npart, st, reduce)
    SSCN_W_SWITCH(h->W[0], SSCN_CALL_X)
#undef SSCN_CALL_X
}

template <class R, int W, bool EMIT>
void go_y(const sscn_handle *h, const void *src, void *dst, hipStream_t st)
{
    const int *g = h->ygrid;
    hipLaunchKernelGGL((k_ysweep<R, kSeg, W, EMIT>), dim3(round8((int64_t)g[0] * g[1] * g[2])), dim3(kYLines, kSegBlock), 0,
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
    hipLaunchKernelGGL((k_zsweep<R, kSeg, W, EMIT>), dim3(round8((int64_t)g[0] * g[1])), dim3(kYLines, kSegBlock), 0, st,
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

template <class R, int W>
hipError_t allow_x_lds_w()
{
    hipError_t e = allow_x_lds((const void *)k_xsweep<R, kSegX, W, false, 8>);
    if (e == hipSuccess)
        e = allow_x_lds((const void *)k_xsweep<R, kSegX, W, false, kXLoad>);
    if (e == hipSuccess)
        e = allow_x_lds((const void *)k_xsweep<R, kSegX, W, true, 8>);
    if (e == hipSuccess)
        e = allow_x_lds((const void *)k_xsweep<R, kSegX, W, true, kXLoad>);
    return e;
}

template <class R>
hipError_t allow_x_lds_all(int W)
{
    hipError_t e = hipSuccess;
#define SSCN_CALL_A(Wc) e = allow_x_lds_w<R, Wc>()
    SSCN_W_SWITCH(W, SSCN_CALL_A)
#undef SSCN_CALL_A
    return e;
}

template void launch_x<SSCN_REAL_T, false>(const sscn_handle *, const void *, void *, int, hipStream_t, bool);
template hipError_t allow_x_lds_all<SSCN_REAL_T>(int);
template void launch_x<SSCN_REAL_T, true>(const sscn_handle *, const void *, void *, int, hipStream_t, bool);
template void launch_y<SSCN_REAL_T, false>(const sscn_handle *, const void *, void *, hipStream_t);
template void launch_y<SSCN_REAL_T, true>(const sscn_handle *, const void *, void *, hipStream_t);
template void launch_z<SSCN_REAL_T, false>(const sscn_handle *, const void *, void *, hipStream_t);
template void launch_z<SSCN_REAL_T, true>(const sscn_handle *, const void *, void *, hipStream_t);

#elif SSCN_PART == 2 || SSCN_PART == 4 || SSCN_PART == 5

// The tile shape of this compilation: 0 (part 2), 1 (part 4) or 2 (part 5).
// The launchers below have the same names in every compilation, so they
// are kept local to each (an unnamed namespace): otherwise the linker would
// keep one compilation's instances for every tile shape.
constexpr int kPartTile = SSCN_PART == 2 ? 0 : SSCN_PART == 4 ? 1 : 2;
constexpr int kPartTileR = kFusedTileR[kPartTile];
constexpr int kPartTileC = kFusedTileC[kPartTile];

namespace {

template <class R, int W, bool RT>
void go_fused(const FusedLaunch &f, int parity, const double *pin, double *pout, int use_pin, hipStream_t st)
{
    constexpr size_t lds = step2d_lds_bytes<R, kSeg, W, kPartTileR, kPartTileC>();
    if (f.one)  // one block per tile, the grid rounded up to the 8 XCDs (see k_step2d)
        hipLaunchKernelGGL((k_step2d<R, kSeg, W, kPartTileR, kPartTileC, kTileNT, RT, true>), dim3(round8(f.grid)),
                           dim3(kTileNT),
                           lds, st, f.inst, f.work, f.nwork, *f.one, parity, pin, pout, use_pin);
    else
        hipLaunchKernelGGL((k_step2d<R, kSeg, W, kPartTileR, kPartTileC, kTileNT, RT, false>), dim3(round8(f.grid)), dim3(kTileNT),
                           lds, st, f.inst, f.work, f.nwork, Inst2D{}, parity, pin, pout, use_pin);
}

template <class R, bool RT>
void launch_fused_tile(const FusedLaunch &f, int parity, const double *pin, double *pout, int use_pin,
                       hipStream_t st)
{
#define SSCN_CALL_F(Wc) go_fused<R, Wc, RT>(f, parity, pin, pout, use_pin, st)
    if constexpr (std::is_same<R, float>::value) {
        if (f.W > 20) {
            if (f.W <= 24)
                go_fused<R, 24, RT>(f, parity, pin, pout, use_pin, st);
            else
                go_fused<R, 32, RT>(f, parity, pin, pout, use_pin, st);
            return;
        }
    }
    SSCN_W_SWITCH_FUSED(R, f.W, SSCN_CALL_F)
#undef SSCN_CALL_F
}

template <class R, int W, bool RT>
hipError_t allow_fused_lds()
{
    constexpr size_t lds = step2d_lds_bytes<R, kSeg, W, kPartTileR, kPartTileC>();
    hipError_t e = hipFuncSetAttribute((const void *)k_step2d<R, kSeg, W, kPartTileR, kPartTileC, kTileNT, RT, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_step2d<R, kSeg, W, kPartTileR, kPartTileC, kTileNT, RT, false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return e;
}

template <class R>
hipError_t allow_fused_lds_tile(int W)
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

}  // namespace

#if SSCN_PART == 2
// The dispatcher over the two tile shapes (FusedLaunch::tile).
template <class R, bool RT>
void launch_fused(const FusedLaunch &f, int parity, const double *pin, double *pout, int use_pin, hipStream_t st)
{
    if (f.tile == 1)
        launch_fused_narrow<R, RT>(f, parity, pin, pout, use_pin, st);
    else if (f.tile == 2)
        launch_fused_small<R, RT>(f, parity, pin, pout, use_pin, st);
    else
        launch_fused_tile<R, RT>(f, parity, pin, pout, use_pin, st);
}

template <class R>
hipError_t allow_fused_lds_all(int W)
{
    hipError_t e = allow_fused_lds_tile<R>(W);
    if (e == hipSuccess)
        e = allow_fused_lds_narrow<R>(W);
    return e == hipSuccess ? allow_fused_lds_small<R>(W) : e;
}

template void launch_fused<SSCN_REAL_T, false>(const FusedLaunch &, int, const double *, double *, int, hipStream_t);
template void launch_fused<SSCN_REAL_T, true>(const FusedLaunch &, int, const double *, double *, int, hipStream_t);
template hipError_t allow_fused_lds_all<SSCN_REAL_T>(int);
#elif SSCN_PART == 4
template <class R, bool RT>
void launch_fused_narrow(const FusedLaunch &f, int parity, const double *pin, double *pout, int use_pin,
                         hipStream_t st)
{
    launch_fused_tile<R, RT>(f, parity, pin, pout, use_pin, st);
}

template <class R>
hipError_t allow_fused_lds_narrow(int W)
{
    return allow_fused_lds_tile<R>(W);
}

template void launch_fused_narrow<SSCN_REAL_T, false>(const FusedLaunch &, int, const double *, double *, int,
                                                      hipStream_t);
template void launch_fused_narrow<SSCN_REAL_T, true>(const FusedLaunch &, int, const double *, double *, int,
                                                     hipStream_t);
template hipError_t allow_fused_lds_narrow<SSCN_REAL_T>(int);
#else
template <class R, bool RT>
void launch_fused_small(const FusedLaunch &f, int parity, const double *pin, double *pout, int use_pin,
                        hipStream_t st)
{
    launch_fused_tile<R, RT>(f, parity, pin, pout, use_pin, st);
}

template <class R>
hipError_t allow_fused_lds_small(int W)
{
    return allow_fused_lds_tile<R>(W);
}

template void launch_fused_small<SSCN_REAL_T, false>(const FusedLaunch &, int, const double *, double *, int,
                                                     hipStream_t);
template void launch_fused_small<SSCN_REAL_T, true>(const FusedLaunch &, int, const double *, double *, int,
                                                    hipStream_t);
template hipError_t allow_fused_lds_small<SSCN_REAL_T>(int);
#endif

#elif SSCN_PART == 3

template <class R, int W, bool RT>
void go_batch_x(const sscn_batch *b, int g, int grid, int use_scale, hipStream_t st)
{
    const int2 *work = b->d_xwork + b->gx_off[g];
    if (b->xshort)
        hipLaunchKernelGGL((k_batch_xsweep<R, kSegX, W, RT, 8>), dim3(std::max(grid, 1)), dim3(256), b->xlds, st,
                           b->d_inst, work, b->d_nx + g, (const double *)b->ypart, use_scale,
                           (const double *)b->d_scale);
    else
        hipLaunchKernelGGL((k_batch_xsweep<R, kSegX, W, RT, kXLoad>), dim3(std::max(grid, 1)), dim3(256), b->xlds, st,
                           b->d_inst, work, b->d_nx + g, (const double *)b->ypart, use_scale,
                           (const double *)b->d_scale);
}

template <class R, int W, bool EMIT>
void go_batch_y(const sscn_batch *b, int g, int grid, hipStream_t st)
{
    // one block per item on a grid of whole XCD rounds (xcd_item)
    hipLaunchKernelGGL((k_batch_ysweep<R, kSeg, W, EMIT>), dim3(round8(std::max(grid, 1))), dim3(kYLines, kSegBlock), 0,
                       st, b->d_inst, b->d_ywork + b->gy_off[g], b->d_ny + g, b->ypart);
}

template <class R, int W, bool EMIT>
void go_batch_z(const sscn_batch *b, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_batch_zsweep<R, kSeg, W, EMIT>), dim3(round8(std::max(grid, 1))), dim3(kYLines, kSegBlock), 0,
                       st, b->d_inst, b->d_zwork, b->d_nzl, b->ypart);
}

// One step of the sweep plan for the listed instances of group g (state in
// buf[0]); all: launch grids covering every instance of the group (graph
// capture), else the current list lengths.  The x-sweep forms the pending
// rescale itself, or, where an instance has many norm partials
// (sscn_batch::prescale), reads it from k_batch_scale, which sums them once
// per instance first.  A batch of 3D instances adds the z-sweep.  ev
// (optional, 4 events): recorded before the rescale reduction and x-sweep,
// before the y-sweep, after it (before the z-sweep) and at the end of the
// step.
template <class R>
void batch_sweep_step(sscn_batch *b, hipStream_t st, int g, bool all, hipEvent_t *ev)
{
    const int grid_x = all ? b->gx_tot[g] : b->gx_cnt[g];
    const int grid_y = all ? b->gy_tot[g] : b->gy_cnt[g];
    auto mark = [&](int t) {
        if (ev)
            (void)hipEventRecord(ev[t], st);
    };
    const bool imag = b->mode == SSCN_IMAG;
    const int sc = (imag && b->pending) ? (b->prescale ? 2 : 1) : 0;
    mark(0);
    if (sc == 2) {
        const int grid_k = all ? b->n : b->grid_k;
        hipLaunchKernelGGL(k_batch_scale, dim3(std::max(grid_k, 1)), dim3(256), 0, st, b->d_inst, b->d_klist, b->d_nk,
                           (const double *)b->ypart, b->d_scale);
    }
#define SSCN_CALL_BX(Wc)                                 \
    do {                                                 \
        if (imag)                                        \
            go_batch_x<R, Wc, false>(b, g, grid_x, sc, st); \
        else                                                \
            go_batch_x<R, Wc, true>(b, g, grid_x, 0, st);   \
    } while (0)
    SSCN_W_SWITCH(b->W, SSCN_CALL_BX);
#undef SSCN_CALL_BX
    mark(1);
    // the last sweep emits the norm partials: y in 2D, z in 3D
    const bool emit_y = imag && !b->dim3;
#define SSCN_CALL_BY(Wc)                             \
    do {                                             \
        if (emit_y)                                  \
            go_batch_y<R, Wc, true>(b, g, grid_y, st);  \
        else                                            \
            go_batch_y<R, Wc, false>(b, g, grid_y, st); \
    } while (0)
    SSCN_W_SWITCH(b->W, SSCN_CALL_BY);
#undef SSCN_CALL_BY
    mark(2);
    if (b->dim3) {
        const int grid_z = all ? b->total_z : b->grid_z;
#define SSCN_CALL_BZ(Wc)                              \
    do {                                              \
        if (imag)                                     \
            go_batch_z<R, Wc, true>(b, grid_z, st);   \
        else                                          \
            go_batch_z<R, Wc, false>(b, grid_z, st);  \
    } while (0)
        SSCN_W_SWITCH(b->Wz, SSCN_CALL_BZ);
#undef SSCN_CALL_BZ
    }
    mark(3);
    if (imag)
        b->pending = true;
}

template <class R, int W>
hipError_t batch_allow_x_lds_w()
{
    hipError_t e = allow_x_lds((const void *)k_batch_xsweep<R, kSegX, W, false, 8>);
    if (e == hipSuccess)
        e = allow_x_lds((const void *)k_batch_xsweep<R, kSegX, W, false, kXLoad>);
    if (e == hipSuccess)
        e = allow_x_lds((const void *)k_batch_xsweep<R, kSegX, W, true, 8>);
    if (e == hipSuccess)
        e = allow_x_lds((const void *)k_batch_xsweep<R, kSegX, W, true, kXLoad>);
    return e;
}

template <class R>
hipError_t batch_allow_x_lds_all(int W)
{
    hipError_t e = hipSuccess;
#define SSCN_CALL_A(Wc) e = batch_allow_x_lds_w<R, Wc>()
    SSCN_W_SWITCH(W, SSCN_CALL_A)
#undef SSCN_CALL_A
    return e;
}

template void batch_sweep_step<SSCN_REAL_T>(sscn_batch *, hipStream_t, int, bool, hipEvent_t *);
template hipError_t batch_allow_x_lds_all<SSCN_REAL_T>(int);

#endif

}  // namespace sscn
