// Host-side definitions shared by the library's translation units: tuning
// constants, the solver and batch handles, the window-size dispatch and the
// kernel launchers.  The launchers are templates defined in sscn_kernels.hip,
// which is compiled once per (part, precision) so that the many window-size
// instantiations of the sweep and fused-step kernels build in parallel.
#pragma once

#include "sscn.h"
#include "sscn_device.hpp"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

using namespace sscn;

namespace sscn {

constexpr int kSeg = 8;             // outputs per thread segment (y, z and the fused step)
#ifndef SSCN_SEGX
#define SSCN_SEGX 8
#endif
constexpr int kSegX = SSCN_SEGX;    // outputs per thread segment of the x-sweeps
constexpr int kGraphSteps = 64;     // most steps per captured graph (single instance)
constexpr int kBatchGraphSteps = 256;  // most steps per captured graph (batch)
constexpr size_t kGraphCache = 4;   // graphs of different step counts kept per handle
constexpr int kRedBlocks = 1024;    // blocks of the grid-stride reductions
#ifndef SSCN_TILE_R
#define SSCN_TILE_R 32
#endif
#ifndef SSCN_TILE_C
#define SSCN_TILE_C 32
#endif
#ifndef SSCN_TILE_NT
#define SSCN_TILE_NT 256
#endif
constexpr int kTileR = SSCN_TILE_R;   // fused 2D step: output tile rows (y)
constexpr int kTileC = SSCN_TILE_C;   // and columns (x)
// The tile shapes of a single instance's fused step (FusedLaunch::tile):
// 0 kTileR x kTileC; 1 kTileR x kTileCn (twice the tiles of half the width,
// for grids whose wide tiles leave most CUs idle or whose real-time step is
// issue-bound); 2 16 x 16 (small grids).  The autotuner times them all.
#ifndef SSCN_TILE_CN
#define SSCN_TILE_CN 16
#endif
constexpr int kTileCn = SSCN_TILE_CN;
constexpr int kFusedTiles = 3;
constexpr int kFusedTileR[kFusedTiles] = {kTileR, kTileR, 16};
constexpr int kFusedTileC[kFusedTiles] = {kTileC, kTileCn, 16};
constexpr int kTileNT = SSCN_TILE_NT; // threads per tile block
constexpr size_t kXLdsCap = 150 * 1024;  // dynamic LDS of an x-sweep block
// Dynamic LDS of a batched x-sweep block at most (bytes) under the capped
// lines-per-block option: every instance's lines per block are halved until
// its staging fits, so that the launch (which reserves the largest
// instance's LDS for every block) holds four blocks of 256 threads per CU in
// the 160 KiB.  Halving leaves some of a block's threads without a segment
// to solve, so the batch autotuner times both options.  SSCN_BATCH_XLDS
// overrides the cap.
#ifndef SSCN_BATCH_XLDS
#define SSCN_BATCH_XLDS 40960
#endif
constexpr size_t kBatchXLds = SSCN_BATCH_XLDS;
// Norm partials of an instance above which the batched x-sweep reads its
// pending rescale from a per-instance reduction (k_batch_scale) instead of
// summing the partials in every block: each wave of an x-sweep block reads
// all of them, which for the 2048 z tiles of a 256 x 256 x 64 instance is
// four times the block's own state.
#ifndef SSCN_BATCH_PRESCALE
#define SSCN_BATCH_PRESCALE 256
#endif
constexpr int kBatchPrescale = SSCN_BATCH_PRESCALE;
// Infinity Cache budget of a group of batched instances (both state
// buffers), MiB; SSCN_BATCH_GROUP_MB overrides it.  0 (the default) puts
// every instance in one group: on the 64-instance complex128 workload (309
// MB in two buffers) two groups of 155 MB measured 1.7 % faster with cached
// state accesses and 10 % slower with streamed ones, so the batch runs as
// one group with streamed accesses.
constexpr int kBatchGroupMB = 0;


}  // namespace sscn

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
    int xLmax = 1;          // largest admissible xL
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
    Inst2D inst_host{};     // the same descriptor, passed by value to the fused step
    int2 *d_work = nullptr;
    int *d_nwork = nullptr;
    int ntiles = 0;
    // the fused step's tile shape (FusedLaunch::tile), whether each shape
    // fits (window and LDS) and its tile count; tile_force >= 0 when
    // SSCN_FUSED_TILE fixes the shape
    int tile = 0, tile_force = -1;
    bool fused_ok_t[kFusedTiles] = {false, false, false};
    int ntiles_t[kFusedTiles] = {0, 0, 0};
    double *partials2 = nullptr;
    int fparity = 0;        // buffer (0 = psi, 1 = work) holding the state
    int pbuf = 0;           // partial buffer holding the pending norm
    float tune_ms[3] = {0, 0, 0};
    std::vector<std::pair<int64_t, hipGraphExec_t>> graphs;  // sscn_step graphs by step count
};

namespace sscn {

template <class R> using V = typename Vec<R>::T;

// Dispatch on the window size W (a template parameter of the sweeps).
#define SSCN_W_SWITCH(Wv, CALL)                                                                             \
    switch (Wv) {                                                                                            \
    case 4: CALL(4); break;                                                                                  \
    case 6: CALL(6); break;                                                                                  \
    case 8: CALL(8); break;                                                                                  \
    case 10: CALL(10); break;                                                                                \
    case 12: CALL(12); break;                                                                                \
    case 13: CALL(13); break;                                                                                \
    case 14: CALL(14); break;                                                                                \
    case 16: CALL(16); break;                                                                                \
    case 20: CALL(20); break;                                                                                \
    case 24: CALL(24); break;                                                                                \
    default: CALL(32); break;                                                                                \
    }

inline unsigned round8(int64_t n) { return (unsigned)((n + 7) / 8 * 8); }

// The rescale of the pending norm (npart > 0 partials) is reduced once by
// k_norm_scale into obs_buf[kScaleSlot], which every x-sweep block reads.
constexpr int kScaleSlot = 48;

#define SSCN_W_SWITCH_FUSED(R, Wv, CALL)                                                                   \
    switch (Wv) {                                                                                            \
    case 4: CALL(4); break;                                                                                  \
    case 6: CALL(6); break;                                                                                  \
    case 8: CALL(8); break;                                                                                  \
    case 10: CALL(10); break;                                                                                \
    case 12: CALL(12); break;                                                                                \
    case 13: CALL(13); break;                                                                                \
    case 14: CALL(14); break;                                                                                \
    case 16: CALL(16); break;                                                                                \
    default: CALL(20); break;                                                                                \
    }

// Launch geometry of one fused 2D step: a work list of (instance, tile)
// over the descriptors inst, or (one != NULL) a single instance whose
// descriptor goes by value with the tiles as work items.
struct FusedLaunch {
    const Inst2D *inst;
    const int2 *work;
    const int *nwork;
    int grid;
    int W;
    const Inst2D *one;
    int tile = 0;  // the tile shape: kFusedTileR[tile] x kFusedTileC[tile]
};

}  // namespace sscn

struct sscn_batch {
    int n = 0, precision = 0, mode = 0, W = 0;
    hipStream_t stream = nullptr, cap = nullptr;
    std::vector<sscn_params> p;
    std::vector<StepArgs> args;
    std::vector<void *> psi, work, tabx, taby;
    std::vector<int> ntiles, nchunk;
    std::vector<char> active;
    std::vector<long long> conv;
    std::vector<Inst2D> hinst;
    Inst2D *d_inst = nullptr;
    int2 *d_work = nullptr, *d_fwork = nullptr, *d_owork = nullptr;
    int *d_nwork = nullptr, *d_nf = nullptr, *d_no = nullptr, *d_obase = nullptr, *d_ocount = nullptr;
    int total_tiles = 0, total_chunks = 0;
    int grid_tiles = 0, grid_chunks = 0;  // list lengths at the last rebuild
    double *part[2] = {nullptr, nullptr};
    double *opart = nullptr, *d_sums = nullptr, *d_mu_prev = nullptr;
    double *vpart = nullptr;  // vortex windings per observable chunk (convergence checks)
    int *d_hits = nullptr, *d_count_prev = nullptr, *d_counts = nullptr;
    long long *d_conv = nullptr;
    double *phase = nullptr;
    int fparity = 0, pbuf = 0;
    bool pending = false;
    int64_t steps = 0;
    hipGraph_t graph = nullptr;  // the convergence run's graph of graph_k steps
    hipGraphExec_t gexec = nullptr;
    int graph_k = 0;
    std::vector<std::pair<int64_t, hipGraphExec_t>> step_graphs;  // sscn_batch_step graphs by step count
    // sweep plan: x line blocks, y tiles, per-instance rescale
    int plan = SSCN_PLAN_AUTO, active_plan = SSCN_PLAN_FUSED;
    bool sweeps_ok = true;
    bool xshort = true;  // every instance has nx * L <= 2048: 8 staged points per x-sweep thread
    // x-sweep lines per block of every instance under the two options: 0 the
    // most the segment count and staging allow, 1 capped at kBatchXLds of LDS
    // per block; xsel the option in use, xforce one forced by
    // SSCN_BATCH_XLINES (-1: none), xtuned once the autotuner has timed them
    std::vector<int> xl_opt[2];
    int xsel = 1, xforce = -1;
    bool xtuned = false;
    float tune_x_ms[2] = {0, 0};
    int xwork_cap = 0;  // entries of d_xwork (the larger option's list)
    std::vector<int> xitems, yitems;
    int total_x = 0, total_y = 0, grid_x = 0, grid_y = 0, grid_k = 0;
    size_t xlds = 0;
    int2 *d_xwork = nullptr, *d_ywork = nullptr;
    int *d_nx = nullptr, *d_ny = nullptr, *d_klist = nullptr, *d_nk = nullptr;  // d_nx, d_ny: one per group
    // Groups of the sweep plan: instances whose two state buffers together
    // fit the Infinity Cache budget run all the steps of a call before the
    // next group's.  Each group owns a fixed region of the x and y work
    // lists (offset, items of all its instances, items of its active ones).
    int ngroups = 1;
    std::vector<int> group;  // group of each instance
    std::vector<int> gx_off, gx_tot, gx_cnt, gy_off, gy_tot, gy_cnt;
    double *ypart = nullptr, *d_scale = nullptr;
    // the pending rescale is summed once per instance (k_batch_scale) before
    // the x-sweep instead of in every x-sweep block: some instance has more
    // than kBatchPrescale norm partials
    bool prescale = false;
    float tune_ms[3] = {0, 0, 0};
    // 3D instances (sweep plan): the z-sweep's window, tables and work list
    bool dim3 = false;
    int Wz = 0;
    std::vector<void *> tabz;
    std::vector<int> zitems;
    int total_z = 0, grid_z = 0;
    int2 *d_zwork = nullptr;
    int *d_nzl = nullptr;
};

namespace sscn {

// Kernel launchers (sscn_kernels.hip), explicitly instantiated for R = double
// and float.
// x-sweep with H1 and the pending rescale (npart > 0 partials of the last
// step's norm; reduce = false reuses the s - 1 the last reducing launch left).
template <class R, bool RT>
void launch_x(const sscn_handle *h, const void *src, void *dst, int npart, hipStream_t st, bool reduce = true);
// y- and z-sweeps; EMIT: write the norm partials of the outputs.
template <class R, bool EMIT>
void launch_y(const sscn_handle *h, const void *src, void *dst, hipStream_t st);
template <class R, bool EMIT>
void launch_z(const sscn_handle *h, const void *src, void *dst, hipStream_t st);
// One fused 2D step over a work list (or one instance).
template <class R, bool RT>
void launch_fused(const FusedLaunch &f, int parity, const double *pin, double *pout, int use_pin, hipStream_t st);
// The launchers of tile shapes 1 and 2 (launch_fused dispatches to them).
template <class R, bool RT>
void launch_fused_narrow(const FusedLaunch &f, int parity, const double *pin, double *pout, int use_pin,
                         hipStream_t st);
template <class R, bool RT>
void launch_fused_small(const FusedLaunch &f, int parity, const double *pin, double *pout, int use_pin,
                        hipStream_t st);
// Raise the dynamic-LDS limit of the fused-step kernels for window W (every
// tile shape).
template <class R>
hipError_t allow_fused_lds_all(int W);
template <class R>
hipError_t allow_fused_lds_narrow(int W);
template <class R>
hipError_t allow_fused_lds_small(int W);
// The same for the x-sweep kernels (kXLdsCap), single-instance and batched.
template <class R>
hipError_t allow_x_lds_all(int W);
template <class R>
hipError_t batch_allow_x_lds_all(int W);
// One step of the batched sweep plan for every listed instance; ev
// (optional): 4 events recorded before the rescale, x- and y-sweep kernels
// and after the y-sweep.
template <class R>
void batch_sweep_step(sscn_batch *b, hipStream_t st, int g, bool all, hipEvent_t *ev = nullptr);

}  // namespace sscn
