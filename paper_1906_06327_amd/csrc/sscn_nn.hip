// C ABI of the learned-initial-state network kernels (include/sscn_nn.h).
#include "sscn_nn.h"
#include "sscn_nn.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

using namespace sscn_nn;

namespace {

thread_local std::string g_nn_err;

int nn_fail(int code, const std::string &msg)
{
    g_nn_err = msg;
    return code;
}

int launched(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return nn_fail(-5, std::string(what) + ": " + hipGetErrorString(e));
    return 0;
}

int blocks(int64_t n) { return (int)std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256)); }

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

extern "C" {

const char *sscn_nn_last_error(void) { return g_nn_err.c_str(); }

}  // extern "C"

namespace {

#ifndef SSCN_NN_CONV_LEGACY
#define SSCN_NN_CONV_LEGACY 0
#endif

// Raise a conv kernel's dynamic-LDS limit once (first launch of each
// instantiation); returns the error of the attribute call.
template <class K>
hipError_t conv_lds_once(K kernel, int bytes)
{
    static hipError_t e = hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return e;
}

// Output-channel tile of a convolution with Cout output channels.
int conv_bn(int Cout) { return Cout % 128 == 0 ? 128 : Cout % 64 == 0 ? 64 : Cout % 32 == 0 ? 32 : 16; }

// K stages of a convolution with Cin input channels.
int conv_stages(int Cin) { return 9 * (Cin % 64 == 0 ? Cin / 64 : Cin % 32 == 0 ? Cin / 32 : Cin / 16); }

// Split-K factor: grids of fewer than 512 blocks (the deep, small layers)
// are split over K so that the launch fills the chip, each part keeping at
// least two stages; 1 = no split.
int conv_splits(int P, int Cin, int Cout)
{
    const int64_t blocks = (int64_t)((P + 127) / 128) * (Cout / conv_bn(Cout));
    if (blocks >= 512)
        return 1;
    const int64_t want = (512 + blocks - 1) / blocks;
    return (int)std::max<int64_t>(1, std::min<int64_t>({want, conv_stages(Cin) / 2, 16}));
}

// Pixel splits of the bias gradient: chunks of about 1024 pixels, at most
// 1024 of them.
int bias_splits(int P) { return std::min(1024, std::max(1, (P + 1023) / 1024)); }

template <int ACT, bool OUTF32, int BN, int WM, int KC>
void go_conv_mfma(const uint16_t *x, int N, int H, int W, int Cin, const uint16_t *w, const float *bias, int Cout,
                  void *y, int ldy, int yoff, float *ws, int nsplit, hipStream_t st)
{
    constexpr int lds = conv_mfma_lds_bytes<BN, KC>();
    const int P = N * H * W;
    if (nsplit > 1) {
        if (conv_lds_once(k_conv3x3_mfma<ACT, OUTF32, BN, WM, KC, true>, lds) != hipSuccess)
            return;  // reported by launched()
        hipLaunchKernelGGL((k_conv3x3_mfma<ACT, OUTF32, BN, WM, KC, true>), dim3((P + 127) / 128, Cout / BN, nsplit),
                           dim3(256), lds, st, x, N, H, W, Cin, w, bias, Cout, (void *)ws, Cout, 0, nsplit);
        const int64_t n = (int64_t)P * Cout;
        const uintptr_t run = OUTF32 ? 16 : 8;  // bytes of 4 output values
        if (Cout % 4 == 0 && ldy % 4 == 0 && yoff % 4 == 0 && reinterpret_cast<uintptr_t>(y) % run == 0 &&
            reinterpret_cast<uintptr_t>(ws) % 16 == 0 && (!bias || reinterpret_cast<uintptr_t>(bias) % 16 == 0)) {
            const int grid = (int)std::min<int64_t>(8192, (n / 4 + 255) / 256);
            hipLaunchKernelGGL((k_conv_split_sum_v4<ACT, OUTF32>), dim3(grid), dim3(256), 0, st, (const float *)ws,
                               nsplit, P, Cout, bias, y, ldy, yoff);
            return;
        }
        const int grid = (int)std::min<int64_t>(8192, (n + 255) / 256);
        hipLaunchKernelGGL((k_conv_split_sum<ACT, OUTF32>), dim3(grid), dim3(256), 0, st, (const float *)ws, nsplit,
                           P, Cout, bias, y, ldy, yoff);
        return;
    }
    if (conv_lds_once(k_conv3x3_mfma<ACT, OUTF32, BN, WM, KC, false>, lds) != hipSuccess)
        return;
    hipLaunchKernelGGL((k_conv3x3_mfma<ACT, OUTF32, BN, WM, KC, false>), dim3((P + 127) / 128, Cout / BN), dim3(256),
                       lds, st, x, N, H, W, Cin, w, bias, Cout, y, ldy, yoff, 1);
}

template <int ACT, bool OUTF32, int BN, int WM>
void go_conv_halo(const uint16_t *x, int N, int H, int W, int Cin, const uint16_t *w, const float *bias, int Cout,
                  void *y, int ldy, int yoff, hipStream_t st, uint16_t *pool)
{
    // narrow layers stage a stencil row of taps per K stage
    constexpr int TG = BN <= 32 ? 3 : 1;
    constexpr int lds = conv_halo_lds_bytes<BN, 32, TG>();
    if (conv_lds_once(k_conv3x3_halo<ACT, OUTF32, BN, WM, 32, TG>, lds) != hipSuccess)
        return;  // reported by launched()
    hipLaunchKernelGGL((k_conv3x3_halo<ACT, OUTF32, BN, WM, 32, TG>), dim3(N * (H / kPatchH) * (W / kPatchW), Cout / BN),
                       dim3(256), lds, st, x, N, H, W, Cin, w, bias, Cout, y, ldy, yoff, pool);
}

// The halo-patch kernel takes images whose sides are multiples of the patch
// (8 x 16) with enough patches to fill the chip (>= 256 blocks).
bool conv_halo_ok(int N, int H, int W, int Cout)
{
    return H % kPatchH == 0 && W % kPatchW == 0 &&
           (int64_t)N * (H / kPatchH) * (W / kPatchW) * (Cout / conv_bn(Cout)) >= 256;
}

template <int ACT, bool OUTF32, int KC>
void launch_conv_kc(const uint16_t *x, int N, int H, int W, int Cin, const uint16_t *w, const float *bias, int Cout,
                    void *y, int ldy, int yoff, float *ws, int nsplit, hipStream_t st)
{
    switch (conv_bn(Cout)) {
    case 128: go_conv_mfma<ACT, OUTF32, 128, 2, KC>(x, N, H, W, Cin, w, bias, Cout, y, ldy, yoff, ws, nsplit, st); break;
    case 64: go_conv_mfma<ACT, OUTF32, 64, 2, KC>(x, N, H, W, Cin, w, bias, Cout, y, ldy, yoff, ws, nsplit, st); break;
    case 32: go_conv_mfma<ACT, OUTF32, 32, 4, KC>(x, N, H, W, Cin, w, bias, Cout, y, ldy, yoff, ws, nsplit, st); break;
    default: go_conv_mfma<ACT, OUTF32, 16, 4, KC>(x, N, H, W, Cin, w, bias, Cout, y, ldy, yoff, ws, nsplit, st); break;
    }
}

// ws: nsplit * P * Cout floats when nsplit > 1 (conv_splits), else unused.
template <int ACT, bool OUTF32>
void launch_conv(const uint16_t *x, int N, int H, int W, int Cin, const uint16_t *w, const float *bias, int Cout,
                 void *y, int ldy, int yoff, hipStream_t st, float *ws = nullptr, int nsplit = 1,
                 uint16_t *pool = nullptr)
{
    const int P = N * H * W;
    if (SSCN_NN_CONV_LEGACY) {
        if (Cout % 64 == 0)
            hipLaunchKernelGGL((k_conv3x3<ACT, OUTF32, 64>), dim3((P + 63) / 64, Cout / 64), dim3(256), 0, st, x, N,
                               H, W, Cin, w, bias, Cout, y, ldy, yoff);
        else if (Cout % 32 == 0)
            hipLaunchKernelGGL((k_conv3x3<ACT, OUTF32, 32>), dim3((P + 63) / 64, Cout / 32), dim3(256), 0, st, x, N,
                               H, W, Cin, w, bias, Cout, y, ldy, yoff);
        else
            hipLaunchKernelGGL((k_conv3x3<ACT, OUTF32, 16>), dim3((P + 63) / 64, Cout / 16), dim3(256), 0, st, x, N,
                               H, W, Cin, w, bias, Cout, y, ldy, yoff);
        return;
    }
    if (nsplit <= 1 && conv_halo_ok(N, H, W, Cout)) {
        switch (conv_bn(Cout)) {
        case 128: go_conv_halo<ACT, OUTF32, 128, 2>(x, N, H, W, Cin, w, bias, Cout, y, ldy, yoff, st, pool); break;
        case 64: go_conv_halo<ACT, OUTF32, 64, 2>(x, N, H, W, Cin, w, bias, Cout, y, ldy, yoff, st, pool); break;
        case 32: go_conv_halo<ACT, OUTF32, 32, 4>(x, N, H, W, Cin, w, bias, Cout, y, ldy, yoff, st, pool); break;
        default: go_conv_halo<ACT, OUTF32, 16, 4>(x, N, H, W, Cin, w, bias, Cout, y, ldy, yoff, st, pool); break;
        }
        return;
    }
    if (Cin % 64 == 0)
        launch_conv_kc<ACT, OUTF32, 64>(x, N, H, W, Cin, w, bias, Cout, y, ldy, yoff, ws, nsplit, st);
    else
        launch_conv_kc<ACT, OUTF32, 32>(x, N, H, W, Cin, w, bias, Cout, y, ldy, yoff, ws, nsplit, st);
}

// Pixel ranges of the weight gradient: about 1024 pixels each, at most
// kWgradSplits of them (each range is one block's sequence of 32-pixel
// chunks, so the large images need many ranges to fill the chip: 1024 took
// a training iteration of the 256^2 network from 10.2 to 8.6 ms against
// 64).
#ifndef SSCN_NN_WGRAD_SPLITS
#define SSCN_NN_WGRAD_SPLITS 1024
#endif
constexpr int kWgradSplits = SSCN_NN_WGRAD_SPLITS;

int wgrad_splits(int P) { return std::min(kWgradSplits, std::max(1, (P + 1023) / 1024)); }

}  // namespace

extern "C" {

int sscn_nn_conv_ws_floats(int N, int H, int W, int Cin, int Cout, int64_t *floats)
{
    if (!floats || N < 1 || H < 1 || W < 1 || Cin < 16 || Cin % 16 || Cout < 16 || Cout % 16)
        return nn_fail(-1, "bad conv_ws_floats arguments");
    const int P = N * H * W;
    const int ns = SSCN_NN_CONV_LEGACY ? 1 : conv_splits(P, Cin, Cout);
    *floats = ns > 1 ? (int64_t)ns * P * Cout : 0;
    return 0;
}

int sscn_nn_conv3x3(const void *x, int N, int H, int W, int Cin, const void *w, const float *bias, int Cout,
                    int act, int out_f32, void *y, int ldy, int yoff, float *ws, int64_t ws_floats, void *stream)
{
    if (!x || !w || !y || N < 1 || H < 1 || W < 1 || Cin < 16 || Cin % 16 || Cout < 16 || Cout % 16 ||
        ldy < yoff + Cout || yoff < 0 || (act != ACT_NONE && act != ACT_LEAKY) || ws_floats < 0)
        return nn_fail(-1, "bad conv3x3 arguments");
    const int P = N * H * W;
    int ns = SSCN_NN_CONV_LEGACY ? 1 : conv_splits(P, Cin, Cout);
    if (!ws || ws_floats < (int64_t)ns * P * Cout)
        ns = 1;  // no (or too small a) workspace: no split
    hipStream_t st = (hipStream_t)stream;
    const uint16_t *xs = (const uint16_t *)x, *wb = (const uint16_t *)w;
    if (act == ACT_LEAKY && !out_f32)
        launch_conv<ACT_LEAKY, false>(xs, N, H, W, Cin, wb, bias, Cout, y, ldy, yoff, st, ws, ns);
    else if (act == ACT_LEAKY)
        launch_conv<ACT_LEAKY, true>(xs, N, H, W, Cin, wb, bias, Cout, y, ldy, yoff, st, ws, ns);
    else if (!out_f32)
        launch_conv<ACT_NONE, false>(xs, N, H, W, Cin, wb, bias, Cout, y, ldy, yoff, st, ws, ns);
    else
        launch_conv<ACT_NONE, true>(xs, N, H, W, Cin, wb, bias, Cout, y, ldy, yoff, st, ws, ns);
    return launched("conv3x3");
}

int sscn_nn_conv3x3_pool(const void *x, int N, int H, int W, int Cin, const void *w, const float *bias, int Cout,
                         int act, void *y, int ldy, int yoff, void *pool_y, float *ws, int64_t ws_floats,
                         void *stream)
{
    if (!pool_y || H % 2 || W % 2)
        return nn_fail(-1, "bad conv3x3_pool arguments");
    if (!x || !w || !y || N < 1 || H < 1 || W < 1 || Cin < 16 || Cin % 16 || Cout < 16 || Cout % 16 ||
        ldy < yoff + Cout || yoff < 0 || (act != ACT_NONE && act != ACT_LEAKY) || ws_floats < 0)
        return nn_fail(-1, "bad conv3x3_pool arguments");
    const int P = N * H * W;
    int ns = SSCN_NN_CONV_LEGACY ? 1 : conv_splits(P, Cin, Cout);
    if (!ws || ws_floats < (int64_t)ns * P * Cout)
        ns = 1;
    // fused where the halo-patch kernel runs with its staged 16-byte stores
    // (the conditions of conv_out_vec_ok); otherwise the two calls
    const bool fused = !SSCN_NN_CONV_LEGACY && ns <= 1 && conv_halo_ok(N, H, W, Cout) && ldy % 8 == 0 &&
                       yoff % 8 == 0 && aligned16(y) && aligned16(pool_y);
    if (!fused) {
        const int r = sscn_nn_conv3x3(x, N, H, W, Cin, w, bias, Cout, act, 0, y, ldy, yoff, ws, ws_floats, stream);
        return r ? r : sscn_nn_pool2(y, ldy, yoff, N, H, W, Cout, pool_y, stream);
    }
    hipStream_t st = (hipStream_t)stream;
    const uint16_t *xs = (const uint16_t *)x, *wb = (const uint16_t *)w;
    if (act == ACT_LEAKY)
        launch_conv<ACT_LEAKY, false>(xs, N, H, W, Cin, wb, bias, Cout, y, ldy, yoff, st, ws, 1, (uint16_t *)pool_y);
    else
        launch_conv<ACT_NONE, false>(xs, N, H, W, Cin, wb, bias, Cout, y, ldy, yoff, st, ws, 1, (uint16_t *)pool_y);
    return launched("conv3x3_pool");
}

int sscn_nn_conv3x3_dgrad(const void *dy, int N, int H, int W, int Cout, const void *w, int Cin,
                          void *wt_scratch, void *dx, int lddx, int dxoff, float *ws, int64_t ws_floats,
                          void *stream)
{
    if (!dy || !w || !wt_scratch || !dx || Cin % 16 || Cout % 16 || Cin < 16 || Cout < 16 || lddx < dxoff + Cin ||
        ws_floats < 0)
        return nn_fail(-1, "bad conv3x3_dgrad arguments");
    hipStream_t st = (hipStream_t)stream;
    const int P = N * H * W;
    int ns = SSCN_NN_CONV_LEGACY ? 1 : conv_splits(P, Cout, Cin);  // the convolution with Cout inputs, Cin outputs
    if (!ws || ws_floats < (int64_t)ns * P * Cin)
        ns = 1;
    hipLaunchKernelGGL(k_wflip, dim3(blocks((int64_t)Cout * 9 * Cin)), dim3(256), 0, st, (const uint16_t *)w, Cout,
                       Cin, (uint16_t *)wt_scratch);
    launch_conv<ACT_NONE, false>((const uint16_t *)dy, N, H, W, Cout, (const uint16_t *)wt_scratch, nullptr, Cin, dx,
                                 lddx, dxoff, st, ws, ns);
    return launched("conv3x3_dgrad");
}

int sscn_nn_wgrad_scratch(int N, int H, int W, int Cin, int Cout, int64_t *floats)
{
    if (!floats)
        return nn_fail(-1, "null argument");
    const int P = N * H * W;
    const int nsplit = wgrad_splits(P);
    *floats = (int64_t)nsplit * Cout * 9 * Cin + (int64_t)bias_splits(P) * Cout;
    return 0;
}

int sscn_nn_conv3x3_wgrad(const void *x, int N, int H, int W, int Cin, const void *dy, int Cout, float *dw,
                          float *db, float *scratch, int64_t scratch_floats, void *stream)
{
    if (!x || !dy || !dw || !scratch || Cin % 16 || Cout % 16 || Cin < 16 || Cout < 16)
        return nn_fail(-1, "bad conv3x3_wgrad arguments");
    int64_t need = 0;
    sscn_nn_wgrad_scratch(N, H, W, Cin, Cout, &need);
    if (scratch_floats < need)
        return nn_fail(-1, "wgrad scratch too small");
    const int P = N * H * W;
    const int nsplit = wgrad_splits(P);
    int chunk = (P + nsplit - 1) / nsplit;
    chunk = (chunk + 15) / 16 * 16;
    hipStream_t st = (hipStream_t)stream;
    const int cw = Cin % 32 == 0 ? 32 : 16;
    // 32 or 16 output channels: several taps per block share the dy tile
    if (Cout == 32)
        hipLaunchKernelGGL(k_conv3x3_wgrad_narrow<32>, dim3(nsplit, 1, 5 * (Cin / cw)), dim3(256), 0, st,
                           (const uint16_t *)x, N, H, W, Cin, (const uint16_t *)dy, Cout, chunk, scratch);
    else if (Cout == 16)
        hipLaunchKernelGGL(k_conv3x3_wgrad_narrow<16>, dim3(nsplit, 1, 3 * (Cin / cw)), dim3(256), 0, st,
                           (const uint16_t *)x, N, H, W, Cin, (const uint16_t *)dy, Cout, chunk, scratch);
    else
        hipLaunchKernelGGL(k_conv3x3_wgrad, dim3(nsplit, (Cout + 63) / 64, 9 * Cin / cw), dim3(256), 0, st,
                           (const uint16_t *)x, N, H, W, Cin, (const uint16_t *)dy, Cout, chunk, scratch);
    const int nw = Cout * 9 * Cin;
    // many ranges (the large images, whose weights are few): one wave per
    // weight; else one thread per weight
    if (nsplit > 64)
        hipLaunchKernelGGL(k_sum_parts_wave, dim3(nw), dim3(64), 0, st, scratch, nsplit, nw, dw);
    else
        hipLaunchKernelGGL(k_sum_splits, dim3(blocks(nw)), dim3(256), 0, st, scratch, nsplit, nw, dw);
    if (db) {
        float *bp = scratch + (size_t)nsplit * nw;
        const int bs = bias_splits(P);
        const int bchunk = (P + bs - 1) / bs;
        if (Cout % 8 == 0 && aligned16(dy))
            hipLaunchKernelGGL(k_bias_grad_v8, dim3(bs), dim3(256), 0, st, (const uint16_t *)dy, P, Cout, bchunk, bp);
        else
            hipLaunchKernelGGL(k_bias_grad, dim3(bs), dim3(256), 0, st, (const uint16_t *)dy, P, Cout, bchunk, bp);
        hipLaunchKernelGGL(k_sum_parts_wave, dim3(Cout), dim3(64), 0, st, bp, bs, Cout, db);
    }
    return launched("conv3x3_wgrad");
}

int sscn_nn_act_bwd(void *dy, const void *y, int64_t n, void *stream)
{
    if (!dy || !y || n < 0)
        return nn_fail(-1, "bad act_bwd arguments");
    if (n % 8 == 0 && aligned16(dy) && aligned16(y))
        hipLaunchKernelGGL(k_act_bwd_v8, dim3(blocks(n / 8)), dim3(256), 0, (hipStream_t)stream, (uint16_t *)dy,
                           (const uint16_t *)y, n / 8);
    else
        hipLaunchKernelGGL(k_act_bwd, dim3(blocks(n)), dim3(256), 0, (hipStream_t)stream, (uint16_t *)dy,
                           (const uint16_t *)y, (int)n);
    return launched("act_bwd");
}

int sscn_nn_pool2(const void *x, int ldx, int xoff, int N, int H, int W, int C, void *y, void *stream)
{
    if (!x || !y || H % 2 || W % 2 || C < 1 || xoff < 0 || ldx < xoff + C)
        return nn_fail(-1, "bad pool2 arguments");
    const uint16_t *xs = (const uint16_t *)x + xoff;
    if (C % 8 == 0 && ldx % 8 == 0 && aligned16(xs) && aligned16(y))
        hipLaunchKernelGGL(k_pool2_v8, dim3(blocks((int64_t)N * H * W * C / 32)), dim3(256), 0, (hipStream_t)stream,
                           xs, ldx, N, H, W, C, (uint16_t *)y);
    else
        hipLaunchKernelGGL(k_pool2, dim3(blocks((int64_t)N * H * W * C / 4)), dim3(256), 0, (hipStream_t)stream,
                           xs, ldx, N, H, W, C, (uint16_t *)y);
    return launched("pool2");
}

int sscn_nn_pool2_bwd(const void *dy, int N, int H, int W, int C, void *dx, void *stream)
{
    if (!dy || !dx || H % 2 || W % 2)
        return nn_fail(-1, "bad pool2_bwd arguments");
    if (C % 8 == 0 && aligned16(dy) && aligned16(dx))
        hipLaunchKernelGGL(k_pool2_bwd_v8, dim3(blocks((int64_t)N * H * W * C / 8)), dim3(256), 0,
                           (hipStream_t)stream, (const uint16_t *)dy, N, H, W, C, (uint16_t *)dx);
    else
        hipLaunchKernelGGL(k_pool2_bwd, dim3(blocks((int64_t)N * H * W * C)), dim3(256), 0, (hipStream_t)stream,
                           (const uint16_t *)dy, N, H, W, C, (uint16_t *)dx);
    return launched("pool2_bwd");
}

int sscn_nn_up2(const void *x, int N, int H, int W, int C, void *y, int ldy, int yoff, void *stream)
{
    if (!x || !y || ldy < yoff + C)
        return nn_fail(-1, "bad up2 arguments");
    if (C % 8 == 0 && ldy % 8 == 0 && yoff % 8 == 0 && aligned16(x) && aligned16(y))
        hipLaunchKernelGGL(k_up2_v8, dim3(blocks((int64_t)N * 4 * H * W * C / 8)), dim3(256), 0, (hipStream_t)stream,
                           (const uint16_t *)x, N, H, W, C, (uint16_t *)y, ldy, yoff);
    else
        hipLaunchKernelGGL(k_up2, dim3(blocks((int64_t)N * 4 * H * W * C)), dim3(256), 0, (hipStream_t)stream,
                           (const uint16_t *)x, N, H, W, C, (uint16_t *)y, ldy, yoff);
    return launched("up2");
}

int sscn_nn_up2_bwd(const void *dy, int ldy, int yoff, int N, int H, int W, int C, void *dx, void *stream)
{
    if (!dy || !dx || ldy < yoff + C)
        return nn_fail(-1, "bad up2_bwd arguments");
    if (C % 8 == 0 && ldy % 8 == 0 && yoff % 8 == 0 && aligned16(dy) && aligned16(dx))
        hipLaunchKernelGGL(k_up2_bwd_v8, dim3(blocks((int64_t)N * H * W * C / 8)), dim3(256), 0, (hipStream_t)stream,
                           (const uint16_t *)dy, ldy, yoff, N, H, W, C, (uint16_t *)dx);
    else
        hipLaunchKernelGGL(k_up2_bwd, dim3(blocks((int64_t)N * H * W * C)), dim3(256), 0, (hipStream_t)stream,
                           (const uint16_t *)dy, ldy, yoff, N, H, W, C, (uint16_t *)dx);
    return launched("up2_bwd");
}

int sscn_nn_chan_copy(const void *src, int lds, int soff, void *dst, int ldd, int doff, int P, int C,
                      int accumulate, void *stream)
{
    if (!src || !dst || lds < soff + C || ldd < doff + C)
        return nn_fail(-1, "bad chan_copy arguments");
    if (C % 8 == 0 && lds % 8 == 0 && soff % 8 == 0 && ldd % 8 == 0 && doff % 8 == 0 && aligned16(src) &&
        aligned16(dst))
        hipLaunchKernelGGL(k_chan_copy_v8, dim3(blocks((int64_t)P * C / 8)), dim3(256), 0, (hipStream_t)stream,
                           (const uint16_t *)src, lds, soff, (uint16_t *)dst, ldd, doff, P, C, accumulate);
    else
        hipLaunchKernelGGL(k_chan_copy, dim3(blocks((int64_t)P * C)), dim3(256), 0, (hipStream_t)stream,
                           (const uint16_t *)src, lds, soff, (uint16_t *)dst, ldd, doff, P, C, accumulate);
    return launched("chan_copy");
}

int sscn_nn_loss(const float *pred, int ld, const float *psi, int B, int K, int S, double *stats, void *dpred,
                 void *stream)
{
    if (!pred || !psi || !stats || ld < 2 || B < 1 || K < 1 || S < 1)
        return nn_fail(-1, "bad loss arguments");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_loss_stats, dim3(B * K), dim3(256), 0, st, pred, ld, psi, K, S, stats);
    if (dpred)
        hipLaunchKernelGGL(k_loss_grad, dim3(blocks((int64_t)B * S)), dim3(256), 0, st, pred, ld, psi, B, K, S, stats,
                           (uint16_t *)dpred);
    return launched("loss");
}

int sscn_nn_psi_to_f32(const void *psi, int precision, int64_t S, float scale, float *out, void *stream)
{
    if (!psi || !out || S < 1 || (precision != 0 && precision != 1))
        return nn_fail(-1, "bad psi_to_f32 arguments");
    hipStream_t st = (hipStream_t)stream;
    if (precision == 0)
        hipLaunchKernelGGL(k_psi_to_f32<double>, dim3(blocks(2 * S)), dim3(256), 0, st, (const double *)psi, S, scale,
                           out);
    else
        hipLaunchKernelGGL(k_psi_to_f32<float>, dim3(blocks(2 * S)), dim3(256), 0, st, (const float *)psi, S, scale,
                           out);
    return launched("psi_to_f32");
}

int sscn_nn_f32_to_psi(const float *pred, int ld, int64_t S, double scale, void *psi, int precision, void *stream)
{
    if (!pred || !psi || ld < 2 || S < 1 || (precision != 0 && precision != 1))
        return nn_fail(-1, "bad f32_to_psi arguments");
    hipStream_t st = (hipStream_t)stream;
    if (precision == 0)
        hipLaunchKernelGGL(k_f32_to_psi<double>, dim3(blocks(2 * S)), dim3(256), 0, st, pred, ld, S, scale,
                           (double *)psi);
    else
        hipLaunchKernelGGL(k_f32_to_psi<float>, dim3(blocks(2 * S)), dim3(256), 0, st, pred, ld, S, scale,
                           (float *)psi);
    return launched("f32_to_psi");
}

int sscn_nn_sumsq(const float *a, int64_t n, double *work, void *stream)
{
    if (!a || !work || n < 0)
        return nn_fail(-1, "bad sumsq arguments");
    const int np = (int)std::min<int64_t>(256, std::max<int64_t>(1, (n + 4095) / 4096));
    hipLaunchKernelGGL(k_sumsq_part, dim3(np), dim3(256), 0, (hipStream_t)stream, a, n, work + 1);
    hipLaunchKernelGGL(k_sumsq_fin, dim3(1), dim3(256), 0, (hipStream_t)stream, (const double *)(work + 1), np,
                       work);
    return launched("sumsq");
}

int sscn_nn_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr, float b1, float b2, float eps,
                 int t, const double *gsq, float max_norm, void *wbf16, void *stream)
{
    if (!w || !m || !v || !g || n < 0 || t < 1 || (gsq && !(max_norm > 0.f)))
        return nn_fail(-1, "bad adam arguments");
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(blocks(n)), dim3(256), 0, (hipStream_t)stream, w, m, v, g, (int)n, lr, b1, b2,
                       eps, c1, c2, gsq, max_norm, (uint16_t *)wbf16);
    return launched("adam");
}

int sscn_nn_f32_to_bf16(const float *a, void *b, int64_t n, void *stream)
{
    if (!a || !b || n < 0)
        return nn_fail(-1, "bad f32_to_bf16 arguments");
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(blocks(n)), dim3(256), 0, (hipStream_t)stream, a, (uint16_t *)b, (int)n);
    return launched("f32_to_bf16");
}

}  // extern "C"
