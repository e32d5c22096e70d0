// Kernels of the learned initial state: a small U-Net whose 3x3
// convolutions run on the gfx950 matrix cores (bf16 operands, fp32
// accumulation), with the elementwise, resampling, loss and Adam kernels of
// its training.  Activations and gradients are NHWC bf16 (channels fastest);
// a convolution's weights are [Cout][3][3][Cin] bf16 with an fp32 master
// copy.  Channel counts of every convolution are multiples of 16.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sscn_nn {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// bf16 <-> fp32 (round to nearest even; NaN kept quiet)
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u)
        return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

enum { ACT_NONE = 0, ACT_LEAKY = 1 };
constexpr float kLeak = 0.1f;

// One 16x16x16 bf16 matrix-core product per call: with lane l, m = l % 16
// and g = l / 16, the lane supplies A[m][4g..4g+3] and B[4g..4g+3][m] and
// receives D[4g..4g+3][m].
__device__ __forceinline__ v4f mfma16(v4s a, v4s b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ v4s load4(const uint16_t *p)
{
    const uint2 u = *reinterpret_cast<const uint2 *>(p);
    v4s r;
    r[0] = (short)(u.x & 0xffffu);
    r[1] = (short)(u.x >> 16);
    r[2] = (short)(u.y & 0xffffu);
    r[3] = (short)(u.y >> 16);
    return r;
}

// 3x3 convolution, padding 1, as an implicit GEMM: M = N*H*W pixels,
// N = Cout, K = 9*Cin.  A wave computes 16 pixels x 16 output channels;
// a block of 4 waves 64 pixels x 16 channels.  Output channel co of pixel p
// goes to y[p*ldy + yoff + co] with bias and activation applied, bf16 or
// fp32.  Grid: (ceil(P/64), Cout/16).
template <int ACT, bool OUTF32>
__global__ __launch_bounds__(256) void k_conv3x3(const uint16_t *__restrict__ x, int N, int H, int W, int Cin,
                                                 const uint16_t *__restrict__ w, const float *__restrict__ bias,
                                                 int Cout, void *__restrict__ y, int ldy, int yoff)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 15, g = lane >> 4;
    const int P = N * H * W;
    const int p0 = (blockIdx.x * 4 + wave) * 16;
    const int co0 = blockIdx.y * 16;
    const int p = p0 + m;
    int n = 0, yy = 0, xx = 0;
    if (p < P) {
        n = p / (H * W);
        const int r = p - n * H * W;
        yy = r / W;
        xx = r - yy * W;
    }
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    const v4s zero = {0, 0, 0, 0};
    const uint16_t *wrow = w + (size_t)(co0 + m) * 9 * Cin;
    for (int tap = 0; tap < 9; ++tap) {
        const int sy = yy + tap / 3 - 1, sx = xx + tap % 3 - 1;
        const bool ok = p < P && sy >= 0 && sy < H && sx >= 0 && sx < W;
        const uint16_t *xr = x + ((size_t)(n * H + sy) * W + sx) * Cin;
        for (int c0 = 0; c0 < Cin; c0 += 16) {
            const v4s a = ok ? load4(xr + c0 + 4 * g) : zero;
            const v4s b = load4(wrow + tap * Cin + c0 + 4 * g);
            acc = mfma16(a, b, acc);
        }
    }
    const int co = co0 + m;
    const float bv = bias ? bias[co] : 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int pp = p0 + 4 * g + i;
        if (pp < P) {
            float v = acc[i] + bv;
            if (ACT == ACT_LEAKY)
                v = v > 0.f ? v : kLeak * v;
            if (OUTF32)
                reinterpret_cast<float *>(y)[(size_t)pp * ldy + yoff + co] = v;
            else
                reinterpret_cast<uint16_t *>(y)[(size_t)pp * ldy + yoff + co] = f2bf(v);
        }
    }
}

// Weights of the input-gradient convolution: wt[ci][8 - tap][co] = w[co][tap][ci].
__global__ __launch_bounds__(256) void k_wflip(const uint16_t *__restrict__ w, int Cout, int Cin,
                                               uint16_t *__restrict__ wt)
{
    const int n = Cout * 9 * Cin;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
        const int co = e / (9 * Cin), r = e - co * 9 * Cin;
        const int tap = r / Cin, ci = r - tap * Cin;
        wt[((size_t)ci * 9 + (8 - tap)) * Cout + co] = w[e];
    }
}

// Weight gradient, split over pixel ranges: part[s][co][tap][ci] =
// sum over pixels p of split s of dy[p][co] * x[p shifted by tap][ci].
// GEMM M = Cout, N = 9*Cin, K = pixels; a wave computes 16 co x 16 (tap, ci)
// over its pixel range.  Grid: (nsplit, Cout/16, 9*Cin/16), 64 threads.
__global__ __launch_bounds__(64) void k_conv3x3_wgrad(const uint16_t *__restrict__ x, int N, int H, int W,
                                                      int Cin, const uint16_t *__restrict__ dy, int Cout,
                                                      int chunk, float *__restrict__ part)
{
    const int lane = threadIdx.x;
    const int m = lane & 15, g = lane >> 4;
    const int s = blockIdx.x, co0 = blockIdx.y * 16, col0 = blockIdx.z * 16;
    const int P = N * H * W;
    const int pb = s * chunk, pe = min(P, pb + chunk);
    const int col = col0 + m;  // (tap, ci) of this lane's B column
    const int tap = col / Cin, ci = col - tap * Cin;
    const int dyo = tap / 3 - 1, dxo = tap % 3 - 1;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = pb; k0 < pe; k0 += 16) {
        v4s a, b;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int p = k0 + 4 * g + i;
            short av = 0, bv = 0;
            if (p < pe) {
                av = (short)dy[(size_t)p * Cout + co0 + m];
                const int n = p / (H * W), r = p - n * H * W;
                const int yy = r / W, xx = r - (r / W) * W;
                const int sy = yy + dyo, sx = xx + dxo;
                if (sy >= 0 && sy < H && sx >= 0 && sx < W)
                    bv = (short)x[((size_t)(n * H + sy) * W + sx) * Cin + ci];
            }
            a[i] = av;
            b[i] = bv;
        }
        acc = mfma16(a, b, acc);
    }
    // D[row = co0 + 4g + i][col0 + m]
    const int ncols = 9 * Cin;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        part[((size_t)s * Cout + co0 + 4 * g + i) * ncols + col0 + m] = acc[i];
}

// out[e] = sum over s of part[s][e] in a fixed order (fp32).
__global__ __launch_bounds__(256) void k_sum_splits(const float *__restrict__ part, int nsplit, int n,
                                                    float *__restrict__ out)
{
    for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
        float acc = 0.f;
        for (int s = 0; s < nsplit; ++s)
            acc += part[(size_t)s * n + e];
        out[e] = acc;
    }
}

// Bias gradient partials: part[s][c] = sum over the pixels of split s of dy.
__global__ __launch_bounds__(256) void k_bias_grad(const uint16_t *__restrict__ dy, int P, int C, int chunk,
                                                   float *__restrict__ part)
{
    const int s = blockIdx.x;
    const int pb = s * chunk, pe = min(P, pb + chunk);
    for (int c = threadIdx.x; c < C; c += 256) {
        float acc = 0.f;
        for (int p = pb; p < pe; ++p)
            acc += bf2f(dy[(size_t)p * C + c]);
        part[(size_t)s * C + c] = acc;
    }
}

// Gradient through the leaky ReLU, from the layer's output y (same sign as
// its input): d = dy * (y > 0 ? 1 : leak), in place on dy.
__global__ __launch_bounds__(256) void k_act_bwd(uint16_t *__restrict__ dy, const uint16_t *__restrict__ y, int n)
{
    for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
        const float g = bf2f(dy[e]);
        dy[e] = f2bf(bf2f(y[e]) > 0.f ? g : kLeak * g);
    }
}

// 2x2 average pooling (H, W even) and its gradient.
__global__ __launch_bounds__(256) void k_pool2(const uint16_t *__restrict__ x, int N, int H, int W, int C,
                                               uint16_t *__restrict__ y)
{
    const int Ho = H / 2, Wo = W / 2;
    const int n = N * Ho * Wo * C;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
        const int c = e % C, q = e / C;
        const int j = q % Wo, i = (q / Wo) % Ho, b = q / (Wo * Ho);
        const size_t base = ((size_t)(b * H + 2 * i) * W + 2 * j) * C + c;
        const float s = bf2f(x[base]) + bf2f(x[base + C]) + bf2f(x[base + (size_t)W * C]) +
                        bf2f(x[base + (size_t)W * C + C]);
        y[e] = f2bf(0.25f * s);
    }
}

__global__ __launch_bounds__(256) void k_pool2_bwd(const uint16_t *__restrict__ dy, int N, int H, int W, int C,
                                                   uint16_t *__restrict__ dx)
{
    const int n = N * H * W * C;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
        const int c = e % C, q = e / C;
        const int j = q % W, i = (q / W) % H, b = q / (W * H);
        dx[e] = f2bf(0.25f * bf2f(dy[((size_t)(b * (H / 2) + i / 2) * (W / 2) + j / 2) * C + c]));
    }
}

// Nearest 2x upsampling into channels [yoff, yoff + C) of a tensor with ldy
// channels, and its gradient (sum of the 4 children).
__global__ __launch_bounds__(256) void k_up2(const uint16_t *__restrict__ x, int N, int H, int W, int C,
                                             uint16_t *__restrict__ y, int ldy, int yoff)
{
    const int Ho = 2 * H, Wo = 2 * W;
    const int n = N * Ho * Wo * C;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
        const int c = e % C, q = e / C;
        const int j = q % Wo, i = (q / Wo) % Ho, b = q / (Wo * Ho);
        y[(size_t)q * ldy + yoff + c] = x[((size_t)(b * H + i / 2) * W + j / 2) * C + c];
    }
}

__global__ __launch_bounds__(256) void k_up2_bwd(const uint16_t *__restrict__ dy, int ldy, int yoff, int N, int H,
                                                 int W, int C, uint16_t *__restrict__ dx)
{
    const int n = N * H * W * C;
    const int Wo = 2 * W;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
        const int c = e % C, q = e / C;
        const int j = q % W, i = (q / W) % H, b = q / (W * H);
        const size_t r0 = (size_t)(b * 2 * H + 2 * i) * Wo + 2 * j;
        const float s = bf2f(dy[r0 * ldy + yoff + c]) + bf2f(dy[(r0 + 1) * ldy + yoff + c]) +
                        bf2f(dy[(r0 + Wo) * ldy + yoff + c]) + bf2f(dy[(r0 + Wo + 1) * ldy + yoff + c]);
        dx[e] = f2bf(s);
    }
}

// dst[p][doff + c] = src[p][soff + c] (accumulate: +=), c < C, p < P.
__global__ __launch_bounds__(256) void k_chan_copy(const uint16_t *__restrict__ src, int lds_, int soff,
                                                   uint16_t *__restrict__ dst, int ldd, int doff, int P, int C,
                                                   int accumulate)
{
    const int n = P * C;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
        const int c = e % C, p = e / C;
        const float v = bf2f(src[(size_t)p * lds_ + soff + c]);
        uint16_t *d = dst + (size_t)p * ldd + doff + c;
        *d = f2bf(accumulate ? bf2f(*d) + v : v);
    }
}

// Phase-aligned loss against K candidate targets per sample (the images of
// one target under the symmetries of the problem).  Prediction in channels
// 0,1 of pred (fp32, ld channels, S = H*W points per sample); targets psi
// [B][K][S] interleaved fp32.  stats[b][k] = {Re <psi_bk, pred_b>,
// Im <psi_bk, pred_b>, |pred_b|^2, |psi_bk|^2}.  One 256-thread block per
// (b, k), fixed-order reduction.
__global__ __launch_bounds__(256) void k_loss_stats(const float *__restrict__ pred, int ld,
                                                    const float *__restrict__ psi, int K, int S,
                                                    double *__restrict__ stats)
{
    __shared__ double red[4][8];
    const int bk = blockIdx.x, b = bk / K;
    double a[4] = {0, 0, 0, 0};
    for (int q = threadIdx.x; q < S; q += 256) {
        const float pr = pred[((size_t)b * S + q) * ld], pi = pred[((size_t)b * S + q) * ld + 1];
        const float tr = psi[((size_t)bk * S + q) * 2], ti = psi[((size_t)bk * S + q) * 2 + 1];
        a[0] += (double)tr * pr + (double)ti * pi;
        a[1] += (double)tr * pi - (double)ti * pr;
        a[2] += (double)pr * pr + (double)pi * pi;
        a[3] += (double)tr * tr + (double)ti * ti;
    }
    for (int k = 0; k < 4; ++k) {
        double v = a[k];
        for (int off = 32; off >= 1; off >>= 1)
            v += __shfl_xor(v, off, 64);
        if ((threadIdx.x & 63) == 0)
            red[k][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4)
        stats[(size_t)bk * 4 + threadIdx.x] =
            (red[threadIdx.x][0] + red[threadIdx.x][1]) + (red[threadIdx.x][2] + red[threadIdx.x][3]);
}

// Loss of sample b against candidate k: |pred|^2 + |psi_k|^2 - 2 |<psi_k, pred>|,
// the minimum over the global phase phi of |pred - e^{i phi} psi_k|^2.
__device__ __forceinline__ double cand_loss(const double *st)
{
    return st[2] + st[3] - 2.0 * sqrt(st[0] * st[0] + st[1] * st[1]);
}

// Loss gradient: the sample's loss is that of its nearest candidate k* (the
// first on ties); with e^{i phi} = <psi_k*, pred> / |<psi_k*, pred>| its
// gradient is 2 (pred - e^{i phi} psi_k*), scaled by 1/B and written as bf16
// into channels 0,1 of dpred (ld channels, the other channels zero).
__global__ __launch_bounds__(256) void k_loss_grad(const float *__restrict__ pred, int ld,
                                                   const float *__restrict__ psi, int B, int K, int S,
                                                   const double *__restrict__ stats, uint16_t *__restrict__ dpred)
{
    const int n = B * S;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
        const int b = e / S, q = e - b * S;
        int kb = 0;
        double lb = cand_loss(stats + (size_t)b * K * 4);
        for (int k = 1; k < K; ++k) {
            const double l = cand_loss(stats + ((size_t)b * K + k) * 4);
            if (l < lb) {
                lb = l;
                kb = k;
            }
        }
        const double *st = stats + ((size_t)b * K + kb) * 4;
        const double dr = st[0], di = st[1];
        const double mag = sqrt(dr * dr + di * di);
        const float cr = mag > 0 ? (float)(dr / mag) : 1.f, ci = mag > 0 ? (float)(di / mag) : 0.f;
        const size_t t = ((size_t)b * K + kb) * S + q;
        const float tr = psi[t * 2], ti = psi[t * 2 + 1];
        const float gr = 2.f * (pred[(size_t)e * ld] - (cr * tr - ci * ti)) / B;
        const float gi = 2.f * (pred[(size_t)e * ld + 1] - (cr * ti + ci * tr)) / B;
        for (int c = 0; c < ld; ++c)
            dpred[(size_t)e * ld + c] = c == 0 ? f2bf(gr) : c == 1 ? f2bf(gi) : (uint16_t)0;
    }
}

// Complex state <-> fp32 pairs: out[2q], out[2q+1] = scale * (Re, Im) psi[q]
// (complex128 or complex64 interleaved), and psi[q] = scale * (pred[q*ld],
// pred[q*ld + 1]).
template <class T>
__global__ __launch_bounds__(256) void k_psi_to_f32(const T *__restrict__ psi, int64_t S, float scale,
                                                    float *__restrict__ out)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < 2 * S; e += (int64_t)gridDim.x * 256)
        out[e] = (float)((double)psi[e] * (double)scale);
}

template <class T>
__global__ __launch_bounds__(256) void k_f32_to_psi(const float *__restrict__ pred, int ld, int64_t S, double scale,
                                                    T *__restrict__ psi)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < 2 * S; e += (int64_t)gridDim.x * 256)
        psi[e] = (T)((double)pred[(e >> 1) * ld + (e & 1)] * scale);
}

// Adam on fp32 master weights, then the bf16 copy the kernels read.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ wm, float *__restrict__ m, float *__restrict__ v,
                                              const float *__restrict__ g, int n, float lr, float b1, float b2,
                                              float eps, float c1, float c2, uint16_t *__restrict__ wbf)
{
    for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
        const float ge = g[e];
        const float me = b1 * m[e] + (1.f - b1) * ge;
        const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
        m[e] = me;
        v[e] = ve;
        const float w = wm[e] - lr * (me / c1) / (sqrtf(ve / c2) + eps);
        wm[e] = w;
        if (wbf)
            wbf[e] = f2bf(w);
    }
}

__global__ __launch_bounds__(256) void k_f32_to_bf16(const float *__restrict__ a, uint16_t *__restrict__ b, int n)
{
    for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256)
        b[e] = f2bf(a[e]);
}

}  // namespace sscn_nn
