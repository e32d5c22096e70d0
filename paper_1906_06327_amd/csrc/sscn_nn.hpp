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

// Eight bf16 values of a 16-byte word to fp32 and back (round to nearest
// even).
__device__ __forceinline__ void unpack8(const uint4 &u, float (&f)[8])
{
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[2 * i] = bf2f((uint16_t)(w[i] & 0xffffu));
        f[2 * i + 1] = bf2f((uint16_t)(w[i] >> 16));
    }
}

__device__ __forceinline__ uint4 pack8(const float (&f)[8])
{
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        w[i] = (uint32_t)f2bf(f[2 * i]) | ((uint32_t)f2bf(f[2 * i + 1]) << 16);
    return make_uint4(w[0], w[1], w[2], w[3]);
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

// Staged tiles of the convolution kernels: rows of 32 bf16 values padded to
// 40 (80 bytes), so that the 8-byte fragment reads of a wave's lanes spread
// over the LDS banks.
constexpr int kConvBK = 32;
constexpr int kConvLd = kConvBK + 8;

__device__ __forceinline__ v4s lds4(const uint16_t *p)
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
// N = Cout, K = 9*Cin.  A block computes 64 pixels x BN output channels
// (BN | Cout).  The K loop takes chunks of KC = 32 (16 if Cin is an odd
// multiple of 16) input channels of one tap: the block stages the chunk's
// 64 x KC input values and BN x KC weights in LDS with one 16-byte load per
// thread each (double-buffered, the next chunk's loads in flight during the
// current chunk's matrix-core products); wave w multiplies pixels 16w..16w+15
// with every 16-channel fragment of the block.  Output channel co of pixel p
// goes to y[p*ldy + yoff + co] with bias and activation applied, bf16 or
// fp32.  Grid: (ceil(P/64), Cout/BN).
template <int ACT, bool OUTF32, int BN>
__global__ __launch_bounds__(256) void k_conv3x3(const uint16_t *__restrict__ x, int N, int H, int W, int Cin,
                                                 const uint16_t *__restrict__ w, const float *__restrict__ bias,
                                                 int Cout, void *__restrict__ y, int ldy, int yoff)
{
    constexpr int NF = BN / 16;
    __shared__ __align__(16) uint16_t sA[2][64 * kConvLd];
    __shared__ __align__(16) uint16_t sB[2][BN * kConvLd];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m = lane & 15, g = lane >> 4;
    const int P = N * H * W;
    const int p0 = blockIdx.x * 64;
    const int co0 = blockIdx.y * BN;
    const int kc = (Cin % 32 == 0) ? 32 : 16;
    const int ncc = Cin / kc;
    const int nk = 9 * ncc;
    // staging roles: thread t stages 8 channels (part t % 4) of pixel t / 4
    // and 8 k-values of weight row t / 4
    const int sp = tid >> 2, part = tid & 3;
    const bool pact = part * 8 < kc;
    const int pa = p0 + sp;
    int an = 0, ay = 0, ax = 0;
    if (pa < P) {
        an = pa / (H * W);
        const int r = pa - an * H * W;
        ay = r / W;
        ax = r - ay * W;
    }
    auto load_chunk = [&](int kk, uint4 &ra, uint4 &rb) {
        const int tap = kk / ncc, c0 = (kk - tap * ncc) * kc;
        ra = make_uint4(0u, 0u, 0u, 0u);
        rb = make_uint4(0u, 0u, 0u, 0u);
        if (pact && pa < P) {
            const int sy = ay + tap / 3 - 1, sx = ax + tap % 3 - 1;
            if (sy >= 0 && sy < H && sx >= 0 && sx < W)
                ra = *reinterpret_cast<const uint4 *>(x + ((size_t)(an * H + sy) * W + sx) * Cin + c0 + part * 8);
        }
        if (pact && sp < BN)
            rb = *reinterpret_cast<const uint4 *>(w + ((size_t)(co0 + sp) * 9 + tap) * Cin + c0 + part * 8);
    };
    auto store_chunk = [&](int buf, const uint4 &ra, const uint4 &rb) {
        if (pact) {
            *reinterpret_cast<uint4 *>(&sA[buf][sp * kConvLd + part * 8]) = ra;
            if (sp < BN)
                *reinterpret_cast<uint4 *>(&sB[buf][sp * kConvLd + part * 8]) = rb;
        }
    };
    v4f acc[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f)
        acc[f] = v4f{0.f, 0.f, 0.f, 0.f};
    uint4 ra, rb;
    load_chunk(0, ra, rb);
    store_chunk(0, ra, rb);
    __syncthreads();
    for (int kk = 0; kk < nk; ++kk) {
        const int cur = kk & 1;
        if (kk + 1 < nk)
            load_chunk(kk + 1, ra, rb);
        for (int k16 = 0; k16 < kc / 16; ++k16) {
            const v4s a = lds4(&sA[cur][(wave * 16 + m) * kConvLd + k16 * 16 + 4 * g]);
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const v4s b = lds4(&sB[cur][(f * 16 + m) * kConvLd + k16 * 16 + 4 * g]);
                acc[f] = mfma16(a, b, acc[f]);
            }
        }
        if (kk + 1 < nk)
            store_chunk(cur ^ 1, ra, rb);
        __syncthreads();
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const int co = co0 + f * 16 + m;
        const float bv = bias ? bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int pp = p0 + wave * 16 + 4 * g + i;
            if (pp < P) {
                float v = acc[f][i] + bv;
                if (ACT == ACT_LEAKY)
                    v = v > 0.f ? v : kLeak * v;
                if (OUTF32)
                    reinterpret_cast<float *>(y)[(size_t)pp * ldy + yoff + co] = v;
                else
                    reinterpret_cast<uint16_t *>(y)[(size_t)pp * ldy + yoff + co] = f2bf(v);
            }
        }
    }
}

// 3x3 convolution on the gfx950 double-K matrix cores: the same implicit
// GEMM (M = N*H*W pixels, N = Cout, K = 9*Cin), in block tiles of BM = 128
// pixels x BN output channels with more products per staged byte.
//
// - v_mfma_f32_16x16x32_bf16: a lane supplies 8 consecutive k of row
//   m = lane % 16 of A and of column m of B (k group lane / 16), and receives
//   D[4 (lane / 16) + r][lane % 16], r = 0..3.  The order of k within a
//   fragment is the same for A and B, so it does not enter the sum.
// - The 4 waves tile the block WM x (4 / WM); a wave owns a TM x TN sub-tile
//   of FM x FN 16 x 16 fragments, so every A fragment it reads from LDS
//   feeds FN products and every B fragment FM.
// - A K stage is KC = 64 consecutive k (64 input channels of one tap) when
//   Cin is a multiple of 64, else 32 (Cin a multiple of 32) or 16 (the
//   input layer: the upper 16 k of each staged row stay zero).  The stage's
//   128 x KC inputs and BN x KC weights go to LDS with 16-byte loads, double
//   buffered: the next stage's loads are in flight during the current
//   stage's products.  LDS rows are padded by 8 bf16 against bank
//   conflicts.
// Output as k_conv3x3.  Grid: (ceil(P / 128), Cout / BN), 256 threads.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ v4f mfma16x32(v8bf a, v8bf b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ v8bf lds8(const uint16_t *p)
{
    const uint4 u = *reinterpret_cast<const uint4 *>(p);
    v8bf r;
    __builtin_memcpy(&r, &u, 16);
    return r;
}

template <int KC>
constexpr int conv_mfma_ld() { return KC + 8; }

template <int BN, int KC>
constexpr int conv_mfma_lds_bytes() { return 2 * (128 + BN) * conv_mfma_ld<KC>() * 2; }

// Staging of a block's 128 x BN outputs for vector stores: rows of BN
// values padded by 16 bytes.
template <bool F32, int BN>
constexpr int conv_out_ld() { return BN + (F32 ? 4 : 8); }
template <bool F32, int BN>
constexpr int conv_out_lds_bytes() { return 128 * conv_out_ld<F32, BN>() * (F32 ? 4 : 2); }

// True if output rows y + p * ldy + off (in values) start on 16 bytes for
// every pixel p, so that a pixel's run of channels can leave in 16-byte
// stores.
template <bool F32>
__device__ __forceinline__ bool conv_out_vec_ok(const void *y, int ldy, int off)
{
    constexpr int q = F32 ? 4 : 8;
    return ldy % q == 0 && off % q == 0 && (reinterpret_cast<uintptr_t>(y) & 15) == 0;
}

// The block's 128 x BN outputs, act(acc + bias), stored through LDS: each
// wave writes its fragments (lane m, g of fragment (i, j) holds pixels
// 4g..4g+3 of row block i, channel m of column block j) into a [128][BN]
// staging tile, then every thread stores 16-byte runs of one pixel's
// channels.  A fragment store of the lanes would otherwise write 2- or
// 4-byte values, 16 channels of 4 pixels per instruction.  pix(pm) is the
// output pixel of block pixel pm (-1: none); outputs go to y[pix * ldy +
// off + c], c < BN, with conv_out_vec_ok(y, ldy, off).  The staging tile
// reuses the kernel's LDS: the caller's last use of it must be behind a
// barrier.
template <int ACT, bool F32, int BN, int WM, int FM, int FN, class Pix>
__device__ __forceinline__ void conv_store_vec(const v4f (&acc)[FM][FN], const float *bias, void *y, int ldy, int off,
                                               void *smem, Pix pix)
{
    constexpr int WN = 4 / WM, TM = 128 / WM, TN = BN / WN;
    constexpr int OE = F32 ? 4 : 2;
    constexpr int LDO = conv_out_ld<F32, BN>();
    constexpr int NPART = BN * OE / 16;  // 16-byte parts of a pixel's outputs
    static_assert(NPART >= 2 && 128 * NPART % 256 == 0, "whole parts per thread");
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m = lane & 15, g = lane >> 4;
    const int wm = wave % WM, wn = wave / WM;
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int c = wn * TN + j * 16 + m;
        const float bv = bias ? bias[c] : 0.f;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int pm = wm * TM + i * 16 + 4 * g + r;
                float v = acc[i][j][r] + bv;
                if (ACT == ACT_LEAKY)
                    v = v > 0.f ? v : kLeak * v;
                if (F32)
                    reinterpret_cast<float *>(smem)[pm * LDO + c] = v;
                else
                    reinterpret_cast<uint16_t *>(smem)[pm * LDO + c] = f2bf(v);
            }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 128 * NPART / 256; ++s) {
        const int e = tid + 256 * s;
        const int pm = e / NPART, part = e - pm * NPART;
        const int64_t pp = pix(pm);
        if (pp >= 0) {
            const uint4 v = *reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(smem) +
                                                             (size_t)pm * LDO * OE + part * 16);
            *reinterpret_cast<uint4 *>(reinterpret_cast<char *>(y) + ((size_t)pp * ldy + off) * OE + part * 16) = v;
        }
    }
}

template <int ACT, bool OUTF32, int BN, int WM, int KC, bool SPLIT>
__global__ __launch_bounds__(256, 2) void k_conv3x3_mfma(const uint16_t *__restrict__ x, int N, int H, int W,
                                                         int Cin, const uint16_t *__restrict__ w,
                                                         const float *__restrict__ bias, int Cout,
                                                         void *__restrict__ y, int ldy, int yoff, int nsplit)
{
    constexpr int BM = 128, WN = 4 / WM;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 16, FN = TN / 16;
    constexpr int LD = conv_mfma_ld<KC>();
    constexpr int KQ = KC / 8;               // 16-byte parts of a staged row
    constexpr int NA = BM * KQ / 256;        // A loads per thread and stage
    constexpr int NB = (BN * KQ + 255) / 256;  // B loads per thread and stage
    static_assert(WM * WN == 4 && FM >= 1 && FN >= 1, "4 waves tile the block");
    static_assert(BM * KQ % 256 == 0, "A parts divide over the threads");
    extern __shared__ __align__(16) uint16_t conv_smem[];
    uint16_t *sA = conv_smem;                 // [2][BM][LD]
    uint16_t *sB = conv_smem + 2 * BM * LD;   // [2][BN][LD]
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m = lane & 15, g = lane >> 4;
    const int wm = wave % WM, wn = wave / WM;
    const int P = N * H * W;
    const int p0 = blockIdx.x * BM;
    const int co0 = blockIdx.y * BN;
    const int kc = Cin % KC == 0 ? KC : 16;  // channels per stage (16: the input layer, KC = 32)
    const int ncc = Cin / kc;
    const int nk_all = 9 * ncc;
    // split K (SPLIT): block z takes stages [k_begin, k_end) and writes its
    // fp32 partial sums to y + z * P * Cout ([z][p][co]), summed by
    // k_conv_split_sum in a fixed order
    const int z = SPLIT ? (int)blockIdx.z : 0;
    const int k_begin = SPLIT ? (int)((int64_t)nk_all * z / nsplit) : 0;
    const int k_end = SPLIT ? (int)((int64_t)nk_all * (z + 1) / nsplit) : nk_all;
    // staging roles: A part e = tid + 256 i: pixel e / KQ, 8 channels (e % KQ);
    // B part e: weight row e / KQ, 8 k-values (e % KQ)
    int an[NA], ay[NA], ax[NA];
    bool aok[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const int pa = p0 + (tid + 256 * i) / KQ;
        aok[i] = pa < P;
        const int pp = aok[i] ? pa : 0;
        an[i] = pp / (H * W);
        const int r = pp - an[i] * H * W;
        ay[i] = r / W;
        ax[i] = r - ay[i] * W;
    }
    struct Regs {
        uint4 a[NA], b[NB];
    };
    auto load_stage = [&](int kk, Regs &rg) {
        const int tap = kk / ncc, c0 = (kk - tap * ncc) * kc;
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int part = (tid + 256 * i) % KQ;
            rg.a[i] = make_uint4(0u, 0u, 0u, 0u);
            const int sy = ay[i] + dy, sx = ax[i] + dx;
            if (aok[i] && part * 8 < kc && sy >= 0 && sy < H && sx >= 0 && sx < W)
                rg.a[i] = *reinterpret_cast<const uint4 *>(x + ((size_t)(an[i] * H + sy) * W + sx) * Cin + c0 + part * 8);
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int e = tid + 256 * i;
            const int row = e / KQ, part = e % KQ;
            rg.b[i] = make_uint4(0u, 0u, 0u, 0u);
            if (e < BN * KQ && part * 8 < kc)
                rg.b[i] = *reinterpret_cast<const uint4 *>(w + ((size_t)(co0 + row) * 9 + tap) * Cin + c0 + part * 8);
        }
    };
    auto store_stage = [&](int buf, const Regs &rg) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int e = tid + 256 * i;
            *reinterpret_cast<uint4 *>(&sA[(buf * BM + e / KQ) * LD + (e % KQ) * 8]) = rg.a[i];
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int e = tid + 256 * i;
            if (e < BN * KQ)
                *reinterpret_cast<uint4 *>(&sB[(buf * BN + e / KQ) * LD + (e % KQ) * 8]) = rg.b[i];
        }
    };
    v4f acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    auto compute = [&](int buf) {
        const uint16_t *cA = sA + (buf * BM + wm * TM) * LD;
        const uint16_t *cB = sB + (buf * BN + wn * TN) * LD;
#pragma unroll
        for (int k32 = 0; k32 < KC / 32; ++k32) {
            v8bf av[FM], bv[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                av[i] = lds8(cA + (i * 16 + m) * LD + k32 * 32 + 8 * g);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                bv[j] = lds8(cB + (j * 16 + m) * LD + k32 * 32 + 8 * g);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = mfma16x32(av[i], bv[j], acc[i][j]);
        }
    };
    // Two register sets, so a stage's global loads are issued two stages
    // before their data is written to LDS (about two stages of products hide
    // their latency); two LDS buffers, one barrier per stage.  The loop is
    // unrolled by two so that the register sets are addressed statically.
    Regs r0, r1;
    const int nk = k_end - k_begin;
    if (nk > 0)
        load_stage(k_begin, r0);
    if (nk > 1)
        load_stage(k_begin + 1, r1);
    if (nk > 0)
        store_stage(0, r0);
    __syncthreads();
    for (int t = 0; t < nk; t += 2) {
        // stage t in LDS buffer 0, its successor's loads in r1
        if (t + 2 < nk)
            load_stage(k_begin + t + 2, r0);
        compute(0);
        if (t + 1 < nk)
            store_stage(1, r1);
        __syncthreads();
        if (t + 1 >= nk)
            break;
        // stage t + 1 in LDS buffer 1, stage t + 2's loads in r0
        if (t + 3 < nk)
            load_stage(k_begin + t + 3, r1);
        compute(1);
        if (t + 2 < nk)
            store_stage(0, r0);
        __syncthreads();
    }
    // the loop ended on a barrier: the staging LDS is free
    auto pix = [&](int pm) -> int64_t { return p0 + pm < P ? (int64_t)p0 + pm : -1; };
    if constexpr (SPLIT && conv_out_lds_bytes<true, BN>() <= conv_mfma_lds_bytes<BN, KC>()) {
        float *part = reinterpret_cast<float *>(y) + (size_t)z * P * Cout;
        if (conv_out_vec_ok<true>(part, Cout, co0)) {
            conv_store_vec<ACT_NONE, true, BN, WM>(acc, nullptr, part, Cout, co0, conv_smem, pix);
            return;
        }
    }
    if constexpr (!SPLIT && conv_out_lds_bytes<OUTF32, BN>() <= conv_mfma_lds_bytes<BN, KC>()) {
        if (conv_out_vec_ok<OUTF32>(y, ldy, yoff)) {
            conv_store_vec<ACT, OUTF32, BN, WM>(acc, bias ? bias + co0 : nullptr, y, ldy, yoff + co0, conv_smem, pix);
            return;
        }
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int co = co0 + wn * TN + j * 16 + m;
        const float bv = (!SPLIT && bias) ? bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int pp = p0 + wm * TM + i * 16 + 4 * g + r;
                if (pp < P) {
                    if (SPLIT) {
                        reinterpret_cast<float *>(y)[((size_t)z * P + pp) * Cout + co] = acc[i][j][r];
                        continue;
                    }
                    float v = acc[i][j][r] + bv;
                    if (ACT == ACT_LEAKY)
                        v = v > 0.f ? v : kLeak * v;
                    if (OUTF32)
                        reinterpret_cast<float *>(y)[(size_t)pp * ldy + yoff + co] = v;
                    else
                        reinterpret_cast<uint16_t *>(y)[(size_t)pp * ldy + yoff + co] = f2bf(v);
                }
            }
    }
}

// 3x3 convolution from a staged halo patch (images with W % 16 == 0 and
// H % 8 == 0).  The block's 128 output pixels are an 8 x 16 patch of one
// image; for each chunk of KC input channels the block stages the patch's
// 10 x 18 input pixels once in LDS, and the 9 taps read their A fragments
// from it at shifted positions (fragment rows are 16 consecutive pixels of a
// patch row, so a shifted fragment is 16 consecutive staged pixels).  That
// loads each input value about 1.4 times instead of 9.  K stages are
// (chunk, group of TG taps) with the weights of TG taps per stage (TG = 3,
// a row of the stencil, for narrow layers: more products per barrier),
// double-buffered and loaded two stages ahead as in k_conv3x3_mfma; the
// next chunk's patch is loaded into registers during the current chunk's
// first stage and written over the one patch buffer behind a barrier after
// its last (one buffer: less LDS per block, more blocks per CU).  Output as
// k_conv3x3.  pool (bf16 outputs only; NULL for none): also the 2 x 2
// average pooling of the outputs, N x H/2 x W/2 x Cout, from the staged
// tile; the caller passes it only where the staged stores apply
// (conv_out_vec_ok) and pool is 16-byte aligned.
// Grid: (N (H / 8) (W / 16), Cout / BN), 256 threads.
constexpr int kPatchH = 8, kPatchW = 16;
constexpr int kHaloPix = (kPatchH + 2) * (kPatchW + 2);

template <int BN, int KC, int TG>
constexpr int conv_halo_lds_bytes() { return (kHaloPix + 2 * TG * BN) * conv_mfma_ld<KC>() * 2; }

template <int ACT, bool OUTF32, int BN, int WM, int KC, int TG>
__global__ __launch_bounds__(256, 2) void k_conv3x3_halo(const uint16_t *__restrict__ x, int N, int H, int W,
                                                         int Cin, const uint16_t *__restrict__ w,
                                                         const float *__restrict__ bias, int Cout,
                                                         void *__restrict__ y, int ldy, int yoff,
                                                         uint16_t *__restrict__ pool)
{
    constexpr int BM = 128, WN = 4 / WM;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 16, FN = TN / 16;
    constexpr int LD = conv_mfma_ld<KC>();
    constexpr int KQ = KC / 8;
    constexpr int NP = (kHaloPix * KQ + 255) / 256;  // patch loads per thread and chunk
    constexpr int NB = (TG * BN * KQ + 255) / 256;   // weight loads per thread and stage
    constexpr int SPC = 9 / TG;                      // stages per chunk
    static_assert(WM * WN == 4 && FM >= 1 && FN >= 1, "4 waves tile the block");
    static_assert(BM == kPatchH * kPatchW, "the block's pixels are one patch");
    static_assert(TG == 1 || TG == 3, "whole stencil rows or single taps");
    extern __shared__ __align__(16) uint16_t conv_smem[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m = lane & 15, g = lane >> 4;
    const int wm = wave % WM, wn = wave / WM;
    const int tiles_x = W / kPatchW, tiles_y = H / kPatchH;
    const int bx = blockIdx.x % tiles_x, rest = blockIdx.x / tiles_x;
    const int by = rest % tiles_y, bn = rest / tiles_y;
    const int y0 = by * kPatchH - 1, x0 = bx * kPatchW - 1;  // image position of staged pixel 0
    const int co0 = blockIdx.y * BN;
    const int kc = Cin % KC == 0 ? KC : 16;
    const int ncc = Cin / kc;
    const int nk = SPC * ncc;
    uint16_t *sP = conv_smem;                  // [kHaloPix][LD]
    uint16_t *sB = conv_smem + kHaloPix * LD;  // [2][TG][BN][LD]
    uint4 rp[NP];
    auto load_patch = [&](int c) {
        const int c0 = c * kc;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int e = tid + 256 * i;
            const int pix = e / KQ, part = e % KQ;
            const int sy = y0 + pix / (kPatchW + 2), sx = x0 + pix % (kPatchW + 2);
            rp[i] = make_uint4(0u, 0u, 0u, 0u);
            if (pix < kHaloPix && part * 8 < kc && sy >= 0 && sy < H && sx >= 0 && sx < W)
                rp[i] = *reinterpret_cast<const uint4 *>(x + ((size_t)(bn * H + sy) * W + sx) * Cin + c0 + part * 8);
        }
    };
    auto store_patch = [&](int buf) {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int e = tid + 256 * i;
            if (e < kHaloPix * KQ)
                *reinterpret_cast<uint4 *>(&sP[(buf * kHaloPix + e / KQ) * LD + (e % KQ) * 8]) = rp[i];
        }
    };
    struct Regs {
        uint4 b[NB];
    };
    // stage s: chunk s / SPC, taps TG (s % SPC) .. + TG - 1; staged weight
    // row tg * BN + co holds tap TG (s % SPC) + tg of output channel co0 + co
    auto load_w = [&](int s, Regs &rg) {
        const int c = s / SPC, tap0 = (s - SPC * c) * TG, c0 = c * kc;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int e = tid + 256 * i;
            const int row = e / KQ, part = e % KQ;
            const int tg = row / BN, co = row - tg * BN;
            rg.b[i] = make_uint4(0u, 0u, 0u, 0u);
            if (e < TG * BN * KQ && part * 8 < kc)
                rg.b[i] = *reinterpret_cast<const uint4 *>(w + ((size_t)(co0 + co) * 9 + tap0 + tg) * Cin + c0 + part * 8);
        }
    };
    auto store_w = [&](int buf, const Regs &rg) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int e = tid + 256 * i;
            if (e < TG * BN * KQ)
                *reinterpret_cast<uint4 *>(&sB[(buf * TG * BN + e / KQ) * LD + (e % KQ) * 8]) = rg.b[i];
        }
    };
    v4f acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    // stage s: chunk s / SPC (patch buffer (s / SPC) & 1), weights in buffer wb
    auto compute = [&](int s, int wb) {
        const int c = s / SPC, tap0 = (s - SPC * c) * TG;
        const uint16_t *cP = sP;
#pragma unroll
        for (int tg = 0; tg < TG; ++tg) {
            const int tap = tap0 + tg;
            const int dy = tap / 3, dx = tap % 3;  // offsets into the staged patch (halo 1)
            const uint16_t *cB = sB + ((wb * TG + tg) * BN + wn * TN) * LD;
#pragma unroll
            for (int k32 = 0; k32 < KC / 32; ++k32) {
                v8bf av[FM], bv[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    const int py = (wm * TM + i * 16) / kPatchW;  // the fragment's patch row
                    av[i] = lds8(cP + ((py + dy) * (kPatchW + 2) + dx + m) * LD + k32 * 32 + 8 * g);
                }
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    bv[j] = lds8(cB + (j * 16 + m) * LD + k32 * 32 + 8 * g);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = mfma16x32(av[i], bv[j], acc[i][j]);
            }
        }
    };
    // the patch of the next chunk: loaded at its predecessor's first stage;
    // stored after the barrier that ends its predecessor's last, then a
    // barrier before the first stage that reads it
    auto patch_load = [&](int s) {
        const int c = s / SPC, q = s - SPC * c;
        if (q == 0 && c + 1 < ncc)
            load_patch(c + 1);
    };
    auto patch_flush = [&](int s) {
        const int c = s / SPC, q = s - SPC * c;
        if (q == SPC - 1 && c + 1 < ncc) {
            store_patch(0);
            __syncthreads();
        }
    };
    Regs r0, r1;
    load_patch(0);
    load_w(0, r0);
    if (nk > 1)
        load_w(1, r1);
    store_patch(0);
    store_w(0, r0);
    __syncthreads();
    for (int t = 0; t < nk; t += 2) {
        if (t + 2 < nk)
            load_w(t + 2, r0);
        patch_load(t);
        compute(t, 0);
        if (t + 1 < nk)
            store_w(1, r1);
        __syncthreads();
        patch_flush(t);
        if (t + 1 >= nk)
            break;
        if (t + 3 < nk)
            load_w(t + 3, r1);
        patch_load(t + 1);
        compute(t + 1, 1);
        if (t + 2 < nk)
            store_w(0, r0);
        __syncthreads();
        patch_flush(t + 1);
    }
    // the loop ended on a barrier: the staging LDS is free
    if constexpr (conv_out_lds_bytes<OUTF32, BN>() <= conv_halo_lds_bytes<BN, KC, TG>()) {
        if (conv_out_vec_ok<OUTF32>(y, ldy, yoff)) {
            auto pix = [&](int pm) -> int64_t {
                return (int64_t)(bn * H + by * kPatchH + pm / kPatchW) * W + bx * kPatchW + pm % kPatchW;
            };
            conv_store_vec<ACT, OUTF32, BN, WM>(acc, bias ? bias + co0 : nullptr, y, ldy, yoff + co0, conv_smem, pix);
            if constexpr (!OUTF32) {
                // the 2 x 2 averages of the staged outputs (the bf16 values
                // just stored), with the arithmetic of k_pool2_v8: the patch
                // holds 4 x 8 whole pooling windows
                if (pool) {
                    constexpr int LDO = conv_out_ld<false, BN>(), NQ = BN / 8;
                    constexpr int QH = kPatchH / 2, QW = kPatchW / 2;
                    const uint16_t *so = conv_smem;
                    const int Ho = H / 2, Wo = W / 2;
                    for (int e = tid; e < QH * QW * NQ; e += 256) {
                        const int pq = e / NQ, part = e - pq * NQ;
                        const int pi = pq / QW, pj = pq - pi * QW;
                        const int pm = 2 * pi * kPatchW + 2 * pj;
                        float a[8], b[8], c[8], d[8], o[8];
                        unpack8(*reinterpret_cast<const uint4 *>(so + pm * LDO + part * 8), a);
                        unpack8(*reinterpret_cast<const uint4 *>(so + (pm + 1) * LDO + part * 8), b);
                        unpack8(*reinterpret_cast<const uint4 *>(so + (pm + kPatchW) * LDO + part * 8), c);
                        unpack8(*reinterpret_cast<const uint4 *>(so + (pm + kPatchW + 1) * LDO + part * 8), d);
#pragma unroll
                        for (int t = 0; t < 8; ++t)
                            o[t] = 0.25f * (a[t] + b[t] + c[t] + d[t]);
                        const size_t q = (size_t)(bn * Ho + by * QH + pi) * Wo + bx * QW + pj;
                        *reinterpret_cast<uint4 *>(pool + q * Cout + co0 + part * 8) = pack8(o);
                    }
                }
            }
            return;
        }
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int co = co0 + wn * TN + j * 16 + m;
        const float bv = bias ? bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int pm = wm * TM + i * 16 + 4 * g + r;  // pixel of the patch
                const size_t pp = (size_t)(bn * H + by * kPatchH + pm / kPatchW) * W + bx * kPatchW + pm % kPatchW;
                float v = acc[i][j][r] + bv;
                if (ACT == ACT_LEAKY)
                    v = v > 0.f ? v : kLeak * v;
                if (OUTF32)
                    reinterpret_cast<float *>(y)[pp * ldy + yoff + co] = v;
                else
                    reinterpret_cast<uint16_t *>(y)[pp * ldy + yoff + co] = f2bf(v);
            }
    }
}

// The split-K sums: y[p * ldy + yoff + c] = act(sum over z of part[z][p][c]
// (z = 0, 1, ... in order) + bias[c]), bf16 or fp32.  Grid-stride over the
// P * C outputs.
template <int ACT, bool OUTF32>
__global__ __launch_bounds__(256) void k_conv_split_sum(const float *__restrict__ part, int nsplit, int P, int C,
                                                       const float *__restrict__ bias, void *__restrict__ y,
                                                       int ldy, int yoff)
{
    const int64_t n = (int64_t)P * C;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int c = (int)(e % C);
        const int64_t p = e / C;
        float v = 0.f;
        for (int z = 0; z < nsplit; ++z)
            v += part[(size_t)z * n + e];
        if (bias)
            v += bias[c];
        if (ACT == ACT_LEAKY)
            v = v > 0.f ? v : kLeak * v;
        if (OUTF32)
            reinterpret_cast<float *>(y)[p * ldy + yoff + c] = v;
        else
            reinterpret_cast<uint16_t *>(y)[p * ldy + yoff + c] = f2bf(v);
    }
}

// The same sums four channels per thread (16-byte partial and bias loads),
// for C, ldy and yoff multiples of 4 and y aligned to the output's 4-value
// run: the same arithmetic per value, so the same bits.
template <int ACT, bool OUTF32>
__global__ __launch_bounds__(256) void k_conv_split_sum_v4(const float *__restrict__ part, int nsplit, int P, int C,
                                                          const float *__restrict__ bias, void *__restrict__ y,
                                                          int ldy, int yoff)
{
    const int64_t n = (int64_t)P * C, n4 = n / 4;
    for (int64_t e4 = (int64_t)blockIdx.x * 256 + threadIdx.x; e4 < n4; e4 += (int64_t)gridDim.x * 256) {
        const int64_t e = e4 * 4;
        const int c = (int)(e % C);
        const int64_t p = e / C;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int z = 0; z < nsplit; ++z) {
            const float4 q = *reinterpret_cast<const float4 *>(part + (size_t)z * n + e);
            v.x += q.x;
            v.y += q.y;
            v.z += q.z;
            v.w += q.w;
        }
        if (bias) {
            const float4 b = *reinterpret_cast<const float4 *>(bias + c);
            v.x += b.x;
            v.y += b.y;
            v.z += b.z;
            v.w += b.w;
        }
        if (ACT == ACT_LEAKY) {
            v.x = v.x > 0.f ? v.x : kLeak * v.x;
            v.y = v.y > 0.f ? v.y : kLeak * v.y;
            v.z = v.z > 0.f ? v.z : kLeak * v.z;
            v.w = v.w > 0.f ? v.w : kLeak * v.w;
        }
        if (OUTF32) {
            *reinterpret_cast<float4 *>(reinterpret_cast<float *>(y) + p * ldy + yoff + c) = v;
        } else {
            uint2 o;
            o.x = (uint32_t)f2bf(v.x) | ((uint32_t)f2bf(v.y) << 16);
            o.y = (uint32_t)f2bf(v.z) | ((uint32_t)f2bf(v.w) << 16);
            *reinterpret_cast<uint2 *>(reinterpret_cast<uint16_t *>(y) + p * ldy + yoff + c) = o;
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
// sum over the pixels p of split s of dy[p][co] * x[p shifted by tap][ci].
// GEMM M = Cout, N = 9*Cin, K = pixels.  A block computes 64 output
// channels (co0..co0+63, those below Cout) x CW columns (one tap, CW = 32 or
// 16 input channels) over its split; pixel chunks of 32 are staged in LDS
// transposed (channel rows, pixel columns) so that every fragment read is
// 8 contiguous bytes; wave w owns channels co0 + 16w .. +15.  Grid: (nsplit,
// ceil(Cout/64), 9*Cin/CW), 256 threads.
__global__ __launch_bounds__(256) void k_conv3x3_wgrad(const uint16_t *__restrict__ x, int N, int H, int W,
                                                      int Cin, const uint16_t *__restrict__ dy, int Cout,
                                                      int chunk, float *__restrict__ part)
{
    __shared__ __align__(16) uint16_t sA[64 * kConvLd];  // dy^T: 64 channels x 32 pixels
    __shared__ __align__(16) uint16_t sB[32 * kConvLd];  // x^T: CW channels x 32 pixels
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m = lane & 15, g = lane >> 4;
    const int s = blockIdx.x, co0 = blockIdx.y * 64;
    const int CW = (Cin % 32 == 0) ? 32 : 16;
    const int ncw = Cin / CW;
    const int tap = blockIdx.z / ncw, ci0 = (blockIdx.z - tap * ncw) * CW;
    const int dyo = tap / 3 - 1, dxo = tap % 3 - 1;
    const int P = N * H * W;
    const int pb = s * chunk, pe = min(P, pb + chunk);
    v4f acc[2] = {v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}};
    // staging roles: dy: thread t takes 8 channels (t % 8) of pixel t / 8;
    // x: thread t < 4 CW takes 8 channels (t % (CW/8)) of pixel t / (CW/8)
    const int ap = tid >> 3, apart = tid & 7;
    const int bq = CW / 8;
    const int bp = tid / bq, bpart = tid - bp * bq;
    for (int k0 = pb; k0 < pe; k0 += 32) {
        uint4 ra = make_uint4(0u, 0u, 0u, 0u), rb = make_uint4(0u, 0u, 0u, 0u);
        {
            const int p = k0 + ap;
            if (p < pe && co0 + apart * 8 < Cout)
                ra = *reinterpret_cast<const uint4 *>(dy + (size_t)p * Cout + co0 + apart * 8);
        }
        if (bp < 32) {
            const int p = k0 + bp;
            if (p < pe) {
                const int n = p / (H * W), r = p - n * H * W;
                const int yy = r / W, xx = r - yy * W;
                const int sy = yy + dyo, sx = xx + dxo;
                if (sy >= 0 && sy < H && sx >= 0 && sx < W)
                    rb = *reinterpret_cast<const uint4 *>(x + ((size_t)(n * H + sy) * W + sx) * Cin + ci0 + bpart * 8);
            }
        }
        __syncthreads();  // the previous chunk's fragment reads are done
        {
            const uint16_t *va = reinterpret_cast<const uint16_t *>(&ra);
#pragma unroll
            for (int j = 0; j < 8; ++j)
                sA[(apart * 8 + j) * kConvLd + ap] = va[j];
            if (bp < 32) {
                const uint16_t *vb = reinterpret_cast<const uint16_t *>(&rb);
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    sB[(bpart * 8 + j) * kConvLd + bp] = vb[j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k16 = 0; k16 < 2; ++k16) {
            const v4s a = lds4(&sA[(wave * 16 + m) * kConvLd + k16 * 16 + 4 * g]);
#pragma unroll
            for (int f = 0; f < 2; ++f)
                if (f * 16 < CW) {
                    const v4s b = lds4(&sB[(f * 16 + m) * kConvLd + k16 * 16 + 4 * g]);
                    acc[f] = mfma16(a, b, acc[f]);
                }
        }
    }
    // D[row = co0 + 16 wave + 4g + i][col = tap*Cin + ci0 + 16f + m]
    const int ncols = 9 * Cin;
#pragma unroll
    for (int f = 0; f < 2; ++f)
        if (f * 16 < CW) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = co0 + wave * 16 + 4 * g + i;
                if (co < Cout)
                    part[((size_t)s * Cout + co) * ncols + tap * Cin + ci0 + f * 16 + m] = acc[f][i];
            }
        }
}

// The weight gradient for layers with CO = 32 or 16 output channels: the
// same GEMM, but a block stages the dy tile of its CO channels once and
// applies it to TPB = 64 / CO taps (the x tiles of those taps staged side
// by side), so that the four waves are all busy: wave w takes output rows
// 16 (w % (CO / 16)) .. + 15 of tap slot w / (CO / 16).  Block z covers
// taps TPB * (z / ncw) .. + TPB - 1 (those past the ninth idle) and input
// channels (z % ncw) CW .. + CW - 1.  Each wave's products run in the same
// order as in k_conv3x3_wgrad.
template <int CO>
__global__ __launch_bounds__(256) void k_conv3x3_wgrad_narrow(const uint16_t *__restrict__ x, int N, int H, int W,
                                                             int Cin, const uint16_t *__restrict__ dy, int Cout,
                                                             int chunk, float *__restrict__ part)
{
    constexpr int TPB = 64 / CO, FR = CO / 16;
    __shared__ __align__(16) uint16_t sA[CO * kConvLd];        // dy^T: CO channels x 32 pixels
    __shared__ __align__(16) uint16_t sB[TPB * 32 * kConvLd];  // x^T per tap slot: CW channels x 32 pixels
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m = lane & 15, g = lane >> 4;
    const int s = blockIdx.x;
    const int CW = (Cin % 32 == 0) ? 32 : 16;
    const int ncw = Cin / CW;
    const int tap0 = TPB * (blockIdx.z / ncw), ci0 = (blockIdx.z % ncw) * CW;
    const int P = N * H * W;
    const int pb = s * chunk, pe = min(P, pb + chunk);
    const int wfr = wave % FR, wslot = wave / FR;
    const bool wtap = tap0 + wslot < 9;
    v4f acc[2] = {v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}};
    // staging roles: dy: thread t < 4 CO takes 8 channels (t % (CO/8)) of
    // pixel t / (CO/8); x: item e < TPB 32 (CW/8) (thread t takes e = t,
    // t + 256) is tap slot e / (4 CW), then 8 channels of one of the 32
    // pixels
    constexpr int aq = CO / 8;
    constexpr int NBX = (TPB * 32 * 4 + 255) / 256;  // x items per thread at CW = 32
    const int ap = tid / aq, apart = tid - ap * aq;
    const int bq = CW / 8;
    const int nbx = TPB * 32 * bq;
    for (int k0 = pb; k0 < pe; k0 += 32) {
        uint4 ra = make_uint4(0u, 0u, 0u, 0u), rb[NBX];
        if (ap < 32) {
            const int p = k0 + ap;
            if (p < pe)
                ra = *reinterpret_cast<const uint4 *>(dy + (size_t)p * Cout + apart * 8);
        }
#pragma unroll
        for (int i = 0; i < NBX; ++i) {
            const int e = tid + 256 * i;
            rb[i] = make_uint4(0u, 0u, 0u, 0u);
            const int bslot = e / (32 * bq), bt = e - bslot * 32 * bq;
            const int bp = bt / bq, bpart = bt - bp * bq;
            const int btap = tap0 + bslot;
            const int p = k0 + bp;
            if (e < nbx && btap < 9 && p < pe) {
                const int n = p / (H * W), r = p - n * H * W;
                const int yy = r / W, xx = r - yy * W;
                const int sy = yy + btap / 3 - 1, sx = xx + btap % 3 - 1;
                if (sy >= 0 && sy < H && sx >= 0 && sx < W)
                    rb[i] = *reinterpret_cast<const uint4 *>(x + ((size_t)(n * H + sy) * W + sx) * Cin + ci0 +
                                                             bpart * 8);
            }
        }
        __syncthreads();  // the previous chunk's fragment reads are done
        {
            const uint16_t *va = reinterpret_cast<const uint16_t *>(&ra);
            if (ap < 32) {
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    sA[(apart * 8 + j) * kConvLd + ap] = va[j];
            }
#pragma unroll
            for (int i = 0; i < NBX; ++i) {
                const int e = tid + 256 * i;
                if (e < nbx) {
                    const int bslot = e / (32 * bq), bt = e - bslot * 32 * bq;
                    const int bp = bt / bq, bpart = bt - bp * bq;
                    const uint16_t *vb = reinterpret_cast<const uint16_t *>(&rb[i]);
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        sB[(bslot * 32 + bpart * 8 + j) * kConvLd + bp] = vb[j];
                }
            }
        }
        __syncthreads();
        if (wtap) {
#pragma unroll
            for (int k16 = 0; k16 < 2; ++k16) {
                const v4s a = lds4(&sA[(wfr * 16 + m) * kConvLd + k16 * 16 + 4 * g]);
#pragma unroll
                for (int f = 0; f < 2; ++f)
                    if (f * 16 < CW) {
                        const v4s b = lds4(&sB[(wslot * 32 + f * 16 + m) * kConvLd + k16 * 16 + 4 * g]);
                        acc[f] = mfma16(a, b, acc[f]);
                    }
            }
        }
    }
    if (!wtap)
        return;
    // D[row = 16 wfr + 4g + i][col = tap Cin + ci0 + 16f + m]
    const int ncols = 9 * Cin, tap = tap0 + wslot;
#pragma unroll
    for (int f = 0; f < 2; ++f)
        if (f * 16 < CW) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = wfr * 16 + 4 * g + i;
                part[((size_t)s * Cout + co) * ncols + tap * Cin + ci0 + f * 16 + m] = acc[f][i];
            }
        }
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

// Bias gradient partials: part[s][c] = sum over the pixels of split s of
// dy[p][c].  Thread t sums channel t % C over pixels t / C, t / C + 256 / C,
// ... (C <= 256 divides 256 or not: threads beyond (256 / C) C idle); the
// per-thread sums are added in fixed order through LDS.
__global__ __launch_bounds__(256) void k_bias_grad(const uint16_t *__restrict__ dy, int P, int C, int chunk,
                                                   float *__restrict__ part)
{
    __shared__ float red[256];
    const int s = blockIdx.x;
    const int pb = s * chunk, pe = min(P, pb + chunk);
    for (int c0 = 0; c0 < C; c0 += 256) {
        const int cw = min(256, C - c0);
        const int rows = 256 / cw;
        const int t = threadIdx.x, c = t % cw, r = t / cw;
        float acc = 0.f;
        if (r < rows)
            for (int p = pb + r; p < pe; p += rows)
                acc += bf2f(dy[(size_t)p * C + c0 + c]);
        red[t] = acc;
        __syncthreads();
        if (t < cw) {
            float v = 0.f;
            for (int k = 0; k < rows; ++k)
                v += red[k * cw + t];
            part[(size_t)s * C + c0 + t] = v;
        }
        __syncthreads();
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
__global__ __launch_bounds__(256) void k_pool2(const uint16_t *__restrict__ x, int ldx, int N, int H, int W, int C,
                                               uint16_t *__restrict__ y)
{
    const int Ho = H / 2, Wo = W / 2;
    const int n = N * Ho * Wo * C;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
        const int c = e % C, q = e / C;
        const int j = q % Wo, i = (q / Wo) % Ho, b = q / (Wo * Ho);
        const size_t base = ((size_t)(b * H + 2 * i) * W + 2 * j) * ldx + c;
        const float s = bf2f(x[base]) + bf2f(x[base + ldx]) + bf2f(x[base + (size_t)W * ldx]) +
                        bf2f(x[base + (size_t)W * ldx + ldx]);
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

// The same five kernels on groups of 8 channels (one 16-byte access per
// operand and thread); every channel count and channel offset a multiple of
// 8.  The arithmetic per element is that of the scalar kernels above, so the
// results are the same bits.
__global__ __launch_bounds__(256) void k_pool2_v8(const uint16_t *__restrict__ x, int ldx, int N, int H, int W,
                                                  int C, uint16_t *__restrict__ y)
{
    const int Ho = H / 2, Wo = W / 2, C8 = C / 8;
    const int64_t n = (int64_t)N * Ho * Wo * C8;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int c8 = (int)(e % C8);
        const int64_t q = e / C8;
        const int j = (int)(q % Wo), i = (int)((q / Wo) % Ho), b = (int)(q / ((int64_t)Wo * Ho));
        const size_t base = ((size_t)(b * H + 2 * i) * W + 2 * j) * ldx + 8 * c8;
        float a[8], bb[8], c[8], d[8], o[8];
        unpack8(*reinterpret_cast<const uint4 *>(x + base), a);
        unpack8(*reinterpret_cast<const uint4 *>(x + base + ldx), bb);
        unpack8(*reinterpret_cast<const uint4 *>(x + base + (size_t)W * ldx), c);
        unpack8(*reinterpret_cast<const uint4 *>(x + base + (size_t)W * ldx + ldx), d);
#pragma unroll
        for (int t = 0; t < 8; ++t)
            o[t] = 0.25f * (a[t] + bb[t] + c[t] + d[t]);
        *reinterpret_cast<uint4 *>(y + (size_t)q * C + 8 * c8) = pack8(o);
    }
}

__global__ __launch_bounds__(256) void k_pool2_bwd_v8(const uint16_t *__restrict__ dy, int N, int H, int W, int C,
                                                      uint16_t *__restrict__ dx)
{
    const int C8 = C / 8;
    const int64_t n = (int64_t)N * H * W * C8;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int c8 = (int)(e % C8);
        const int64_t q = e / C8;
        const int j = (int)(q % W), i = (int)((q / W) % H), b = (int)(q / ((int64_t)W * H));
        float g[8];
        unpack8(*reinterpret_cast<const uint4 *>(dy + ((size_t)(b * (H / 2) + i / 2) * (W / 2) + j / 2) * C + 8 * c8), g);
#pragma unroll
        for (int t = 0; t < 8; ++t)
            g[t] = 0.25f * g[t];
        *reinterpret_cast<uint4 *>(dx + (size_t)q * C + 8 * c8) = pack8(g);
    }
}

__global__ __launch_bounds__(256) void k_up2_v8(const uint16_t *__restrict__ x, int N, int H, int W, int C,
                                                uint16_t *__restrict__ y, int ldy, int yoff)
{
    const int Ho = 2 * H, Wo = 2 * W, C8 = C / 8;
    const int64_t n = (int64_t)N * Ho * Wo * C8;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int c8 = (int)(e % C8);
        const int64_t q = e / C8;
        const int j = (int)(q % Wo), i = (int)((q / Wo) % Ho), b = (int)(q / ((int64_t)Wo * Ho));
        *reinterpret_cast<uint4 *>(y + (size_t)q * ldy + yoff + 8 * c8) =
            *reinterpret_cast<const uint4 *>(x + ((size_t)(b * H + i / 2) * W + j / 2) * C + 8 * c8);
    }
}

__global__ __launch_bounds__(256) void k_up2_bwd_v8(const uint16_t *__restrict__ dy, int ldy, int yoff, int N, int H,
                                                    int W, int C, uint16_t *__restrict__ dx)
{
    const int C8 = C / 8, Wo = 2 * W;
    const int64_t n = (int64_t)N * H * W * C8;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int c8 = (int)(e % C8);
        const int64_t q = e / C8;
        const int j = (int)(q % W), i = (int)((q / W) % H), b = (int)(q / ((int64_t)W * H));
        const size_t r0 = (size_t)(b * 2 * H + 2 * i) * Wo + 2 * j;
        float a[8], bb[8], c[8], d[8], o[8];
        unpack8(*reinterpret_cast<const uint4 *>(dy + r0 * ldy + yoff + 8 * c8), a);
        unpack8(*reinterpret_cast<const uint4 *>(dy + (r0 + 1) * ldy + yoff + 8 * c8), bb);
        unpack8(*reinterpret_cast<const uint4 *>(dy + (r0 + Wo) * ldy + yoff + 8 * c8), c);
        unpack8(*reinterpret_cast<const uint4 *>(dy + (r0 + Wo + 1) * ldy + yoff + 8 * c8), d);
#pragma unroll
        for (int t = 0; t < 8; ++t)
            o[t] = a[t] + bb[t] + c[t] + d[t];
        *reinterpret_cast<uint4 *>(dx + (size_t)q * C + 8 * c8) = pack8(o);
    }
}

__global__ __launch_bounds__(256) void k_chan_copy_v8(const uint16_t *__restrict__ src, int lds_, int soff,
                                                      uint16_t *__restrict__ dst, int ldd, int doff, int P, int C,
                                                      int accumulate)
{
    const int C8 = C / 8;
    const int64_t n = (int64_t)P * C8;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int c8 = (int)(e % C8);
        const int64_t p = e / C8;
        const uint4 sv = *reinterpret_cast<const uint4 *>(src + (size_t)p * lds_ + soff + 8 * c8);
        uint4 *d = reinterpret_cast<uint4 *>(dst + (size_t)p * ldd + doff + 8 * c8);
        if (!accumulate) {
            *d = sv;  // bf16 -> fp32 -> bf16 is exact
        } else {
            float a[8], b[8];
            unpack8(sv, a);
            unpack8(*d, b);
#pragma unroll
            for (int t = 0; t < 8; ++t)
                a[t] = b[t] + a[t];
            *d = pack8(a);
        }
    }
}

__global__ __launch_bounds__(256) void k_act_bwd_v8(uint16_t *__restrict__ dy, const uint16_t *__restrict__ y,
                                                   int64_t n8)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n8; e += (int64_t)gridDim.x * 256) {
        float g[8], v[8];
        unpack8(reinterpret_cast<const uint4 *>(dy)[e], g);
        unpack8(reinterpret_cast<const uint4 *>(y)[e], v);
#pragma unroll
        for (int t = 0; t < 8; ++t)
            g[t] = v[t] > 0.f ? g[t] : kLeak * g[t];
        reinterpret_cast<uint4 *>(dy)[e] = pack8(g);
    }
}

// Bias gradient partials as k_bias_grad, 8 channels per thread (16-byte
// loads; C a multiple of 8): thread t takes channel group q0 + t % qw and
// pixels t / qw, t / qw + 256 / qw, ... of the split (qw = the groups of one
// pass, at most 256), and the per-thread sums are added in fixed order
// through LDS.
__global__ __launch_bounds__(256) void k_bias_grad_v8(const uint16_t *__restrict__ dy, int P, int C, int chunk,
                                                      float *__restrict__ part)
{
    __shared__ float red[256 * 8];
    const int s = blockIdx.x;
    const int pb = s * chunk, pe = min(P, pb + chunk);
    const int C8 = C / 8;
    for (int q0 = 0; q0 < C8; q0 += 256) {
        const int qw = min(256, C8 - q0);
        const int rows = 256 / qw;
        const int t = threadIdx.x, q = t % qw, r = t / qw;
        float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (r < rows)
            for (int p = pb + r; p < pe; p += rows) {
                float v[8];
                unpack8(*reinterpret_cast<const uint4 *>(dy + (size_t)p * C + 8 * (q0 + q)), v);
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    acc[k] += v[k];
            }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            red[t * 8 + k] = acc[k];
        __syncthreads();
        for (int e = t; e < qw * 8; e += 256) {
            const int gq = e / 8, k = e % 8;
            float v = 0.f;
            for (int rr = 0; rr < rows; ++rr)
                v += red[(rr * qw + gq) * 8 + k];
            part[(size_t)s * C + 8 * (q0 + gq) + k] = v;
        }
        __syncthreads();
    }
}

// out[e] = sum over s of part[s][e] for few outputs and many parts: one
// wave per output, lane l adding parts l, l + 64, ..., then a butterfly over
// the 64 lanes (a fixed order).
__global__ __launch_bounds__(64) void k_sum_parts_wave(const float *__restrict__ part, int nsplit, int n,
                                                       float *__restrict__ out)
{
    const int e = blockIdx.x, lane = threadIdx.x;
    float acc = 0.f;
    for (int s = lane; s < nsplit; s += 64)
        acc += part[(size_t)s * n + e];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        acc += __shfl_xor(acc, off, 64);
    if (lane == 0)
        out[e] = acc;
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

// Sum of squares, first pass: block b sums a[e]^2 in fp64 over e = b*256 +
// t + k*gridDim*256 (t = thread, fixed order), then over its threads in a
// fixed tree; part[b] = the block's sum.
__global__ __launch_bounds__(256) void k_sumsq_part(const float *__restrict__ a, int64_t n, double *__restrict__ part)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const double x = a[e];
        acc += x * x;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = red[0];
}

// Second pass, one block: out[0] = sum of part[0 .. np), np <= 256, in a
// fixed tree.
__global__ __launch_bounds__(256) void k_sumsq_fin(const double *__restrict__ part, int np, double *__restrict__ out)
{
    __shared__ double red[256];
    red[threadIdx.x] = threadIdx.x < np ? part[threadIdx.x] : 0.0;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[0] = red[0];
}

// Adam on fp32 master weights, then the bf16 copy the kernels read.  With
// gsq (the squared global gradient norm, on the device) the gradient is
// first scaled by min(1, max_norm / sqrt(*gsq)).
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ wm, float *__restrict__ m, float *__restrict__ v,
                                              const float *__restrict__ g, int n, float lr, float b1, float b2,
                                              float eps, float c1, float c2, const double *__restrict__ gsq,
                                              float max_norm, uint16_t *__restrict__ wbf)
{
    float gs = 1.f;
    if (gsq) {
        const double q = *gsq, mn = max_norm;
        if (q > mn * mn)
            gs = (float)(mn / sqrt(q));
    }
    for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
        const float ge = gs * g[e];
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
