// Device code of the SSCN solver for gfx950 (CDNA4, wave64).
//
// One SSCN step (paper Sec. 2, Eqs. (eq1)-(eq3), (split)) is:
//   H1:  psi <- exp(-i tau (V + g|s psi|^2)) s psi       (s: pending rescale)
//   x :  Crank-Nicolson along x for every (j,k) line     (Eqs. (eqD.9:kn1),
//   y :  along y, rotation coefficient y_j -> -x_i        (eqD.11), (eq5))
//   z :  along z (3D), no rotation term
// and, in imaginary time, the FP64 norm of the result, whose rescale s is
// folded into the next step's H1.
//
// Each line solve uses the Cayley form of Crank-Nicolson: with
// A = I + K, K = (i tau/2) H_line (tridiagonal: A0 = 1 + k0 on the diagonal,
// A- below, A+ above) the paper's right-hand side is b = (2I - A) psi, so
//   psi' = A^{-1} b = 2 A^{-1} psi - psi = psi + 2 delta,  (I + K) delta = -K psi.
// Solving for the small correction delta keeps the rounding of the O(1)
// diagonal (1 + k0 in the storage precision) out of the result: only small
// quantities are rounded, which is what lets complex64 sweeps track the FP64
// oracle.  Every line system is strictly diagonally
// dominant, so the influence of a right-hand-side entry decays geometrically
// with distance; a line is cut into segments of S outputs, each solved by
// Thomas elimination over its own window of W extra rows on each side.  W is
// chosen on the host from a decay bound so that the truncation is below the
// arithmetic's rounding; when that would need W > 32 the whole-line exact
// kernels are used instead.
//
// The elimination factors are data independent.  Every window uses the fixed
// point c* = A+ / (A0 - A- c*), r* = 1/(A0 - A- c*) of the Thomas recurrence,
// which is the exact factorisation of T_abs, the line matrix with its first
// diagonal entry A0 replaced by A0 - A- c* (a window starting inside the line
// thereby sees the eliminated semi-infinite line before it).  The true matrix
// is T = T_abs + (A- c*) e_1 e_1^T, so by the Sherman-Morrison formula
//   T^{-1} b = T_abs^{-1} b - gamma (T_abs^{-1} b)_1 z,   z = T_abs^{-1} e_1,
//   gamma = A- c* / (1 + A- c* z_1);
// z decays away from the wall, and the host tabulates zeta_u = 2 gamma z_u for
// the first W rows.  The sweep kernels apply out_u -= delta_1 zeta_u there.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sscn_types.hpp"

#include <type_traits>

namespace sscn {

// Largest number of state elements one thread of the x-sweep stages.
constexpr int kXLoad = 16;

// Waves per SIMD the bandwidth-bound sweep kernels are compiled for (the
// register budget: 512 / kSweepWaves VGPRs per lane).
#ifndef SSCN_SWEEP_WAVES
#define SSCN_SWEEP_WAVES 1
#endif
constexpr int kSweepWaves = SSCN_SWEEP_WAVES;

// The batched sweeps stream the state (nontemporal loads and stores where a
// point is touched once): their working set exceeds the caches.
#ifndef SSCN_BATCH_STREAM
#define SSCN_BATCH_STREAM 1
#endif
constexpr bool kBatchStream = SSCN_BATCH_STREAM != 0;


template <class R> struct Cx {
    R re, im;
};

template <class R> __device__ __forceinline__ Cx<R> cx(R a, R b) { return Cx<R>{a, b}; }
template <class R> __device__ __forceinline__ Cx<R> operator+(Cx<R> a, Cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R> __device__ __forceinline__ Cx<R> operator-(Cx<R> a, Cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R> __device__ __forceinline__ Cx<R> operator*(Cx<R> a, Cx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R> __device__ __forceinline__ Cx<R> operator*(R s, Cx<R> a) { return {s * a.re, s * a.im}; }
template <class R> __device__ __forceinline__ R norm2(Cx<R> a) { return a.re * a.re + a.im * a.im; }
template <class R> __device__ __forceinline__ Cx<R> recip(Cx<R> a)
{
    R inv = R(1) / (a.re * a.re + a.im * a.im);
    return {a.re * inv, -a.im * inv};
}

// storage vector type of one complex element
template <class R> struct Vec;
template <> struct Vec<double> { using T = double2; };
template <> struct Vec<float> { using T = float2; };

// State values are read and written through the global address space (a
// C-style cast: the only cast that changes the address space): every state
// buffer is device memory, and pointers loaded from a work-list descriptor
// would otherwise be accessed as generic (flat) pointers, whose loads also
// count against the LDS wait counter.
template <class R> struct GVec;
template <> struct GVec<double> {
    typedef double V __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(1))) V T;
};
template <> struct GVec<float> {
    typedef float V __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(1))) V T;
};

template <class R> __device__ __forceinline__ Cx<R> ld(const typename Vec<R>::T *p, int64_t i)
{
    const typename GVec<R>::V v = ((const typename GVec<R>::T *)p)[i];
    return {v.x, v.y};
}
template <class R> __device__ __forceinline__ void st(typename Vec<R>::T *p, int64_t i, Cx<R> a)
{
    typename GVec<R>::V v;
    v.x = a.re;
    v.y = a.im;
    ((typename GVec<R>::T *)p)[i] = v;
}

// A complex value (a pivot-table entry) read through the global address space.
template <class R> __device__ __forceinline__ Cx<R> ldg(const Cx<R> *p, int64_t i)
{
    const typename GVec<R>::V v = ((const typename GVec<R>::T *)p)[i];
    return {v.x, v.y};
}

// Streaming forms for state the kernel touches once (nontemporal hint: the
// line is not kept in the caches for reuse).  A sweep over a state larger
// than the caches reads each point once and writes it once; the hint lets
// the memory system stream those accesses.
template <class R> __device__ __forceinline__ Cx<R> ld_stream(const typename Vec<R>::T *p, int64_t i)
{
    const typename GVec<R>::V v = __builtin_nontemporal_load(((const typename GVec<R>::T *)p) + i);
    return {v.x, v.y};
}
template <class R> __device__ __forceinline__ void st_stream(typename Vec<R>::T *p, int64_t i, Cx<R> a)
{
    typename GVec<R>::V v;
    v.x = a.re;
    v.y = a.im;
    __builtin_nontemporal_store(v, ((typename GVec<R>::T *)p) + i);
}

// Line coefficients for a line whose rotation coefficient is `rot`.
template <class R> struct LineCoef {
    Cx<R> A0, k0, Ap, Am;
    R kr, ki, ur, ui, wr, wi;  // k0, the mean u of A+ and A-, and their half difference w = q rot
};

template <class R>
__device__ __forceinline__ LineCoef<R> line_coef(const AxisCoef &c, double rot)
{
    LineCoef<R> L;
    L.A0 = {R(c.a0r), R(c.a0i)};
    L.k0 = {R(c.k0r), R(c.k0i)};
    L.Ap = {R(c.ur + c.qr * rot), R(c.ui + c.qi * rot)};
    L.Am = {R(c.ur - c.qr * rot), R(c.ui - c.qi * rot)};
    L.kr = R(c.k0r);
    L.ki = R(c.k0i);
    L.ur = R(c.ur);
    L.ui = R(c.ui);
    L.wr = R(c.qr * rot);
    L.wi = R(c.qi * rot);
    return L;
}

// -(K v)_u for the line operator K = A - I.
template <class R>
__device__ __forceinline__ Cx<R> minus_kv(const LineCoef<R> &L, Cx<R> vm, Cx<R> v0, Cx<R> vp)
{
    const Cx<R> t = L.k0 * v0 + L.Am * vm + L.Ap * vp;
    return Cx<R>{-t.re, -t.im};
}

// The same with the coefficient structure of one time mode, A+- = u +- w:
// K v = k0 v0 + u (vm + vp) + w (vp - vm).  Imaginary time (ST = 1): k0 and
// u are real and w is imaginary; real time (ST = 2): k0 and u are imaginary
// and w is real (tau = -i dt or dt in k0 = i tau / 2h^2, u = -i tau / 4h^2,
// w = tau rot / 4h).  ST = 0: general complex coefficients.
template <class R, int ST>
__device__ __forceinline__ Cx<R> minus_kv_st(const LineCoef<R> &L, Cx<R> vm, Cx<R> v0, Cx<R> vp)
{
    if constexpr (ST == 0) {
        return minus_kv(L, vm, v0, vp);
    } else {
        const Cx<R> sm = {vm.re + vp.re, vm.im + vp.im};
        const Cx<R> df = {vp.re - vm.re, vp.im - vm.im};
        if constexpr (ST == 1)
            return Cx<R>{-(L.kr * v0.re + L.ur * sm.re - L.wi * df.im),
                         -(L.kr * v0.im + L.ur * sm.im + L.wi * df.re)};
        else
            return Cx<R>{-(-L.ki * v0.im - L.ui * sm.im + L.wr * df.re),
                         -(L.ki * v0.re + L.ui * sm.re + L.wr * df.im)};
    }
}

// a * y + t and t - a * y with the multiplications fused, so that a chain
// of them through y is two dependent FMAs deep per link.
template <class R>
__device__ __forceinline__ Cx<R> cfma(Cx<R> a, Cx<R> y, Cx<R> t)
{
    return Cx<R>{fma(a.re, y.re, fma(-a.im, y.im, t.re)), fma(a.re, y.im, fma(a.im, y.re, t.im))};
}
template <class R>
__device__ __forceinline__ Cx<R> cfnma(Cx<R> a, Cx<R> y, Cx<R> t)
{
    return Cx<R>{fma(-a.re, y.re, fma(a.im, y.im, t.re)), fma(-a.re, y.im, fma(-a.im, y.re, t.im))};
}
// Component-wise select (compiles to conditional moves, not branches).
template <class R>
__device__ __forceinline__ Cx<R> csel(bool c, Cx<R> a, Cx<R> b)
{
    return Cx<R>{c ? a.re : b.re, c ? a.im : b.im};
}

// Windowed solve of (I + K) delta = -K v for the S unknowns s..s+S-1 of a line
// with unknowns 1..n-1, by Thomas elimination with the fixed-point factors
// (cst, rst) from row s-W on; then io[r] = v_{s+r} + 2 delta_{s+r} and
// d_first = delta_s (both uncorrected for the wall; see above).
// ld(r) returns v_{s-W-1+r}, r = 0..S+2W+1 (zero outside the unknowns
// 1..n-1): the callers read the window straight from the values they staged
// in LDS, so a window never sits in registers as a whole.
//
// In FP64 the solve is done in the Cayley form instead: (I + K) z = v and
// psi' = 2 z - v, with z_first = z_s (uncorrected) in d_first.  It needs no
// right-hand side -K v per row, and the wall correction is the same (it
// depends on the matrix only: out_u -= z_1 zeta_u).  The delta form keeps
// the rounding of 1 + k0 out of FP32 sweeps, where it matters.
//
// FP64 (Cayley form) runs the elimination on scaled unknowns: with y = r*
// yt and z = r* zt the recurrences are yt_u = v_u + alpha yt_{u-1} (alpha =
// -A- r*) and zt_u = yt_u - c* zt_{u+1}, and r* multiplies only the S
// outputs.  Rows of the window outside the unknowns 1..n-1 must see the
// walls' zeros.  The right-hand side is the window value itself, which is
// zero outside the unknowns, so rows before the near wall stay zero by
// themselves; rows beyond the far wall are zeroed in the back substitution
// (their yt times 0).  The mask is a product with 0 or 1, not a branch, so
// the window is one basic block.  The FP32 delta form does the same with
// ISSUE = true (the fused step, bound by instruction issue): scaled
// unknowns, and the right-hand side and coupling of rows outside the
// unknowns multiplied by 0, so their eliminated values are exactly zero.
// With ISSUE = false (the bandwidth-bound sweeps) it keeps the plain
// recurrence with those rows skipped.
//
// Only the S eliminated values of the output rows are kept.  The back
// substitution enters them with zt at the first row after them, which is the
// sum over the W rows after the outputs of (-c*)^t times their eliminated
// values (the back recurrence unrolled, the rows beyond the far wall masked):
// the forward pass accumulates that sum as it goes, so the registers a
// window needs do not grow with W.
template <class R, int S, int W, int ST = 0, bool ISSUE = false, class Ld>
__device__ __forceinline__ void window_solve(int s, int n, const LineCoef<R> &L, Cx<R> cst, Cx<R> rst, Ld ld,
                                             Cx<R> (&io)[S], Cx<R> &d_first)
{
    constexpr int NR = S + 2 * W;
    const Cx<R> zero = {R(0), R(0)};
    const Cx<R> ma = L.Am * rst;
    const Cx<R> alpha = {-ma.re, -ma.im};
    const Cx<R> mc = {-cst.re, -cst.im};
    if constexpr (std::is_same<R, double>::value) {
        Cx<R> ym[S];
        Cx<R> yp = zero, zs = zero, pw = {R(1), R(0)};
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            yp = cfma(alpha, yp, ld(r + 1));
            const R m = (s - W + r <= n - 1) ? R(1) : R(0);
            if (r >= W && r < W + S)
                ym[r - W] = m * yp;
            if (r >= W + S) {
                zs = cfma(pw, m * yp, zs);
                if (r + 1 < NR)
                    pw = pw * mc;
            }
        }
        // psi' = 2 r* zt - v, one complex multiply-add per output
        const Cx<R> r2 = {R(2) * rst.re, R(2) * rst.im};
        Cx<R> zn = zs;
#pragma unroll
        for (int r = W + S - 1; r >= W; --r) {
            const Cx<R> zt = cfnma(cst, zn, ym[r - W]);
            const Cx<R> v = ld(r + 1);
            io[r - W] = cfma(r2, zt, Cx<R>{-v.re, -v.im});
            if (r == W)
                d_first = rst * zt;
            zn = zt;
        }
        return;
    }

    if constexpr (ISSUE) {
        Cx<R> ym[S];
        Cx<R> yp = zero, zs = zero, pw = {R(1), R(0)};
        Cx<R> vm = ld(0), v0 = ld(1);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const Cx<R> vp = ld(r + 2);
            const int u = s - W + r;
            const R m = (u >= 1 && u <= n - 1) ? R(1) : R(0);
            yp = cfma(m * alpha, yp, m * minus_kv_st<R, ST>(L, vm, v0, vp));
            if (r >= W && r < W + S)
                ym[r - W] = yp;
            if (r >= W + S) {
                zs = cfma(pw, yp, zs);
                if (r + 1 < NR)
                    pw = pw * mc;
            }
            vm = v0;
            v0 = vp;
        }
        const Cx<R> r2 = {R(2) * rst.re, R(2) * rst.im};
        Cx<R> zn = zs;
#pragma unroll
        for (int r = W + S - 1; r >= W; --r) {
            const Cx<R> zt = cfnma(cst, zn, ym[r - W]);
            io[r - W] = cfma(r2, zt, ld(r + 1));  // v + 2 r* zt
            if (r == W)
                d_first = rst * zt;
            zn = zt;
        }
        return;
    }

    // delta form: d'_u = r* rhs_u + alpha d'_{u-1}, d_u = d'_u - c* d_{u+1}
    Cx<R> dm[S];
    Cx<R> dprev = zero, ds = zero, pw = {R(1), R(0)};
    Cx<R> vm = ld(0), v0 = ld(1);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const Cx<R> vp = ld(r + 2);
        const int u = s - W + r;
        const bool valid = (u >= 1) && (u <= n - 1);
        Cx<R> dp = zero;
        if (valid)
            dp = rst * minus_kv_st<R, ST>(L, vm, v0, vp) + alpha * dprev;
        dprev = dp;
        if (r >= W && r < W + S)
            dm[r - W] = dp;
        if (r >= W + S) {
            ds = cfma(pw, dp, ds);
            if (r + 1 < NR)
                pw = pw * mc;
        }
        vm = v0;
        v0 = vp;
    }
    Cx<R> dnext = ds;
#pragma unroll
    for (int r = W + S - 1; r >= W; --r) {
        const Cx<R> d = dm[r - W] - cst * dnext;
        io[r - W] = ld(r + 1) + R(2) * d;
        if (r == W)
            d_first = d;
        dnext = d;
    }
}

// Block index remapping for the strided sweeps.  Consecutive hardware
// workgroup ids go to the 8 XCDs in turn; the remap gives each XCD a
// contiguous range of logical blocks, so the windows of neighbouring
// segments (which share halo rows) run under the same L2.  Returns -1 for
// the padding blocks of a grid rounded up to a multiple of 8.
__device__ __forceinline__ int xcd_logical_block(int nblocks)
{
    const int b = blockIdx.x;
    const int per = (nblocks + 7) / 8;
    const int l = (b % 8) * per + b / 8;
    return l < nblocks ? l : -1;
}

// The work-list item of this block in a launch of at least 8 ceil(n / 8)
// blocks over a list of n items (n read on the device, so a launch captured
// for a longer list stays valid when the list shrinks): as
// xcd_logical_block, each XCD takes a contiguous run of the list, whose
// neighbouring items share halo rows in that XCD's L2.  -1 for the blocks
// beyond the list.
__device__ __forceinline__ int xcd_item(int n)
{
    const int b = blockIdx.x;
    const int per = (n + 7) / 8;
    const int l = (b % 8) * per + b / 8;
    return (b / 8 < per && l < n) ? l : -1;
}

// One DPP lane permutation of a double within rows of 16 lanes (CTRL: a
// gfx9 DPP control code; every lane reads an active lane of its own row).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum of v over the 64 lanes of a wave (all lanes active), the same bits in
// every lane and in every wave that sums the same values: pairs (lane xor
// 1), then quads (xor 2), then halves of rows mirrored (lane i with 7 - i),
// then rows mirrored (i with 15 - i), all with DPP row permutations, so each
// lane of a 16-lane row holds the row's sum; then the four row sums in the
// fixed order (r0 + r1) + (r2 + r3).
__device__ __forceinline__ double wave_sum_f64(double v)
{
    v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Deterministic block sum of one double over a 256-thread block; the result
// is valid in thread 0.  Fixed reduction order, no atomics.
__device__ __forceinline__ double block_sum_256(double v, double *red)
{
    v = wave_sum_f64(v);
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    __syncthreads();
    if ((tid & 63) == 0)
        red[tid >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (tid == 0)
        r = (red[0] + red[1]) + (red[2] + red[3]);
    return r;
}

__device__ __forceinline__ double block_max_256(double v, double *red)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v = fmax(v, __shfl_xor(v, off, 64));
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    __syncthreads();
    if ((tid & 63) == 0)
        red[tid >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (tid == 0)
        r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    return r;
}

// Deterministic block sum over NT threads (NT/64 waves), valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum_nt(double v, double *red)
{
    v = wave_sum_f64(v);
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    __syncthreads();
    if ((tid & 63) == 0)
        red[tid >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (tid == 0)
        for (int w = 0; w < NT / 64; ++w)
            r += red[w];
    return r;
}

// Fixed-order sum of n FP64 partials by one wave (all 64 lanes active): lane
// l adds ((p_l + p_{l+64}) + (p_{l+128} + p_{l+192})), then p_{l+256},
// p_{l+320}, ... in turn; then the DPP wave sum.  Every wave of every kernel
// that sums the same partials gets the same bits, so the rescale of a pending
// norm is the same number whether it is folded into the next step or applied
// by a kernel of its own, and a run restarted from a saved state repeats the
// uninterrupted run bit for bit.  (The fused step prefetches the first four
// partials itself and combines them in this order.)
__device__ __forceinline__ double wave_partials_sum(const double *part, int n)
{
    const int lane = (threadIdx.x + threadIdx.y * blockDim.x) & 63;
    double pp[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        pp[k] = lane + 64 * k < n ? part[lane + 64 * k] : 0.0;
    double v = (pp[0] + pp[1]) + (pp[2] + pp[3]);
    for (int t = lane + 256; t < n; t += 64)
        v += part[t];
    return wave_sum_f64(v);
}

// s - 1 of the rescale s = 1 / sqrt(dV tot) that normalises a state whose
// sum of |psi|^2 is tot (the one expression every path evaluates).
__device__ __forceinline__ double norm_scale_m1(double tot, double dV) { return 1.0 / sqrt(dV * tot) - 1.0; }

__device__ __forceinline__ void sin_cos(double x, double *s, double *c) { sincos(x, s, c); }
__device__ __forceinline__ void sin_cos(float x, float *s, float *c) { sincosf(x, s, c); }

// e^x - 1 by its Taylor series x sum_{k < NT} x^k / (k+1)! (Horner).
template <class R, int NT>
__device__ __forceinline__ R expm1_taylor(R x)
{
    R c = R(1);
    R inv[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        c = c / R(k + 1);  // 1 / (k+1)!, folded at compile time
        inv[k] = c;
    }
    R q = inv[NT - 1];
#pragma unroll
    for (int k = NT - 2; k >= 0; --k)
        q = fma(q, x, inv[k]);
    return x * q;
}

// The series truncated where the first omitted term is below 2^-60 (FP64)
// or 2^-30 (FP32) of the sum: for |x| <= 1/4, 13 and 8 terms; for |x| <= 1
// (the sum is then at least 1 - 1/e of its first term), 19 and 12 terms.
template <class R>
__device__ __forceinline__ R expm1_series(R x)
{
    return expm1_taylor<R, std::is_same<R, double>::value ? 13 : 8>(x);
}

template <class R>
__device__ __forceinline__ R expm1_wide(R x)
{
    return expm1_taylor<R, std::is_same<R, double>::value ? 19 : 12>(x);
}

// e^x - 1: the short series where |x| <= 1/4, the long one where |x| <= 1,
// else the library expm1.  The H1 factors of the imaginary-time step have
// arguments dt times the local energy; at the corners of the large grids
// (the harmonic potential grows to several hundred there) they pass 1/4 but
// stay below 1 at the time steps used, so the library branch is rare.
template <class R>
__device__ __forceinline__ R expm1_small(R x)
{
    const R ax = fabs(x);
    if (ax <= R(0.25))
        return expm1_series(x);
    if (ax <= R(1))
        return expm1_wide(x);
    return expm1(x);
}

// e[c] <- e^{e[c]} - 1 for the NP arguments a thread holds, with one branch
// for all of them (so the NP series evaluations interleave): by the range of
// the largest |e[c]|, the short series, the long series or the library
// expm1 for all.
template <class R, int NP>
__device__ __forceinline__ void expm1_all(R (&e)[NP])
{
    R amax = R(0);
#pragma unroll
    for (int c = 0; c < NP; ++c)
        amax = fmax(amax, fabs(e[c]));
    if (amax <= R(0.25)) {
#pragma unroll
        for (int c = 0; c < NP; ++c)
            e[c] = expm1_series(e[c]);
    } else if (amax <= R(1)) {
#pragma unroll
        for (int c = 0; c < NP; ++c)
            e[c] = expm1_wide(e[c]);
    } else {
#pragma unroll
        for (int c = 0; c < NP; ++c)
            e[c] = expm1(e[c]);
    }
}

// e^{-i th} - 1 = (cos th - 1) - i sin th for |th| <= 1/4 by the Taylor
// series of cos th - 1 (in th^2, Horner) and sin th, truncated where the
// first omitted term is below 2^-60 (FP64: 7 and 8 terms) or 2^-30 (FP32: 4
// and 4 terms) of the sum.
template <class R>
__device__ __forceinline__ Cx<R> expim1_series(R th)
{
    constexpr bool dbl = std::is_same<R, double>::value;
    constexpr int NC = dbl ? 7 : 4, NS = dbl ? 8 : 4;
    R cc[NC], sc[NS];
    R f = R(1);
#pragma unroll
    for (int k = 1; k <= 2 * NS; ++k) {  // 1/k!, folded at compile time
        f = f / R(k);
        const R sg = ((k / 2) % 2) ? R(-1) : R(1);
        if (k % 2 == 0 && k / 2 <= NC)
            cc[k / 2 - 1] = sg * f;  // (-1)^m / (2m)!, m = k/2
        if (k % 2 == 1 && (k - 1) / 2 < NS)
            sc[(k - 1) / 2] = sg * f;  // (-1)^m / (2m+1)!, m = (k-1)/2
    }
    const R t = th * th;
    R pc = cc[NC - 1];
#pragma unroll
    for (int m = NC - 2; m >= 0; --m)
        pc = fma(pc, t, cc[m]);
    R ps = sc[NS - 1];
#pragma unroll
    for (int m = NS - 2; m >= 0; --m)
        ps = fma(ps, t, sc[m]);
    return Cx<R>{t * pc, -(th * ps)};
}

// e^{-i th} - 1 from one library sincos of th/2: -2 sin^2(th/2) - i 2
// sin(th/2) cos(th/2).
template <class R>
__device__ __forceinline__ Cx<R> expim1_lib(R th)
{
    R sh, ch;
    sin_cos(R(0.5) * th, &sh, &ch);
    return Cx<R>{R(-2) * sh * sh, R(-2) * sh * ch};
}

// e^{-i th[c]} - 1 for the NP arguments a thread holds, with one branch for
// all of them: the series if every |th[c]| <= 1/4, else the library.
template <class R, int NP>
__device__ __forceinline__ void expim1_all(const R (&th)[NP], Cx<R> (&f)[NP])
{
    R amax = R(0);
#pragma unroll
    for (int c = 0; c < NP; ++c)
        amax = fmax(amax, fabs(th[c]));
    if (amax <= R(0.25)) {
#pragma unroll
        for (int c = 0; c < NP; ++c)
            f[c] = expim1_series(th[c]);
    } else {
#pragma unroll
        for (int c = 0; c < NP; ++c)
            f[c] = expim1_lib(th[c]);
    }
}

// Pointwise H1 factor exp(-i tau w) applied as v + (exp(-i tau w) - 1) v, so
// that only the small difference from 1 is rounded: real time (tau = dt)
// exp(-i dt w) - 1 = (cos(dt w) - 1) - i sin(dt w); imaginary time
// (tau = -i dt) expm1(-dt w).
template <class R, bool RT>
__device__ __forceinline__ Cx<R> h1_apply(Cx<R> v, R w, R dt)
{
    if constexpr (RT) {
        const R th = dt * w;
        Cx<R> f;
        if (fabs(th) <= R(0.25))
            f = expim1_series(th);
        else
            f = expim1_lib(th);
        return v + f * v;
    } else {
        return v + expm1_small(-dt * w) * v;
    }
}

// psi <- s psi applied as psi + (s - 1) psi with s - 1 formed in FP64.
template <class R>
__device__ __forceinline__ Cx<R> rescale(Cx<R> v, R sm1)
{
    return v + sm1 * v;
}

// ---------------------------------------------------------------------------
// Pivot table of one line type (x-lines by j, y-lines by i, one for z):
// tab[0] = c*, tab[1] = r*, tab[1 + u] = zeta_u (u = 1..W).  Stride W + 2.

// x-sweep with the H1 sub-step and the pending rescale (s - 1 read from
// sm1p, NULL for none) fused in front.  A block owns L whole x-lines (L a
// power of two, L * nseg <= 256, nx * L <= 256 * KX).  Staging and the
// write-back give each line 256 / L consecutive threads that load (store)
// its points u = m, m + 256/L, ... coalesced; the staged lines sit in LDS
// padded every S elements so that the solve threads, which own consecutive
// segments (thread p: segment p % nseg of line p / nseg), hit distinct banks.
// A block loads its line group into registers (xsweep_load), then finishes
// it (xsweep_finish).  Making the kernels persistent, with the next group's
// loads issued during the current group's solve, measured slower than one
// group per block with the hardware dealing blocks to the CUs.  src may
// equal dst: a line is owned by exactly one block and loaded before that
// block writes it.

// The values one thread stages for a line group: KX state points and two
// pivot-table entries.
template <class R, int KX>
struct XStage {
    Cx<R> pre[KX];
    Cx<R> tpre[2];
};

// Issue the loads of the line group starting at line0 (L lines).
template <class R, int S, int W, int KX, bool NT = false>
__device__ __forceinline__ void xsweep_load(const typename Vec<R>::T *src, const StepArgs &a, int L,
                                            const Cx<R> *__restrict__ tab, int line0, XStage<R, KX> &g)
{
    const int nx = a.nx, ny = a.ny;
    const int nlines = ny * (a.dim == 3 ? a.nz : 1);
    const int tid = threadIdx.x;
    const int tpl = 256 / L;
    const int sl = tid / tpl, sm = tid - sl * tpl;
    const int sline = line0 + sl;
    const int sj = sline % ny, sk = sline / ny;
    const bool sact = sline < nlines && sj > 0 && (a.dim == 2 || sk > 0);
    const int64_t sbase = (int64_t)sline * nx;
#pragma unroll
    for (int c = 0; c < KX; ++c) {
        const int u = sm + c * tpl;
        g.pre[c] = Cx<R>{R(0), R(0)};
        if (sact && u >= 1 && u <= nx - 1)
            g.pre[c] = NT ? ld_stream<R>(src, sbase + u) : ld<R>(src, sbase + u);
    }
#pragma unroll
    for (int c2 = 0; c2 < 2; ++c2) {
        const int te = tid + c2 * 256;
        g.tpre[c2] = Cx<R>{R(0), R(0)};
        if (te < L * (W + 2)) {
            const int tl = te / (W + 2), c = te - tl * (W + 2);
            const int tline = line0 + tl;
            if (tline < nlines)
                g.tpre[c2] = ldg(tab, (int64_t)(tline % ny) * (W + 2) + c);
        }
    }
}

// The rest of the group from its loaded values: rescale and H1 into LDS,
// the windowed solves, the wall terms and the write-back.  The staged lines
// use the padded layout of x_row_index: the zero entries around the
// unknowns let each window read the row at compile-time offsets from its
// segment's base entry.
template <class R, int S, int W, bool RT, int KX, bool NT = false>
__device__ __forceinline__ void xsweep_finish(typename Vec<R>::T *dst, const StepArgs &a, int L, double sm1,
                                              int line0, XStage<R, KX> &g, unsigned char *smem)
{
    constexpr int OFF = x_row_off(S, W);
    constexpr int OFFE = x_row_index(OFF, S);  // entry of point u = 0
    Cx<R> *lin = reinterpret_cast<Cx<R> *>(smem);
    const int nx = a.nx, ny = a.ny;
    const int LS = x_row_len(nx, S, W);
    Cx<R> *ltab = lin + (size_t)L * LS;      // L rows of W + 2 table entries
    Cx<R> *d1 = ltab + (size_t)L * (W + 2);  // delta_1 of each staged line
    const int nlines = ny * (a.dim == 3 ? a.nz : 1);
    const int nseg = (nx - 2) / S + 1;
    const int tid = threadIdx.x;
    const int tpl = 256 / L;
    const int sl = tid / tpl, sm = tid - sl * tpl;
    const int sline = line0 + sl;
    const int sj = sline % ny, sk = sline / ny;
    const bool sact = sline < nlines && sj > 0 && (a.dim == 2 || sk > 0);
    const int64_t sbase = (int64_t)sline * nx;
    // LDS entry of point u >= 0 of a staged line
    auto xe = [](int u) { return OFFE + u + u / S; };
    Cx<R>(&pre)[KX] = g.pre;
    const R sr = R(RT ? 0.0 : sm1);  // the pending rescale, s - 1
    if constexpr (RT || !std::is_same<R, double>::value) {
        Cx<R> *row = lin + sl * LS;
        const double y = a.y0 + sj * a.hy, z = a.z0 + sk * a.hz;
        const double vyz = a.vy * y * y + (a.dim == 3 ? a.vz * z * z : 0.0);
#pragma unroll
        for (int c = 0; c < KX; ++c) {
            const int u = sm + c * tpl;
            if (u >= 1 && u <= nx - 1) {
                Cx<R> v = {R(0), R(0)};
                if (sact) {
                    v = rescale(pre[c], sr);
                    const double x = a.x0 + u * a.hx;
                    const R w = R(a.vx * x * x + vyz) + R(a.g) * norm2(v);
                    v = h1_apply<R, RT>(v, w, R(a.dt));
                }
                row[xe(u)] = v;
            }
        }
    } else {
        // imaginary time: every argument -dt w first (zero off the line, whose
        // staged value is zero anyway), then their expm1 together
        Cx<R> *row = lin + sl * LS;
        const double y = a.y0 + sj * a.hy, z = a.z0 + sk * a.hz;
        const double vyz = a.vy * y * y + (a.dim == 3 ? a.vz * z * z : 0.0);
        R ex[KX];
#pragma unroll
        for (int c = 0; c < KX; ++c) {
            const int u = sm + c * tpl;
            pre[c] = rescale(pre[c], sr);
            const double x = a.x0 + u * a.hx;
            const R arg = -R(a.dt) * (R(a.vx * x * x + vyz) + R(a.g) * norm2(pre[c]));
            ex[c] = (sact && u >= 1 && u <= nx - 1) ? arg : R(0);
        }
        expm1_all(ex);
#pragma unroll
        for (int c = 0; c < KX; ++c) {
            const int u = sm + c * tpl;
            if (u >= 1 && u <= nx - 1)
                row[xe(u)] = pre[c] + ex[c] * pre[c];
        }
    }
    // zeros around the unknowns: points -OFF..0 and nx..nx-1+S+W of each line
    {
        constexpr int NPAD = OFF + 1 + S + W;
        for (int e = tid; e < L * NPAD; e += 256) {
            const int pl = e / NPAD, pk = e - pl * NPAD;
            const int U = pk <= OFF ? pk : nx + OFF + (pk - OFF - 1);  // U = u + OFF
            lin[pl * LS + x_row_index(U, S)] = Cx<R>{R(0), R(0)};
        }
    }
#pragma unroll
    for (int c2 = 0; c2 < 2; ++c2)
        if (tid + c2 * 256 < L * (W + 2))
            ltab[tid + c2 * 256] = g.tpre[c2];
    __syncthreads();

    const int l = tid / nseg, q = tid - l * nseg;
    const int line = line0 + l;
    const int j = line % ny, k = line / ny;
    const bool active = l < L && line < nlines && j > 0 && (a.dim == 2 || k > 0);
    const int s0 = 1 + q * S;
    Cx<R> io[S];
    if (active) {
        const LineCoef<R> Lc = line_coef<R>(a.ax[0], a.omega * (a.y0 + j * a.hy));
        // window value r: point u = s0 - W - 1 + r = q S - W + r, i.e. U = u +
        // OFF = q S + (OFF - W + r) >= 0, at entry q (S + 1) + x_row_index(OFF
        // - W + r, S) (OFF is a multiple of S): a constant offset per r
        const Cx<R> *seg = lin + l * LS + q * (S + 1);
        auto ld = [&](int r) -> Cx<R> { return seg[x_row_index(OFF - W + r, S)]; };
        Cx<R> df;
        window_solve<R, S, W, RT ? 2 : 1>(s0, nx, Lc, ltab[l * (W + 2)], ltab[l * (W + 2) + 1], ld, io, df);
        if (q == 0)
            d1[l] = df;
    }
    __syncthreads();
    if (active) {
        // the outputs back into the row; points beyond nx - 1 land in the
        // row's trailing zeros, which nothing reads any more
        Cx<R> *seg = lin + l * LS + q * (S + 1) + OFFE + 1;  // entry of point s0
        if (q * S < W) {  // the wall rows 1..W lie in the first segments
            const Cx<R> df = d1[l];
#pragma unroll
            for (int r = 0; r < S; ++r)
                if (s0 + r <= W)
                    io[r] = io[r] - df * ltab[l * (W + 2) + 1 + s0 + r];
        }
#pragma unroll
        for (int r = 0; r < S; ++r)
            seg[x_row_index(1 + r, S) - 1] = io[r];
    }
    __syncthreads();
    if (sact) {
        const Cx<R> *row = lin + sl * LS;
#pragma unroll
        for (int c = 0; c < KX; ++c) {
            const int u = sm + c * tpl;
            if (u >= 1 && u <= nx - 1) {
                if (NT)
                    st_stream<R>(dst, sbase + u, row[xe(u)]);
                else
                    st<R>(dst, sbase + u, row[xe(u)]);
            }
        }
    }
}

// KX: staged points per thread, nx * L <= 256 * KX (fewer registers for
// short lines, hence more waves per SIMD in this bandwidth-bound kernel).
// Block b takes line group b (lines b L .. b L + L - 1).
template <class R, int S, int W, bool RT, int KX>
__global__ __launch_bounds__(256, kSweepWaves) void k_xsweep(const typename Vec<R>::T *src, typename Vec<R>::T *dst,
                                                StepArgs a, int L, const double *__restrict__ sm1p,
                                                const Cx<R> *__restrict__ tab)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    XStage<R, KX> g;
    xsweep_load<R, S, W, KX>(src, a, L, tab, blockIdx.x * L, g);
    xsweep_finish<R, S, W, RT, KX>(dst, a, L, sm1p ? *sm1p : 0.0, blockIdx.x * L, g, smem_raw);
}

// s - 1 of the pending rescale, s = 1/sqrt(dV sum of the npart norm
// partials), summed in fixed order by one block.
static __global__ __launch_bounds__(256) void k_norm_scale(const double *partials, int npart, double dV, double *out)
{
    const double sm1 = norm_scale_m1(wave_partials_sum(partials, npart), dV);
    if (threadIdx.x == 0)
        out[0] = sm1;
}

// ---------------------------------------------------------------------------
// Strided sweeps (y: stride nx, z: stride nx*ny).  A block (kYLines x
// kSegBlock threads) takes kYLines consecutive lines and kSegBlock
// consecutive segments; it stages the tile of kSegBlock*S + 2W + 2 rows x
// kYLines lines those windows cover in LDS with one coalesced pass (each row
// a contiguous run), so the halo rows shared by neighbouring segments are
// read once.  Thread (tx, ty) solves segment ty of line tx from LDS and
// writes its outputs straight to global memory (coalesced across tx).  The
// tile is tall (8 segments, 64 output rows) so that the 2W + 2 halo rows
// add little to the reads, and narrow (32 lines) so that its LDS leaves room
// for three blocks per CU at W = 14 in FP64.  src != dst.  With EMIT the
// block writes the FP64 partial sum of |psi'|^2 of its outputs at its
// logical block index.  Grid: 1-D, rounded up to a multiple of 8 logical
// blocks (gx line tiles x gy segment groups x gz planes).
#ifndef SSCN_Y_LINES
#define SSCN_Y_LINES 32
#endif
constexpr int kYLines = SSCN_Y_LINES;
constexpr int kSegBlock = 256 / kYLines;
static_assert(kYLines * kSegBlock == 256, "strided sweep blocks have 256 threads");

template <class R, int S, int W, bool NT = false>
__device__ __forceinline__ void strided_sweep_tile(const typename Vec<R>::T *__restrict__ src,
                                                   typename Vec<R>::T *__restrict__ dst, int n, int64_t base,
                                                   int64_t stride, int nlines, int line0, int by, bool plane_ok,
                                                   const LineCoef<R> &Lc, const Cx<R> *__restrict__ trow,
                                                   bool emit, double &acc)
{
    constexpr int TR = kSegBlock * S + 2 * W + 2;
    constexpr int LN = kYLines;
    constexpr int K = (TR * LN + 255) / 256;
    __shared__ Cx<R> tile[TR * LN];
    __shared__ Cx<R> d1[LN];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = tx + LN * ty;
    const int row0 = by * kSegBlock * S - W;  // line index u of tile row 0
    Cx<R> pre[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
        const int e = tid + c * 256;
        const int rr = e / LN, col = e - rr * LN;
        const int u = row0 + rr;
        const bool in = e < TR * LN && plane_ok && u >= 1 && u <= n - 1 && line0 + col < nlines;
        pre[c] = csel(in, ld<R>(src, in ? base + (int64_t)u * stride + line0 + col : (int64_t)0),
                      Cx<R>{R(0), R(0)});
    }
#pragma unroll
    for (int c = 0; c < K; ++c) {
        const int e = tid + c * 256;
        if (e < TR * LN)
            tile[e] = pre[c];
    }
    __syncthreads();
    const int nseg = (n - 2) / S + 1;
    const int q = by * kSegBlock + ty;
    const int s0 = 1 + q * S;
    const bool active = trow != nullptr && q < nseg;
    Cx<R> io[S];
    if (active) {
        Cx<R> df;
        window_solve<R, S, W>(s0, n, Lc, ldg(trow, 0), ldg(trow, 1), [&](int r) { return tile[(ty * S + r) * LN + tx]; },
                              io, df);
        if (q == 0)
            d1[tx] = df;
    }
    if (by == 0) {  // the wall rows 1..W lie in the first segment group
        __syncthreads();
        if (active && s0 <= W) {
            const Cx<R> df = d1[tx];
#pragma unroll
            for (int r = 0; r < S; ++r) {
                const int u = s0 + r;
                if (u <= W)
                    io[r] = io[r] - df * ldg(trow, 1 + u);
            }
        }
    }
    if (active) {
#pragma unroll
        for (int r = 0; r < S; ++r) {
            const int u = s0 + r;
            if (u <= n - 1) {
                if (NT)
                    st_stream<R>(dst, base + (int64_t)u * stride + line0 + tx, io[r]);
                else
                    st<R>(dst, base + (int64_t)u * stride + line0 + tx, io[r]);
                if (emit)
                    acc += (double)io[r].re * (double)io[r].re + (double)io[r].im * (double)io[r].im;
            }
        }
    }
}

// One y tile: columns bx*kYLines .. +kYLines-1 of plane bz, segment group
// by; the norm partial of its outputs (EMIT) goes to *partial.
template <class R, int S, int W, bool EMIT, bool NT = false>
__device__ __forceinline__ void ysweep_block(const typename Vec<R>::T *__restrict__ src,
                                             typename Vec<R>::T *__restrict__ dst, const StepArgs &a, int bx, int by,
                                             int bz, double *partial, const Cx<R> *__restrict__ tab, double *red)
{
    const int nx = a.nx, ny = a.ny;
    const int i = bx * kYLines + threadIdx.x;
    const bool plane_ok = (a.dim == 2 || bz > 0);
    const Cx<R> *trow = nullptr;
    LineCoef<R> Lc{};
    if (i > 0 && i < nx && plane_ok) {
        Lc = line_coef<R>(a.ax[1], -a.omega * (a.x0 + i * a.hx));
        trow = tab + (size_t)i * (W + 2);
    }
    double acc = 0.0;
    strided_sweep_tile<R, S, W, NT>(src, dst, ny, (int64_t)bz * nx * ny, nx, nx, bx * kYLines, by, plane_ok, Lc,
                                    trow, EMIT, acc);
    if (EMIT) {
        const double b = block_sum_256(acc, red);
        if (threadIdx.x == 0 && threadIdx.y == 0)
            *partial = b;
    }
}

template <class R, int S, int W, bool EMIT>
__global__ __launch_bounds__(256, kSweepWaves) void k_ysweep(const typename Vec<R>::T *__restrict__ src,
                                                typename Vec<R>::T *__restrict__ dst, StepArgs a,
                                                double *partials, int gx, int gy, int gz,
                                                const Cx<R> *__restrict__ tab)
{
    __shared__ double red[8];
    const int lb = xcd_logical_block(gx * gy * gz);
    if (lb < 0)
        return;
    const int by = lb % gy, rest = lb / gy;
    const int bx = rest % gx, bz = rest / gx;
    ysweep_block<R, S, W, EMIT>(src, dst, a, bx, by, bz, partials + lb, tab, red);
}

template <class R, int S, int W, bool EMIT>
__global__ __launch_bounds__(256, kSweepWaves) void k_zsweep(const typename Vec<R>::T *__restrict__ src,
                                                typename Vec<R>::T *__restrict__ dst, StepArgs a,
                                                double *partials, int gx, int gy,
                                                const Cx<R> *__restrict__ tab)
{
    __shared__ double red[8];
    const int lb = xcd_logical_block(gx * gy);
    if (lb < 0)
        return;
    const int by = lb % gy, bx = lb / gy;
    const int nx = a.nx, ny = a.ny;
    const int pidx = bx * kYLines + threadIdx.x;
    const int i = pidx % nx, j = pidx / nx;
    const Cx<R> *trow = nullptr;
    LineCoef<R> Lc{};
    if (pidx < nx * ny && i > 0 && j > 0) {
        Lc = line_coef<R>(a.ax[2], 0.0);
        trow = tab;
    }
    double acc = 0.0;
    strided_sweep_tile<R, S, W>(src, dst, a.nz, 0, (int64_t)nx * ny, nx * ny, bx * kYLines, by, true, Lc, trow,
                                EMIT, acc);
    if (EMIT) {
        const double b = block_sum_256(acc, red);
        if (threadIdx.x == 0 && threadIdx.y == 0)
            partials[lb] = b;
    }
}

// ---------------------------------------------------------------------------
// Fused 2D step: one launch advances every listed (instance, tile) item by a
// whole SSCN step.  An item is a TR x TC tile of outputs; the block stages
// the tile plus a halo of W+1 rows and columns from the current buffer,
// applies the pending rescale and H1 to every staged point, solves the
// x-lines of all staged rows for the TC output columns, then the y-lines of
// the TC columns for the TR output rows, and writes the tile to the other
// buffer with its FP64 partial |psi'|^2.  Halos make neighbouring tiles
// independent, so one launch needs no grid-wide synchronisation; the two
// buffers of an instance alternate from step to step.  Blocks loop over the
// work list, so the same launch serves one grid or a batch of instances of
// different sizes and parameters.
struct Inst2D {
    int nx, ny, tiles_x, tiles_y, poff, active;
    int xl, ygx, ygy, ypoff;  // sweep plan: x lines per block, y tile grid, offset of its partials
    // 3D instances (nz > 1, sweep plan only): the z tile grid and the offset
    // of its partials; eoff / ecount: the norm partials of the sweep that
    // emits them (y in 2D, z in 3D), which the next x-sweep sums
    int nz, zgx, zgy, zpoff, eoff, ecount;
    double hx, hy, x0, y0, vx, vy, g, omega, dt, dV;
    double hz, z0, vz;
    AxisCoef ax[3];
    void *buf[2];
    const void *tab[3];   // pivot tables of x-lines (by j), y-lines (by i) and z-lines (one)
};

// stage-buffer row stride: >= SC + SC/S + 1 and = 4 (mod 16), so that the
// 8 (b128) or 16 (b64) lanes served together hit distinct banks
constexpr int stage_stride(int SC, int S)
{
    int v = SC + SC / S + 1;
    while (v % 16 != 4)
        ++v;
    return v;
}

// Dynamic LDS of the fused step, in complex elements: the staged tile.
constexpr size_t step2d_lds_elems(int S, int W, int TR, int TC)
{
    return (size_t)(TR + 2 * W + 2) * stage_stride(TC + 2 * W + 2, S);
}

template <class R, int S, int W, int TR, int TC>
constexpr size_t step2d_lds_bytes()
{
    return step2d_lds_elems(S, W, TR, TC) * sizeof(Cx<R>);
}

// One step of a 2D instance per tile.  ONE: a single instance passed by
// value (tile = work item) instead of a work list of (instance, tile).  The
// x-windows have S outputs; the y-windows S/2, so that the TC x (2 TR / S)
// y-segments of a tile occupy all NT threads.
template <class R, int S, int W, int TR, int TC, int NT, bool RT, bool ONE>
__global__ __launch_bounds__(NT) void k_step2d(const Inst2D *__restrict__ insts, const int2 *__restrict__ work,
                                               const int *__restrict__ nwork, Inst2D one, int parity,
                                               const double *__restrict__ pin, double *__restrict__ pout,
                                               int use_pin)
{
    constexpr int H = W + 1;
    constexpr int SR = TR + 2 * H, SC = TC + 2 * H;
    constexpr int SCP = stage_stride(SC, S);
    constexpr int NST = (SR * SC + NT - 1) / NT;
    constexpr int NSX = TC / S;
    constexpr int NXI = (SR * NSX + NT - 1) / NT;  // x-segments per thread
    constexpr int SY = S / 2, NSY = TR / SY;
    constexpr int ST = RT ? 2 : 1;
    constexpr int PP = 4;  // norm partials prefetched per thread
    static_assert(TC % S == 0 && TR % SY == 0 && TC * NSY <= NT && TC + SR <= NT, "tile shape");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // SR x SCP staged points, H1 applied; the x-solve writes its outputs
    // (the TC tile columns of every row) back in place
    Cx<R> *st1 = reinterpret_cast<Cx<R> *>(smem_raw);
    auto sx = [&](int rr, int cc) -> Cx<R> & { return st1[rr * SCP + cc + cc / S]; };
    __shared__ Cx<R> d1x[SR];
    __shared__ Cx<R> d1y[TC];
    __shared__ Cx<R> tpx[SR][2];  // (c*, r*) of the x-line of each staged row
    __shared__ Cx<R> tpy[TC][2];  // (c*, r*) of the y-line of each tile column
    __shared__ double red[20];
    const int tid = threadIdx.x;
    const int nw = ONE ? one.tiles_x * one.tiles_y : *nwork;
    // one block per tile on a grid of at least 8 ceil(nw / 8) blocks; the
    // hardware deals consecutive blocks to the 8 XCDs in turn, and the remap
    // gives each XCD a contiguous run of tiles, so that the halos
    // neighbouring tiles share are fetched once into that XCD's L2
    const int it0 = ONE ? xcd_logical_block(nw) : xcd_item(nw);
    if (it0 < 0)
        return;
    for (int it = it0; it < nw; it += gridDim.x) {
        int ik = 0, tile = it;
        if (!ONE) {
            const int2 wk = work[it];
            ik = wk.x;
            tile = wk.y;
        }
        const Inst2D &I = ONE ? one : insts[ik];
        const int nx = I.nx, ny = I.ny;
        // complex128: tiles ordered column by column within groups of GR
        // tile rows, so that each XCD's contiguous run of tiles is a compact
        // block (4 x 8 tiles on a 16 x 16 tile grid) whose shared halos its
        // L2 keeps; complex64 keeps the row-major order (GR = 1), which
        // measured faster for its tile shape
        constexpr int GR = sizeof(R) == 8 ? 4 : 1;
        int tyi, txi;
        if constexpr (GR > 1) {
            const int grp = tile / (GR * I.tiles_x), loc = tile - grp * GR * I.tiles_x;
            const int rows = min(GR, I.tiles_y - GR * grp);
            tyi = GR * grp + loc % rows;
            txi = loc / rows;
        } else {
            tyi = tile / I.tiles_x;
            txi = tile - tyi * I.tiles_x;
        }
        const int r0 = 1 + tyi * TR, c0 = 1 + txi * TC;  // first output row j / column i
        const int jb = r0 - H, ib = c0 - H;              // staged origin
        const typename Vec<R>::T *src = reinterpret_cast<const typename Vec<R>::T *>(I.buf[parity]);
        typename Vec<R>::T *dst = reinterpret_cast<typename Vec<R>::T *>(I.buf[parity ^ 1]);
        const Cx<R> *tabx = reinterpret_cast<const Cx<R> *>(I.tab[0]);
        const Cx<R> *taby = reinterpret_cast<const Cx<R> *>(I.tab[1]);

        // norm partials of the previous step first (their wait does not
        // wait for the state), then every load of the staged tile
        // (every wave sums all np partials itself, lane l taking l, l + 64,
        // ..., so that the rescale needs no block barrier)
        const int np = I.tiles_x * I.tiles_y;
        const int lane = tid & 63;
        double pp[PP];
#pragma unroll
        for (int k = 0; k < PP; ++k) {
            pp[k] = 0.0;
            if (!RT && use_pin && lane + k * 64 < np)
                pp[k] = pin[I.poff + lane + k * 64];
        }
        // every load is issued (from a clamped in-bounds address where the
        // point lies outside the grid) before any is consumed
        Cx<R> pre[NST];
#pragma unroll
        for (int c = 0; c < NST; ++c) {
            const int e = tid + c * NT;
            const int rr = e / SC, cc = e - rr * SC;
            const int j = jb + rr, i = ib + cc;
            const bool in = e < SR * SC && j >= 1 && j <= ny - 1 && i >= 1 && i <= nx - 1;
            pre[c] = ld<R>(src, in ? (int64_t)j * nx + i : (int64_t)0);
            pre[c] = csel(in, pre[c], Cx<R>{R(0), R(0)});
        }
        // pivot pairs (c*, r*) of the x-lines of the staged rows and of the
        // y-lines of the tile columns
        // (thread t < TC: y-line of column c0 + t; TC <= t < TC + SR: x-line
        // of staged row t - TC; the table row index clamped into the grid)
        const Cx<R> *prow = tid < TC ? taby + (size_t)min(max(c0 + tid, 1), nx - 1) * (W + 2)
                                     : tabx + (size_t)min(max(jb + tid - TC, 1), ny - 1) * (W + 2);
        const Cx<R> pv0 = prow[0], pv1 = prow[1];
        double sm1 = 0.0;
        if (!RT && use_pin) {
            double v = (pp[0] + pp[1]) + (pp[2] + pp[3]);
            for (int t = lane + PP * 64; t < np; t += 64)
                v += pin[I.poff + t];
            sm1 = norm_scale_m1(wave_sum_f64(v), I.dV);
        }
        const R sr = R(sm1);
        // rescale and H1 on every staged point (a point outside the grid
        // holds zero and stays zero)
        if constexpr (RT) {
            // real time: all angles dt w first, then e^{-i dt w} - 1
            // together, then v + (e^{-i dt w} - 1) v
            R th[NST];
#pragma unroll
            for (int c = 0; c < NST; ++c) {
                const int e = tid + c * NT;
                const int rr = e / SC, cc = e - rr * SC;
                const int j = jb + rr, i = ib + cc;
                const double x = I.x0 + i * I.hx, y = I.y0 + j * I.hy;
                th[c] = R(I.dt) * (R(I.vx * x * x + I.vy * y * y) + R(I.g) * norm2(pre[c]));
            }
            Cx<R> f[NST];
            expim1_all(th, f);
#pragma unroll
            for (int c = 0; c < NST; ++c) {
                const int e = tid + c * NT;
                const int rr = e / SC, cc = e - rr * SC;
                if (e < SR * SC)
                    st1[rr * SCP + cc + cc / S] = pre[c] + f[c] * pre[c];
            }
        } else {
            // imaginary time: all arguments -dt w first, then their expm1
            // together, then v + expm1(-dt w) v
            R ex[NST];
#pragma unroll
            for (int c = 0; c < NST; ++c) {
                const int e = tid + c * NT;
                const int rr = e / SC, cc = e - rr * SC;
                const int j = jb + rr, i = ib + cc;
                pre[c] = rescale(pre[c], sr);
                const double x = I.x0 + i * I.hx, y = I.y0 + j * I.hy;
                ex[c] = -R(I.dt) * (R(I.vx * x * x + I.vy * y * y) + R(I.g) * norm2(pre[c]));
            }
            expm1_all(ex);
#pragma unroll
            for (int c = 0; c < NST; ++c) {
                const int e = tid + c * NT;
                const int rr = e / SC, cc = e - rr * SC;
                if (e < SR * SC)
                    st1[rr * SCP + cc + cc / S] = pre[c] + ex[c] * pre[c];
            }
        }
        if (tid < TC) {
            tpy[tid][0] = pv0;
            tpy[tid][1] = pv1;
        } else if (tid - TC < SR) {
            tpx[tid - TC][0] = pv0;
            tpx[tid - TC][1] = pv1;
        }
        __syncthreads();

        // x-lines of every staged row, outputs for the TC tile columns: all
        // windows are read before any output is written back
        Cx<R> xo[NXI][S];
#pragma unroll
        for (int k = 0; k < NXI; ++k) {
            const int p = tid + k * NT;
            const int rr = p / NSX, q = p - rr * NSX;
            const int j = jb + rr;
#pragma unroll
            for (int r = 0; r < S; ++r)
                xo[k][r] = Cx<R>{R(0), R(0)};
            if (p < SR * NSX && j >= 1 && j <= ny - 1) {
                const LineCoef<R> Lc = line_coef<R>(I.ax[0], I.omega * (I.y0 + j * I.hy));
                Cx<R> df;
                const int s = c0 + q * S;
                window_solve<R, S, W, ST, true>(s, nx, Lc, tpx[rr][0], tpx[rr][1],
                                                [&](int r) { return sx(rr, q * S + r); }, xo[k], df);
                if (s == 1)
                    d1x[rr] = df;
#pragma unroll
                for (int r = 0; r < S; ++r)
                    xo[k][r] = csel(s + r <= nx - 1, xo[k][r], Cx<R>{R(0), R(0)});
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NXI; ++k) {
            const int p = tid + k * NT;
            const int rr = p / NSX, q = p - rr * NSX;
            if (p < SR * NSX) {
#pragma unroll
                for (int r = 0; r < S; ++r)
                    sx(rr, H + q * S + r) = xo[k][r];
            }
        }
        __syncthreads();
        if (c0 == 1) {  // wall rows of the x-lines: Sherman-Morrison term
            for (int p = tid; p < SR * W; p += NT) {
                const int rr = p / W, u = 1 + (p - rr * W);
                const int j = jb + rr;
                if (j >= 1 && j <= ny - 1 && u <= nx - 1 && u - c0 < TC)
                    sx(rr, H + u - c0) = sx(rr, H + u - c0) - d1x[rr] * tabx[(size_t)j * (W + 2) + 1 + u];
            }
            __syncthreads();
        }

        // y-lines of the TC columns, outputs for the TR tile rows
        const int col = tid % TC, q = tid / TC;
        const int i = c0 + col;
        const bool act = q < NSY && i <= nx - 1;
        const int s = r0 + q * SY;
        Cx<R> io[SY];
        if (act) {
            const LineCoef<R> Lc = line_coef<R>(I.ax[1], -I.omega * (I.x0 + i * I.hx));
            Cx<R> df;
            window_solve<R, SY, W, ST, true>(s, ny, Lc, tpy[col][0], tpy[col][1],
                                             [&](int r) { return sx(q * SY + r, H + col); }, io, df);
            if (s == 1)
                d1y[col] = df;
        }
        if (r0 == 1)
            __syncthreads();
        double acc = 0.0;
        if (act) {
            const Cx<R> *trow = taby + (size_t)i * (W + 2);
#pragma unroll
            for (int r = 0; r < SY; ++r) {
                const int u = s + r;
                if (u <= ny - 1) {
                    Cx<R> o = io[r];
                    if (r0 == 1 && u <= W)
                        o = o - d1y[col] * trow[1 + u];
                    st<R>(dst, (int64_t)u * nx + i, o);
                    if (!RT)
                        acc += (double)o.re * (double)o.re + (double)o.im * (double)o.im;
                }
            }
        }
        if (!RT) {
            const double b = block_sum_nt<NT>(acc, red);
            if (tid == 0)
                pout[I.poff + tile] = b;
        }
        __syncthreads();  // LDS reuse by the next item
    }
}

// ---------------------------------------------------------------------------
// Exact whole-line path (used when the decay bound would need W > 32).

// Pointwise H1 with the pending rescale, src -> dst.
template <class R, bool RT>
__global__ __launch_bounds__(256) void k_h1(const typename Vec<R>::T *src, typename Vec<R>::T *dst, StepArgs a,
                                            const double *partials, int npart)
{
    double sm1 = 0.0;
    if (!RT && npart > 0)
        sm1 = norm_scale_m1(wave_partials_sum(partials, npart), a.dV);
    const R sr = R(sm1);
    const int64_t n = (int64_t)a.nx * a.ny * (a.dim == 3 ? a.nz : 1);
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        const int i = (int)(p % a.nx);
        const int64_t rest = p / a.nx;
        const int j = (int)(rest % a.ny), k = (int)(rest / a.ny);
        Cx<R> v = rescale(ld<R>(src, p), sr);
        const double x = a.x0 + i * a.hx, y = a.y0 + j * a.hy;
        double V = a.vx * x * x + a.vy * y * y;
        if (a.dim == 3) {
            const double z = a.z0 + k * a.hz;
            V += a.vz * z * z;
        }
        const R w = R(V) + R(a.g) * norm2(v);
        st<R>(dst, p, h1_apply<R, RT>(v, w, R(a.dt)));
    }
}

// One thread per line; textbook Thomas over the whole line with the
// elimination factors in a global workspace (2 complex per point).
template <class R>
__global__ __launch_bounds__(256) void k_line_exact(const typename Vec<R>::T *src, typename Vec<R>::T *dst,
                                                    StepArgs a, int axis, Cx<R> *ws)
{
    const int nx = a.nx, ny = a.ny, nz = (a.dim == 3 ? a.nz : 1);
    int n, nlines;
    if (axis == 0) { n = nx; nlines = ny * nz; }
    else if (axis == 1) { n = ny; nlines = nx * nz; }
    else { n = nz; nlines = nx * ny; }
    const int line = blockIdx.x * 256 + threadIdx.x;
    if (line >= nlines)
        return;
    int64_t base, stride;
    double rot;
    bool wall;
    if (axis == 0) {
        const int j = line % ny, k = line / ny;
        base = ((int64_t)k * ny + j) * nx; stride = 1;
        rot = a.omega * (a.y0 + j * a.hy);
        wall = (j == 0) || (a.dim == 3 && k == 0);
    } else if (axis == 1) {
        const int i = line % nx, k = line / nx;
        base = (int64_t)k * nx * ny + i; stride = nx;
        rot = -a.omega * (a.x0 + i * a.hx);
        wall = (i == 0) || (a.dim == 3 && k == 0);
    } else {
        const int i = line % nx, j = line / nx;
        base = (int64_t)j * nx + i; stride = (int64_t)nx * ny;
        rot = 0.0;
        wall = (i == 0) || (j == 0);
    }
    if (wall)
        return;
    const LineCoef<R> Lc = line_coef<R>(a.ax[axis], rot);
    Cx<R> *cpw = ws + (int64_t)line * 2 * n;
    Cx<R> *dpw = cpw + n;
    const Cx<R> zero = {R(0), R(0)};
    Cx<R> cprev = zero, dprev = zero, vm = zero;
    Cx<R> v0 = ld<R>(src, base + stride);
    for (int u = 1; u <= n - 1; ++u) {
        const Cx<R> vp = (u + 1 <= n - 1) ? ld<R>(src, base + (u + 1) * stride) : zero;
        const Cx<R> rr = recip(Lc.A0 - Lc.Am * cprev);
        cprev = Lc.Ap * rr;
        dprev = (minus_kv(Lc, vm, v0, vp) - Lc.Am * dprev) * rr;
        cpw[u] = cprev;
        dpw[u] = dprev;
        vm = v0;
        v0 = vp;
    }
    Cx<R> dnext = zero;
    for (int u = n - 1; u >= 1; --u) {
        const Cx<R> d = dpw[u] - cpw[u] * dnext;
        const Cx<R> v = ld<R>(src, base + u * stride);
        st<R>(dst, base + u * stride, v + R(2) * d);
        dnext = d;
    }
}

// ---------------------------------------------------------------------------
// Reductions and small kernels.

// FP64 partial sums of |psi|^2 over a grid-stride range (one per block).
template <class R>
__global__ __launch_bounds__(256) void k_norm_partials(const typename Vec<R>::T *psi, int64_t n, double *partials)
{
    __shared__ double red[8];
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        const Cx<R> v = ld<R>(psi, p);
        acc += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
    }
    const double b = block_sum_256(acc, red);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = b;
}

// psi_dst = s psi_src with s = 1/sqrt(dV sum partials).  folded (the
// renormalisation that ends a run of steps): always psi + (s - 1) psi, the
// form the steps fold into their next H1, so that n steps in one call and n
// calls of one step leave the same bits.  An imaginary-time step only lowers
// the norm (s >= 1), where s - 1 from FP64 is at least as accurate as s.
// Otherwise (a given state of arbitrary scale): the same form near s = 1,
// and the product s psi for |s - 1| >= 1/4, since s - 1 rounded to FP32
// would carry a relative error of ulp(1) / s for s << 1.
template <class R>
__global__ __launch_bounds__(256) void k_rescale(const typename Vec<R>::T *src, typename Vec<R>::T *dst, int64_t n,
                                                 double dV, const double *partials, int npart, int folded)
{
    const double tot = wave_partials_sum(partials, npart);
    const double sm1 = norm_scale_m1(tot, dV);
    if (folded || fabs(sm1) < 0.25) {
        const R sr = R(sm1);
        for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256)
            st<R>(dst, p, rescale(ld<R>(src, p), sr));
    } else {
        const R sc = R(1.0 / sqrt(dV * tot));
        for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
            const Cx<R> v = ld<R>(src, p);
            st<R>(dst, p, Cx<R>{v.re * sc, v.im * sc});
        }
    }
}

template <class R>
__global__ __launch_bounds__(256) void k_copy(const typename Vec<R>::T *src, typename Vec<R>::T *dst, int64_t n)
{
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256)
        dst[p] = src[p];
}

// Precision conversion between the two storage layouts.
template <class RS, class RD>
__global__ __launch_bounds__(256) void k_convert(const typename Vec<RS>::T *src, typename Vec<RD>::T *dst, int64_t n)
{
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        const Cx<RS> v = ld<RS>(src, p);
        st<RD>(dst, p, Cx<RD>{RD(v.re), RD(v.im)});
    }
}

// Zero every wall point (index 0 on any axis).
// Density profiles (the paper's density outputs): out[e] for e < nout of
// `kind` (see sscn_density): full |psi|^2, integrals over the other axes
// (sums times the spacings, in a fixed order), or the cut through the
// centre index of the other axes.
template <class R>
__global__ __launch_bounds__(256) void k_density(const typename Vec<R>::T *__restrict__ psi, int nx, int ny,
                                                 int nz, double hx, double hy, double hz, int kind, int64_t nout,
                                                 double *__restrict__ out)
{
    auto dens = [&](int i, int j, int k) -> double {
        const Cx<R> v = ld<R>(psi, ((int64_t)k * ny + j) * nx + i);
        return (double)v.re * (double)v.re + (double)v.im * (double)v.im;
    };
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nout; e += (int64_t)gridDim.x * 256) {
        double r = 0.0;
        if (kind == 0) {
            const int i = (int)(e % nx);
            const int64_t t = e / nx;
            r = dens(i, (int)(t % ny), (int)(t / ny));
        } else if (kind == 1) {  // integral over z: (j, i)
            const int i = (int)(e % nx), j = (int)(e / nx);
            for (int k = 0; k < nz; ++k)
                r += dens(i, j, k);
            r *= nz > 1 ? hz : 1.0;
        } else if (kind == 2) {  // integral over y, z: i
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    r += dens((int)e, j, k);
            r *= hy * (nz > 1 ? hz : 1.0);
        } else if (kind == 3) {  // integral over x, z: j
            for (int k = 0; k < nz; ++k)
                for (int i = 0; i < nx; ++i)
                    r += dens(i, (int)e, k);
            r *= hx * (nz > 1 ? hz : 1.0);
        } else if (kind == 4) {  // integral over x, y: k
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i)
                    r += dens(i, j, (int)e);
            r *= hx * hy;
        } else if (kind == 5) {  // cut along x through (ny/2, nz/2)
            r = dens((int)e, ny / 2, nz / 2);
        } else if (kind == 6) {  // cut along y
            r = dens(nx / 2, (int)e, nz / 2);
        } else {  // cut along z
            r = dens(nx / 2, ny / 2, (int)e);
        }
        out[e] = r;
    }
}

// Centred embedding (continuation start): dst[k][j][i] = src[k-oz][j-oy][i-ox]
// where that index lies inside src, else zero; zero on the walls of dst.
template <class R>
__global__ __launch_bounds__(256) void k_embed(const typename Vec<R>::T *__restrict__ src, int nxs, int nys,
                                               int nzs, typename Vec<R>::T *__restrict__ dst, int nx, int ny,
                                               int nz, int ox, int oy, int oz, int dim)
{
    const int64_t n = (int64_t)nx * ny * nz;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int i = (int)(e % nx);
        const int64_t r = e / nx;
        const int j = (int)(r % ny), k = (int)(r / ny);
        const int is = i - ox, js = j - oy, ks = k - oz;
        const bool wall = i == 0 || j == 0 || (dim == 3 && k == 0);
        const bool in = !wall && is >= 0 && is < nxs && js >= 0 && js < nys && ks >= 0 && ks < nzs;
        Cx<R> v = {R(0), R(0)};
        if (in)
            v = ld<R>(src, ((int64_t)ks * nys + js) * nxs + is);
        st<R>(dst, e, v);
    }
}

// Product state of the 3D form of Eq. (fun): dst[k][j][i] = xy[j][i] c g_k
// with g_k = exp(-z_k^2 / (2 d_z^2)), z_k = z0 + k hz, c given.
template <class R>
__global__ __launch_bounds__(256) void k_extend_z(const typename Vec<R>::T *__restrict__ xy, int nx, int ny,
                                                  typename Vec<R>::T *__restrict__ dst, int nz, double z0,
                                                  double hz, double dz, double c)
{
    const int64_t nxy = (int64_t)nx * ny, n = nxy * nz;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int k = (int)(e / nxy);
        const double t = (z0 + k * hz) / dz;
        const double f = c * exp(-0.5 * t * t);
        const Cx<R> v = ld<R>(xy, e - k * nxy);
        st<R>(dst, e, Cx<R>{R((double)v.re * f), R((double)v.im * f)});
    }
}

// Keys' cubic convolution weights (a = -1/2) of the samples at offsets -1,
// 0, 1, 2 from a point at fraction t in [0, 1) past the sample at offset 0:
// W(t + 1), W(t), W(1 - t), W(2 - t) with W the piecewise cubic of the
// kernel (expanded in t).
__device__ __forceinline__ void keys_weights(double t, double (&w)[4])
{
    w[0] = ((-t + 2.0) * t - 1.0) * t * 0.5;
    w[1] = ((3.0 * t - 5.0) * t * t + 2.0) * 0.5;
    w[2] = ((-3.0 * t + 4.0) * t + 1.0) * t * 0.5;
    w[3] = (t - 1.0) * t * t * 0.5;
}

// Grid-to-grid interpolation: dst point (x, y) (both grids centred,
// x_i = -n h / 2 + i h) takes the cubic-convolution interpolant of src at
// (ca x - sa y, sa x + ca y); src samples beyond its grid are zero; dst
// walls (index 0) are zero.  FP64 arithmetic in both precisions.
template <class R>
__global__ __launch_bounds__(256) void k_resample(const typename Vec<R>::T *__restrict__ src, int nxs, int nys,
                                                  double hxs, double hys, typename Vec<R>::T *__restrict__ dst,
                                                  int nx, int ny, double hx, double hy, double ca, double sa)
{
    const int64_t n = (int64_t)nx * ny;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        const int i = (int)(p % nx), j = (int)(p / nx);
        double re = 0.0, im = 0.0;
        const double x = -0.5 * nx * hx + i * hx, y = -0.5 * ny * hy + j * hy;
        const double u = (ca * x - sa * y + 0.5 * nxs * hxs) / hxs;
        const double v = (sa * x + ca * y + 0.5 * nys * hys) / hys;
        // beyond the source grid by more than the stencil: zero (and the
        // integer conversion below stays in range)
        if (i > 0 && j > 0 && u > -2.0 && u < nxs + 1.0 && v > -2.0 && v < nys + 1.0) {
            const double fu = floor(u), fv = floor(v);
            const int i0 = (int)fu, j0 = (int)fv;
            double wx[4], wy[4];
            keys_weights(u - fu, wx);
            keys_weights(v - fv, wy);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int js = j0 - 1 + b;
                if (js < 0 || js >= nys)
                    continue;
                double rr = 0.0, ri = 0.0;
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int is = i0 - 1 + a;
                    if (is < 0 || is >= nxs)
                        continue;
                    const Cx<R> f = ld<R>(src, (int64_t)js * nxs + is);
                    rr += wx[a] * (double)f.re;
                    ri += wx[a] * (double)f.im;
                }
                re += wy[b] * rr;
                im += wy[b] * ri;
            }
        }
        st<R>(dst, p, Cx<R>{R(re), R(im)});
    }
}

// Angular moments of the density about the origin, one block of 1024
// threads: out[2k], out[2k + 1] = hx hy sum |psi|^2 (cos k phi, sin k phi),
// k = 0..kmax (kmax <= 8); a point at the origin enters k = 0 only.  Each
// thread sums a grid-stride share, then a fixed-order block sum.
template <class R>
__global__ __launch_bounds__(1024) void k_angular_moments(const typename Vec<R>::T *__restrict__ psi, int nx, int ny,
                                                          double hx, double hy, int kmax, double *__restrict__ out)
{
    __shared__ double red[16];
    double c[9], s[9];
#pragma unroll
    for (int k = 0; k < 9; ++k)
        c[k] = s[k] = 0.0;
    const int64_t n = (int64_t)nx * ny;
    for (int64_t p = threadIdx.x; p < n; p += 1024) {
        const int i = (int)(p % nx), j = (int)(p / nx);
        const double x = -0.5 * nx * hx + i * hx, y = -0.5 * ny * hy + j * hy;
        const Cx<R> v = ld<R>(psi, p);
        const double d = (double)v.re * (double)v.re + (double)v.im * (double)v.im;
        // e^{i phi}, zero at the origin (the grid point 2i = nx, 2j = ny,
        // found by index: a contracted x = -nx hx / 2 + i hx need not be 0
        // there), so that the origin adds to k = 0 only
        const bool origin = 2 * i == nx && 2 * j == ny;
        const double r = sqrt(x * x + y * y);
        const double er = origin ? 0.0 : x / r, ei = origin ? 0.0 : y / r;
        double pr = 1.0, pi = 0.0;  // e^{i k phi}, k = 0 first
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            c[k] += d * pr;
            s[k] += d * pi;
            const double t = pr * er - pi * ei;
            pi = pr * ei + pi * er;
            pr = t;
        }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int k = 0; k <= kmax && k < 9; ++k) {
        for (int part = 0; part < 2; ++part) {
            const double w = wave_sum_f64(part ? s[k] : c[k]);
            if (lane == 0)
                red[wave] = w;
            __syncthreads();
            if (threadIdx.x == 0) {
                double t = 0.0;
                for (int q = 0; q < 16; ++q)
                    t += red[q];
                out[2 * k + part] = hx * hy * t;
            }
            __syncthreads();
        }
    }
}

template <class R>
__global__ __launch_bounds__(256) void k_zero_walls(typename Vec<R>::T *psi, StepArgs a)
{
    const int64_t n = (int64_t)a.nx * a.ny * (a.dim == 3 ? a.nz : 1);
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        const int i = (int)(p % a.nx);
        const int64_t rest = p / a.nx;
        const int j = (int)(rest % a.ny), k = (int)(rest / a.ny);
        if (i == 0 || j == 0 || (a.dim == 3 && k == 0))
            st<R>(psi, p, Cx<R>{R(0), R(0)});
    }
}

// Initial state of Eq. (fun) (not normalised; the host normalises after).
// Counter-based uniform numbers for the random phase R(x, y) of Eq. (fun):
// u = 2^-53 (h(seed XOR q) >> 11) for the point index q = j nx + i, with h
// the output function of the SplitMix64 generator (Steele, Lea and Flood,
// 2014): advance the state by the golden-ratio increment 0x9E3779B97F4A7C15,
// then two xor-shift-multiply rounds and a final xor-shift.  Integer
// arithmetic only, so every implementation gives the same bits.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double seed_uniform(uint64_t seed, int64_t q)
{
    return (double)(splitmix64(seed ^ (uint64_t)q) >> 11) * 0x1.0p-53;
}

// out[j nx + i] = seed_uniform(seed, j nx + i) for an ny x nx plane.
static __global__ __launch_bounds__(256) void k_phase_seed(double *out, int nx, int ny, uint64_t seed)
{
    const int64_t n = (int64_t)nx * ny;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
        out[q] = seed_uniform(seed, q);
}

// Initial state of Eq. (fun); the random phase from the host array phase
// (NULL: none) or, with seeded, from seed_uniform(seed, j nx + i).
template <class R>
__global__ __launch_bounds__(256) void k_init(typename Vec<R>::T *psi, StepArgs a, int kind, const double *phase,
                                              double dxy, double dz, int seeded = 0, uint64_t seed = 0)
{
    const double pi = 3.14159265358979323846;
    const int64_t n = (int64_t)a.nx * a.ny * (a.dim == 3 ? a.nz : 1);
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        const int i = (int)(p % a.nx);
        const int64_t rest = p / a.nx;
        const int j = (int)(rest % a.ny), k = (int)(rest / a.ny);
        double re = 0.0, im = 0.0;
        if (i > 0 && j > 0 && (a.dim == 2 || k > 0)) {
            const double x = a.x0 + i * a.hx, y = a.y0 + j * a.hy;
            double fr = 1.0, fi = 0.0;
            if (kind == 1) { fr = x; fi = y; }
            const double amp = exp(-(x * x + y * y) / (2.0 * dxy * dxy)) / sqrt(pi * dxy * dxy);
            re = fr * amp;
            im = fi * amp;
            if (phase || seeded) {
                const int64_t q = (int64_t)j * a.nx + i;
                double sn, cs;
                sincos(2.0 * pi * (seeded ? seed_uniform(seed, q) : phase[q]), &sn, &cs);
                const double r2 = re * cs - im * sn, i2 = re * sn + im * cs;
                re = r2;
                im = i2;
            }
            if (a.dim == 3) {
                const double z = a.z0 + k * a.hz;
                const double fz = pow(pi * dz * dz, -0.25) * exp(-z * z / (2.0 * dz * dz));
                re *= fz;
                im *= fz;
            }
        }
        st<R>(psi, p, Cx<R>{R(re), R(im)});
    }
}

// Observables: 15 FP64 sums + max density (index 13) per block (see
// sscn_obs.sums).
constexpr int kObsN = 16;
template <class R>
__device__ __forceinline__ Cx<double> at(const typename Vec<R>::T *psi, const StepArgs &a, int i, int j, int k)
{
    const int nz = a.dim == 3 ? a.nz : 1;
    if (i < 0 || j < 0 || k < 0 || i >= a.nx || j >= a.ny || k >= nz)
        return Cx<double>{0.0, 0.0};
    const Cx<R> v = ld<R>(psi, ((int64_t)k * a.ny + j) * a.nx + i);
    return Cx<double>{(double)v.re, (double)v.im};
}

// The 13 sums and the max of the observables at grid point p (see sscn_obs).
template <class R>
__device__ __forceinline__ void obs_point(const typename Vec<R>::T *psi, const StepArgs &a, int64_t p,
                                          double (&s)[kObsN])
{
    const int i = (int)(p % a.nx);
    const int64_t rest = p / a.nx;
    const int j = (int)(rest % a.ny), k = (int)(rest / a.ny);
    const double x = a.x0 + i * a.hx, y = a.y0 + j * a.hy;
    const double z = a.dim == 3 ? a.z0 + k * a.hz : 0.0;
    const Cx<double> v = at<R>(psi, a, i, j, k);
    const double dens = v.re * v.re + v.im * v.im;
    double V = a.vx * x * x + a.vy * y * y;
    if (a.dim == 3)
        V += a.vz * z * z;
    const Cx<double> xp = at<R>(psi, a, i + 1, j, k), xm = at<R>(psi, a, i - 1, j, k);
    const Cx<double> yp = at<R>(psi, a, i, j + 1, k), ym = at<R>(psi, a, i, j - 1, k);
    const Cx<double> fx = (1.0 / a.hx) * (xp - v), fy = (1.0 / a.hy) * (yp - v);
    Cx<double> fz = {0.0, 0.0};
    if (a.dim == 3)
        fz = (1.0 / a.hz) * (at<R>(psi, a, i, j, k + 1) - v);
    const double kin_r = fx.re * fx.re + fy.re * fy.re + fz.re * fz.re;
    const double kin = norm2(fx) + norm2(fy) + norm2(fz);
    const Cx<double> cxd = (1.0 / (2.0 * a.hx)) * (xp - xm), cyd = (1.0 / (2.0 * a.hy)) * (yp - ym);
    const Cx<double> lz = y * cxd - x * cyd;  // (y d/dx - x d/dy) psi
    // fourth-order central differences (-f[i+2] + 8 f[i+1] - 8 f[i-1] + f[i-2]) / (12 h)
    const Cx<double> qx = (1.0 / (12.0 * a.hx)) * (8.0 * (xp - xm) - (at<R>(psi, a, i + 2, j, k) - at<R>(psi, a, i - 2, j, k)));
    const Cx<double> qy = (1.0 / (12.0 * a.hy)) * (8.0 * (yp - ym) - (at<R>(psi, a, i, j + 2, k) - at<R>(psi, a, i, j - 2, k)));
    Cx<double> qz = {0.0, 0.0};
    if (a.dim == 3)
        qz = (1.0 / (12.0 * a.hz)) * (8.0 * (at<R>(psi, a, i, j, k + 1) - at<R>(psi, a, i, j, k - 1)) -
                                      (at<R>(psi, a, i, j, k + 2) - at<R>(psi, a, i, j, k - 2)));
    const Cx<double> lz4 = y * qx - x * qy;
    s[0] += dens;
    s[1] += v.re * v.re;
    s[2] += 0.5 * kin_r;
    s[3] += V * v.re * v.re;
    s[4] += a.g * dens * v.re * v.re;
    s[5] += a.omega * v.re * lz.im;
    s[6] += 0.5 * kin;
    s[7] += V * dens;
    s[8] += a.g * dens * dens;
    s[9] += a.omega * (v.re * lz.im - v.im * lz.re);  // Im(conj(v) lz)
    s[10] += x * x * dens;
    s[11] += y * y * dens;
    s[12] += z * z * dens;
    s[13] = fmax(s[13], __dadd_rn(__dmul_rn(v.re, v.re), __dmul_rn(v.im, v.im)));  // as k_plane_max
    s[14] += 0.5 * (norm2(qx) + norm2(qy) + norm2(qz));
    s[15] += a.omega * (v.re * lz4.im - v.im * lz4.re);  // Im(conj(v) lz4)
}

template <class R>
__device__ __forceinline__ void obs_block_write(double (&s)[kObsN], double *red, double *out)
{
#pragma unroll
    for (int t = 0; t < kObsN; ++t) {
        const double b = t == 13 ? block_max_256(s[t], red) : block_sum_256(s[t], red);
        if (threadIdx.x == 0)
            out[t] = b;
    }
}

template <class R>
__global__ __launch_bounds__(256) void k_observables(const typename Vec<R>::T *psi, StepArgs a, double *partials)
{
    __shared__ double red[8];
    const int64_t n = (int64_t)a.nx * a.ny * (a.dim == 3 ? a.nz : 1);
    double s[kObsN];
#pragma unroll
    for (int t = 0; t < kObsN; ++t)
        s[t] = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256)
        obs_point<R>(psi, a, p, s);
    obs_block_write<R>(s, red, partials + (int64_t)blockIdx.x * kObsN);
}

// Fixed-order final reduction of nblk rows of nval partials: values with
// maxmask bit set take the max, the others the sum.  One 256-thread block.
static __global__ __launch_bounds__(256) void k_reduce_final(const double *partials, int nblk, int nval, unsigned maxmask,
                                                      double *out)
{
    __shared__ double red[8];
    for (int v = 0; v < nval; ++v) {
        const bool mx = (maxmask >> v) & 1u;
        double acc = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 256) {
            const double x = partials[(int64_t)b * nval + v];
            acc = mx ? fmax(acc, x) : acc + x;
        }
        const double r = mx ? block_max_256(acc, red) : block_sum_256(acc, red);
        if (threadIdx.x == 0)
            out[v] = r;
        __syncthreads();
    }
}

// Max density over the plane k0 (one partial per block).
template <class R>
__global__ __launch_bounds__(256) void k_plane_max(const typename Vec<R>::T *psi, StepArgs a, int k0, double *partials)
{
    __shared__ double red[8];
    const int64_t n = (int64_t)a.nx * a.ny;
    double m = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        const Cx<R> v = ld<R>(psi, (int64_t)k0 * n + p);
        const double re = v.re, im = v.im;
        m = fmax(m, __dadd_rn(__dmul_rn(re, re), __dmul_rn(im, im)));
    }
    const double b = block_max_256(m, red);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = b;
}

// Vortex windings counted at plaquette (i, j) of plane k0 (corners (i, j),
// (i+1, j), (i+1, j+1), (i, j+1)): w = round(sum of the wrapped phase
// differences counter-clockwise / 2 pi) when w > 0, no corner is exactly
// zero and the largest density within `box` points reaches thr; else 0.
template <class R>
__device__ __forceinline__ int plaquette_count(const typename Vec<R>::T *psi, const StepArgs &a, int k0, int i, int j,
                                               double thr, int box)
{
    const double two_pi = 6.283185307179586476925286766559;
    const Cx<double> c00 = at<R>(psi, a, i, j, k0), c10 = at<R>(psi, a, i + 1, j, k0);
    const Cx<double> c11 = at<R>(psi, a, i + 1, j + 1, k0), c01 = at<R>(psi, a, i, j + 1, k0);
    auto zero = [](Cx<double> c) { return c.re == 0.0 && c.im == 0.0; };
    if (zero(c00) || zero(c10) || zero(c11) || zero(c01))
        return 0;
    // arg(b conj(a)) with the products rounded as written (no contraction)
    auto darg = [](Cx<double> b, Cx<double> c) {
        const double re = __dadd_rn(__dmul_rn(b.re, c.re), __dmul_rn(b.im, c.im));
        const double im = __dsub_rn(__dmul_rn(b.im, c.re), __dmul_rn(b.re, c.im));
        return atan2(im, re);
    };
    const double sum = darg(c10, c00) + darg(c11, c10) + darg(c01, c11) + darg(c00, c01);
    const int w = (int)llround(sum / two_pi);
    if (w <= 0)
        return 0;
    double local = 0.0;
    for (int jj = j - box; jj <= j + 1 + box; ++jj)
        for (int ii = i - box; ii <= i + 1 + box; ++ii) {
            const Cx<double> v = at<R>(psi, a, ii, jj, k0);
            local = fmax(local, __dadd_rn(__dmul_rn(v.re, v.re), __dmul_rn(v.im, v.im)));
        }
    return local >= thr ? w : 0;
}

// Vortex count on plane k0: per plaquette winding of the wrapped phase
// differences, masked by the largest density within `box` points.
template <class R>
__global__ __launch_bounds__(256) void k_vortex(const typename Vec<R>::T *psi, StepArgs a, int k0, double frac,
                                                int box, const double *dmax, double *partials)
{
    __shared__ double red[8];
    const int nx = a.nx, ny = a.ny;
    const int64_t n = (int64_t)(nx - 1) * (ny - 1);
    const double thr = frac * dmax[0];
    double cnt = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        const int i = (int)(p % (nx - 1)), j = (int)(p / (nx - 1));
        cnt += plaquette_count<R>(psi, a, k0, i, j, thr, box);
    }
    const double b = block_sum_256(cnt, red);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = b;
}

// ---------------------------------------------------------------------------
// Batched instances: per-instance chunks of kChunk points as work items.
constexpr int kChunk = 4096;

__device__ __forceinline__ StepArgs inst_args(const Inst2D &I)
{
    StepArgs a{};
    const bool d3 = I.nz > 1;
    a.dim = d3 ? 3 : 2;
    a.nx = I.nx;
    a.ny = I.ny;
    a.nz = d3 ? I.nz : 1;
    a.hx = I.hx;
    a.hy = I.hy;
    a.hz = d3 ? I.hz : 1.0;
    a.x0 = I.x0;
    a.y0 = I.y0;
    a.z0 = d3 ? I.z0 : 0.0;
    a.vx = I.vx;
    a.vy = I.vy;
    a.vz = d3 ? I.vz : 0.0;
    a.g = I.g;
    a.omega = I.omega;
    a.dt = I.dt;
    a.dV = I.dV;
    a.ax[0] = I.ax[0];
    a.ax[1] = I.ax[1];
    a.ax[2] = d3 ? I.ax[2] : I.ax[1];
    return a;
}

// Points of an instance's state.
__device__ __forceinline__ int64_t inst_points(const Inst2D &I) { return (int64_t)I.nx * I.ny * (I.nz > 1 ? I.nz : 1); }

// End of a batched stepping call: for every listed (instance, chunk) item,
// buf[0] = s buf[parity] with s = 1/sqrt(dV sum of the instance's partials)
// (imaginary time, rescale = 1) or a plain copy (rescale = 0).
// With scale != NULL, s - 1 of instance k is scale[k] (sweep plan).
template <class R>
__global__ __launch_bounds__(256) void k_batch_finish(const Inst2D *__restrict__ insts, const int2 *__restrict__ fwork,
                                                      const int *__restrict__ nf, int parity,
                                                      const double *__restrict__ partials, int rescale_on,
                                                      const double *__restrict__ scale)
{
    const int nfw = *nf;
    for (int it = blockIdx.x; it < nfw; it += gridDim.x) {
        const int2 wk = fwork[it];
        const Inst2D &I = insts[wk.x];
        const int64_t n = inst_points(I);
        double sm1 = 0.0;
        if (rescale_on && scale)
            sm1 = scale[wk.x];
        else if (rescale_on)
            sm1 = norm_scale_m1(wave_partials_sum(partials + I.poff, I.tiles_x * I.tiles_y), I.dV);
        const R sr = R(sm1);
        const typename Vec<R>::T *src = reinterpret_cast<const typename Vec<R>::T *>(I.buf[parity]);
        typename Vec<R>::T *dst = reinterpret_cast<typename Vec<R>::T *>(I.buf[0]);
        const int64_t base = (int64_t)wk.y * kChunk;
        Cx<R> v[kChunk / 256];
#pragma unroll
        for (int c = 0; c < kChunk / 256; ++c) {
            const int64_t p = base + threadIdx.x + c * 256;
            v[c] = Cx<R>{R(0), R(0)};
            if (p < n)
                v[c] = ld<R>(src, p);
        }
#pragma unroll
        for (int c = 0; c < kChunk / 256; ++c) {
            const int64_t p = base + threadIdx.x + c * 256;
            if (p < n)
                st<R>(dst, p, rescale(v[c], sr));
        }
        __syncthreads();
    }
}

// Observables of every listed (instance, chunk) item into opart[item * kObsN].
template <class R>
__global__ __launch_bounds__(256) void k_batch_obs(const Inst2D *__restrict__ insts, const int2 *__restrict__ owork,
                                                   const int *__restrict__ no, double *__restrict__ opart)
{
    __shared__ double red[8];
    const int now = *no;
    for (int it = blockIdx.x; it < now; it += gridDim.x) {
        const int2 wk = owork[it];
        const Inst2D &I = insts[wk.x];
        const StepArgs a = inst_args(I);
        const typename Vec<R>::T *psi = reinterpret_cast<const typename Vec<R>::T *>(I.buf[0]);
        const int64_t n = inst_points(I);
        const int64_t base = (int64_t)wk.y * kChunk;
        double s[kObsN];
#pragma unroll
        for (int t = 0; t < kObsN; ++t)
            s[t] = 0.0;
        for (int c = threadIdx.x; c < kChunk; c += 256)
            if (base + c < n)
                obs_point<R>(psi, a, base + c, s);
        obs_block_write<R>(s, red, opart + (int64_t)it * kObsN);
        __syncthreads();
    }
}

// Per instance (one block each): fixed-order sum of its items' partials
// (items obase[k] .. obase[k] + ocount[k] - 1 of the current list; ocount 0
// for instances not listed) into sums[k * kObsN ..].
static __global__ __launch_bounds__(256) void k_batch_obs_final(int ninst, const int *__restrict__ obase,
                                                                const int *__restrict__ ocount,
                                                                const double *__restrict__ opart,
                                                                double *__restrict__ sums)
{
    __shared__ double red[8];
    const int k = blockIdx.x;
    if (k >= ninst)
        return;
    const int cnt = ocount[k], b0 = obase[k];
    if (cnt == 0)
        return;
    double acc[kObsN];
    for (int v = 0; v < kObsN; ++v) {
        const bool mx = v == 13;
        double x = 0.0;
        for (int b = threadIdx.x; b < cnt; b += 256) {
            const double y = opart[(int64_t)(b0 + b) * kObsN + v];
            x = mx ? fmax(x, y) : x + y;
        }
        acc[v] = mx ? block_max_256(x, red) : block_sum_256(x, red);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int v = 0; v < kObsN; ++v)
            sums[(int64_t)k * kObsN + v] = acc[v];
}

// Vortex windings of every listed (instance, chunk) item: the plaquettes
// p = chunk * kChunk .. + kChunk - 1 of the (nx - 1) (ny - 1) plaquettes,
// counted as plaquette_count with the instance's max density sums[k * kObsN
// + 13] (from k_batch_obs_final); one partial per item into vpart[item].
template <class R>
__global__ __launch_bounds__(256) void k_batch_vortex(const Inst2D *__restrict__ insts, const int2 *__restrict__ owork,
                                                      const int *__restrict__ no, const double *__restrict__ sums,
                                                      double frac, int box, double *__restrict__ vpart)
{
    __shared__ double red[8];
    const int now = *no;
    for (int it = blockIdx.x; it < now; it += gridDim.x) {
        const int2 wk = owork[it];
        const Inst2D &I = insts[wk.x];
        const StepArgs a = inst_args(I);
        const typename Vec<R>::T *psi = reinterpret_cast<const typename Vec<R>::T *>(I.buf[0]);
        const int64_t n = (int64_t)(I.nx - 1) * (I.ny - 1);
        const int64_t base = (int64_t)wk.y * kChunk;
        const double thr = frac * sums[(int64_t)wk.x * kObsN + 13];
        double cnt = 0.0;
        for (int c = threadIdx.x; c < kChunk; c += 256) {
            const int64_t p = base + c;
            if (p < n)
                cnt += plaquette_count<R>(psi, a, I.nz > 1 ? I.nz / 2 : 0, (int)(p % (I.nx - 1)),
                                          (int)(p / (I.nx - 1)), thr, box);
        }
        const double b = block_sum_256(cnt, red);
        if (threadIdx.x == 0)
            vpart[it] = b;
        __syncthreads();
    }
}

// Convergence bookkeeping of every listed instance (one thread each), the
// criterion of sscn_converge: mu of the real-part form (from sums), its
// change since the last check d; when d < tol the instance's vortex count c
// (sum of its vpart items, exact in FP64) is compared with the count at the
// previous hit, and hits counts consecutive checks with d < tol and an
// unchanged count (a changed count restarts the run of hits at 1); an
// instance is flagged converged (conv[k] = step) at two hits.  counts[k]
// receives every listed instance's current count.
static __global__ __launch_bounds__(256) void k_batch_conv(int ninst, const int *__restrict__ obase,
                                                           const int *__restrict__ ocount,
                                                           const double *__restrict__ vpart,
                                                           const double *__restrict__ sums,
                                                           double *__restrict__ mu_prev, int *__restrict__ hits,
                                                           int *__restrict__ count_prev, int *__restrict__ counts,
                                                           long long *__restrict__ conv, double tol, long long step)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ninst || ocount[k] == 0)
        return;
    double c = 0.0;
    for (int b = 0; b < ocount[k]; ++b)
        c += vpart[obase[k] + b];
    const int cnt = (int)c;
    counts[k] = cnt;
    const double *s = sums + (int64_t)k * kObsN;
    const double mu = (s[2] + s[3] + s[4] + s[5]) / s[1];
    const double prev = mu_prev[k];
    if (conv[k] < 0) {
        if (prev == prev && fabs(mu - prev) < tol) {
            hits[k] = (count_prev[k] < 0 || cnt == count_prev[k]) ? hits[k] + 1 : 1;
            count_prev[k] = cnt;
            if (hits[k] >= 2)
                conv[k] = step;
        } else {
            hits[k] = 0;
            count_prev[k] = -1;
        }
    }
    mu_prev[k] = mu;
}

// ---------------------------------------------------------------------------
// Batched sweep plan (2D instances): the x- and y-sweeps of every listed
// instance in one launch each, over work lists of (instance, x line block)
// and (instance, y tile).  State in buf[0]; the x-sweep writes buf[1] and
// the y-sweep writes buf[0] back with one norm partial per y tile at
// partials[I.ypoff + tile].

// s - 1 of the pending rescale of each listed instance, from its partials.
static __global__ __launch_bounds__(256) void k_batch_scale(const Inst2D *__restrict__ insts, const int *__restrict__ klist,
                                                     const int *__restrict__ nk, const double *__restrict__ partials,
                                                     double *__restrict__ scale)
{
    const int nkk = *nk;
    for (int it = blockIdx.x; it < nkk; it += gridDim.x) {
        const int k = klist[it];
        const Inst2D &I = insts[k];
        const double sm1 = norm_scale_m1(wave_partials_sum(partials + I.eoff, I.ecount), I.dV);
        if (threadIdx.x == 0)
            scale[k] = sm1;
    }
}

// One work-list item (instance, first line) per block.  use_scale = 1: the
// pending rescale of the instance is formed here, from the norm partials the
// previous step's last sweep left at partials[I.eoff ..] (every wave sums
// them in the fixed order of wave_partials_sum while its state loads are in
// flight, so every block, and the finish pass, gets the same bits); 2: it
// is read from scale[instance], where k_batch_scale left it (the same sum,
// once per instance, for instances with many partials); 0: none.
template <class R, int S, int W, bool RT, int KX>
__global__ __launch_bounds__(256, kSweepWaves) void k_batch_xsweep(const Inst2D *__restrict__ insts, const int2 *__restrict__ xwork,
                                                      const int *__restrict__ nitems,
                                                      const double *__restrict__ partials, int use_scale,
                                                      const double *__restrict__ scale)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int it = blockIdx.x;
    if (it >= *nitems)
        return;
    const int2 wk = xwork[it];
    const Inst2D &I = insts[wk.x];
    const StepArgs a = inst_args(I);
    XStage<R, KX> g;
    xsweep_load<R, S, W, KX, kBatchStream>(reinterpret_cast<const typename Vec<R>::T *>(I.buf[0]), a, I.xl,
                                   reinterpret_cast<const Cx<R> *>(I.tab[0]), wk.y, g);
    const double sm1 = use_scale == 1   ? norm_scale_m1(wave_partials_sum(partials + I.eoff, I.ecount), I.dV)
                       : use_scale == 2 ? scale[wk.x]
                                        : 0.0;
    // 2D: buf[0] -> buf[1]; 3D: in place (a block loads its lines whole
    // before it writes them), so that the y- and z-sweeps end in buf[0]
    xsweep_finish<R, S, W, RT, KX, kBatchStream>(reinterpret_cast<typename Vec<R>::T *>(I.buf[I.nz > 1 ? 0 : 1]), a,
                                                 I.xl, sm1, wk.y, g, smem_raw);
}

// One item per block, XCD-aware (xcd_item): the launch has at least
// 8 ceil(nitems / 8) blocks.
template <class R, int S, int W, bool EMIT>
__global__ __launch_bounds__(256, kSweepWaves) void k_batch_ysweep(const Inst2D *__restrict__ insts, const int2 *__restrict__ ywork,
                                                      const int *__restrict__ nitems, double *__restrict__ partials)
{
    __shared__ double red[8];
    const int it = xcd_item(*nitems);
    if (it < 0)
        return;
    const int2 wk = ywork[it];
    const Inst2D &I = insts[wk.x];
    const StepArgs a = inst_args(I);
    // item wk.y: segment group by of column tile bx in plane bz
    const int by = wk.y % I.ygy, rest = wk.y / I.ygy;
    const int bx = rest % I.ygx, bz = rest / I.ygx;
    // 2D: buf[1] -> buf[0] with the norm partials; 3D: buf[0] -> buf[1]
    const int from = I.nz > 1 ? 0 : 1;
    ysweep_block<R, S, W, EMIT, kBatchStream>(reinterpret_cast<const typename Vec<R>::T *>(I.buf[from]),
                                              reinterpret_cast<typename Vec<R>::T *>(I.buf[1 - from]), a, bx, by, bz,
                                              partials + I.ypoff + wk.y, reinterpret_cast<const Cx<R> *>(I.tab[1]),
                                              red);
}

// Batched z-sweep of 3D instances, one item (instance, z tile) per block,
// XCD-aware: buf[1] -> buf[0] with the norm partials of the outputs (EMIT) at
// partials[I.zpoff + tile].  Tile t: segment group t % zgy of the column
// group t / zgy (32 consecutive (i, j) columns of the plane).
template <class R, int S, int W, bool EMIT>
__global__ __launch_bounds__(256, kSweepWaves) void k_batch_zsweep(const Inst2D *__restrict__ insts, const int2 *__restrict__ zwork,
                                                      const int *__restrict__ nitems, double *__restrict__ partials)
{
    __shared__ double red[8];
    const int it = xcd_item(*nitems);
    if (it < 0)
        return;
    const int2 wk = zwork[it];
    const Inst2D &I = insts[wk.x];
    const StepArgs a = inst_args(I);
    const int by = wk.y % I.zgy, bx = wk.y / I.zgy;
    const int nx = I.nx, ny = I.ny;
    const int pidx = bx * kYLines + threadIdx.x;
    const int i = pidx % nx, j = pidx / nx;
    const Cx<R> *trow = nullptr;
    LineCoef<R> Lc{};
    if (pidx < nx * ny && i > 0 && j > 0) {
        Lc = line_coef<R>(a.ax[2], 0.0);
        trow = reinterpret_cast<const Cx<R> *>(I.tab[2]);
    }
    double acc = 0.0;
    strided_sweep_tile<R, S, W, kBatchStream>(reinterpret_cast<const typename Vec<R>::T *>(I.buf[1]),
                                              reinterpret_cast<typename Vec<R>::T *>(I.buf[0]), I.nz, 0,
                                              (int64_t)nx * ny, nx * ny, bx * kYLines, by, true, Lc, trow, EMIT, acc);
    if (EMIT) {
        const double b = block_sum_256(acc, red);
        if (threadIdx.x == 0 && threadIdx.y == 0)
            partials[I.zpoff + wk.y] = b;
    }
}

}  // namespace sscn
