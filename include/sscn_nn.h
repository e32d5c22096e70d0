/*
 * sscn_nn.h -- C ABI of the kernels of the learned initial state.
 *
 * A small convolutional U-Net proposes the initial state of an imaginary-
 * time run in place of the one-vortex random-phase state of Eq. (fun)
 * (paper, Sec. 2).  The paper itself accelerates convergence by starting
 * from a converged state of neighbouring parameters (Sec. 3 and Fig. 3); the
 * network generalises that idea from converged states the solver produces.
 * These entry points are the network's forward and backward building blocks;
 * the layer sequence and the training loop live in
 * paper_1906_06327_amd/nn.py.
 *
 * Tensors are DEVICE buffers, NHWC (channels fastest).  Activations and
 * activation gradients are bf16 (uint16 bit patterns); weights of a 3x3
 * convolution are bf16 [Cout][3][3][Cin]; biases, weight/bias gradients and
 * the Adam state are fp32.  Channel counts of every convolution are
 * multiples of 16 (pad with zeros).  "ld"/"off" arguments address channel
 * slices: element (pixel p, channel c) of a slice is at p*ld + off + c.
 * Every call enqueues on `stream` (a hipStream_t, NULL = null stream) and
 * returns 0, or -1 for bad arguments, -5 for a HIP launch error;
 * sscn_nn_last_error() describes the last failure of the calling thread.
 * Reductions are fixed-order (no atomics): results are deterministic.
 */
#ifndef SSCN_NN_H
#define SSCN_NN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* y = act(conv3x3(x, w) + bias), zero padding 1, stride 1.  Matrix-core
 * implicit GEMM (bf16 x bf16 -> fp32): block tiles of 128 pixels x up to
 * 128 output channels on the gfx950 16x16x32 bf16 instructions.  act: 0
 * none, 1 leaky ReLU (0.1).  out_f32: y is fp32 instead of bf16.  bias may
 * be NULL.  ws (device, ws_floats fp32 elements, may be NULL): workspace
 * for splitting the K sum of small layers (a grid of fewer than 512 blocks)
 * over more blocks; the partial sums are added in a fixed order, so results
 * do not depend on the split.  With ws NULL or smaller than
 * sscn_nn_conv_ws_floats reports, the layer runs unsplit (same values up
 * to fp32 rounding order). */
int sscn_nn_conv3x3(const void *x, int N, int H, int W, int Cin, const void *w, const float *bias, int Cout,
                    int act, int out_f32, void *y, int ldy, int yoff, float *ws, int64_t ws_floats, void *stream);

/* A convolution with bf16 outputs (as sscn_nn_conv3x3 with out_f32 = 0)
 * followed by the 2 x 2 average pooling of its outputs (as sscn_nn_pool2 of
 * y, ldy, yoff with C = Cout) into pool_y, N x H/2 x W/2 x Cout bf16: the
 * encoder's second convolution of a level and the pooling into the next
 * (Sec. 3, the network's contracting path).  H and W even.  Where the
 * halo-patch kernel runs with its staged 16-byte stores (sides multiples of
 * 8 x 16, ldy and yoff multiples of 8, y and pool_y 16-byte aligned, no K
 * split) the pooling is taken from the staged output tile in the same
 * kernel; otherwise the two operations run one after the other.  Both give
 * the same bits.  Returns -1 for bad arguments, like sscn_nn_conv3x3. */
int sscn_nn_conv3x3_pool(const void *x, int N, int H, int W, int Cin, const void *w, const float *bias, int Cout,
                         int act, void *y, int ldy, int yoff, void *pool_y, float *ws, int64_t ws_floats,
                         void *stream);

/* fp32 workspace elements a convolution of these sizes uses to split its K
 * sum (0: it is not split).  For the input gradient of a convolution with
 * Cin inputs and Cout outputs, ask for (Cin = Cout, Cout = Cin). */
int sscn_nn_conv_ws_floats(int N, int H, int W, int Cin, int Cout, int64_t *floats);

/* Input gradient of a convolution: dx = conv3x3(dy, w flipped and
 * transposed), bf16.  wt_scratch: 9*Cin*Cout bf16 elements.  ws, ws_floats:
 * as sscn_nn_conv3x3 (the convolution with Cout inputs and Cin outputs). */
int sscn_nn_conv3x3_dgrad(const void *dy, int N, int H, int W, int Cout, const void *w, int Cin,
                          void *wt_scratch, void *dx, int lddx, int dxoff, float *ws, int64_t ws_floats,
                          void *stream);

/* Size (floats) of the scratch sscn_nn_conv3x3_wgrad needs. */
int sscn_nn_wgrad_scratch(int N, int H, int W, int Cin, int Cout, int64_t *floats);

/* Weight gradient dw[co][tap][ci] = sum_p dy[p][co] x[p + tap][ci] (matrix
 * cores, split over pixel ranges and summed in fixed order) and bias
 * gradient db[co] = sum_p dy[p][co] (db may be NULL).  fp32 outputs. */
int sscn_nn_conv3x3_wgrad(const void *x, int N, int H, int W, int Cin, const void *dy, int Cout, float *dw,
                          float *db, float *scratch, int64_t scratch_floats, void *stream);

/* In place: dy *= (y > 0 ? 1 : 0.1), the leaky-ReLU gradient from the
 * layer's output y. */
int sscn_nn_act_bwd(void *dy, const void *y, int64_t n, void *stream);

/* 2x2 average pooling (H, W even; y is N x H/2 x W/2 x C) of channels
 * xoff .. xoff + C - 1 of x, whose pixels are ldx >= xoff + C channels apart
 * (x may be a channel slice of a wider tensor, such as the decoder's
 * concatenation buffer that the encoder's last convolution writes into),
 * and its gradient (dy is N x H/2 x W/2 x C, dx is N x H x W x C). */
int sscn_nn_pool2(const void *x, int ldx, int xoff, int N, int H, int W, int C, void *y, void *stream);
int sscn_nn_pool2_bwd(const void *dy, int N, int H, int W, int C, void *dx, void *stream);

/* Nearest 2x upsampling of x (N x H x W x C) into a channel slice of y
 * (N x 2H x 2W, ldy channels), and its gradient into dx (N x H x W x C). */
int sscn_nn_up2(const void *x, int N, int H, int W, int C, void *y, int ldy, int yoff, void *stream);
int sscn_nn_up2_bwd(const void *dy, int ldy, int yoff, int N, int H, int W, int C, void *dx, void *stream);

/* Copy (accumulate = 0) or add (accumulate = 1) a channel slice: dst slice
 * (ldd, doff) of P pixels x C channels from the src slice (lds, soff). */
int sscn_nn_chan_copy(const void *src, int lds, int soff, void *dst, int ldd, int doff, int P, int C,
                      int accumulate, void *stream);

/* Phase-aligned loss of B samples of S points against K candidate targets
 * each (the images of one converged state under the symmetries of the
 * rotating problem).  Prediction pred: fp32, ld channels, Re and Im in
 * channels 0 and 1; targets psi: fp32 [B][K][S] interleaved Re, Im.
 * stats[(b*K + k)*4 + 0..3] = Re<psi_bk,pred_b>, Im<psi_bk,pred_b>,
 * |pred_b|^2, |psi_bk|^2 (fp64, device).  The loss of (b, k) is
 * |pred|^2 + |psi|^2 - 2|<psi,pred>|, i.e. |pred - e^{i phi} psi|^2
 * minimised over the global phase phi; the loss of sample b is the least
 * over k.  If dpred is not NULL it receives the gradient of the batch-mean
 * loss (through the least candidate, the first on ties), bf16, ld channels
 * (channels beyond 1 zero). */
int sscn_nn_loss(const float *pred, int ld, const float *psi, int B, int K, int S, double *stats, void *dpred,
                 void *stream);

/* Solver state to training target and back.  psi_to_f32: out[2q + 0/1] =
 * scale * Re/Im psi[q] for S points of a complex128 (precision 0) or
 * complex64 (precision 1) interleaved device buffer.  f32_to_psi: psi[q] =
 * scale * (pred[q*ld], pred[q*ld + 1]), written in the given precision. */
int sscn_nn_psi_to_f32(const void *psi, int precision, int64_t S, float scale, float *out, void *stream);
int sscn_nn_f32_to_psi(const float *pred, int ld, int64_t S, double scale, void *psi, int precision, void *stream);

/* Squared 2-norm of n fp32 values a (device), summed in fp64 in a fixed
 * order (reproducible run to run).  work: device buffer of at least 257
 * doubles owned by the caller; on completion work[0] holds the sum and
 * work[1..256] are overwritten (partials).  Stream-ordered, no host sync. */
int sscn_nn_sumsq(const float *a, int64_t n, double *work, void *stream);

/* One Adam step (t >= 1) on fp32 master weights w with state m, v and
 * gradient g; if wbf16 is not NULL the updated weights are also written
 * there as bf16.  Global-norm clipping: if gsq is not NULL it points to the
 * squared norm of the whole gradient (device, e.g. work[0] of
 * sscn_nn_sumsq over every parameter's gradient) and g is scaled by
 * min(1, max_norm / sqrt(*gsq)) before the update; max_norm must then be
 * > 0.  gsq NULL: no clipping, max_norm ignored.  Returns -1 on bad
 * arguments. */
int sscn_nn_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr, float b1, float b2, float eps,
                 int t, const double *gsq, float max_norm, void *wbf16, void *stream);

/* b = bf16(a), round to nearest even. */
int sscn_nn_f32_to_bf16(const float *a, void *b, int64_t n, void *stream);

const char *sscn_nn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SSCN_NN_H */
