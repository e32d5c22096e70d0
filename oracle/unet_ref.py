"""Reference U-Net of the learned initial state (numpy, FP64 accumulation).

TEST INFRASTRUCTURE ONLY: plain numpy versions of every network operation
and of the whole forward/backward pass, used to check the GPU kernels and
their gradients.  Shares no code with the GPU library.

Tensors are NHWC.  With ``bf16=True`` every value the GPU stores in bf16 is
rounded to bf16 at the same point (activations after bias and activation,
pooled values, gradients after each kernel), while all sums are FP64, so the
GPU result differs only by its FP32 accumulation order; with ``bf16=False``
the pass is plain FP64 (used for the finite-difference pins).
"""
import numpy as np

LEAK = 0.1


def bf16(a):
    """Round to the nearest bf16 (ties to even) and return float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _r(a, on):
    return bf16(a) if on else np.asarray(a, dtype=np.float64)


def conv3x3(x, w, b=None, act=0):
    """y[n,i,j,o] = sum_{ky,kx,c} xpad[n,i+ky,j+kx,c] w[o,ky,kx,c] + b[o], then
    leaky ReLU if act."""
    N, H, W, C = x.shape
    xp = np.zeros((N, H + 2, W + 2, C))
    xp[:, 1:-1, 1:-1, :] = x
    y = np.zeros((N, H, W, w.shape[0]))
    for ky in range(3):
        for kx in range(3):
            y += np.einsum("nhwc,oc->nhwo", xp[:, ky:ky + H, kx:kx + W, :], w[:, ky, kx, :])
    if b is not None:
        y += b
    if act:
        y = np.where(y > 0, y, LEAK * y)
    return y


def conv3x3_dgrad(dy, w):
    """Gradient with respect to the convolution's input."""
    wt = np.transpose(w[:, ::-1, ::-1, :], (3, 1, 2, 0))  # [c][ky][kx][o], flipped
    return conv3x3(dy, wt)


def conv3x3_wgrad(x, dy):
    N, H, W, C = x.shape
    xp = np.zeros((N, H + 2, W + 2, C))
    xp[:, 1:-1, 1:-1, :] = x
    dw = np.zeros((dy.shape[3], 3, 3, C))
    for ky in range(3):
        for kx in range(3):
            dw[:, ky, kx, :] = np.einsum("nhwo,nhwc->oc", dy, xp[:, ky:ky + H, kx:kx + W, :])
    return dw, dy.sum(axis=(0, 1, 2))


def act_bwd(dy, y):
    return np.where(y > 0, dy, LEAK * dy)


def pool2(x):
    N, H, W, C = x.shape
    return 0.25 * x.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def pool2_bwd(dy):
    return 0.25 * np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2)


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_bwd(dy):
    N, H, W, C = dy.shape
    return dy.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def _cands(psi):
    """Targets as (B, K, H, W, 2): a single target per sample is K = 1."""
    return psi[:, None] if psi.ndim == 4 else psi


def loss_stats(pred, psi):
    """Per sample b and candidate k: Re<psi_bk,pred_b>, Im<psi_bk,pred_b>,
    |pred_b|^2, |psi_bk|^2 (pred (B, H, W, 2), psi (B, [K,] H, W, 2) real and
    imaginary pairs).  Shape (B, K, 4)."""
    psi = _cands(psi)
    pr, pi = pred[:, None, ..., 0], pred[:, None, ..., 1]
    tr, ti = psi[..., 0], psi[..., 1]
    ax = (2, 3)
    pp = np.broadcast_to((pr * pr + pi * pi).sum(ax), tr.shape[:2])
    return np.stack([(tr * pr + ti * pi).sum(ax), (tr * pi - ti * pr).sum(ax),
                     pp, (tr * tr + ti * ti).sum(ax)], axis=2)


def loss_value(pred, psi):
    """min over candidates k and global phases phi of |pred - e^{i phi} psi_k|^2."""
    s = loss_stats(pred, psi)
    return (s[..., 2] + s[..., 3] - 2.0 * np.hypot(s[..., 0], s[..., 1])).min(axis=1)


def loss_grad(pred, psi):
    """Gradient of the batch-mean loss with respect to pred (through the
    nearest candidate, the first on ties)."""
    psi = _cands(psi)
    s = loss_stats(pred, psi)
    lk = s[..., 2] + s[..., 3] - 2.0 * np.hypot(s[..., 0], s[..., 1])
    kb = np.argmin(lk, axis=1)
    B = pred.shape[0]
    g = np.zeros_like(pred)
    for b in range(B):
        sr, si = s[b, kb[b], 0], s[b, kb[b], 1]
        mag = np.hypot(sr, si)
        cr, ci = (sr / mag, si / mag) if mag > 0 else (1.0, 0.0)
        tr, ti = psi[b, kb[b], ..., 0], psi[b, kb[b], ..., 1]
        g[b, ..., 0] = 2.0 * (pred[b, ..., 0] - (cr * tr - ci * ti)) / B
        g[b, ..., 1] = 2.0 * (pred[b, ..., 1] - (cr * ti + ci * tr)) / B
    return g


def layer_specs(chans, bott, in_ch=16, out_ch=16):
    """(name, Cin, Cout, act) of every convolution of the U-Net, in order."""
    specs, cin = [], in_ch
    for lv, c in enumerate(chans):
        specs += [(f"enc{lv}a", cin, c, 1), (f"enc{lv}b", c, c, 1)]
        cin = c
    specs += [("bota", cin, bott, 1), ("botb", bott, bott, 1)]
    cup = bott
    for lv in range(len(chans) - 1, -1, -1):
        cout = chans[lv - 1] if lv > 0 else chans[0]
        specs += [(f"dec{lv}a", cup + chans[lv], cout, 1), (f"dec{lv}b", cout, cout, 1)]
        cup = cout
    specs += [("out", cup, out_ch, 0)]
    return specs


def unet_forward(x, params, chans, bott, bf16_on=True):
    """Returns (output (N,H,W,16) float64, cache of activations)."""
    A = {}
    rb = bf16_on
    Wt = {k: (_r(v[0], rb), np.asarray(v[1], np.float64)) for k, v in params.items()}
    cur = _r(x, rb)
    A["x"] = cur
    for lv, c in enumerate(chans):
        A[f"enc{lv}a"] = _r(conv3x3(cur, *Wt[f"enc{lv}a"], act=1), rb)
        A[f"enc{lv}b"] = _r(conv3x3(A[f"enc{lv}a"], *Wt[f"enc{lv}b"], act=1), rb)
        A[f"pool{lv}"] = _r(pool2(A[f"enc{lv}b"]), rb)
        cur = A[f"pool{lv}"]
    A["bota"] = _r(conv3x3(cur, *Wt["bota"], act=1), rb)
    A["botb"] = _r(conv3x3(A["bota"], *Wt["botb"], act=1), rb)
    cur = A["botb"]
    for lv in range(len(chans) - 1, -1, -1):
        A[f"cat{lv}"] = np.concatenate([up2(cur), A[f"enc{lv}b"]], axis=3)
        A[f"dec{lv}a"] = _r(conv3x3(A[f"cat{lv}"], *Wt[f"dec{lv}a"], act=1), rb)
        A[f"dec{lv}b"] = _r(conv3x3(A[f"dec{lv}a"], *Wt[f"dec{lv}b"], act=1), rb)
        cur = A[f"dec{lv}b"]
    out = conv3x3(cur, *Wt["out"], act=0)
    if rb:
        out = np.asarray(out, np.float32).astype(np.float64)
    A["out"] = out
    A["_W"] = Wt
    return out, A


def unet_backward(dout, A, chans, bott, bf16_on=True):
    """Gradients {name: (dw, db)} of every convolution for output gradient
    dout, following the GPU's order and rounding points."""
    rb = bf16_on
    Wt = A["_W"]
    G = {}
    d = _r(dout, rb)
    G["out"] = conv3x3_wgrad(A["dec0b"], d)
    g = _r(conv3x3_dgrad(d, Wt["out"][0]), rb)
    L = len(chans)
    cups = {}
    cup = bott
    for lv in range(L - 1, -1, -1):
        cups[lv] = cup
        cup = chans[lv - 1] if lv > 0 else chans[0]
    gskip = {}
    for lv in range(0, L):
        g = _r(act_bwd(g, A[f"dec{lv}b"]), rb)
        G[f"dec{lv}b"] = conv3x3_wgrad(A[f"dec{lv}a"], g)
        g = _r(conv3x3_dgrad(g, Wt[f"dec{lv}b"][0]), rb)
        g = _r(act_bwd(g, A[f"dec{lv}a"]), rb)
        G[f"dec{lv}a"] = conv3x3_wgrad(A[f"cat{lv}"], g)
        gcat = _r(conv3x3_dgrad(g, Wt[f"dec{lv}a"][0]), rb)
        gskip[lv] = gcat[..., cups[lv]:]
        g = _r(up2_bwd(gcat[..., :cups[lv]]), rb)
    g = _r(act_bwd(g, A["botb"]), rb)
    G["botb"] = conv3x3_wgrad(A["bota"], g)
    g = _r(conv3x3_dgrad(g, Wt["botb"][0]), rb)
    g = _r(act_bwd(g, A["bota"]), rb)
    G["bota"] = conv3x3_wgrad(A[f"pool{L - 1}"], g)
    g = _r(conv3x3_dgrad(g, Wt["bota"][0]), rb)
    for lv in range(L - 1, -1, -1):
        g = _r(pool2_bwd(g), rb)
        g = _r(g + gskip[lv], rb)
        g = _r(act_bwd(g, A[f"enc{lv}b"]), rb)
        G[f"enc{lv}b"] = conv3x3_wgrad(A[f"enc{lv}a"], g)
        g = _r(conv3x3_dgrad(g, Wt[f"enc{lv}b"][0]), rb)
        g = _r(act_bwd(g, A[f"enc{lv}a"]), rb)
        inp = A[f"pool{lv - 1}"] if lv > 0 else A["x"]
        G[f"enc{lv}a"] = conv3x3_wgrad(inp, g)
        g = _r(conv3x3_dgrad(g, Wt[f"enc{lv}a"][0]), rb)
    G["_dx"] = g
    return G


def clip_scale(grads, max_norm):
    """Global-norm clipping factor: min(1, max_norm / ||g||) with ||g|| the
    2-norm of every gradient array in `grads` taken together."""
    norm = np.sqrt(sum(float(np.sum(np.asarray(g, dtype=np.float64) ** 2)) for g in grads))
    return 1.0 if norm <= max_norm else max_norm / norm


def adam(w, m, v, g, lr, b1, b2, eps, t, gscale=1.0):
    """One Adam step (bias-corrected moments) on the gradient gscale * g."""
    g = gscale * np.asarray(g, dtype=np.float64)
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    w = w - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return w, m, v
