"""U-Net of the learned initial state, on the kernels of include/sscn_nn.h.

The network maps, on a fixed 2D grid, the coordinates and the problem
parameters (Omega, g, nu) to a complex wave function that seeds an
imaginary-time run in place of the one-vortex random-phase state of
Eq. (fun).  Every arithmetic step runs in libsscn.so's kernels (matrix-core
bf16 3x3 convolutions with fp32 accumulation, pooling, upsampling, the
phase-aligned loss, Adam); this module only sequences the layers and owns
the buffers (torch tensors used as device memory).

Architecture (input 16 channels, H = W divisible by 16): encoder levels of
channels `chans` with two leaky-ReLU 3x3 convolutions each, 2x2 average
pooling between levels, a bottleneck of `bott` channels, and a decoder that
upsamples (nearest 2x), concatenates the encoder output of the same level
and applies two convolutions; a final 3x3 convolution writes 16 fp32
channels of which 0 and 1 are Re and Im of psi.
"""
import ctypes

import numpy as np

from . import lib as _sscn_lib

IN_CH = 16
OUT_CH = 16


def _nn():
    L = _sscn_lib()
    if not getattr(L, "_nn_ready", False):
        vp, ci, i64, cf = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_float
        L.sscn_nn_conv3x3.argtypes = [vp, ci, ci, ci, ci, vp, vp, ci, ci, ci, vp, ci, ci, vp, i64, vp]
        L.sscn_nn_conv3x3_pool.argtypes = [vp, ci, ci, ci, ci, vp, vp, ci, ci, vp, ci, ci, vp, vp, i64, vp]
        L.sscn_nn_conv_ws_floats.argtypes = [ci, ci, ci, ci, ci, ctypes.POINTER(i64)]
        L.sscn_nn_conv3x3_dgrad.argtypes = [vp, ci, ci, ci, ci, vp, ci, vp, vp, ci, ci, vp, i64, vp]
        L.sscn_nn_wgrad_scratch.argtypes = [ci, ci, ci, ci, ci, ctypes.POINTER(i64)]
        L.sscn_nn_conv3x3_wgrad.argtypes = [vp, ci, ci, ci, ci, vp, ci, vp, vp, vp, i64, vp]
        L.sscn_nn_act_bwd.argtypes = [vp, vp, i64, vp]
        L.sscn_nn_pool2.argtypes = [vp, ci, ci, ci, ci, ci, ci, vp, vp]
        L.sscn_nn_pool2_bwd.argtypes = [vp, ci, ci, ci, ci, vp, vp]
        L.sscn_nn_up2.argtypes = [vp, ci, ci, ci, ci, vp, ci, ci, vp]
        L.sscn_nn_up2_bwd.argtypes = [vp, ci, ci, ci, ci, ci, ci, vp, vp]
        L.sscn_nn_chan_copy.argtypes = [vp, ci, ci, vp, ci, ci, ci, ci, ci, vp]
        L.sscn_nn_loss.argtypes = [vp, ci, vp, ci, ci, ci, vp, vp, vp]
        L.sscn_nn_psi_to_f32.argtypes = [vp, ci, i64, cf, vp, vp]
        L.sscn_nn_f32_to_psi.argtypes = [vp, ci, i64, ctypes.c_double, vp, ci, vp]
        L.sscn_nn_sumsq.argtypes = [vp, i64, vp, vp]
        L.sscn_nn_adam.argtypes = [vp, vp, vp, vp, i64, cf, cf, cf, cf, ci, vp, cf, vp, vp]
        L.sscn_nn_f32_to_bf16.argtypes = [vp, vp, i64, vp]
        L.sscn_nn_last_error.restype = ctypes.c_char_p
        L._nn_ready = True
    return L


def _ck(code):
    if code != 0:
        raise RuntimeError("sscn_nn: " + _nn().sscn_nn_last_error().decode())


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


# ---------------------------------------------------------------------------
# thin wrappers (argument marshalling only)

def conv_ws_floats(N, H, W, Cin, Cout):
    n = ctypes.c_int64()
    _ck(_nn().sscn_nn_conv_ws_floats(N, H, W, Cin, Cout, ctypes.byref(n)))
    return n.value


def conv3x3(x, N, H, W, Cin, w, b, Cout, act, y, ldy=None, yoff=0, out_f32=False, ws=None, stream=None):
    _ck(_nn().sscn_nn_conv3x3(_p(x), N, H, W, Cin, _p(w), _p(b), Cout, int(act), int(out_f32), _p(y),
                              ldy or Cout, yoff, _p(ws), ws.numel() if ws is not None else 0, stream))


def conv3x3_pool(x, N, H, W, Cin, w, b, Cout, act, y, pool, ldy=None, yoff=0, ws=None, stream=None):
    _ck(_nn().sscn_nn_conv3x3_pool(_p(x), N, H, W, Cin, _p(w), _p(b), Cout, int(act), _p(y), ldy or Cout, yoff,
                                   _p(pool), _p(ws), ws.numel() if ws is not None else 0, stream))


def conv3x3_dgrad(dy, N, H, W, Cout, w, Cin, wt, dx, lddx=None, dxoff=0, ws=None, stream=None):
    _ck(_nn().sscn_nn_conv3x3_dgrad(_p(dy), N, H, W, Cout, _p(w), Cin, _p(wt), _p(dx), lddx or Cin,
                                    dxoff, _p(ws), ws.numel() if ws is not None else 0, stream))


def wgrad_scratch(N, H, W, Cin, Cout):
    n = ctypes.c_int64()
    _ck(_nn().sscn_nn_wgrad_scratch(N, H, W, Cin, Cout, ctypes.byref(n)))
    return n.value


def conv3x3_wgrad(x, N, H, W, Cin, dy, Cout, dw, db, scratch, stream=None):
    _ck(_nn().sscn_nn_conv3x3_wgrad(_p(x), N, H, W, Cin, _p(dy), Cout, _p(dw), _p(db), _p(scratch),
                                    scratch.numel(), stream))


def act_bwd(dy, y, stream=None):
    _ck(_nn().sscn_nn_act_bwd(_p(dy), _p(y), dy.numel(), stream))


def pool2(x, N, H, W, C, y, ldx=None, xoff=0, stream=None):
    _ck(_nn().sscn_nn_pool2(_p(x), ldx or C, xoff, N, H, W, C, _p(y), stream))


def pool2_bwd(dy, N, H, W, C, dx, stream=None):
    _ck(_nn().sscn_nn_pool2_bwd(_p(dy), N, H, W, C, _p(dx), stream))


def up2(x, N, H, W, C, y, ldy, yoff, stream=None):
    _ck(_nn().sscn_nn_up2(_p(x), N, H, W, C, _p(y), ldy, yoff, stream))


def up2_bwd(dy, ldy, yoff, N, H, W, C, dx, stream=None):
    _ck(_nn().sscn_nn_up2_bwd(_p(dy), ldy, yoff, N, H, W, C, _p(dx), stream))


def chan_copy(src, lds, soff, dst, ldd, doff, P, C, accumulate=False, stream=None):
    _ck(_nn().sscn_nn_chan_copy(_p(src), lds, soff, _p(dst), ldd, doff, P, C, int(accumulate), stream))


def loss(pred, ld, psi, B, K, S, stats, dpred=None, stream=None):
    _ck(_nn().sscn_nn_loss(_p(pred), ld, _p(psi), B, K, S, _p(stats), _p(dpred), stream))


def psi_to_f32(psi, S, scale, out, stream=None):
    prec = 0 if psi.dtype == _complex128() else 1
    _ck(_nn().sscn_nn_psi_to_f32(_p(psi), prec, int(S), float(scale), _p(out), stream))


def f32_to_psi(pred, ld, S, scale, psi, stream=None):
    prec = 0 if psi.dtype == _complex128() else 1
    _ck(_nn().sscn_nn_f32_to_psi(_p(pred), ld, int(S), float(scale), _p(psi), prec, stream))


def _complex128():
    import torch
    return torch.complex128


def sumsq(a, work, stream=None):
    """work[0] = sum of a**2 (fp64, fixed order); work: >= 257 float64 on the device."""
    if work.numel() < 257:
        raise ValueError("sumsq needs a work buffer of at least 257 doubles")
    _ck(_nn().sscn_nn_sumsq(_p(a), a.numel(), _p(work), stream))


def adam(w, m, v, g, lr, b1, b2, eps, t, wbf=None, gsq=None, max_norm=0.0, stream=None):
    """One Adam step; gsq (a one-element float64 device tensor holding the
    squared global gradient norm) turns on clipping to max_norm."""
    _ck(_nn().sscn_nn_adam(_p(w), _p(m), _p(v), _p(g), w.numel(), float(lr), float(b1), float(b2),
                           float(eps), int(t), _p(gsq), float(max_norm), _p(wbf), stream))


def f32_to_bf16(a, b, stream=None):
    _ck(_nn().sscn_nn_f32_to_bf16(_p(a), _p(b), a.numel(), stream))


# ---------------------------------------------------------------------------

def layer_specs(chans=(16, 32, 64, 64), bott=128):
    """(name, Cin, Cout, act) of every convolution, in forward order."""
    specs = []
    cin = IN_CH
    for lv, c in enumerate(chans):
        specs += [(f"enc{lv}a", cin, c, 1), (f"enc{lv}b", c, c, 1)]
        cin = c
    specs += [("bota", cin, bott, 1), ("botb", bott, bott, 1)]
    cup = bott
    for lv in range(len(chans) - 1, -1, -1):
        cout = chans[lv - 1] if lv > 0 else chans[0]
        specs += [(f"dec{lv}a", cup + chans[lv], cout, 1), (f"dec{lv}b", cout, cout, 1)]
        cup = cout
    specs += [("out", cup, OUT_CH, 0)]
    return specs


def init_params(specs, seed=0):
    """He-normal weights (fp32, [Cout][3][3][Cin]) and zero biases."""
    rng = np.random.default_rng(seed)
    out = {}
    for name, cin, cout, act in specs:
        std = np.sqrt(2.0 / (9 * cin)) * (1.0 if act else 0.1)
        out[name] = (rng.standard_normal((cout, 3, 3, cin)).astype(np.float32) * std,
                     np.zeros(cout, np.float32))
    return out


class UNet:
    """Forward, backward and Adam of the U-Net for batches of N samples of
    H x W points (H, W divisible by 2^len(chans))."""

    def __init__(self, N, H, W, chans=(16, 32, 64, 64), bott=128, seed=0, params=None):
        import torch
        self.torch = torch
        self.N, self.H, self.W = N, H, W
        self.chans, self.bott = tuple(chans), bott
        self.specs = layer_specs(self.chans, bott)
        self.dev = torch.device("cuda")
        p0 = params if params is not None else init_params(self.specs, seed)
        f32, bf = torch.float32, torch.int16
        self.w32, self.wbf, self.b, self.gw, self.gb, self.m, self.v = {}, {}, {}, {}, {}, {}, {}
        # every parameter gradient is a view into one flat buffer, so that
        # the global gradient norm is one reduction
        ngrad = sum(int(np.prod(p0[n][0].shape)) + p0[n][1].size for n, _, _, _ in self.specs)
        self.gflat = torch.zeros(ngrad, dtype=f32, device=self.dev)
        self.gwork = torch.zeros(257, dtype=torch.float64, device=self.dev)
        off = 0
        for name, cin, cout, act in self.specs:
            w, b = p0[name]
            self.w32[name] = torch.tensor(w, dtype=f32, device=self.dev)
            self.b[name] = torch.tensor(b, dtype=f32, device=self.dev)
            self.wbf[name] = torch.empty(w.shape, dtype=bf, device=self.dev)
            f32_to_bf16(self.w32[name], self.wbf[name])
            self.gw[name] = self.gflat[off:off + w.size].view(w.shape)
            off += w.size
            self.gb[name] = self.gflat[off:off + b.size]
            off += b.size
            for d in (self.m, self.v):
                d[name] = (torch.zeros_like(self.w32[name]), torch.zeros_like(self.b[name]))
        self.t = 0
        self._alloc()

    def _act(self, H, W, C):
        return self.torch.zeros((self.N, H, W, C), dtype=self.torch.int16, device=self.dev)

    def _alloc(self):
        N, H, W = self.N, self.H, self.W
        self.acts = {}   # forward outputs of every layer (bf16)
        self.shapes = {}  # name -> (H, W, Cin, Cout) of each convolution
        self.pools = []
        self.cats = []
        h, w = H, W
        for lv, c in enumerate(self.chans):
            self.shapes[f"enc{lv}a"] = (h, w)
            self.shapes[f"enc{lv}b"] = (h, w)
            h, w = h // 2, w // 2
        self.shapes["bota"] = self.shapes["botb"] = (h, w)
        for lv in range(len(self.chans) - 1, -1, -1):
            h, w = h * 2, w * 2
            self.shapes[f"dec{lv}a"] = self.shapes[f"dec{lv}b"] = (h, w)
        self.shapes["out"] = (H, W)
        for name, cin, cout, act in self.specs:
            hh, ww = self.shapes[name]
            if name == "out":
                self.acts[name] = self.torch.zeros((N, hh, ww, cout), dtype=self.torch.float32,
                                                   device=self.dev)
            else:
                self.acts[name] = self._act(hh, ww, cout)
        h, w = H, W
        self.pool = {}
        for lv, c in enumerate(self.chans):
            self.pool[lv] = self._act(h // 2, w // 2, c)
            h, w = h // 2, w // 2
        self.cat = {}
        cup = self.bott
        for lv in range(len(self.chans) - 1, -1, -1):
            hh, ww = self.shapes[f"dec{lv}a"]
            self.cat[lv] = self._act(hh, ww, cup + self.chans[lv])
            cup = self.chans[lv - 1] if lv > 0 else self.chans[0]
        # gradient buffers, one per activation, and scratch
        self.gacts = {k: self._act(*v.shape[1:]) for k, v in self.acts.items()}
        self.gpool = {k: self._act(*v.shape[1:]) for k, v in self.pool.items()}
        self.gcat = {k: self._act(*v.shape[1:]) for k, v in self.cat.items()}
        self.gin = self._act(H, W, IN_CH)
        maxw = max(cin * cout * 9 for _, cin, cout, _ in self.specs)
        self.wt = self.torch.empty(maxw, dtype=self.torch.int16, device=self.dev)
        # one fp32 scratch for the weight gradients and for the split-K
        # partial sums of the small layers (used one call at a time)
        need = max(max(wgrad_scratch(N, *self.shapes[n], cin, cout), conv_ws_floats(N, *self.shapes[n], cin, cout),
                       conv_ws_floats(N, *self.shapes[n], cout, cin)) for n, cin, cout, _ in self.specs)
        self.scratch = self.torch.empty(need, dtype=self.torch.float32, device=self.dev)
        self.stats = self.torch.zeros(4 * N, dtype=self.torch.float64, device=self.dev)

    # -- forward ----------------------------------------------------------
    def _cup_of(self):
        """Channels of the upsampled half of each level's concatenation
        buffer (the output channels of the level below)."""
        spec = {s[0]: s for s in self.specs}
        out, cup = {}, self.bott
        for lv in range(len(self.chans) - 1, -1, -1):
            out[lv] = cup
            cup = spec[f"dec{lv}b"][2]
        return out

    def forward(self, x):
        """x: (N, H, W, 16) bf16 tensor.  Returns the fp32 (N, H, W, 16)
        output; channels 0, 1 are Re, Im of psi."""
        N = self.N
        self.x = x
        spec = {s[0]: s for s in self.specs}

        def conv(name, inp, out=None, ldy=None, yoff=0):
            _, cin, cout, act = spec[name]
            h, w = self.shapes[name]
            conv3x3(inp, N, h, w, cin, self.wbf[name], self.b[name], cout, act,
                    out if out is not None else self.acts[name], ldy=ldy, yoff=yoff,
                    out_f32=(name == "out"), ws=self.scratch)

        # the encoder's second convolution of each level writes straight into
        # the skip half of that level's concatenation buffer (channels cup ..
        # cup + c - 1 of ld) and pools its outputs into the next level's
        # input; the decoder fills the other half by upsampling
        cup_of = self._cup_of()
        cur = x
        for lv, c in enumerate(self.chans):
            ld = cup_of[lv] + c
            conv(f"enc{lv}a", cur)
            _, cin, _, act = spec[f"enc{lv}b"]
            h, w = self.shapes[f"enc{lv}b"]
            conv3x3_pool(self.acts[f"enc{lv}a"], N, h, w, cin, self.wbf[f"enc{lv}b"], self.b[f"enc{lv}b"], c, act,
                         self.cat[lv], self.pool[lv], ldy=ld, yoff=cup_of[lv], ws=self.scratch)
            cur = self.pool[lv]
        conv("bota", cur)
        conv("botb", self.acts["bota"])
        cur, cup = self.acts["botb"], self.bott
        for lv in range(len(self.chans) - 1, -1, -1):
            h, w = self.shapes[f"dec{lv}a"]
            ld = cup + self.chans[lv]
            up2(cur, N, h // 2, w // 2, cup, self.cat[lv], ld, 0)
            conv(f"dec{lv}a", self.cat[lv])
            conv(f"dec{lv}b", self.acts[f"dec{lv}a"])
            cur = self.acts[f"dec{lv}b"]
            cup = spec[f"dec{lv}b"][2]
        conv("out", cur)
        return self.acts["out"]

    # -- backward ---------------------------------------------------------
    def backward(self, dout):
        """dout: (N, H, W, 16) bf16 gradient of the output.  Fills
        self.gw / self.gb (fp32) and self.gin (input gradient)."""
        N = self.N
        spec = {s[0]: s for s in self.specs}

        def conv_bwd(name, inp, dy, dinp, lddx=None, dxoff=0):
            _, cin, cout, act = spec[name]
            h, w = self.shapes[name]
            conv3x3_wgrad(inp, N, h, w, cin, dy, cout, self.gw[name], self.gb[name], self.scratch)
            if dinp is not None:
                conv3x3_dgrad(dy, N, h, w, cout, self.wbf[name], cin, self.wt, dinp, lddx=lddx,
                              dxoff=dxoff, ws=self.scratch)

        lv0 = len(self.chans) - 1
        top = self.acts["dec0b"]
        conv_bwd("out", top, dout, self.gacts["dec0b"])
        cup_of = self._cup_of()
        for lv in range(0, lv0 + 1):
            h, w = self.shapes[f"dec{lv}a"]
            act_bwd(self.gacts[f"dec{lv}b"], self.acts[f"dec{lv}b"])
            conv_bwd(f"dec{lv}b", self.acts[f"dec{lv}a"], self.gacts[f"dec{lv}b"], self.gacts[f"dec{lv}a"])
            act_bwd(self.gacts[f"dec{lv}a"], self.acts[f"dec{lv}a"])
            conv_bwd(f"dec{lv}a", self.cat[lv], self.gacts[f"dec{lv}a"], self.gcat[lv])
            ld = cup_of[lv] + self.chans[lv]
            below = self.gacts[f"dec{lv + 1}b"] if lv < lv0 else self.gacts["botb"]
            up2_bwd(self.gcat[lv], ld, 0, N, h // 2, w // 2, cup_of[lv], below)
        act_bwd(self.gacts["botb"], self.acts["botb"])
        conv_bwd("botb", self.acts["bota"], self.gacts["botb"], self.gacts["bota"])
        act_bwd(self.gacts["bota"], self.acts["bota"])
        conv_bwd("bota", self.pool[lv0], self.gacts["bota"], self.gpool[lv0])
        for lv in range(lv0, -1, -1):
            c = self.chans[lv]
            h, w = self.shapes[f"enc{lv}b"]
            pool2_bwd(self.gpool[lv], N, h, w, c, self.gacts[f"enc{lv}b"])
            ld = cup_of[lv] + c
            chan_copy(self.gcat[lv], ld, cup_of[lv], self.gacts[f"enc{lv}b"], c, 0, N * h * w, c,
                      accumulate=True)
            # the layer's output lives in the concatenation buffer (forward)
            chan_copy(self.cat[lv], ld, cup_of[lv], self.acts[f"enc{lv}b"], c, 0, N * h * w, c)
            act_bwd(self.gacts[f"enc{lv}b"], self.acts[f"enc{lv}b"])
            conv_bwd(f"enc{lv}b", self.acts[f"enc{lv}a"], self.gacts[f"enc{lv}b"], self.gacts[f"enc{lv}a"])
            act_bwd(self.gacts[f"enc{lv}a"], self.acts[f"enc{lv}a"])
            inp = self.pool[lv - 1] if lv > 0 else self.x
            dinp = self.gpool[lv - 1] if lv > 0 else self.gin
            conv_bwd(f"enc{lv}a", inp, self.gacts[f"enc{lv}a"], dinp)

    def loss_and_grad(self, psi_target, grad=True):
        """Phase-aligned loss against fp32 targets of shape (N, H, W, 2) or
        (N, K, H, W, 2) (K candidate images per sample, the nearest counts);
        writes the output gradient into gacts['out'] if grad and returns the
        per-sample loss (host numpy, synchronises)."""
        S = self.H * self.W
        K = 1 if psi_target.dim() == 4 else int(psi_target.shape[1])
        if self.stats.numel() < 4 * self.N * K:
            self.stats = self.torch.zeros(4 * self.N * K, dtype=self.torch.float64, device=self.dev)
        loss(self.acts["out"], OUT_CH, psi_target, self.N, K, S, self.stats,
             self.gacts["out"] if grad else None)
        st = self.stats[:4 * self.N * K].view(self.N, K, 4).cpu().numpy()
        return (st[..., 2] + st[..., 3] - 2.0 * np.hypot(st[..., 0], st[..., 1])).min(axis=1)

    def grad_sqnorm(self):
        """Enqueue the squared global norm of the parameter gradients into
        gwork[0] (device); returns that one-element view."""
        sumsq(self.gflat, self.gwork)
        return self.gwork[:1]

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, max_norm=None, gsq=None):
        """One Adam step on every parameter; with max_norm the gradients are
        first scaled so that their global norm is at most max_norm (gsq: the
        grad_sqnorm() of this step if already enqueued)."""
        self.t += 1
        if max_norm is None:
            gsq = None
        elif gsq is None:
            gsq = self.grad_sqnorm()
        mn = float(max_norm) if max_norm is not None else 0.0
        for name, _, _, _ in self.specs:
            m, v = self.m[name], self.v[name]
            adam(self.w32[name], m[0], v[0], self.gw[name], lr, b1, b2, eps, self.t, self.wbf[name], gsq, mn)
            adam(self.b[name], m[1], v[1], self.gb[name], lr, b1, b2, eps, self.t, None, gsq, mn)

    def params_numpy(self):
        return {n: (self.w32[n].cpu().numpy(), self.b[n].cpu().numpy()) for n, _, _, _ in self.specs}
