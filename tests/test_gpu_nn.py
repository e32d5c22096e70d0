"""GPU tests of the learned-initial-state network kernels against the numpy
reference oracle/unet_ref.py, called through the C ABI of include/sscn_nn.h.

The convolution tests also check the matrix-core operand and result layout
the kernels assume: any transposition or lane mix-up changes the result far
beyond the tolerances.  Tolerances: products of bf16 operands are exact in
fp32, so an fp32 output differs from the FP64 sum only by fp32 accumulation
(bounded by 1e-5 times the sum of absolute terms for these depths); a bf16
output can additionally sit one bf16 step (2^-7 relative) away where the
two sums straddle a rounding boundary.
"""
import numpy as np
import pytest

from oracle import unet_ref as U

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def nn():
    _need_gpu()
    from paper_1906_06327_amd import nn as N
    return N


def to_bf(a):
    """numpy -> device bf16 bit patterns (int16) and the float64 values."""
    t = torch.tensor(np.asarray(a, np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).cuda(), t.float().numpy().astype(np.float64)


def from_bf(t):
    return t.cpu().view(torch.bfloat16).float().numpy().astype(np.float64)


def f32(a):
    return torch.tensor(np.asarray(a, np.float32)).cuda()


def close_bf(gpu, ref, absum, name):
    bad = np.abs(gpu - ref) > 2.0 ** -7 * np.abs(ref) + 2e-5 * absum + 1e-30
    assert not bad.any(), f"{name}: {bad.sum()} of {bad.size} outside tolerance"


@pytest.mark.parametrize("N,H,W,Cin,Cout,act", [(3, 13, 11, 48, 32, 1), (1, 8, 8, 16, 16, 0),
                                                 (2, 24, 20, 160, 64, 1),
                                                 # every block shape and K stage of the matrix-core
                                                 # kernel, with pixel counts that leave a ragged
                                                 # last block: BN 128 / 64 / 32 / 16, stages of 64,
                                                 # 32 and 16 channels
                                                 (2, 9, 13, 64, 128, 1), (1, 10, 10, 128, 256, 0),
                                                 (2, 7, 9, 96, 64, 1), (1, 16, 16, 16, 32, 1),
                                                 (1, 5, 6, 32, 48, 0), (1, 12, 12, 512, 256, 1),
                                                 # the halo-patch kernel (sides multiples of 8 x 16,
                                                 # >= 256 patch blocks): BN 32 with 16- and 32-channel
                                                 # chunks, 64, 128 (two column blocks) and 16
                                                 (8, 64, 64, 16, 32, 1), (8, 64, 64, 96, 32, 1),
                                                 (8, 64, 64, 64, 64, 0), (4, 64, 64, 64, 256, 1),
                                                 (8, 64, 64, 32, 16, 0)])
def test_conv3x3(nn, N, H, W, Cin, Cout, act):
    rng = np.random.default_rng(N * 1000 + Cin)
    xd, x = to_bf(rng.standard_normal((N, H, W, Cin)))
    wd, w = to_bf(rng.standard_normal((Cout, 3, 3, Cin)) / np.sqrt(9 * Cin))
    b = rng.standard_normal(Cout).astype(np.float32)
    ref = U.conv3x3(x, w, b.astype(np.float64), act=act)
    absum = U.conv3x3(np.abs(x), np.abs(w), np.abs(b).astype(np.float64))
    y32 = torch.zeros((N, H, W, Cout), dtype=torch.float32, device="cuda")
    nn.conv3x3(xd, N, H, W, Cin, wd, f32(b), Cout, act, y32, out_f32=True)
    g = y32.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(g - ref) <= 1e-5 * absum + 1e-30)
    # with a workspace, small grids split their K sum over more blocks
    nws = nn.conv_ws_floats(N, H, W, Cin, Cout)
    if nws > 0:
        ws = torch.full((nws,), float("nan"), dtype=torch.float32, device="cuda")
        y32.zero_()
        nn.conv3x3(xd, N, H, W, Cin, wd, f32(b), Cout, act, y32, out_f32=True, ws=ws)
        gs = y32.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(gs - ref) <= 1e-5 * absum + 1e-30)
    # bf16 output into a channel slice of a wider tensor
    ld, off = Cout + 32, 16
    ybf = torch.full((N, H, W, ld), 7, dtype=torch.int16, device="cuda")
    nn.conv3x3(xd, N, H, W, Cin, wd, f32(b), Cout, act, ybf, ldy=ld, yoff=off)
    gb = from_bf(ybf)
    close_bf(gb[..., off:off + Cout], ref, absum, "conv bf16")
    untouched = ybf.cpu().numpy()
    assert np.all(untouched[..., :off] == 7) and np.all(untouched[..., off + Cout:] == 7)
    # the same values where the rows are not 16-byte aligned (per-value
    # stores instead of the staged 16-byte runs)
    ld2, off2 = Cout + 6, 2
    yb2 = torch.full((N, H, W, ld2), 7, dtype=torch.int16, device="cuda")
    nn.conv3x3(xd, N, H, W, Cin, wd, f32(b), Cout, act, yb2, ldy=ld2, yoff=off2)
    g2 = yb2.cpu().numpy()
    assert np.array_equal(g2[..., off2:off2 + Cout], untouched[..., off:off + Cout])
    assert np.all(g2[..., :off2] == 7) and np.all(g2[..., off2 + Cout:] == 7)
    # split K sums into both slices: four channels per thread where 4-value
    # runs are 8-byte aligned, one where not, with the same bits
    if nws > 0:
        got = []
        for l, o in ((ld, off), (ld2, off2)):
            ys = torch.full((N, H, W, l), 7, dtype=torch.int16, device="cuda")
            nn.conv3x3(xd, N, H, W, Cin, wd, f32(b), Cout, act, ys, ldy=l, yoff=o, ws=ws)
            gs = ys.cpu().numpy()
            close_bf(from_bf(ys)[..., o:o + Cout], ref, absum, "conv bf16 split")
            assert np.all(gs[..., :o] == 7) and np.all(gs[..., o + Cout:] == 7)
            got.append(gs[..., o:o + Cout])
        assert np.array_equal(got[0], got[1])


@pytest.mark.parametrize("N,H,W,Cin,Cout,ld,off,split", [
    # halo-patch shapes with aligned channel slices: pooling fused
    # (>= 256 patch blocks; BN 32, 64 with two input chunks, 128)
    (8, 64, 64, 16, 32, 64, 32, False), (8, 64, 64, 64, 64, 64, 0, False), (8, 64, 64, 32, 128, 192, 64, False),
    # the same where the rows are not 16-byte aligned, a small image (no
    # halo kernel) and a split K sum: convolution, then the pooling kernel
    (8, 64, 64, 16, 32, 38, 2, False), (2, 12, 10, 32, 48, 48, 0, False), (1, 16, 16, 128, 256, 512, 256, True)])
def test_conv_pool_fused(nn, N, H, W, Cin, Cout, ld, off, split):
    """sscn_nn_conv3x3_pool gives the bits of sscn_nn_conv3x3 followed by
    sscn_nn_pool2, fused or not."""
    rng = np.random.default_rng(H * W + Cin)
    xd, _ = to_bf(rng.standard_normal((N, H, W, Cin)))
    wd, _ = to_bf(rng.standard_normal((Cout, 3, 3, Cin)) / np.sqrt(9 * Cin))
    b = f32(rng.standard_normal(Cout))
    ws = None
    if split:
        nws = nn.conv_ws_floats(N, H, W, Cin, Cout)
        assert nws > 0
        ws = torch.empty(nws, dtype=torch.float32, device="cuda")
    y1 = torch.full((N, H, W, ld), 7, dtype=torch.int16, device="cuda")
    p1 = torch.full((N, H // 2, W // 2, Cout), 7, dtype=torch.int16, device="cuda")
    nn.conv3x3(xd, N, H, W, Cin, wd, b, Cout, 1, y1, ldy=ld, yoff=off, ws=ws)
    nn.pool2(y1, N, H, W, Cout, p1, ldx=ld, xoff=off)
    y2 = torch.full((N, H, W, ld), 7, dtype=torch.int16, device="cuda")
    p2 = torch.full((N, H // 2, W // 2, Cout), 9, dtype=torch.int16, device="cuda")
    nn.conv3x3_pool(xd, N, H, W, Cin, wd, b, Cout, 1, y2, p2, ldy=ld, yoff=off, ws=ws)
    assert torch.equal(y1, y2)
    assert torch.equal(p1, p2)


def test_conv3x3_dgrad_and_wgrad(nn):
    rng = np.random.default_rng(7)
    N, H, W, Cin, Cout = 2, 12, 10, 32, 48
    xd, x = to_bf(rng.standard_normal((N, H, W, Cin)))
    wd, w = to_bf(rng.standard_normal((Cout, 3, 3, Cin)) / np.sqrt(9 * Cin))
    dyd, dy = to_bf(rng.standard_normal((N, H, W, Cout)))
    wt = torch.empty(9 * Cin * Cout, dtype=torch.int16, device="cuda")
    ld, off = Cin + 16, 16
    dx = torch.zeros((N, H, W, ld), dtype=torch.int16, device="cuda")
    nn.conv3x3_dgrad(dyd, N, H, W, Cout, wd, Cin, wt, dx, lddx=ld, dxoff=off)
    ref = U.conv3x3_dgrad(dy, w)
    absum = U.conv3x3_dgrad(np.abs(dy), np.abs(w))
    close_bf(from_bf(dx)[..., off:], ref, absum, "dgrad")
    assert np.all(dx.cpu().numpy()[..., :off] == 0)
    # the same with the K sum split over blocks (a workspace)
    nws = nn.conv_ws_floats(N, H, W, Cout, Cin)
    assert nws > 0
    dx2 = torch.zeros((N, H, W, ld), dtype=torch.int16, device="cuda")
    nn.conv3x3_dgrad(dyd, N, H, W, Cout, wd, Cin, wt, dx2, lddx=ld, dxoff=off,
                     ws=torch.empty(nws, dtype=torch.float32, device="cuda"))
    close_bf(from_bf(dx2)[..., off:], ref, absum, "dgrad split")
    assert np.all(dx2.cpu().numpy()[..., :off] == 0)

    scr = torch.empty(nn.wgrad_scratch(N, H, W, Cin, Cout), dtype=torch.float32, device="cuda")
    dw = torch.zeros((Cout, 3, 3, Cin), dtype=torch.float32, device="cuda")
    db = torch.zeros(Cout, dtype=torch.float32, device="cuda")
    nn.conv3x3_wgrad(xd, N, H, W, Cin, dyd, Cout, dw, db, scr)
    rdw, rdb = U.conv3x3_wgrad(x, dy)
    adw, _ = U.conv3x3_wgrad(np.abs(x), np.abs(dy))
    assert np.all(np.abs(dw.cpu().numpy() - rdw) <= 1e-5 * adw + 1e-30)
    assert np.allclose(db.cpu().numpy(), rdb, rtol=1e-5, atol=1e-4)


def test_wgrad_many_splits_and_ragged_tail(nn):
    # P = 2 * 45 * 37 = 3330 pixels: several pixel splits, last one partial
    rng = np.random.default_rng(8)
    N, H, W, Cin, Cout = 2, 45, 37, 16, 16
    xd, x = to_bf(rng.standard_normal((N, H, W, Cin)))
    dyd, dy = to_bf(rng.standard_normal((N, H, W, Cout)))
    scr = torch.empty(nn.wgrad_scratch(N, H, W, Cin, Cout), dtype=torch.float32, device="cuda")
    dw = torch.zeros((Cout, 3, 3, Cin), dtype=torch.float32, device="cuda")
    db = torch.zeros(Cout, dtype=torch.float32, device="cuda")
    nn.conv3x3_wgrad(xd, N, H, W, Cin, dyd, Cout, dw, db, scr)
    rdw, rdb = U.conv3x3_wgrad(x, dy)
    adw, _ = U.conv3x3_wgrad(np.abs(x), np.abs(dy))
    assert np.all(np.abs(dw.cpu().numpy() - rdw) <= 1e-5 * adw + 1e-30)
    assert np.allclose(db.cpu().numpy(), rdb, rtol=1e-5, atol=1e-3)
    # deterministic: a second call gives the same bits
    dw2 = torch.zeros_like(dw)
    nn.conv3x3_wgrad(xd, N, H, W, Cin, dyd, Cout, dw2, None, scr)
    assert torch.equal(dw, dw2)


@pytest.mark.parametrize("Cin,Cout", [(32, 32), (16, 32), (64, 32), (32, 16), (48, 16)])
def test_wgrad_narrow_outputs(nn, Cin, Cout):
    """32 and 16 output channels take the weight-gradient kernel whose
    blocks apply one staged dy tile to 2 or 4 taps (the ninth tap alone in
    the last group), with 32- and 16-channel input slices, over several
    pixel ranges with a partial last one; against the reference, and two
    calls give the same bits."""
    rng = np.random.default_rng(13)
    N, H, W = 2, 29, 41
    xd, x = to_bf(rng.standard_normal((N, H, W, Cin)))
    dyd, dy = to_bf(rng.standard_normal((N, H, W, Cout)))
    scr = torch.empty(nn.wgrad_scratch(N, H, W, Cin, Cout), dtype=torch.float32, device="cuda")
    dw = torch.zeros((Cout, 3, 3, Cin), dtype=torch.float32, device="cuda")
    db = torch.zeros(Cout, dtype=torch.float32, device="cuda")
    nn.conv3x3_wgrad(xd, N, H, W, Cin, dyd, Cout, dw, db, scr)
    rdw, rdb = U.conv3x3_wgrad(x, dy)
    adw, _ = U.conv3x3_wgrad(np.abs(x), np.abs(dy))
    assert np.all(np.abs(dw.cpu().numpy() - rdw) <= 1e-5 * adw + 1e-30)
    assert np.allclose(db.cpu().numpy(), rdb, rtol=1e-5, atol=1e-3)
    dw2 = torch.zeros_like(dw)
    nn.conv3x3_wgrad(xd, N, H, W, Cin, dyd, Cout, dw2, None, scr)
    assert torch.equal(dw, dw2)


def test_wgrad_wave_summed_ranges(nn):
    """An image large enough for more than 64 pixel ranges (2 x 192 x 192 =
    73 728 pixels: 72 ranges), whose partial weight gradients are summed one
    wave per weight, against the reference; two calls give the same bits."""
    rng = np.random.default_rng(12)
    N, H, W, Cin, Cout = 2, 192, 192, 16, 16
    xd, x = to_bf(rng.standard_normal((N, H, W, Cin)))
    dyd, dy = to_bf(rng.standard_normal((N, H, W, Cout)))
    scr = torch.empty(nn.wgrad_scratch(N, H, W, Cin, Cout), dtype=torch.float32, device="cuda")
    dw = torch.zeros((Cout, 3, 3, Cin), dtype=torch.float32, device="cuda")
    nn.conv3x3_wgrad(xd, N, H, W, Cin, dyd, Cout, dw, None, scr)
    rdw, _ = U.conv3x3_wgrad(x, dy)
    adw, _ = U.conv3x3_wgrad(np.abs(x), np.abs(dy))
    assert np.all(np.abs(dw.cpu().numpy() - rdw) <= 1e-5 * adw + 1e-30)
    dw2 = torch.zeros_like(dw)
    nn.conv3x3_wgrad(xd, N, H, W, Cin, dyd, Cout, dw2, None, scr)
    assert torch.equal(dw, dw2)


@pytest.mark.parametrize("Cout", [48, 512])
def test_bias_gradient_channel_groups(nn, Cout):
    """The bias gradient's 16-byte kernel with channel groups that do not
    divide the 256 threads (48: 6 groups, 42 pixel rows) and with 64 groups
    (512), over several pixel splits with a partial last one, against the
    plain sum; two calls give the same bits."""
    rng = np.random.default_rng(11)
    N, H, W, Cin = 1, 40, 52, 16
    xd, x = to_bf(rng.standard_normal((N, H, W, Cin)))
    dyd, dy = to_bf(rng.standard_normal((N, H, W, Cout)))
    scr = torch.empty(nn.wgrad_scratch(N, H, W, Cin, Cout), dtype=torch.float32, device="cuda")
    dw = torch.zeros((Cout, 3, 3, Cin), dtype=torch.float32, device="cuda")
    db = torch.zeros(Cout, dtype=torch.float32, device="cuda")
    nn.conv3x3_wgrad(xd, N, H, W, Cin, dyd, Cout, dw, db, scr)
    ref = dy.reshape(-1, Cout).astype(np.float64).sum(axis=0)
    asum = np.abs(dy).reshape(-1, Cout).astype(np.float64).sum(axis=0)
    assert np.all(np.abs(db.cpu().numpy() - ref) <= 1e-5 * asum + 1e-6)
    db2 = torch.zeros_like(db)
    nn.conv3x3_wgrad(xd, N, H, W, Cin, dyd, Cout, dw, db2, scr)
    assert torch.equal(db, db2)


# C = 32 with channel offsets that are multiples of 8 takes the 16-byte
# kernels, C = 20 with odd offsets the element-wise ones
@pytest.mark.parametrize("C,uoff,soff,doff,cc", [(32, 16, 8, 8, 24), (20, 4, 3, 5, 12)])
def test_elementwise_and_resampling(nn, C, uoff, soff, doff, cc):
    rng = np.random.default_rng(9)
    N, H, W = 2, 8, 6
    xd, x = to_bf(rng.standard_normal((N, H, W, C)))
    # pooling and its gradient
    y = torch.zeros((N, H // 2, W // 2, C), dtype=torch.int16, device="cuda")
    nn.pool2(xd, N, H, W, C, y)
    assert np.array_equal(from_bf(y), U.bf16(U.pool2(x)))
    # the same channels read as a slice of a wider tensor (offset uoff, pixel
    # stride C + uoff + 8), e.g. the skip half of a concatenation buffer
    ldw = C + uoff + 8
    wide = torch.zeros((N, H, W, ldw), dtype=torch.int16, device="cuda")
    wide[..., uoff:uoff + C] = xd
    ys = torch.zeros_like(y)
    nn.pool2(wide, N, H, W, C, ys, ldx=ldw, xoff=uoff)
    assert torch.equal(ys, y)
    dx = torch.zeros_like(xd)
    nn.pool2_bwd(y, N, H, W, C, dx)
    assert np.array_equal(from_bf(dx), U.bf16(U.pool2_bwd(from_bf(y))))
    # upsampling into a channel slice and its gradient
    ld = C + uoff
    up = torch.zeros((N, 2 * H, 2 * W, ld), dtype=torch.int16, device="cuda")
    nn.up2(xd, N, H, W, C, up, ld, uoff)
    assert np.array_equal(from_bf(up)[..., uoff:], U.up2(x))
    g = torch.zeros_like(xd)
    nn.up2_bwd(up, ld, uoff, N, H, W, C, g)
    assert np.array_equal(from_bf(g), U.bf16(U.up2_bwd(U.up2(x))))
    # channel copy and accumulate
    dst = torch.zeros((N, H, W, 48), dtype=torch.int16, device="cuda")
    nn.chan_copy(xd, C, 0, dst, 48, doff, N * H * W, cc)
    nn.chan_copy(xd, C, soff, dst, 48, doff, N * H * W, cc, accumulate=True)
    got = from_bf(dst)
    assert np.array_equal(got[..., doff:doff + cc], U.bf16(x[..., 0:cc] + x[..., soff:soff + cc]))
    assert np.all(got[..., :doff] == 0) and np.all(got[..., doff + cc:] == 0)
    # leaky-ReLU gradient
    dyd, dy = to_bf(rng.standard_normal((N, H, W, C)))
    nn.act_bwd(dyd, xd)
    # the kernel scales by the fp32 value of 0.1 in fp32 arithmetic
    scaled = (np.float32(U.LEAK) * dy.astype(np.float32)).astype(np.float64)
    assert np.array_equal(from_bf(dyd), U.bf16(np.where(x > 0, dy, scaled)))


@pytest.mark.parametrize("K", [1, 3])
def test_loss_and_adam(nn, K):
    rng = np.random.default_rng(10 + K)
    B, H, W, ld = 3, 9, 7, 16
    pred = rng.standard_normal((B, H, W, ld)).astype(np.float32)
    psi = rng.standard_normal((B, K, H, W, 2)).astype(np.float32)
    if K > 1:
        psi[1, 2] = 0.8 * pred[1, ..., :2]  # sample 1's nearest image is its last candidate
    stats = torch.zeros(4 * B * K, dtype=torch.float64, device="cuda")
    dpred = torch.full((B, H, W, ld), 5, dtype=torch.int16, device="cuda")
    nn.loss(f32(pred), ld, f32(psi), B, K, H * W, stats, dpred)
    rs = U.loss_stats(pred[..., :2].astype(np.float64), psi.astype(np.float64))
    assert np.allclose(stats.cpu().numpy().reshape(B, K, 4), rs, rtol=1e-13, atol=1e-12)
    rg = U.loss_grad(pred[..., :2].astype(np.float64), psi.astype(np.float64))
    got = from_bf(dpred)
    scale = 2.0 * (np.abs(pred[..., :2]) + np.abs(psi).sum(-1).max(1)[..., None]) / B
    close_bf(got[..., :2], rg, scale, "loss grad")
    assert np.all(got[..., 2:] == 0)

    n = 1000
    w = rng.standard_normal(n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    wd, md, vd = f32(w), f32(m), f32(v)
    wbf = torch.zeros(n, dtype=torch.int16, device="cuda")
    rw, rm, rv = w.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for t in range(1, 4):
        gr = rng.standard_normal(n).astype(np.float32)
        nn.adam(wd, md, vd, f32(gr), 1e-2, 0.9, 0.999, 1e-8, t, wbf)
        rw, rm, rv = U.adam(rw, rm, rv, gr.astype(np.float64), 1e-2, 0.9, 0.999, 1e-8, t)
    assert np.allclose(wd.cpu().numpy(), rw, rtol=1e-5, atol=1e-6)
    assert np.array_equal(from_bf(wbf), U.bf16(wd.cpu().numpy()))


@pytest.mark.parametrize("n", [1, 255, 4097, 3 * 4096 * 256 + 17])
def test_sumsq(nn, n):
    """Fixed-order fp64 sum of squares: one block, a ragged tail, and more
    elements than 256 blocks of 4096 (every block strides)."""
    a = np.random.default_rng(n).standard_normal(n).astype(np.float32)
    work = torch.full((257,), 7.0, dtype=torch.float64, device="cuda")
    nn.sumsq(f32(a), work)
    ref = float(np.sum(a.astype(np.float64) ** 2))
    got = float(work[0])
    assert abs(got - ref) <= 1e-13 * ref, (got, ref)
    nn.sumsq(f32(a), work)
    assert float(work[0]) == got  # reproducible bit for bit


def test_adam_global_norm_clipping(nn):
    """Two gradient arrays clipped together: the device scale read from the
    sumsq result matches the oracle's clip_scale; a bound above the norm
    leaves the step unclipped."""
    rng = np.random.default_rng(21)
    sizes = (600, 37)
    ws = [rng.standard_normal(k).astype(np.float32) for k in sizes]
    dev = [[f32(w), f32(np.zeros_like(w)), f32(np.zeros_like(w))] for w in ws]
    ref = [[w.astype(np.float64), np.zeros(len(w)), np.zeros(len(w))] for w in ws]
    flat = torch.zeros(sum(sizes), dtype=torch.float32, device="cuda")
    work = torch.zeros(257, dtype=torch.float64, device="cuda")
    for t, max_norm in ((1, 3.0), (2, 3.0), (3, 1e6)):
        gs = [(rng.standard_normal(k) * 2.0).astype(np.float32) for k in sizes]
        flat.copy_(torch.tensor(np.concatenate(gs)))
        nn.sumsq(flat, work)
        sc = U.clip_scale([g.astype(np.float64) for g in gs], max_norm)
        assert (sc < 1.0) == (max_norm < 10.0)
        off = 0
        for k, (d, r, g) in enumerate(zip(dev, ref, gs)):
            nn.adam(d[0], d[1], d[2], flat[off:off + sizes[k]], 1e-2, 0.9, 0.999, 1e-8, t,
                    gsq=work[:1], max_norm=max_norm)
            r[0], r[1], r[2] = U.adam(r[0], r[1], r[2], g.astype(np.float64), 1e-2, 0.9, 0.999, 1e-8, t,
                                      gscale=sc)
            off += sizes[k]
    for d, r in zip(dev, ref):
        assert np.allclose(d[0].cpu().numpy(), r[0], rtol=1e-5, atol=1e-6)
        assert np.allclose(d[1].cpu().numpy(), r[1], rtol=1e-5, atol=1e-7)
        assert np.allclose(d[2].cpu().numpy(), r[2], rtol=1e-4, atol=1e-9)


def test_state_conversions(nn):
    rng = np.random.default_rng(12)
    S = 1000
    for dt in (torch.complex128, torch.complex64):
        z = (rng.standard_normal(S) + 1j * rng.standard_normal(S))
        zt = torch.tensor(z).to(dt).cuda()
        out = torch.zeros(2 * S, dtype=torch.float32, device="cuda")
        nn.psi_to_f32(zt, S, 0.5, out)
        zz = zt.cpu().numpy().astype(np.complex128) * 0.5
        ref = np.stack([zz.real, zz.imag], axis=1).reshape(-1)
        assert np.array_equal(out.cpu().numpy(), ref.astype(np.float32))
        pred = torch.tensor(rng.standard_normal((S, 16)).astype(np.float32)).cuda()
        back = torch.zeros(S, dtype=dt, device="cuda")
        nn.f32_to_psi(pred, 16, S, 2.0, back)
        pn = pred.cpu().numpy().astype(np.float64)
        want = (2.0 * pn[:, 0] + 2.0j * pn[:, 1]).astype(np.complex128 if dt == torch.complex128 else np.complex64)
        assert np.array_equal(back.cpu().numpy(), want)


@pytest.mark.parametrize("chans,bott,N,H", [((16, 32), 32, 2, 16), ((16, 32, 64, 64), 128, 2, 32),
                                            # the learned start's network at full size: 6 levels,
                                            # 32-64-128-256-256 and a 256-channel bottleneck, 256 x 256
                                            ((32, 64, 128, 256, 256), 256, 1, 256)])
def test_unet_forward_backward(nn, chans, bott, N, H):
    """Whole network on the GPU against the reference with the same bf16
    rounding points.  The two differ only where fp32 and FP64 accumulation
    tip a bf16 rounding the other way, and such flips propagate, so the
    comparison is in relative L2 norm: 2e-2 for the output; for a weight
    gradient, 5e-2 or the whole effect of bf16 rounding on that gradient
    (the bf16 reference against the FP64 reference), whichever is larger:
    the GPU gradient must be as close to the bf16 reference as bf16
    arithmetic itself is to exact arithmetic.  A wrong index or operand
    layout gives errors of order one."""
    print(f"[gpu-nn] whole network chans={chans} bott={bott} N={N} H={H}", flush=True)
    rng = np.random.default_rng(11)
    net = nn.UNet(N, H, H, chans=chans, bott=bott, seed=3)
    # non-zero biases so the bias path is exercised
    for name in net.b:
        net.b[name].copy_(torch.tensor(0.05 * rng.standard_normal(net.b[name].numel()), dtype=torch.float32))
    params = {k: (v[0].astype(np.float64), v[1].astype(np.float64)) for k, v in net.params_numpy().items()}
    xin = np.zeros((N, H, H, 16))
    xin[..., :5] = rng.standard_normal((N, H, H, 5))
    xd, _ = to_bf(xin)
    out = net.forward(xd).cpu().numpy().astype(np.float64)
    ref, A = U.unet_forward(xin, params, chans, bott, bf16_on=True)
    rel = np.linalg.norm(out - ref) / np.linalg.norm(ref)
    assert rel < 2e-2, rel
    psi = rng.standard_normal((N, H, H, 2)).astype(np.float32)
    lossv = net.loss_and_grad(f32(psi))
    rloss = U.loss_value(out[..., :2], psi.astype(np.float64))
    assert np.allclose(lossv, rloss, rtol=1e-9)
    dout = np.zeros((N, H, H, 16))
    dout[..., :2] = U.loss_grad(out[..., :2], psi.astype(np.float64))
    net.backward(net.gacts["out"])
    G = U.unet_backward(dout, A, chans, bott, bf16_on=True)
    out64, A64 = U.unet_forward(U.bf16(xin), params, chans, bott, bf16_on=False)
    dout64 = np.zeros_like(dout)
    dout64[..., :2] = U.loss_grad(out64[..., :2], psi.astype(np.float64))
    G64 = U.unet_backward(dout64, A64, chans, bott, bf16_on=False)

    def rel(a, b):
        return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)

    for name, _, _, _ in net.specs:
        for k, got in enumerate((net.gw[name].cpu().numpy(), net.gb[name].cpu().numpy())):
            err, floor = rel(got, G[name][k]), rel(G64[name][k], G[name][k])
            assert err < max(5e-2, floor), (name, k, err, floor)


def test_unet_training_reduces_loss(nn):
    """Adam on a fixed batch of smooth targets: the loss must fall well
    below its initial value."""
    N, H = 4, 32
    net = nn.UNet(N, H, H, chans=(16, 32), bott=32, seed=5)
    ax = np.linspace(-1, 1, H)
    X, Y = np.meshgrid(ax, ax)
    xin = np.zeros((N, H, H, 16))
    psi = np.zeros((N, H, H, 2))
    for k in range(N):
        xin[k, ..., 0], xin[k, ..., 1], xin[k, ..., 2] = X, Y, 0.25 * k
        amp = np.exp(-(X ** 2 + Y ** 2) / (0.2 + 0.1 * k))
        psi[k, ..., 0] = amp * np.cos(2 * X)
        psi[k, ..., 1] = amp * np.sin(2 * Y)
    xd, _ = to_bf(xin)
    pd = f32(psi)
    first = None
    for it in range(300):
        net.forward(xd)
        lv = net.loss_and_grad(pd).mean()
        first = lv if first is None else first
        net.backward(net.gacts["out"])
        net.adam_step(lr=2e-3)
    assert np.isfinite(lv) and lv < 0.2 * first, (first, lv)
