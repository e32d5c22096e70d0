"""Pins of the reference U-Net (oracle/unet_ref.py): every backward formula
against central finite differences of the FP64 forward pass, the loss
against a brute-force minimisation over the global phase, and bf16 rounding
against its definition, Adam and global-norm clipping against closed forms."""
import numpy as np
import pytest

from oracle import unet_ref as U


def fd(f, x, idx, eps=1e-6):
    xp = x.copy()
    xm = x.copy()
    xp[idx] += eps
    xm[idx] -= eps
    return (f(xp) - f(xm)) / (2 * eps)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5e-3, 3.0e38, 0.0])
    r = U.bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0  # tie to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert r[2] == 1.0 + 2 ** -7
    # every result has at most 8 significant bits
    m, _ = np.frexp(r[np.isfinite(r) & (r != 0)])
    assert np.all(m * 2 ** 8 == np.round(m * 2 ** 8))


def test_conv_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 5, 6, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    dy = rng.standard_normal((2, 5, 6, 4))

    def L_of_x(xx):
        return float((U.conv3x3(xx, w, b) * dy).sum())

    def L_of_w(ww):
        return float((U.conv3x3(x, ww, b) * dy).sum())

    dx = U.conv3x3_dgrad(dy, w)
    dw, db = U.conv3x3_wgrad(x, dy)
    for idx in [(0, 0, 0, 0), (1, 4, 5, 2), (0, 2, 3, 1)]:
        assert abs(dx[idx] - fd(L_of_x, x, idx)) < 1e-6
    for idx in [(0, 0, 0, 0), (3, 2, 1, 2), (1, 1, 1, 1)]:
        assert abs(dw[idx] - fd(L_of_w, w, idx)) < 1e-6
    assert np.allclose(db, dy.sum(axis=(0, 1, 2)))


def test_resampling_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 8, 6, 3))
    y = rng.standard_normal((2, 4, 3, 3))
    # <pool(x), y> = <x, pool_bwd(y)> and <up(y), x> = <y, up_bwd(x)>
    assert np.isclose((U.pool2(x) * y).sum(), (x * U.pool2_bwd(y)).sum())
    assert np.isclose((U.up2(y) * x).sum(), (y * U.up2_bwd(x)).sum())


def test_loss_is_minimum_over_global_phase():
    rng = np.random.default_rng(3)
    pred = rng.standard_normal((3, 4, 5, 2))
    psi = rng.standard_normal((3, 4, 5, 2))
    val = U.loss_value(pred, psi)
    p = pred[..., 0] + 1j * pred[..., 1]
    t = psi[..., 0] + 1j * psi[..., 1]
    phis = np.linspace(0, 2 * np.pi, 20001)
    for b in range(3):
        brute = min(np.sum(np.abs(p[b] - np.exp(1j * f) * t[b]) ** 2) for f in phis[::50])
        fine = np.array([np.sum(np.abs(p[b] - np.exp(1j * f) * t[b]) ** 2) for f in phis])
        assert val[b] <= brute + 1e-12
        assert abs(val[b] - fine.min()) < 1e-6
    g = U.loss_grad(pred, psi)
    f = lambda pp: float(U.loss_value(pp, psi).mean())
    for idx in [(0, 1, 2, 0), (2, 3, 4, 1), (1, 0, 0, 1)]:
        assert abs(g[idx] - fd(f, pred, idx)) < 1e-6


@pytest.mark.parametrize("chans,bott", [((16, 16), 16), ((16, 32), 32)])
def test_unet_backprop_matches_finite_differences(chans, bott):
    rng = np.random.default_rng(4)
    specs = U.layer_specs(chans, bott)
    params = {n: (rng.standard_normal((co, 3, 3, ci)) * np.sqrt(2 / (9 * ci)),
                  0.1 * rng.standard_normal(co)) for n, ci, co, _ in specs}
    x = rng.standard_normal((2, 8, 8, 16))
    psi = rng.standard_normal((2, 8, 8, 2))

    def total(pp):
        out, _ = U.unet_forward(x, pp, chans, bott, bf16_on=False)
        return float(U.loss_value(out[..., :2], psi).mean())

    out, A = U.unet_forward(x, params, chans, bott, bf16_on=False)
    dout = np.zeros_like(out)
    dout[..., :2] = U.loss_grad(out[..., :2], psi)
    G = U.unet_backward(dout, A, chans, bott, bf16_on=False)
    for name in ("enc0a", "dec0a", "bota", "out", f"dec{len(chans) - 1}b"):
        w, b = params[name]
        for idx in [(0, 0, 0, 0), (w.shape[0] - 1, 2, 1, w.shape[3] - 1)]:
            def f_w(ww, name=name):
                pp = dict(params)
                pp[name] = (ww, params[name][1])
                return total(pp)
            num = fd(f_w, w, idx, eps=1e-5)
            assert abs(G[name][0][idx] - num) <= 1e-6 + 1e-5 * abs(num), (name, idx)
        def f_b(bb, name=name):
            pp = dict(params)
            pp[name] = (params[name][0], bb)
            return total(pp)
        num = fd(f_b, b, (0,), eps=1e-5)
        assert abs(G[name][1][0] - num) <= 1e-6 + 1e-5 * abs(num), name


def test_loss_over_candidates_is_least_candidate():
    rng = np.random.default_rng(5)
    pred = rng.standard_normal((2, 4, 5, 2))
    cands = rng.standard_normal((2, 3, 4, 5, 2))
    cands[1, 2] = pred[1] * 0.9  # sample 1 has a near candidate
    each = np.stack([U.loss_value(pred, cands[:, k]) for k in range(3)], axis=1)
    assert np.allclose(U.loss_value(pred, cands), each.min(axis=1))
    assert np.argmin(each[1]) == 2
    g = U.loss_grad(pred, cands)
    f = lambda pp: float(U.loss_value(pp, cands).mean())
    for idx in [(0, 1, 2, 0), (1, 3, 4, 1)]:
        assert abs(g[idx] - fd(f, pred, idx)) < 1e-6


def test_adam_closed_forms():
    """Adam with zero initial moments: the first step moves every weight by
    lr g / (|g| + eps) (the bias corrections turn the moments back into g
    and g^2), and a constant gradient keeps moving it by the same amount at
    every later step; with eps = 0 the step does not depend on the
    gradient's scale, so a clipping factor changes nothing once the
    moments are built from clipped gradients alone."""
    rng = np.random.default_rng(5)
    w0 = rng.standard_normal(50)
    g = rng.standard_normal(50) * 10.0 ** rng.uniform(-3, 3, 50)
    lr, eps = 1e-2, 1e-8
    m = v = np.zeros(50)
    w = w0
    for t in range(1, 6):
        w, m, v = U.adam(w, m, v, g, lr, 0.9, 0.999, eps, t)
        assert np.allclose(w, w0 - t * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-12)
    wa, _, _ = U.adam(w0, np.zeros(50), np.zeros(50), g, lr, 0.9, 0.999, 0.0, 1)
    wb, _, _ = U.adam(w0, np.zeros(50), np.zeros(50), g, lr, 0.9, 0.999, 0.0, 1, gscale=1e-3)
    assert np.allclose(wa, wb, rtol=0, atol=1e-14)
    assert np.allclose(wa, w0 - lr * np.sign(g), rtol=0, atol=1e-14)


def test_clip_scale_is_global_norm():
    a, b = np.array([3.0]), np.array([[0.0, 4.0]])
    assert U.clip_scale([a, b], 1.0) == pytest.approx(0.2, rel=1e-15)
    assert U.clip_scale([a, b], 5.0) == 1.0
    assert U.clip_scale([a, b], 10.0) == 1.0
    rng = np.random.default_rng(6)
    gs = [rng.standard_normal(s) for s in ((7, 3), (11,), (2, 2, 5))]
    c = U.clip_scale(gs, 0.5)
    assert np.sqrt(sum(np.sum((c * x) ** 2) for x in gs)) == pytest.approx(0.5, rel=1e-14)
