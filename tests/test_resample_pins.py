"""Pins of the oracle's grid-to-grid interpolation and angular moments (the
learned initial state's resampling), against what the mathematics fixes:
the reproduction properties of Keys' kernel, a brute-force double sum over
every source sample, exact grid permutations, the convergence order, and
the orientation of a pattern of known angle."""
import math

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def grid(n, h):
    return -0.5 * n * h + h * np.arange(n)


def test_keys_kernel_values_and_reproduction():
    # W(0) = 1, W(+-1) = W(+-2) = 0 (interpolating), support (-2, 2)
    assert O.keys_cubic(0.0) == 1.0
    for s in (1.0, -1.0, 2.0, -2.0, 2.5, -3.0):
        assert O.keys_cubic(s) == 0.0
    # W(1/2) = 9/16, W(3/2) = -1/16 (Keys' kernel at a = -1/2)
    assert abs(O.keys_cubic(0.5) - 9 / 16) < 1e-15
    assert abs(O.keys_cubic(1.5) + 1 / 16) < 1e-15
    # sums over the four samples reproduce 1, t and t^2 (third-order kernel)
    t = np.linspace(0.0, 0.999, 23)
    for m in range(3):
        rep = sum(O.keys_cubic(t - d) * float(d) ** m for d in (-1, 0, 1, 2))
        assert np.max(np.abs(rep - t ** m)) < 1e-13, m
    # ... but not t^3 (the kernel is not of fourth order)
    rep3 = sum(O.keys_cubic(t - d) * float(d) ** 3 for d in (-1, 0, 1, 2))
    assert np.max(np.abs(rep3 - t ** 3)) > 1e-3


def test_resample_identity_and_walls():
    rng = np.random.default_rng(1)
    f = rng.standard_normal((30, 41)) + 1j * rng.standard_normal((30, 41))
    f[0, :] = 0
    f[:, 0] = 0
    g = O.resample(f, (0.13, 0.17), (30, 41), (0.13, 0.17))
    # the source index of each point is recomputed from its coordinate, so
    # the copy holds to rounding
    assert np.max(np.abs(g - f)) < 1e-14 * np.max(np.abs(f))


def test_resample_equals_brute_force_double_sum():
    """The 4 x 4 stencil equals the sum over every source sample of
    W((X - X_i)/hx) W((Y - Y_j)/hy) f_ij (written out independently)."""
    rng = np.random.default_rng(2)
    nys, nxs, hxs, hys = 11, 13, 0.3, 0.25
    f = rng.standard_normal((nys, nxs)) + 1j * rng.standard_normal((nys, nxs))
    ny, nx, hx, hy, ang = 9, 10, 0.37, 0.29, 0.41
    g = O.resample(f, (hxs, hys), (ny, nx), (hx, hy), ang)
    xs, ys = grid(nxs, hxs), grid(nys, hys)
    for j in range(1, ny):
        for i in range(1, nx):
            x, y = grid(nx, hx)[i], grid(ny, hy)[j]
            X = math.cos(ang) * x - math.sin(ang) * y
            Y = math.sin(ang) * x + math.cos(ang) * y
            acc = 0j
            for jj in range(nys):
                for ii in range(nxs):
                    acc += O.keys_cubic((X - xs[ii]) / hxs) * O.keys_cubic((Y - ys[jj]) / hys) * f[jj, ii]
            assert abs(g[j, i] - acc) < 1e-13 * max(1.0, abs(acc)), (j, i)
    assert np.all(g[0, :] == 0) and np.all(g[:, 0] == 0)


def test_resample_reproduces_quadratics():
    """A quadratic polynomial sampled on the source grid is interpolated
    exactly wherever the stencil stays inside the grid."""
    nys, nxs, hs = 40, 44, 0.2
    xs, ys = grid(nxs, hs), grid(nys, hs)
    XS, YS = np.meshgrid(xs, ys)
    poly = lambda X, Y: 0.3 + 1.1 * X - 0.7 * Y + 0.25 * X * X - 0.4 * X * Y + 0.15 * Y * Y  # noqa: E731
    f = poly(XS, YS) * (1 + 0.5j)
    ny, nx, h, ang = 25, 25, 0.23, 0.3
    g = O.resample(f, (hs, hs), (ny, nx), (h, h), ang)
    x = grid(nx, h)
    X, Y = np.meshgrid(x, x)
    XR, YR = math.cos(ang) * X - math.sin(ang) * Y, math.sin(ang) * X + math.cos(ang) * Y
    exact = poly(XR, YR) * (1 + 0.5j)
    inside = (np.abs(XR) < xs[-3]) & (np.abs(YR) < ys[-3]) & (XR > xs[2]) & (YR > ys[2])
    inside[0, :] = inside[:, 0] = False
    assert inside.sum() > 300
    assert np.max(np.abs(g - exact)[inside]) < 1e-12


def test_resample_quarter_turn_is_a_permutation():
    """On a square grid, x_i -> -x_i maps interior index i to n - i, so a
    rotation by pi/2 permutes interior points: out[j][i] = f[i][n - j]."""
    n, h = 20, 0.15
    rng = np.random.default_rng(3)
    f = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    f[0, :] = 0
    f[:, 0] = 0
    g = O.resample(f, (h, h), (n, n), (h, h), math.pi / 2)
    ref = np.zeros_like(f)
    for j in range(1, n):
        for i in range(1, n):
            ref[j, i] = f[i, n - j]  # source point (-y_j, x_i)
    assert np.max(np.abs(g - ref)) < 1e-12


def test_resample_third_order_convergence():
    """A smooth field resampled onto a fixed grid from sources of spacing h
    and h/2: the error falls by about 2^3."""
    def field(X, Y):
        return np.exp(-(X * X + 0.7 * Y * Y) / 2) * np.exp(1j * (0.8 * X - 0.3 * Y))
    nx, h = 37, 0.21
    x = grid(nx, h)
    X, Y = np.meshgrid(x, x)
    ang = 0.2
    XR, YR = math.cos(ang) * X - math.sin(ang) * Y, math.sin(ang) * X + math.cos(ang) * Y
    exact = field(XR, YR)
    exact[0, :] = exact[:, 0] = 0
    errs = []
    for hs in (0.2, 0.1):
        ns = int(round(16.0 / hs))
        xs = grid(ns, hs)
        XS, YS = np.meshgrid(xs, xs)
        f = field(XS, YS)
        f[0, :] = f[:, 0] = 0
        errs.append(np.max(np.abs(O.resample(f, (hs, hs), (nx, nx), (h, h), ang) - exact)))
    ratio = errs[0] / errs[1]
    assert 6.0 < ratio < 12.0, (errs, ratio)


def test_angular_moments_orientation():
    """A ring density with a 6-fold modulation at angle alpha: arg(M_6) / 6
    recovers alpha, up to the square grid's aliasing, which falls fast as
    the grid is refined; the odd orders vanish (the density and the grid's
    interior points are symmetric under the half turn; the even orders 2
    and 4 do not, as the square grid aliases the 6-fold pattern into
    them)."""
    errs = {}
    for n, h in ((64, 0.2), (128, 0.1)):
        x = grid(n, h)
        X, Y = np.meshgrid(x, x)
        phi = np.arctan2(Y, X)
        R2 = X * X + Y * Y
        for alpha in (0.0, 0.3, -0.7, 1.0):
            rho = (R2 / 4) * np.exp(-R2 / 4) * (1 + 0.3 * np.cos(6 * (phi - alpha)))
            psi = np.sqrt(rho).astype(np.complex128)
            psi[0, :] = psi[:, 0] = 0
            m = O.angular_moments(psi, h, h, 6)
            got = np.angle(m[6]) / 6
            d = (got - alpha + math.pi / 6) % (math.pi / 3) - math.pi / 6
            errs[(n, alpha)] = abs(d)
            for k in (1, 3, 5):
                assert abs(m[k]) < 1e-12 * abs(m[0]), (k, abs(m[k]))
    for alpha in (0.3, -0.7, 1.0):
        assert errs[(128, alpha)] < 2e-5, errs
        assert errs[(128, alpha)] < errs[(64, alpha)] / 8, errs
    assert errs[(64, 0.0)] < 1e-12 and errs[(128, 0.0)] < 1e-12
