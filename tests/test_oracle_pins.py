"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a dense
LAPACK solve, a dense textbook Crank-Nicolson propagator built from the line
Hamiltonians, a numerical ODE integration, closed-form energies, exact
eigenvalues/eigenvectors, conservation laws, symmetries, or synthetic
states with a known vortex content.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import eigh_tridiagonal

import oracle as O
import workloads as W
from tests import _dense as D


# --------------------------------------------------------------------------
# Line solve (Thomas) against a dense LU solve with pivoting.

@pytest.mark.parametrize("n", [1, 2, 8, 33, 64])
@pytest.mark.parametrize("mode", [0, 1])
def test_thomas_matches_dense_solve(n, mode):
    rng = np.random.default_rng(100 + n + 7 * mode)
    dt, h = 0.01, 0.1
    tau = dt if mode == 1 else -1j * dt
    rot = rng.uniform(-3, 3)
    A0 = 1 + 1j * tau / (2 * h * h)
    # a diagonally dominant system with the paper's structure plus noise
    a = -(1j * tau / (4 * h)) * (1 / h - 1j * rot) * (1 + 0.1 * rng.standard_normal(n))
    c = -(1j * tau / (4 * h)) * (1 / h + 1j * rot) * (1 + 0.1 * rng.standard_normal(n))
    b = A0 * np.ones(n, dtype=complex)
    d = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    M = np.diag(b) + np.diag(c[:-1], 1) + np.diag(a[1:], -1)
    ref = np.linalg.solve(M, d)
    got = O.thomas(a, b, c, d)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


# --------------------------------------------------------------------------
# Each sweep against the dense textbook CN propagator of the line Hamiltonian.

@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("mode", [0, 1])
def test_sweep_2d_matches_dense_cayley(axis, mode):
    p = O.make_params(dim=2, nx=13, ny=11, hx=0.3, hy=0.25, gamma=1.0,
                      nu=1.3, g=5.0, omega=0.7, dt=0.02, mode=mode)
    psi = W.random_field(3, (11, 13))
    got = O.sweep(p, psi, axis)
    ref = D.apply_axis(psi, p, axis)
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("mode", [0, 1])
def test_sweep_3d_matches_dense_cayley(axis, mode):
    p = O.make_params(dim=3, nx=8, ny=9, nz=6, hx=0.4, hy=0.35, hz=0.2,
                      gamma=1.0, nu=1.1, lam=3.0, g=2.0, omega=0.5, dt=0.01,
                      mode=mode)
    psi = W.random_field(4, (6, 9, 8))
    got = O.sweep(p, psi, axis)
    ref = D.apply_axis(psi, p, axis)
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_real_time_line_hamiltonian_is_hermitian():
    # The split line operators are Hermitian, so real-time CN is unitary.
    for axis in (0, 1, 2):
        H = D.line_hamiltonian(20, 0.1, axis, 2.3, 0.8)
        assert np.allclose(H, H.conj().T, atol=0)


# --------------------------------------------------------------------------
# H1 sub-step against a numerical integration of i dpsi/dt = (V + g|psi|^2) psi.

def _h1_ode(p, psi0, x, y):
    V = 0.5 * (p.gamma ** 2 * x * x + p.nu ** 2 * y * y)

    def rhs(t, u):
        z = u[0] + 1j * u[1]
        w = (V + p.g * abs(z) ** 2) * z
        dz = -1j * w if p.mode == 1 else -w
        return [dz.real, dz.imag]

    sol = solve_ivp(rhs, (0, p.dt), [psi0.real, psi0.imag], rtol=1e-13,
                    atol=1e-15, method="DOP853")
    return sol.y[0, -1] + 1j * sol.y[1, -1]


def test_h1_real_time_is_exact_ode_solution():
    p = O.make_params(dim=2, nx=6, ny=6, hx=0.5, hy=0.5, gamma=1.0, nu=1.2,
                      g=50.0, omega=0.3, dt=0.01, mode=1)
    psi = W.random_field(5, (6, 6)) * 4
    got = O.h1(p, psi)
    x = D.coords(6, 0.5)
    for j in range(1, 6):
        for i in range(1, 6):
            ref = _h1_ode(p, psi[j, i], x[i], x[j])
            assert abs(got[j, i] - ref) <= 1e-11 * max(abs(ref), 1e-300)
    # |psi| is invariant pointwise
    assert np.max(np.abs(np.abs(got) - np.abs(psi))) <= 1e-15


def test_h1_imaginary_time_first_order():
    # g = 0: exp(-dt V) psi is the exact imaginary-time solution.  g > 0: the
    # frozen-density form differs from the exact ODE solution at O(dt^2).
    x = D.coords(6, 0.5)
    errs = []
    for dt in (0.004, 0.002):
        for g in (0.0, 20.0):
            p = O.make_params(dim=2, nx=6, ny=6, hx=0.5, hy=0.5, gamma=1.0,
                              nu=1.2, g=g, dt=dt, mode=0)
            psi = W.random_field(6, (6, 6)) * 2
            got = O.h1(p, psi)
            e = max(abs(got[j, i] - _h1_ode(p, psi[j, i], x[i], x[j]))
                    for j in range(1, 6) for i in range(1, 6))
            if g == 0.0:
                assert e <= 1e-12
            else:
                errs.append(e)
    ratio = errs[0] / errs[1]
    assert 3.6 < ratio < 4.4  # O(dt^2) per sub-step


# --------------------------------------------------------------------------
# Full step against the dense brute force.

@pytest.mark.parametrize("mode", [0, 1])
def test_step_2d_matches_dense_bruteforce(mode):
    p = O.make_params(dim=2, nx=12, ny=12, hx=0.45, hy=0.45, gamma=1.0, nu=1.2,
                      g=40.0, omega=0.6, dt=0.01, mode=mode)
    psi = W.random_field(7, (12, 12)) / math.sqrt(0.45 * 0.45)
    got = O.step(p, psi, 3)
    ref = psi
    for _ in range(3):
        ref = D.dense_step(p, ref)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("mode", [0, 1])
def test_step_3d_matches_dense_bruteforce(mode):
    p = O.make_params(dim=3, nx=8, ny=8, nz=6, hx=0.5, hy=0.5, hz=0.3,
                      gamma=1.0, nu=1.1, lam=2.5, g=30.0, omega=0.5, dt=0.01,
                      mode=mode)
    psi = W.random_field(8, (6, 8, 8)) / math.sqrt(0.5 * 0.5 * 0.3)
    got = O.step(p, psi, 2)
    ref = D.dense_step(p, D.dense_step(p, psi))
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


# --------------------------------------------------------------------------
# g = 0: imaginary time is power iteration on a fixed linear map.

def test_g0_fixed_point_is_dominant_eigenvector():
    n, h, dt = 12, 0.5, 0.05
    p = O.make_params(dim=2, nx=n, ny=n, hx=h, hy=h, gamma=1.0, nu=1.25,
                      g=0.0, omega=0.35, dt=dt, mode=0)
    m = n - 1
    V = D.potential_grid(p)[1:, 1:].reshape(-1)
    x = D.coords(n, h)
    N = m * m
    Cx = np.zeros((N, N), complex)
    Cy = np.zeros((N, N), complex)
    for j in range(m):      # rows (x-lines at y_{j+1})
        C = D.cn_matrix(D.line_hamiltonian(n, h, 0, x[j + 1], p.omega), dt, 0)
        Cx[j * m:(j + 1) * m, j * m:(j + 1) * m] = C
    for i in range(m):      # columns (y-lines at x_{i+1})
        C = D.cn_matrix(D.line_hamiltonian(n, h, 1, x[i + 1], p.omega), dt, 0)
        idx = np.arange(m) * m + i
        Cy[np.ix_(idx, idx)] = C
    M = Cy @ Cx @ np.diag(np.exp(-dt * V))
    w, v = np.linalg.eig(M)
    top = v[:, np.argmax(np.abs(w))]
    psi = O.init_state(p, 0, W.phase_field(1, n, n), 1.0)
    psi = O.step(p, psi, 1500)
    u = psi[1:, 1:].reshape(-1)
    u = u / np.linalg.norm(u)
    top = top / np.linalg.norm(top)
    phase = np.vdot(top, u)
    assert np.linalg.norm(u - phase / abs(phase) * top) <= 1e-10


# --------------------------------------------------------------------------
# Closed forms at g = 0.

def _tri_ground(n, h, w):
    xs = D.coords(n, h)[1:]
    d = 1.0 / h ** 2 + 0.5 * w * w * xs * xs
    e = -0.5 / h ** 2 * np.ones(n - 2)
    return eigh_tridiagonal(d, e, eigvals_only=True, select="i",
                            select_range=(0, 0))[0]


def test_g0_separable_ground_energy_converges_as_dt_squared():
    # Omega = 0: the discrete ground energy is eigmin(T_x) + eigmin(T_y)
    # exactly; the split-step fixed point reaches it with an O(dt^2) error.
    n, h = 40, 0.25
    E0 = _tri_ground(n, h, 1.0) + _tri_ground(n, h, 1.5)
    assert abs(E0 - 1.25) < 0.01  # continuum (gamma + nu) / 2
    errs = []
    for dt in (0.02, 0.01):
        p = O.make_params(dim=2, nx=n, ny=n, hx=h, hy=h, gamma=1.0, nu=1.5,
                          g=0.0, omega=0.0, dt=dt, mode=0)
        psi = O.step(p, O.init_state(p, 0, None, 1.0), int(40 / dt))
        ob = O.observables(p, psi)
        errs.append(ob["mu_full"] - E0)
        assert abs(ob["mu"] - ob["mu_full"]) < 1e-12
        assert abs(ob["energy"] - ob["mu"]) < 1e-12  # g = 0
    assert 0 < errs[1] < errs[0] < 2e-4
    assert 3.6 < errs[0] / errs[1] < 4.4


def test_g0_rotating_anisotropic_closed_form():
    # Rotating anisotropic oscillator: E0 = (w1 + w2)/2 with
    # w^4 - (gamma^2 + nu^2 + 2 Omega^2) w^2 + (gamma^2-Omega^2)(nu^2-Omega^2) = 0.
    gam, nu, om = 1.0, 1.05, 0.9
    a = gam ** 2 + nu ** 2 + 2 * om ** 2
    b = (gam ** 2 - om ** 2) * (nu ** 2 - om ** 2)
    r = math.sqrt(a * a - 4 * b)
    E0 = 0.5 * (math.sqrt((a + r) / 2) + math.sqrt((a - r) / 2))
    assert abs(E0 - 1.0239613) < 1e-7
    errs = []
    for n, h in ((80, 0.25), (100, 0.2)):
        p = O.make_params(dim=2, nx=n, ny=n, hx=h, hy=h, gamma=gam, nu=nu,
                          g=0.0, omega=om, dt=0.01, mode=0)
        psi = O.step(p, O.init_state(p, 0, None, 1.0), 8000)
        errs.append(O.observables(p, psi)["mu_full"] - E0)
    assert abs(errs[0]) < 0.006 and abs(errs[1]) < 0.004
    assert 1.35 < errs[0] / errs[1] < 1.8  # O(h^2): (0.25/0.2)^2 = 1.56


def test_observables_closed_forms():
    # Gaussian ground state of the anisotropic trap: mu = E = (gamma+nu)/2,
    # rms_x = 1/sqrt(2 gamma), and the one-vortex state (x + iy) e^{-r^2/2}
    # of the isotropic trap: E = 2 - Omega (L_z = 1).  Errors are O(h^2).
    gam, nu = 1.0, 1.4
    errs = []
    for n, h in ((96, 0.2), (192, 0.1)):
        p = O.make_params(dim=2, nx=n, ny=n, hx=h, hy=h, gamma=gam, nu=nu,
                          g=0.0, omega=0.3, dt=1e-3, mode=0)
        x = D.coords(n, h)
        Y, X = np.meshgrid(x, x, indexing="ij")
        psi = np.exp(-(gam * X ** 2 + nu * Y ** 2) / 2).astype(complex)
        psi[0, :] = 0
        psi[:, 0] = 0
        ob = O.observables(p, psi)
        errs.append(abs(ob["mu"] - (gam + nu) / 2))
        assert abs(ob["mu_full"] - (gam + nu) / 2) < 0.01
        assert abs(ob["rms_x"] - 1 / math.sqrt(2 * gam)) < 1e-6
        assert abs(ob["rms_y"] - 1 / math.sqrt(2 * nu)) < 1e-6
        # vortex state, isotropic trap
        pv = O.make_params(dim=2, nx=n, ny=n, hx=h, hy=h, gamma=1.0, nu=1.0,
                           g=0.0, omega=0.45, dt=1e-3, mode=0)
        v = (X + 1j * Y) * np.exp(-(X ** 2 + Y ** 2) / 2)
        v[0, :] = 0
        v[:, 0] = 0
        obv = O.observables(pv, v)
        assert abs(obv["energy_full"] - (2 - 0.45)) < 0.01
        assert abs(obv["energy"] - (2 - 0.45)) < 0.01
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_observables_gp_identity_and_3d():
    # mu - E = 1/2 g int |psi|^4 (full functional); 3D Gaussian ground state
    # of the trap gives (gamma + nu + lambda) / 2.
    p = O.make_params(dim=3, nx=48, ny=48, nz=40, hx=0.2, hy=0.2, hz=0.1,
                      gamma=1.0, nu=1.2, lam=4.0, g=25.0, omega=0.2, dt=1e-3)
    x = D.coords(48, 0.2)
    z = D.coords(40, 0.1)
    Z, Y, X = np.meshgrid(z, x, x, indexing="ij")
    psi = np.exp(-(X ** 2 + 1.2 * Y ** 2 + 4.0 * Z ** 2) / 2).astype(complex)
    psi[0], psi[:, 0], psi[:, :, 0] = 0, 0, 0
    psi = O.normalize(p, psi)
    ob = O.observables(p, psi)
    s = ob["sums"]
    assert abs((ob["mu_full"] - ob["energy_full"]) - 0.5 * s[8]) < 1e-12
    p0 = O.make_params(dim=3, nx=48, ny=48, nz=40, hx=0.2, hy=0.2, hz=0.1,
                       gamma=1.0, nu=1.2, lam=4.0, g=0.0, omega=0.0, dt=1e-3)
    assert abs(O.observables(p0, psi)["mu"] - (1 + 1.2 + 4) / 2) < 0.02
    assert abs(ob["rms_z"] - 1 / math.sqrt(8.0)) < 1e-4


# --------------------------------------------------------------------------
# Conservation and symmetry.

def test_real_time_is_unitary():
    p = O.make_params(dim=2, nx=48, ny=40, hx=0.3, hy=0.3, gamma=1.0, nu=1.1,
                      g=80.0, omega=0.7, dt=0.005, mode=1)
    psi = O.init_state(p, 1, W.phase_field(2, 40, 48), 1.0)
    out = O.step(p, psi, 2000)
    assert abs(O.observables(p, out)["norm"] - 1.0) < 1e-12


def test_sweep_axis_rotation_symmetry():
    # For hx = hy and nx = ny the y-sweep is the x-sweep conjugated by a
    # 90-degree rotation of the interior grid, in either direction.
    n, h = 16, 0.3
    for mode in (0, 1):
        p = O.make_params(dim=2, nx=n, ny=n, hx=h, hy=h, g=0.0, omega=0.4,
                          dt=0.05, mode=mode)
        psi = W.random_field(9, (n, n))

        def rot_ccw(a):
            out = np.zeros_like(a)
            out[n - np.arange(1, n)[:, None], np.arange(1, n)[None, :]] = a[1:, 1:].T
            return out

        def rot_cw(a):
            out = np.zeros_like(a)
            out[np.arange(1, n)[:, None], n - np.arange(1, n)[None, :]] = a[1:, 1:].T
            return out

        for R in (rot_ccw, rot_cw):
            lhs = O.sweep(p, R(psi), 1)
            rhs = R(O.sweep(p, psi, 0))
            assert np.max(np.abs(lhs - rhs)) < 1e-15


def test_restart_is_bitwise_deterministic():
    p = O.make_params(dim=2, nx=40, ny=36, hx=0.25, hy=0.25, g=60.0,
                      omega=0.5, dt=2e-3, mode=0)
    psi = O.init_state(p, 1, W.phase_field(3, 36, 40), 1.0)
    a = O.step(p, psi, 50)
    b = O.step(p, O.step(p, psi, 20), 30)
    assert np.array_equal(a, b)


def test_real_time_energy_drift_is_first_order_in_dt():
    # From an imaginary-time-relaxed state, real-time propagation keeps the
    # full-functional energy; its excursion shrinks with dt.
    p = O.make_params(dim=2, nx=48, ny=48, hx=0.25, hy=0.25, gamma=1.0,
                      nu=1.0, g=30.0, omega=0.5, dt=0.005, mode=0)
    psi = O.step(p, O.init_state(p, 1, W.phase_field(4, 48, 48), 1.0), 3000)
    dev = []
    for dt in (0.004, 0.002):
        pr = O.make_params(dim=2, nx=48, ny=48, hx=0.25, hy=0.25, gamma=1.0,
                           nu=1.0, g=30.0, omega=0.5, dt=dt, mode=1)
        E0 = O.observables(pr, psi)["energy_full"]
        cur, mx = psi, 0.0
        for _ in range(10):
            cur = O.step(pr, cur, int(0.2 / dt))
            mx = max(mx, abs(O.observables(pr, cur)["energy_full"] - E0))
        dev.append(mx)
    assert dev[0] < 0.05
    assert dev[1] < dev[0]


# --------------------------------------------------------------------------
# Initial state.

def test_initial_state_shape_and_norm():
    p = O.make_params(dim=2, nx=64, ny=64, hx=0.2, hy=0.2)
    ph = W.phase_field(13, 64, 64)
    psi = O.init_state(p, 1, ph, 1.0)
    assert abs(O.observables(p, psi)["norm"] - 1) < 1e-13
    assert np.all(psi[0, :] == 0) and np.all(psi[:, 0] == 0)
    x = D.coords(64, 0.2)
    # ratio to the unmodulated one-vortex profile is a pure phase 2 pi R
    ref = (x[None, :] + 1j * x[:, None]) * np.exp(-(x[None, :] ** 2 + x[:, None] ** 2) / 2)
    keep = np.abs(ref) > 1e-12  # the vortex core sits on the grid point (0, 0)
    keep[0, :] = False
    keep[:, 0] = False
    r = psi[keep] / ref[keep]
    mag = np.abs(r)
    assert np.max(mag) / np.min(mag) - 1 < 1e-12
    diff = np.angle(r * np.exp(-2j * np.pi * ph[keep]))
    assert np.max(np.abs(diff)) < 1e-10
    # one vortex without random phase: winding +1 at the centre (odd n puts
    # the core inside a plaquette; a zero exactly on a grid point is split
    # over four plaquettes and counted in none of them)
    p = O.make_params(dim=2, nx=63, ny=63, hx=0.2, hy=0.2)
    assert O.vortex_count(p, O.init_state(p, 1, None, 1.0)) == 1
    assert O.vortex_count(p, O.init_state(p, 0, None, 1.0)) == 0


def test_initial_state_3d_gaussian_factor():
    p = O.make_params(dim=3, nx=32, ny=32, nz=24, hx=0.3, hy=0.3, hz=0.1, lam=4.0)
    psi = O.init_state(p, 1, None, 1.0, 0.5)
    z = D.coords(24, 0.1)
    col = psi[:, 16, 20]
    ref = np.exp(-z ** 2 / (2 * 0.25))
    ref[0] = 0
    assert np.allclose(col / col[12], ref / ref[12], rtol=1e-12, atol=1e-15)
    assert abs(O.observables(p, psi)["norm"] - 1) < 1e-13


# --------------------------------------------------------------------------
# Vortex counting on synthetic states with known zeros.

def _synthetic(n, h, zeros, anti=(), xi=0.2):
    """A broad envelope times unit-modulus vortex cores of size xi at `zeros`
    (charge +1) and `anti` (charge -1)."""
    x = D.coords(n, h)
    Y, X = np.meshgrid(x, x, indexing="ij")
    Zc = X + 1j * Y
    psi = np.exp(-(X ** 2 + Y ** 2) / (2 * 2.0 ** 2)).astype(complex)
    for z0 in zeros:
        psi = psi * (Zc - z0) / np.sqrt(np.abs(Zc - z0) ** 2 + xi ** 2)
    for z0 in anti:
        psi = psi * np.conj(Zc - z0) / np.sqrt(np.abs(Zc - z0) ** 2 + xi ** 2)
    psi[0, :] = 0
    psi[:, 0] = 0
    return psi


def test_vortex_count_synthetic():
    n, h = 128, 0.1
    p = O.make_params(dim=2, nx=n, ny=n, hx=h, hy=h)
    zeros = [0.03 + 0.02j] + [1.5 * np.exp(1j * (np.pi / 3 * k + 0.1)) for k in range(6)]
    assert O.vortex_count(p, _synthetic(n, h, zeros)) == 7
    # antivortices are not counted
    assert O.vortex_count(p, _synthetic(n, h, zeros[:3], anti=[-2.0 + 1.0j])) == 3
    # a defect far out in the empty region is masked by the density cut
    psi = _synthetic(n, h, zeros[:2] + [5.9 + 0.05j])
    assert O.vortex_count(p, psi) == 2
    assert O.vortex_count(p, psi, density_frac=0.0) == 3


def _field(n_y, n_x, h):
    """A smooth complex field sampled on the paper's grid x_i = -n h/2 + i h
    (h a power of two, so every coordinate is exact)."""
    x = -n_x * h / 2 + h * np.arange(n_x)
    y = -n_y * h / 2 + h * np.arange(n_y)
    X, Y = np.meshgrid(x, y)
    return (X + 1j * Y) * np.exp(-(X ** 2 + 2 * Y ** 2) / 4)


@pytest.mark.parametrize("small,big", [((10, 14), (16, 22)), ((16, 22), (10, 14)), ((10, 22), (16, 14))])
def test_embed_keeps_physical_coordinates(small, big):
    """The embedded value at a point of the new grid is the old grid's value
    at the same (x, y); points the old grid does not cover, and the walls of
    the new grid, are zero (Sec. 3, continuation start)."""
    h = 0.125
    src = _field(*small, h)
    src[0, :] = 0
    src[:, 0] = 0
    out = O.embed(src, big)
    ref = _field(*big, h)
    ny, nx = big
    y = -ny * h / 2 + h * np.arange(ny)
    x = -nx * h / 2 + h * np.arange(nx)
    covered = ((np.abs(y) < small[0] * h / 2)[:, None] | (y == -small[0] * h / 2)[:, None]) & \
              ((np.abs(x) < small[1] * h / 2)[None, :] | (x == -small[1] * h / 2)[None, :])
    covered[0, :] = False
    covered[:, 0] = False
    # the old grid's own wall row and column hold zero
    oy, ox = (ny - small[0]) // 2, (nx - small[1]) // 2
    if 0 <= oy < ny:
        covered[oy, :] = False
    if 0 <= ox < nx:
        covered[:, ox] = False
    assert np.array_equal(out[covered], ref[covered])
    assert np.all(out[~covered] == 0)


def test_embed_round_trip_norm_and_parity():
    rng = np.random.default_rng(3)
    src = rng.standard_normal((6, 12, 10)) + 1j * rng.standard_normal((6, 12, 10))
    src[0], src[:, 0], src[:, :, 0] = 0, 0, 0
    big = O.embed(src, (10, 16, 18))
    assert np.array_equal(O.embed(big, src.shape), src)
    assert np.sum(np.abs(big) ** 2) == pytest.approx(np.sum(np.abs(src) ** 2), rel=1e-15)
    with pytest.raises(ValueError):
        O.embed(src, (10, 16, 17))


def test_functional_fourth_order_closed_forms():
    """The fourth-order functional against closed forms of the continuum:
    the anisotropic Gaussian (E = mu = (gamma + nu) / 2 at g = 0), the
    one-vortex state (x + i y) e^{-r^2/2} of the isotropic trap (E = 2 -
    Omega, L_z = 1), and the GP identity mu - E = g/2 int |psi|^4; the
    error falls as h^4."""
    gam, nu = 1.0, 1.4
    errs = []
    for n, h in ((96, 0.2), (192, 0.1)):
        x = D.coords(n, h)
        Y, X = np.meshgrid(x, x, indexing="ij")
        p = O.make_params(dim=2, nx=n, ny=n, hx=h, hy=h, gamma=gam, nu=nu, g=0.0, omega=0.3, dt=1e-3, mode=0)
        psi = np.exp(-(gam * X ** 2 + nu * Y ** 2) / 2).astype(complex)
        psi[0, :] = 0
        psi[:, 0] = 0
        f = O.functional_fourth_order(p, psi)
        errs.append(abs(f["mu"] - (gam + nu) / 2))
        pv = O.make_params(dim=2, nx=n, ny=n, hx=h, hy=h, gamma=1.0, nu=1.0, g=7.0, omega=0.45, dt=1e-3, mode=0)
        v = (X + 1j * Y) * np.exp(-(X ** 2 + Y ** 2) / 2)
        v[0, :] = 0
        v[:, 0] = 0
        fv = O.functional_fourth_order(pv, v)
        nv = np.sum(np.abs(v) ** 2) * h * h
        inter = 0.5 * 7.0 * np.sum(np.abs(v) ** 4) * h * h / nv
        assert abs(fv["lz"] - 1.0) < 5e-4
        assert abs(fv["energy"] - inter - (2 - 0.45)) < 1e-3
        assert fv["mu"] - fv["energy"] == pytest.approx(inter, rel=1e-12)
        # the C oracle's observables compute the same functional
        ov = O.observables(pv, v)
        assert ov["mu_4th"] == pytest.approx(fv["mu"], rel=1e-12)
        assert ov["energy_4th"] == pytest.approx(fv["energy"], rel=1e-12)
    assert 12 < errs[0] / errs[1] < 20


def test_density_profiles_closed_forms():
    """Integrated densities of the normalised anisotropic Gaussian
    sqrt(gamma nu)/pi e^{-gamma x^2 - nu y^2} are its 1D marginals
    sqrt(gamma/pi) e^{-gamma x^2} (and in y), the cuts through the centre
    are the Gaussian at y = 0 (index ny/2 is y = 0 on the paper's grid), and
    the 3D z profile of a product state is the z marginal."""
    gam, nu, n, h = 1.3, 0.8, 96, 0.2
    x = D.coords(n, h)
    Y, X = np.meshgrid(x, x, indexing="ij")
    psi = (gam * nu) ** 0.25 / np.sqrt(np.pi) * np.exp(-(gam * X ** 2 + nu * Y ** 2) / 2)
    psi[0, :] = 0
    psi[:, 0] = 0
    p = O.make_params(dim=2, nx=n, ny=n, hx=h, hy=h, gamma=gam, nu=nu)
    assert np.allclose(O.density(p, psi, "x"), np.sqrt(gam / np.pi) * np.exp(-gam * x ** 2), atol=1e-12)
    assert np.allclose(O.density(p, psi, "y"), np.sqrt(nu / np.pi) * np.exp(-nu * x ** 2), atol=1e-12)
    assert x[n // 2] == 0.0
    assert np.allclose(O.density(p, psi, "cut_x"), np.sqrt(gam * nu) / np.pi * np.exp(-gam * x ** 2), atol=1e-15)
    assert np.array_equal(O.density(p, psi, "xy"), np.abs(psi) ** 2)
    nz, hz, lam = 40, 0.15, 2.0
    z = D.coords(nz, hz)
    fz = (lam / np.pi) ** 0.25 * np.exp(-lam * z ** 2 / 2)
    fz[0] = 0
    psi3 = fz[:, None, None] * psi[None]
    p3 = O.make_params(dim=3, nx=n, ny=n, nz=nz, hx=h, hy=h, hz=hz, gamma=gam, nu=nu, lam=lam)
    assert np.allclose(O.density(p3, psi3, "z"), fz ** 2, atol=1e-12)
    assert np.allclose(O.density(p3, psi3, "xy"), np.abs(psi) ** 2, atol=1e-12)
    assert np.allclose(O.density(p3, psi3, "x"), np.sqrt(gam / np.pi) * np.exp(-gam * x ** 2), atol=1e-12)


def test_extend_z_gives_the_3d_form_of_eq_fun():
    """The 3D initial state of Eq. (fun) is the 2D one times a Gaussian in z
    (Sec. 2): extending the oracle's normalised 2D state along z and zeroing
    the wall plane reproduces the oracle's own 3D initial state (built by its
    C code from Eq. (fun) directly), normalised."""
    import workloads as W
    n, nz, h, hz, lam = 20, 14, 0.3, 0.15, 4.0
    ph = W.phase_field(5, n, n)
    p2 = O.make_params(dim=2, nx=n, ny=n, hx=h, hy=h, g=10.0, omega=0.5)
    p3 = O.make_params(dim=3, nx=n, ny=n, nz=nz, hx=h, hy=h, hz=hz, lam=lam, g=10.0, omega=0.5)
    d_z = 1.0 / np.sqrt(lam)
    for kind in (0, 1):
        xy = O.init_state(p2, kind=kind, phase=ph, d_xy=1.0)
        ext = O.extend_z(xy, nz, hz, d_z)
        ext[0] = 0
        ref = O.init_state(p3, kind=kind, phase=ph, d_xy=1.0, d_z=d_z)
        assert np.linalg.norm(ext - ref) <= 1e-13 * np.linalg.norm(ref)
        assert abs(h * h * hz * np.sum(np.abs(ext) ** 2) - 1.0) <= 1e-14
    # the Gaussian's width: ratio of planes k and k' is exp(-(z_k^2 - z_k'^2) / (2 d_z^2))
    ext = O.extend_z(np.ones((3, 3)), nz, hz, d_z)
    z = -0.5 * nz * hz + np.arange(nz) * hz
    assert ext[3, 1, 1].real / ext[7, 1, 1].real == pytest.approx(np.exp(-(z[3] ** 2 - z[7] ** 2) / (2 * d_z ** 2)),
                                                                  rel=1e-14)


def test_splitmix64_matches_the_published_generator():
    """The first three outputs of the SplitMix64 generator seeded with 0, as
    its reference implementation (Vigna, splitmix64.c, public domain) prints
    them; the generator's state advances by the increment each call."""
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    state, got = 0, []
    for _ in range(3):
        got.append(O.splitmix64(state))
        state = (state + 0x9E3779B97F4A7C15) & ((1 << 64) - 1)
    assert got == want


def test_splitmix_phase_is_a_53_bit_uniform_per_point():
    ph = O.splitmix_phase(13, 40, 50)
    assert ph.shape == (40, 50)
    assert np.all(ph >= 0.0) and np.all(ph < 1.0)
    # every value is an integer multiple of 2^-53
    assert np.all(np.floor(ph * 2.0 ** 53) == ph * 2.0 ** 53)
    # point (i, j) depends on the seed and its index j nx + i only
    assert ph[3, 7] == (O.splitmix64(13 ^ (3 * 50 + 7)) >> 11) * 2.0 ** -53
    assert O.splitmix_phase(13, 1, 2000)[0, 157] == ph[3, 7]
    # uniform: mean and variance within 5 sigma of 1/2 and 1/12 over 2000 draws
    assert abs(ph.mean() - 0.5) < 5 * np.sqrt(1 / 12 / ph.size)
    assert abs(ph.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / ph.size)
    assert not np.array_equal(O.splitmix_phase(14, 40, 50), ph)
