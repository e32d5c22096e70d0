"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds workload definitions and random draws only: parameter sets
with the shapes of the paper's runs, the random numbers R(x, y) of the
initial state of Eq. (fun), and seeded random fields.  It contains none of the
solver's arithmetic, and imports neither the oracle nor the GPU library.

Arrays are numpy; shapes are (ny, nx) in 2D and (nz, ny, nx) in 3D with x
fastest.  Index 0 of every axis is the Dirichlet wall, so every state drawn
here is zero there.
"""
import math

import numpy as np

# ---------------------------------------------------------------------------
# Workload configurations.  Grid convention: n stored points per axis,
# x_i = -n*h/2 + i*h, so n = 128 and h = 0.1 span [-6.4, 6.4).

CONFIGS = {
    # 2D imaginary time, 128^2, g = 100, Omega = 0.6, 1000 steps.
    "c1": dict(dim=2, nx=128, ny=128, nz=1, hx=0.1, hy=0.1, hz=0.1,
               gamma=1.0, nu=1.0, lam=1.0, g=100.0, omega=0.6, dt=1e-3,
               mode=0, precision=0, steps=1000, seed=13, kind=1, d_xy=1.0),
    # 2D 512^2 on [-12.8, 12.8)^2, anisotropic trap, 20000 imaginary-time
    # steps then 10000 real-time steps; complex128 and complex64 variants.
    "c2": dict(dim=2, nx=512, ny=512, nz=1, hx=0.1, hy=0.1, hz=0.1,
               gamma=1.0, nu=1.05, lam=1.0, g=1000.0, omega=0.9, dt=5e-4,
               mode=0, precision=0, steps=20000, real_steps=10000, seed=13,
               kind=1, d_xy=1.0),
    # 3D 256 x 256 x 64, dz = 0.2, lambda = 4, complex64 sweeps.
    "c3": dict(dim=3, nx=256, ny=256, nz=64, hx=0.1, hy=0.1, hz=0.2,
               gamma=1.0, nu=1.0, lam=4.0, g=2000.0, omega=0.8, dt=2e-4,
               mode=0, precision=1, steps=5000, real_steps=5000, seed=13,
               kind=1, d_xy=1.0, d_z=0.5),
}

# The paper's own preset and Table 1 / Fig. 2(a) run: 2D, h = 0.05, 256
# stored points (the paper's 257-point grid minus its always-zero last row),
# g = 100, Omega = 0.8, Delta = 0.00025.
PAPER_2D_PRESET = dict(dim=2, nx=256, ny=256, nz=1, hx=0.05, hy=0.05,
                       hz=0.05, gamma=1.0, nu=1.0, lam=1.0, g=100.0,
                       omega=0.8, dt=0.00025, mode=0, precision=0, seed=13,
                       kind=1, d_xy=1.0)


def solver_params(cfg, **over):
    """The solver-parameter subset of a config (what both sides consume)."""
    keys = ("dim", "nx", "ny", "nz", "hx", "hy", "hz", "gamma", "nu", "lam",
            "g", "omega", "dt", "mode", "precision")
    d = {k: cfg[k] for k in keys if k in cfg}
    d.update(over)
    if d.get("dim", 2) == 2:
        d["nz"] = 1
    return d


def shape(cfg):
    return (cfg["nz"], cfg["ny"], cfg["nx"]) if cfg["dim"] == 3 else (cfg["ny"], cfg["nx"])


def phase_field(seed, ny, nx):
    """The random number R(x, y) of Eq. (fun), uniform in [0, 1), one per
    (x, y) grid point and constant along z.  numpy PCG64 stream `seed`."""
    return np.random.default_rng(int(seed)).random((int(ny), int(nx)))


def random_field(seed, shp, envelope=True):
    """A seeded complex test field with zero walls (index 0 of every axis).

    With ``envelope`` the complex Gaussian noise is multiplied by a wide
    bump so the field vanishes smoothly towards the walls; the result is
    scaled to unit sum of squares (not the method's normalisation)."""
    rng = np.random.default_rng(int(seed))
    f = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    if envelope:
        for ax, n in enumerate(shp):
            t = (np.arange(n) - n / 2) / (n / 2)
            w = np.exp(-4.0 * t * t)
            sh = [1] * len(shp)
            sh[ax] = n
            f = f * w.reshape(sh)
    idx = [slice(None)] * len(shp)
    for ax in range(len(shp)):
        i2 = list(idx)
        i2[ax] = 0
        f[tuple(i2)] = 0
    f /= np.sqrt(np.sum(np.abs(f) ** 2))
    return np.ascontiguousarray(f.astype(np.complex128))


# ---------------------------------------------------------------------------
# Batched sweep: 64 instances of uneven size and parameters.

BATCH_SIZES = (128, 192, 256, 384, 512)


def batch3d_instances(n=8, seed=2020, h=0.1, hz=0.2, nz=64, dt=2e-4):
    """Parameter draws of a batched 3D imaginary-time sweep: the 3D workload's
    trap (gamma = nu = 1, lambda = 4, h_z = 0.2, 64 points in z, dt = 2e-4)
    with Omega ~ U[0.5, 0.9], g_3D ~ logU[200, 2000] and the in-plane side
    drawn uniformly from the members of {128, 192, 256} whose extent holds
    2 * 1.4 radii of the rotating condensate (largest if none does); the
    radius is the 2D Thomas-Fermi one for g_2D = g_3D sqrt(lambda / (2 pi))
    (the quasi-2D reduction), which over-estimates the 3D one."""
    rng = np.random.default_rng(int(seed))
    lam = 4.0
    out = []
    for t in range(n):
        om = float(rng.uniform(0.5, 0.9))
        g = float(math.exp(rng.uniform(math.log(200.0), math.log(2000.0))))
        a = 1.0 - om * om
        g2 = g * math.sqrt(lam / (2.0 * math.pi))
        mu_tf = math.sqrt(g2 * a / math.pi)
        r_tf = math.sqrt(2.0 * mu_tf) / math.sqrt(a)
        ok = [s for s in (128, 192, 256) if s * h >= 2.0 * 1.4 * r_tf]
        if not ok:
            ok = [256]
        side = int(ok[int(rng.integers(len(ok)))])
        out.append(dict(dim=3, nx=side, ny=side, nz=nz, hx=h, hy=h, hz=hz,
                        gamma=1.0, nu=1.0, lam=lam, g=g, omega=om, dt=dt,
                        mode=0, precision=1, seed=13 + t, kind=1, d_xy=1.0))
    return out


def batch_instances(n=64, seed=2019, h=0.1, dt=1e-3):
    """Parameter draws of the batched 2D imaginary-time sweep.

    Omega ~ U[0.5, 0.95], g ~ logU[100, 3000], nu ~ U[1.0, 1.2], gamma = 1.
    The grid side is drawn uniformly from the members of BATCH_SIZES whose
    extent n*h holds 2 * 1.4 Thomas-Fermi radii, so every instance is
    resolved and contained (largest size if none qualifies)."""
    rng = np.random.default_rng(int(seed))
    out = []
    for t in range(n):
        om = float(rng.uniform(0.5, 0.95))
        g = float(math.exp(rng.uniform(math.log(100.0), math.log(3000.0))))
        nu = float(rng.uniform(1.0, 1.2))
        gam = 1.0
        a = gam * gam - om * om
        b = nu * nu - om * om
        mu_tf = math.sqrt(g * math.sqrt(a * b) / math.pi)
        r_tf = math.sqrt(2.0 * mu_tf) / math.sqrt(a)
        ok = [s for s in BATCH_SIZES if s * h >= 2.0 * 1.4 * r_tf]
        if not ok:
            ok = [BATCH_SIZES[-1]]
        side = int(ok[int(rng.integers(len(ok)))])
        out.append(dict(dim=2, nx=side, ny=side, nz=1, hx=h, hy=h, hz=h,
                        gamma=gam, nu=nu, lam=1.0, g=g, omega=om, dt=dt,
                        mode=0, precision=0, seed=13 + t, kind=1, d_xy=1.0))
    return out
