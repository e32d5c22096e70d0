"""Oracle for the SSCN rotating Gross-Pitaevskii solver (FP64, CPU).

TEST INFRASTRUCTURE ONLY.  A plain, slow, obviously-correct implementation of
what the GPU path computes, written from the paper (Kumar, Loncar,
Muruganandam, Adhikari, Balaz, "C and Fortran OpenMP programs for rotating
Bose-Einstein condensates").  It shares no code with the GPU library and is
used only by the tests, the smoke check and the benchmark's CPU baseline.

The solver's arithmetic (the step, the observables, the vortex count, the
initial state) lives in ``sscn_oracle.c``, marshalled here through ctypes.
Nine plain numpy/Python definitions live in this module: ``embed``
(continuation start), ``extend_z`` (3D product start),
``functional_fourth_order``, ``density``, ``splitmix64`` and
``splitmix_phase`` (the counter-based random phase of the seeded initial
state), and for the learned initial state ``keys_cubic``, ``resample``
(interpolation between grids) and ``angular_moments`` (lattice
orientation).  Each function is pinned in tests/test_oracle_pins.py against
what the paper and the mathematics fix; none is parity unpinned.  Arrays are
complex128 with shape (ny, nx) in 2D and (nz, ny, nx) in 3D (x fastest),
index 0 of every axis being the wall.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


class OrcParams(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int),
                ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double),
                ("hz", ctypes.c_double), ("gamma", ctypes.c_double),
                ("nu", ctypes.c_double), ("lam", ctypes.c_double),
                ("g", ctypes.c_double), ("omega", ctypes.c_double),
                ("dt", ctypes.c_double), ("mode", ctypes.c_int)]


class OrcObs(ctypes.Structure):
    _fields_ = [("norm", ctypes.c_double), ("mu", ctypes.c_double),
                ("energy", ctypes.c_double), ("mu_full", ctypes.c_double),
                ("energy_full", ctypes.c_double), ("mu_4th", ctypes.c_double),
                ("energy_4th", ctypes.c_double), ("rms_x", ctypes.c_double),
                ("rms_y", ctypes.c_double), ("rms_z", ctypes.c_double),
                ("rms_r", ctypes.c_double), ("max_density", ctypes.c_double),
                ("sums", ctypes.c_double * 16)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        cp = ctypes.c_void_p
        P = ctypes.POINTER(OrcParams)
        L.orc_thomas.argtypes = [ctypes.c_int, cp, cp, cp, cp, cp]
        L.orc_h1.argtypes = [P, cp]
        L.orc_sweep.argtypes = [P, ctypes.c_int, cp]
        L.orc_normalize.argtypes = [P, cp]
        L.orc_normalize.restype = ctypes.c_double
        L.orc_step.argtypes = [P, cp, ctypes.c_long]
        L.orc_init_state.argtypes = [P, ctypes.c_int, cp, ctypes.c_double,
                                     ctypes.c_double, cp]
        L.orc_observables.argtypes = [P, cp, ctypes.POINTER(OrcObs)]
        L.orc_vortex_count.argtypes = [P, cp, ctypes.c_double, ctypes.c_int]
        L.orc_vortex_count.restype = ctypes.c_int
        _lib = L
    return _lib


def make_params(dim=2, nx=64, ny=64, nz=1, hx=0.1, hy=0.1, hz=0.1, gamma=1.0,
                nu=1.0, lam=1.0, g=0.0, omega=0.0, dt=1e-3, mode=0, **_ignored):
    """Parameter struct; ``mode`` 0 = imaginary time, 1 = real time."""
    return OrcParams(int(dim), int(nx), int(ny), int(nz if dim == 3 else 1),
                     float(hx), float(hy), float(hz), float(gamma), float(nu),
                     float(lam), float(g), float(omega), float(dt), int(mode))


def shape_of(p):
    return (p.nz, p.ny, p.nx) if p.dim == 3 else (p.ny, p.nx)


def _buf(p, psi):
    a = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    if a.shape != shape_of(p):
        raise ValueError(f"psi shape {a.shape} != {shape_of(p)}")
    return a


def thomas(a, b, c, d):
    """Solve a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = d[i] (textbook Thomas)."""
    a, b, c, d = (np.ascontiguousarray(v, dtype=np.complex128) for v in (a, b, c, d))
    x = np.zeros_like(d)
    lib().orc_thomas(len(d), a.ctypes.data, b.ctypes.data, c.ctypes.data,
                     d.ctypes.data, x.ctypes.data)
    return x


def h1(p, psi):
    out = _buf(p, psi)
    lib().orc_h1(ctypes.byref(p), out.ctypes.data)
    return out


def sweep(p, psi, axis):
    out = _buf(p, psi)
    lib().orc_sweep(ctypes.byref(p), int(axis), out.ctypes.data)
    return out


def normalize(p, psi):
    out = _buf(p, psi)
    lib().orc_normalize(ctypes.byref(p), out.ctypes.data)
    return out


def step(p, psi, nsteps=1):
    out = _buf(p, psi)
    lib().orc_step(ctypes.byref(p), out.ctypes.data, int(nsteps))
    return out


def init_state(p, kind=1, phase=None, d_xy=1.0, d_z=None):
    """Eq. (fun); ``phase`` is the (ny, nx) array of R(x, y) or None."""
    out = np.zeros(shape_of(p), dtype=np.complex128)
    if d_z is None:
        d_z = 1.0 / np.sqrt(p.lam) if p.dim == 3 else 1.0
    ph = None
    if phase is not None:
        ph = np.ascontiguousarray(phase, dtype=np.float64)
        if ph.shape != (p.ny, p.nx):
            raise ValueError("phase must have shape (ny, nx)")
    lib().orc_init_state(ctypes.byref(p), int(kind),
                         ph.ctypes.data if ph is not None else None,
                         float(d_xy), float(d_z), out.ctypes.data)
    return out


OBS_KEYS = ("norm", "mu", "energy", "mu_full", "energy_full", "mu_4th", "energy_4th", "rms_x",
            "rms_y", "rms_z", "rms_r", "max_density")


def observables(p, psi):
    a = _buf(p, psi)
    o = OrcObs()
    lib().orc_observables(ctypes.byref(p), a.ctypes.data, ctypes.byref(o))
    d = {k: getattr(o, k) for k in OBS_KEYS}
    d["sums"] = np.array(list(o.sums))
    return d


def vortex_count(p, psi, density_frac=0.05, box=3):
    a = _buf(p, psi)
    return int(lib().orc_vortex_count(ctypes.byref(p), a.ctypes.data,
                                      float(density_frac), int(box)))


def embed(psi, shape):
    """Continuation start of Sec. 3: place a state (ny, nx) or (nz, ny, nx)
    at the centre of a grid of `shape` with the same spacing, the index
    offset on each axis being half the difference of the sizes (the paper's
    Fortran reads the old grid into I = NX2 - NXOLD2 .. NX2 + NXOLD2).  Points
    of the new grid not covered by the old one are zero, old points falling
    outside the new grid are dropped, and the new grid's walls (index 0) are
    zero.  The size differences must be even, so the two grids' points
    coincide."""
    src = np.asarray(psi, dtype=np.complex128)
    if src.ndim != len(shape) or src.ndim not in (2, 3):
        raise ValueError("shape rank mismatch")
    if any((n - m) % 2 for n, m in zip(shape, src.shape)):
        raise ValueError("grid sizes must differ by an even number of points")
    out = np.zeros(shape, dtype=np.complex128)
    for idx in np.ndindex(*shape):
        if 0 in idx:
            continue
        sidx = tuple(i - (n - m) // 2 for i, n, m in zip(idx, shape, src.shape))
        if all(0 <= si < m for si, m in zip(sidx, src.shape)):
            out[idx] = src[sidx]
    return out


def extend_z(xy, nz, hz, d_z):
    """The 3D form of Eq. (fun) is a 2D function times a Gaussian in z of
    width d_z.  Given a 2D field, return the (nz, ny, nx) product with the
    Gaussian exp(-z^2 / (2 d_z^2)) at z_k = -nz hz / 2 + k hz, divided by
    sqrt(hz sum_{k=1}^{nz-1} exp(-z_k^2 / d_z^2)) so that a 2D field normalised
    on its grid gives a 3D state normalised over the interior; the wall plane
    k = 0 is included (the caller zeroes it)."""
    xy = np.asarray(xy)
    z = -0.5 * nz * hz + np.arange(nz) * hz
    gz = np.exp(-0.5 * (z / d_z) ** 2)
    norm = np.sqrt(hz * np.sum(gz[1:] ** 2))
    out = np.empty((nz,) + xy.shape, dtype=np.complex128)
    for k in range(nz):
        out[k] = xy.astype(np.complex128) * (gz[k] / norm)
    return out


def _d1_fourth(f, axis, h):
    """First derivative along `axis` by the fourth-order central difference
    (-f[i+2] + 8 f[i+1] - 8 f[i-1] + f[i-2]) / (12 h), the field taken as
    zero beyond the grid (the walls)."""
    pad = [(0, 0)] * f.ndim
    pad[axis] = (2, 2)
    fp = np.pad(f, pad)
    n = f.shape[axis]

    def at(k):
        return np.take(fp, np.arange(2 + k, 2 + k + n), axis=axis)
    return (-at(2) + 8 * at(1) - 8 * at(-1) + at(-2)) / (12 * h)


def functional_fourth_order(p, psi):
    """Energy and chemical potential of Eqs. (e2d) / (e3d) in the rotating
    frame, E = integral of 1/2 |grad psi|^2 + V |psi|^2 + g/2 |psi|^4 -
    Omega psi* L_z psi with L_z = -i (x d/dy - y d/dx), and mu = E + g/2
    integral |psi|^4, per unit norm, with every derivative taken by the
    fourth-order central difference and integrals as h^d times plain sums.
    The continuum functional evaluated to O(h^4): the printed values of
    Table 1 are reproduced this way from the converged lattices (the
    library's own mu and E use the operators of the discrete step, whose
    O(h^2) terms grow with the phase gradients of fast rotation)."""
    psi = np.asarray(psi, dtype=np.complex128)
    dim = p.dim
    hs = (p.hz, p.hy, p.hx)[3 - dim:]
    ns = psi.shape
    axes = [-ns[k] * hs[k] / 2 + hs[k] * np.arange(ns[k]) for k in range(dim)]
    grids = np.meshgrid(*axes, indexing="ij")
    X, Y = grids[-1], grids[-2]
    V = 0.5 * (p.gamma ** 2 * X ** 2 + p.nu ** 2 * Y ** 2)
    if dim == 3:
        V = V + 0.5 * p.lam ** 2 * grids[0] ** 2
    dvol = float(np.prod(hs))
    dx = _d1_fourth(psi, dim - 1, p.hx)
    dy = _d1_fourth(psi, dim - 2, p.hy)
    grad2 = np.abs(dx) ** 2 + np.abs(dy) ** 2
    if dim == 3:
        grad2 = grad2 + np.abs(_d1_fourth(psi, 0, p.hz)) ** 2
    dens = np.abs(psi) ** 2
    norm = dens.sum() * dvol
    kin = 0.5 * grad2.sum() * dvol
    pot = (V * dens).sum() * dvol
    inter = 0.5 * p.g * (dens ** 2).sum() * dvol
    lz = (np.conj(psi) * (-1j) * (X * dy - Y * dx)).sum().real * dvol
    energy = (kin + pot + inter - p.omega * lz) / norm
    return {"energy": energy, "mu": energy + inter / norm, "lz": lz / norm, "norm": norm}


DENSITY_KINDS = ("full", "xy", "x", "y", "z", "cut_x", "cut_y", "cut_z")


def density(p, psi, kind):
    """The paper's density outputs (Sec. 3) from a state (ny, nx) or (nz,
    ny, nx): 'full' |psi|^2; 'xy' its integral over z; 'x', 'y', 'z' the
    integrals over the other axes; 'cut_x', 'cut_y', 'cut_z' the values along
    one axis through the centre indices of the others.  Integrals are h
    times plain sums."""
    d = np.abs(np.asarray(psi, dtype=np.complex128)) ** 2
    if d.ndim == 2:
        d = d[None]
    nz, ny, nx = d.shape
    hz = p.hz if nz > 1 else 1.0
    if kind == "full":
        return d if p.dim == 3 else d[0]
    if kind == "xy":
        return d.sum(axis=0) * hz
    if kind == "x":
        return d.sum(axis=(0, 1)) * p.hy * hz
    if kind == "y":
        return d.sum(axis=(0, 2)) * p.hx * hz
    if kind == "z":
        return d.sum(axis=(1, 2)) * p.hx * p.hy
    if kind == "cut_x":
        return d[nz // 2, ny // 2, :]
    if kind == "cut_y":
        return d[nz // 2, :, nx // 2]
    if kind == "cut_z":
        return d[:, ny // 2, nx // 2]
    raise ValueError(kind)


# ---------------------------------------------------------------------------
# Grids of different spacing and extent (the learned initial state).  The
# paper moves states between grids only by centred embedding on a common
# spacing (``embed``); a network that works in coordinates scaled to each
# condensate's size needs interpolation.  The interpolation is Keys' cubic
# convolution (R. G. Keys, "Cubic convolution interpolation for digital
# image processing", IEEE Trans. ASSP 29 (1981)) with a = -1/2, separable in
# x and y; samples beyond a grid are zero, as the walls are.


def keys_cubic(s):
    """Keys' interpolation kernel with a = -1/2:
    W(s) = 3/2 |s|^3 - 5/2 |s|^2 + 1 for |s| <= 1,
    W(s) = -1/2 |s|^3 + 5/2 |s|^2 - 4 |s| + 2 for 1 < |s| < 2, else 0."""
    s = np.abs(np.asarray(s, dtype=np.float64))
    inner = 1.5 * s ** 3 - 2.5 * s ** 2 + 1.0
    outer = -0.5 * s ** 3 + 2.5 * s ** 2 - 4.0 * s + 2.0
    return np.where(s <= 1.0, inner, np.where(s < 2.0, outer, 0.0))


_MASK64 = (1 << 64) - 1


def splitmix64(x):
    """Output of the SplitMix64 generator (Steele, Lea and Flood, 2014) for
    the state x (Python integers, modulo 2^64): the state advances by
    0x9E3779B97F4A7C15, then z = (z ^ z >> 30) * 0xBF58476D1CE4E5B9,
    z = (z ^ z >> 27) * 0x94D049BB133111EB, z ^ z >> 31."""
    z = (x + 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def splitmix_phase(seed, ny, nx):
    """The random number R(x, y) of Eq. (fun) on an ny x nx plane as the
    library's counter-based draw defines it (reading of the unspecified
    generator): R[j, i] = 2^-53 (splitmix64(seed XOR (j nx + i)) >> 11).
    Pure-Python integers, one point at a time."""
    out = np.empty((ny, nx), dtype=np.float64)
    for j in range(ny):
        for i in range(nx):
            out[j, i] = (splitmix64((seed ^ (j * nx + i)) & _MASK64) >> 11) * 2.0 ** -53
    return out


def resample(psi, h_src, shape, h, angle=0.0):
    """Interpolate the state psi (ny_s, nx_s) on its grid of spacings
    h_src = (hx_s, hy_s) onto a grid of `shape` (ny, nx) and spacings
    h = (hx, hy), both grids centred as the solver's (x_i = -n h / 2 + i h),
    sampling the source at the destination points rotated by `angle` about
    the origin: out(x, y) = f(cos a x - sin a y, sin a x + cos a y), with f
    the cubic-convolution interpolant sum_ij W((X - X_i)/hx_s) W((Y - Y_j)/hy_s)
    psi_ij over the source samples (zero beyond the source grid).  The
    destination walls (index 0) are zero."""
    src = np.asarray(psi, dtype=np.complex128)
    nys, nxs = src.shape
    ny, nx = shape
    hxs, hys = h_src
    hx, hy = h
    x = -0.5 * nx * hx + hx * np.arange(nx)
    y = -0.5 * ny * hy + hy * np.arange(ny)
    X, Y = np.meshgrid(x, y)
    ca, sa = np.cos(angle), np.sin(angle)
    XS = ca * X - sa * Y
    YS = sa * X + ca * Y
    u = (XS + 0.5 * nxs * hxs) / hxs  # continuous source indices
    v = (YS + 0.5 * nys * hys) / hys
    i0 = np.floor(u).astype(np.int64)
    j0 = np.floor(v).astype(np.int64)
    out = np.zeros((ny, nx), dtype=np.complex128)
    for b in range(-1, 3):
        js = j0 + b
        wy = keys_cubic(v - js)
        for a in range(-1, 3):
            is_ = i0 + a
            wx = keys_cubic(u - is_)
            ok = (is_ >= 0) & (is_ < nxs) & (js >= 0) & (js < nys)
            vals = np.where(ok, src[np.clip(js, 0, nys - 1), np.clip(is_, 0, nxs - 1)], 0.0)
            out += wx * wy * vals
    out[0, :] = 0
    out[:, 0] = 0
    return out


def angular_moments(psi, hx, hy, kmax):
    """M_k = hx hy sum_ij |psi_ij|^2 exp(i k phi_ij), phi = atan2(y_j, x_i),
    for k = 0..kmax (the angular Fourier components of the density about
    the trap centre).  A point at the origin has no angle: it enters M_0
    only."""
    d = np.abs(np.asarray(psi, dtype=np.complex128)) ** 2
    ny, nx = d.shape
    x = -0.5 * nx * hx + hx * np.arange(nx)
    y = -0.5 * ny * hy + hy * np.arange(ny)
    X, Y = np.meshgrid(x, y)
    phi = np.arctan2(Y, X)
    at_origin = (X == 0) & (Y == 0)
    out = []
    for k in range(kmax + 1):
        f = np.exp(1j * k * phi)
        if k > 0:
            f = np.where(at_origin, 0.0, f)
        out.append(hx * hy * np.sum(d * f))
    return np.array(out)
