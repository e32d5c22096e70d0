"""Oracle for the SSCN rotating Gross-Pitaevskii solver (FP64, CPU).

TEST INFRASTRUCTURE ONLY.  A plain, slow, obviously-correct implementation of
what the GPU path computes, written from the paper (Kumar, Loncar,
Muruganandam, Adhikari, Balaz, "C and Fortran OpenMP programs for rotating
Bose-Einstein condensates").  It shares no code with the GPU library and is
used only by the tests, the smoke check and the benchmark's CPU baseline.

The arithmetic lives in ``sscn_oracle.c``; this module only marshals numpy
arrays through ctypes.  Arrays are complex128 with shape (ny, nx) in 2D and
(nz, ny, nx) in 3D (x fastest), index 0 of every axis being the wall.
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
                ("energy_full", ctypes.c_double), ("rms_x", ctypes.c_double),
                ("rms_y", ctypes.c_double), ("rms_z", ctypes.c_double),
                ("rms_r", ctypes.c_double), ("max_density", ctypes.c_double),
                ("sums", ctypes.c_double * 14)]


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


OBS_KEYS = ("norm", "mu", "energy", "mu_full", "energy_full", "rms_x",
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
