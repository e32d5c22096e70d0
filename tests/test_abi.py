"""Host-side checks of the C ABI (no GPU needed).

The library must load and export every symbol include/sscn.h declares, and
sscn_init must reject ill-posed parameters before it touches the device.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sscn.h")


def _lib():
    import paper_1906_06327_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_1906_06327_amd import build
        build.build()
    return P


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sscn_[a-z_]+)\s*\(", text)))


def test_header_declarations_match_binding():
    P = _lib()
    assert declared_symbols() == sorted(P.EXPORTS)


def test_library_exports_every_declared_symbol():
    P = _lib()
    L = P.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_strerror_codes():
    P = _lib()
    L = P.lib()
    assert L.sscn_strerror(0) == b"ok"
    assert L.sscn_strerror(-2).startswith(b"omega")
    assert L.sscn_strerror(-99) == b"unknown error"


BASE = dict(dim=2, nx=64, ny=64, hx=0.1, hy=0.1, gamma=1.0, nu=1.0, g=10.0,
            omega=0.5, dt=1e-3, mode=0, precision=0)


@pytest.mark.parametrize("over,code", [
    (dict(omega=1.0), -2),                  # Omega >= min(gamma, nu)
    (dict(omega=-1.2, nu=1.1), -2),
    (dict(dim=4), -1),
    (dict(nx=2), -1),
    (dict(dt=0.0), -1),
    (dict(hx=-0.1), -1),
    (dict(mode=2), -1),
    (dict(precision=3), -1),
    # real time with dt*Omega*max|y|/(2h) >= 1: not diagonally dominant
    (dict(mode=1, dt=0.05, omega=0.9, nx=256, ny=256), -3),
])
def test_init_rejects_bad_parameters_before_touching_the_device(over, code):
    P = _lib()
    p = P.make_params(**{**BASE, **over})
    h = ctypes.c_void_p()
    # a dummy non-null state pointer: validation must fail before any use
    rc = P.lib().sscn_init(ctypes.byref(p), ctypes.c_void_p(16), None, ctypes.byref(h))
    assert rc == code
    assert not h.value
    assert len(P.lib().sscn_last_error()) > 0


def test_null_arguments_are_rejected():
    P = _lib()
    L = P.lib()
    p = P.make_params(**BASE)
    h = ctypes.c_void_p()
    assert L.sscn_init(ctypes.byref(p), None, None, ctypes.byref(h)) == -1
    assert L.sscn_step(None, 1) == -1
    assert L.sscn_get_state(None, None) == -1
    L.sscn_destroy(None)  # no-op


def test_fused_tile_launchers_are_local_to_their_compilation():
    """The fused step is compiled once per tile shape (sscn_kernels.hip,
    parts 2, 4 and 5) with launchers of the same names; they must have internal
    linkage, or the linker keeps one shape's instances for both and the
    second shape silently runs the first shape's kernel (the results stay
    right, the work doubles)."""
    import shutil
    import subprocess
    if shutil.which("nm") is None:
        pytest.skip("nm not available")
    P = _lib()
    out = subprocess.run(["nm", "-C", "--defined-only", "--extern-only", P.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    assert "launch_fused_narrow<double, true>" in out  # the dispatch targets are exported
    assert "launch_fused_small<double, true>" in out
    for name in ("launch_fused_tile<", "go_fused<", "allow_fused_lds_tile<", "allow_fused_lds<"):
        assert name not in out, name
