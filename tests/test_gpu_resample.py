"""GPU parity of the grid-to-grid interpolation (sscn_resample) and the
angular density moments (sscn_angular_moments) against the oracle, at
small ragged sizes and at the sizes the learned initial state uses (the
network's 256 x 256 Thomas-Fermi frame to and from the 128..512 grids of
the batched instances)."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1906_06327_amd as P
    P.lib()
    return P


def field(seed, ny, nx):
    f = W.random_field(seed, (ny, nx))
    return f


CASES = [
    # (src ny, nx, hx, hy), (dst ny, nx, hx, hy), angle
    ((33, 47, 0.21, 0.17), (29, 52, 0.19, 0.23), 0.0),
    ((33, 47, 0.21, 0.17), (29, 52, 0.19, 0.23), 0.7),
    ((40, 40, 0.15, 0.15), (40, 40, 0.15, 0.15), math.pi / 2),
    ((20, 24, 0.3, 0.3), (90, 70, 0.1, 0.1), -2.1),      # destination far larger: zeros outside
    ((256, 256, 0.0931, 0.0931), (384, 384, 0.1, 0.1), 0.0),  # network frame -> instance grid
    ((512, 512, 0.1, 0.1), (256, 256, 0.1107, 0.1107), 0.4),  # instance grid -> rotated frame
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_resample_matches_oracle(P, prec, case):
    import torch
    (nys, nxs, hxs, hys), (ny, nx, hx, hy), ang = CASES[case]
    print(f"[gpu-resample] case {case} prec={prec} {nxs}x{nys} -> {nx}x{ny} angle {ang}", flush=True)
    f = field(70 + case, nys, nxs)
    dt = torch.complex128 if prec == 0 else torch.complex64
    src = torch.tensor(f, dtype=dt, device="cuda")
    dst = torch.full((ny, nx), complex(float("nan"), 0.0), dtype=dt, device="cuda")
    P.resample(src, (hxs, hys), dst, (hx, hy), ang)
    got = dst.cpu().numpy().astype(np.complex128)
    ref = O.resample(src.cpu().numpy().astype(np.complex128), (hxs, hys), (ny, nx), (hx, hy), ang)
    scale = max(np.max(np.abs(ref)), 1e-300)
    tol = 1e-13 if prec == 0 else 1e-6
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - ref)) <= tol * scale, np.max(np.abs(got - ref)) / scale
    assert np.all(got[0, :] == 0) and np.all(got[:, 0] == 0)


@pytest.mark.parametrize("prec", [0, 1])
def test_angular_moments_match_oracle(P, prec):
    import torch
    print(f"[gpu-resample] moments prec={prec}", flush=True)
    for (ny, nx, h) in ((64, 64, 0.2), (77, 101, 0.13), (384, 384, 0.1)):
        f = field(90 + nx, ny, nx)
        dt = torch.complex128 if prec == 0 else torch.complex64
        psi = torch.tensor(f, dtype=dt, device="cuda")
        out = P.angular_moments(psi, (h, h), 8)
        got = out.cpu().numpy()
        ref = O.angular_moments(psi.cpu().numpy().astype(np.complex128), h, h, 8)
        m0 = abs(ref[0])
        assert np.max(np.abs((got[:, 0] + 1j * got[:, 1]) - ref)) <= 1e-12 * m0
