"""Host-side logic of the learned start over the batched workload's ranges:
the network frame of an instance, the features, the canonical orientation of
a lattice whose orientation the trap leaves free, and the symmetry images of
a target."""
import math

import numpy as np
import pytest

from paper_1906_06327_amd import learned_start_c4 as L4


def test_frame_spans_the_scaled_radius():
    c = dict(omega=0.8, g=1200.0, nu=1.1)
    a, b = 1 - 0.64, 1.21 - 0.64
    mu = math.sqrt(1200.0 * math.sqrt(a * b) / math.pi)
    r = math.sqrt(2 * mu / a)
    assert abs(L4.frame_h(c) * L4.N_NET - 2 * L4.BOX * r) < 1e-12
    fi = L4.frame_instance(dict(c, gamma=1.0))
    assert fi["nx"] == fi["ny"] == L4.N_NET and fi["hx"] == fi["hy"] == L4.frame_h(c)
    assert fi["precision"] == 1 and fi["mode"] == 0


def test_features_are_the_frame_coordinates_and_scaled_parameters():
    lo = dict(omega=L4.RANGES["omega"][0], g=L4.RANGES["g"][0], nu=L4.RANGES["nu"][0])
    mid = dict(omega=sum(L4.RANGES["omega"]) / 2, g=math.sqrt(L4.RANGES["g"][0] * L4.RANGES["g"][1]),
               nu=sum(L4.RANGES["nu"]) / 2)
    f = L4.features([lo, mid], n=8)
    assert f.shape == (2, 8, 8, 16)
    assert f[0, 2, 5, 0] == np.float32((5 - 4) * 2 / 8) and f[0, 2, 5, 1] == np.float32((2 - 4) * 2 / 8)
    assert np.allclose(f[0, ..., 2:5], -1.0, atol=1e-6)  # the bottom of every range
    assert np.allclose(f[1, ..., 2:5], 0.0, atol=1e-6)   # the centre (log scale for g)
    assert np.all(f[..., 5:] == 0)


@pytest.mark.parametrize("k,theta", [(2, 0.3), (3, -0.5), (6, 0.2)])
def test_canonical_angle_recovers_the_orientation_of_the_dominant_order(k, theta):
    m = np.zeros(9, complex)
    m[0] = 1.0
    m[k] = 0.4 * np.exp(1j * k * theta)  # dominant order k at orientation theta
    m[(k % 8) + 1 if (k % 8) + 1 != k else 2] += 0.05
    ang = L4.canonical_angle(m, nu=1.0)
    # defined modulo 2 pi / k
    d = (ang - theta) * k / (2 * math.pi)
    assert abs(d - round(d)) < 1e-12
    assert L4.canonical_angle(m, nu=L4.NU_ISO) == 0.0  # anisotropic trap: orientation fixed


def test_images_are_the_symmetries_of_the_rotating_problem():
    torch = pytest.importorskip("torch")
    n = 10
    rng = np.random.default_rng(3)
    t = torch.tensor(rng.standard_normal((n, n, 2)), dtype=torch.float32)
    t[0, :] = 0
    t[:, 0] = 0
    ims = L4.images(t)
    assert ims.shape == (4, n, n, 2)
    assert torch.equal(ims[0], t)
    # rotation by pi: (i, j) -> (n - i, n - j); reflections with conjugation
    assert torch.equal(ims[1][3, 4], t[n - 3, n - 4])
    assert ims[2][3, 4, 0] == t[3, n - 4, 0] and ims[2][3, 4, 1] == -t[3, n - 4, 1]
    assert ims[3][3, 4, 0] == t[n - 3, 4, 0] and ims[3][3, 4, 1] == -t[n - 3, 4, 1]
    for k in (1, 2, 3):  # each an involution that keeps the walls
        assert torch.equal(L4.images(ims[k])[k], t)
        assert torch.all(ims[k][0, :] == 0) and torch.all(ims[k][:, 0] == 0)
