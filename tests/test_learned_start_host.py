"""Host-side logic of the learned start: Thomas-Fermi-scaled grids,
network features, symmetry images of a state and the phase-aligned
distance."""
import math

import numpy as np

from paper_1906_06327_amd import learned_start as LS


def test_tf_grid_spans_the_scaled_radius():
    p = LS.tf_instance(0.7, 400.0, 1.1, n=128)
    a, b = 1 - 0.49, 1.21 - 0.49
    mu = math.sqrt(400.0 * math.sqrt(a * b) / math.pi)
    r = math.sqrt(2 * mu / a)
    assert abs(p["hx"] * 128 - 2 * LS.BOX * r) < 1e-12
    assert p["hx"] == p["hy"] and p["nx"] == p["ny"] == 128


def test_features_are_the_scaled_coordinates_and_parameters():
    f = LS.features([(0.7, 316.22776601683796, 1.1), (0.9, 1000.0, 1.2)], n=16)
    assert f.shape == (2, 16, 16, 16)
    assert f[0, 3, 5, 0] == np.float32((5 - 8) / 8) and f[0, 3, 5, 1] == np.float32((3 - 8) / 8)
    assert np.allclose(f[0, ..., 2:5], 0.0, atol=1e-6)  # the centre of every range
    assert np.allclose(f[1, ..., 2:5], 1.0, atol=1e-6)  # the top of every range
    assert np.all(f[..., 5:] == 0)


def test_images_are_involutions_and_keep_the_density_pattern():
    rng = np.random.default_rng(0)
    n = 12
    psi = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    psi[0, :] = 0
    psi[:, 0] = 0
    ims = LS.images(psi)
    assert np.array_equal(ims[0], psi)
    for k in (1, 2, 3):
        again = LS.images(ims[k])[k]
        assert np.array_equal(again, psi)  # each symmetry applied twice is the identity
        assert np.all(ims[k][0, :] == 0) and np.all(ims[k][:, 0] == 0)  # walls stay walls
    # rotation by pi maps the point (i, j) to (n - i, n - j)
    assert ims[1][3, 4] == psi[n - 3, n - 4]
    assert ims[2][3, 4] == np.conj(psi[3, n - 4])


def test_phase_distance():
    rng = np.random.default_rng(1)
    a = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    assert LS.phase_distance(a, 3.0 * np.exp(0.7j) * a) < 1e-7
    e1 = np.zeros(4, complex)
    e2 = np.zeros(4, complex)
    e1[0], e2[1] = 1, 1j
    assert abs(LS.phase_distance(e1, e2) - math.sqrt(2)) < 1e-12
