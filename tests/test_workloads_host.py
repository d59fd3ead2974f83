"""The skewed generators against the closed forms of the densities they
sample (Plummer sphere, Kuzmin disk): the empirical mass fraction inside a
radius must match the cumulative mass of the profile."""
import numpy as np

import workloads as W


def test_plummer_cumulative_mass():
    a = 0.01
    P = W.plummer(400_000, seed=1, a=a, x_max=1.0 - 1e-12)
    r = np.linalg.norm(P - 0.5, axis=1)
    for rr in (0.25 * a, a, 3 * a, 10 * a):
        want = rr ** 3 / (rr ** 2 + a ** 2) ** 1.5
        assert abs((r < rr).mean() - want) < 4e-3
    # isotropic: the mean direction is near zero
    assert np.all(np.abs((P - 0.5).mean(axis=0)) < 0.01 * r.mean() * 10)


def test_kuzmin_cumulative_mass_and_plane():
    a = 0.02
    K = W.kuzmin(400_000, seed=2, a=a, x_max=1.0 - 1e-9)
    assert np.all(K[:, 2] == 0.5)
    R = np.linalg.norm(K[:, :2] - 0.5, axis=1)
    for rr in (0.5 * a, a, 4 * a, 30 * a):
        want = 1.0 - a / np.sqrt(rr ** 2 + a ** 2)
        assert abs((R < rr).mean() - want) < 4e-3


def test_truncation_bounds_the_radius():
    a = 0.01
    P = W.plummer(100_000, seed=3, a=a, x_max=0.999)
    r_max = a / np.sqrt(0.999 ** (-2.0 / 3.0) - 1.0)
    assert np.linalg.norm(P - 0.5, axis=1).max() <= r_max * (1 + 1e-12)
    K = W.kuzmin(100_000, seed=4, a=a, x_max=0.999)
    R_max = a * np.sqrt(1.0 / (1.0 - 0.999) ** 2 - 1.0)
    assert np.linalg.norm(K[:, :2] - 0.5, axis=1).max() <= R_max * (1 + 1e-12)
