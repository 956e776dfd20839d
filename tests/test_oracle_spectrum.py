"""Pins of the oracle's plane power spectrum (Sect. 3.2.2): Parseval's
theorem per plane, and a single plane wave landing on its two modes with the
closed-form power, for each choice of the plane normal."""
import numpy as np
import pytest


@pytest.mark.parametrize("normal", [0, 1, 2])
def test_parseval(orc, normal):
    dims = (6, 5, 4)
    f = np.random.default_rng(normal).standard_normal(int(np.prod(dims)))
    ps = orc.plane_power_spectrum(dims, f, normal)
    a1, a2 = [a for a in range(3) if a != normal]
    assert ps.shape == (dims[a2], dims[a1])
    assert abs(ps.sum() - dims[a1] * dims[a2] * (f ** 2).sum()) < 1e-9 * ps.sum()


@pytest.mark.parametrize("normal", [0, 1, 2])
def test_plane_wave_lands_on_its_modes(orc, normal):
    dims = (8, 6, 10)
    a1, a2 = [a for a in range(3) if a != normal]
    m1, m2 = 3, 2
    i, j, k = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    X = [i, j, k]
    f = np.cos(2 * np.pi * (m1 * X[a1] / dims[a1] + m2 * X[a2] / dims[a2])).transpose(2, 1, 0).reshape(-1)
    ps = orc.plane_power_spectrum(dims, f, normal)
    peak = dims[normal] * (dims[a1] * dims[a2] / 2.0) ** 2
    want = np.zeros_like(ps)
    want[m2, m1] = peak
    want[dims[a2] - m2, dims[a1] - m1] = peak
    assert np.allclose(ps, want, atol=1e-9 * peak)
