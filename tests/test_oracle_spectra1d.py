"""Pins of the 1D spectra (CPU only): single Fourier modes land in the bins
of their wavenumber components with the closed-form energy, and for random
fields every axis sums to the energy of each velocity component measured in
physical space (half the mean square of the inverse transform)."""
import numpy as np

from helpers import kept_mask
from paper_1807_01769_amd import inputs as I


def test_single_mode_3d(oracle_mod):
    n = 16
    h = n // 2 + 1
    u = np.zeros((3, n, n, h), np.complex128)
    # u_z = cos(3x + 2y - z): coefficient 1/2 at m = (3, 2, -1), kx > 0 half
    u[2, n - 1, 2, 3] = 0.5
    s = oracle_mod.spectra1d3d(u)
    want = np.zeros_like(s)
    for a, k in ((0, 3), (1, 2), (2, 1)):
        want[a, 2, k] = 0.25  # 1/2 <u_z^2> = 1/4
    assert np.array_equal(s, want)


def test_axes_sum_to_component_energy_3d(oracle_mod):
    n = 16
    u = I.random_solenoidal_3d(n, seed=51) * kept_mask(n, 3)[None]
    s = oracle_mod.spectra1d3d(u)
    for c in range(3):
        phys = oracle_mod.irfftn(u[c])
        ec = 0.5 * np.mean(phys ** 2)
        for a in range(3):
            assert abs(s[a, c].sum() - ec) <= 1e-13 * ec


def test_single_mode_and_sums_2d(oracle_mod):
    n = 32
    h = n // 2 + 1
    w = np.zeros((n, h), np.complex128)
    w[n - 3, 2] = 0.5  # w = cos(2x - 3y): u = 3/13 cos, v = 2/13 cos
    s = oracle_mod.spectra1d2d(w)
    k2 = 13.0
    eu, ev = 0.25 * (3 / k2) ** 2, 0.25 * (2 / k2) ** 2
    want = np.zeros_like(s)
    want[0, 0, 2] = want[1, 0, 3] = eu
    want[0, 1, 2] = want[1, 1, 3] = ev
    assert np.allclose(s, want, rtol=1e-14, atol=0)
    w = I.random_vorticity_2d(n, 52, lambda k: k * np.exp(-(k / 4.0) ** 2))
    s = oracle_mod.spectra1d2d(w)
    _, E, _ = oracle_mod.diag2d(w, 4)
    for a in range(2):
        assert abs(s[a].sum() - E) <= 1e-13 * E
