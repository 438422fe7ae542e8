"""Pins of the 2D Boussinesq (stratified) reference (CPU only).

A single plane wave is an exact solution of the nonlinear equations (u is
normal to k and every gradient parallel to it, so the advection terms
vanish): an internal gravity wave oscillating at Omega = N |kx| / |k| and
decaying with exp(-nu k^2 t).  The inviscid tendency conserves kinetic plus
potential energy 1/2 <|u|^2> + 1/2 <b^2> / N^2, and with N^2 = 0, b = 0 the
system is the 2D solver."""
import numpy as np

from helpers import kept_mask
from paper_1807_01769_amd import inputs as I


def _plane_wave(n, mx, my, w0, b0):
    s = np.zeros((2, n, n // 2 + 1), np.complex128)
    s[0, my % n, mx] = w0
    s[1, my % n, mx] = b0
    return s


def _wave_exact(n, mx, my, w0, b0, N2, nu, t):
    k2 = float(mx * mx + my * my)
    om = np.sqrt(N2) * abs(mx) / np.sqrt(k2)
    d = np.exp(-nu * k2 * t)
    w = d * (w0 * np.cos(om * t) + 1j * mx * b0 / om * np.sin(om * t))
    b = d * (b0 * np.cos(om * t) + 1j * N2 * mx * w0 / (k2 * om) * np.sin(om * t))
    return _plane_wave(n, mx, my, w, b)


def test_plane_wave_tendency_is_the_linear_coupling(oracle_mod):
    n, N2 = 32, 4.0
    w0, b0 = 0.5 - 0.1j, 0.2j
    s = _plane_wave(n, 3, -2, w0, b0)
    t = oracle_mod.tendency2d_strat(s, N2)
    want = _plane_wave(n, 3, -2, 1j * 3 * b0, 1j * N2 * 3 * w0 / 13.0)
    assert np.abs(t - want).max() <= 1e-14


def test_plane_wave_step_converges_to_gravity_wave(oracle_mod):
    n, N2, nu, T = 32, 9.0, 1e-2, 1.0
    w0, b0 = 0.3, 0.1 + 0.05j
    s0 = _plane_wave(n, 2, 1, w0, b0)
    exact = _wave_exact(n, 2, 1, w0, b0, N2, nu, T)
    errs = []
    for m in (20, 40, 80):
        got = oracle_mod.step2d_strat(s0, nu, T / m, N2, m)
        errs.append(np.abs(got - exact).max())
    assert errs[-1] < 1e-7
    for a, b in zip(errs, errs[1:]):
        assert 13.0 < a / b < 19.0, errs


def test_inviscid_energy_conservation(oracle_mod):
    n, N2 = 32, 2.5
    w = I.random_vorticity_2d(n, 81, lambda k: k * np.exp(-(k / 4.0) ** 2))
    b = I.random_vorticity_2d(n, 82, lambda k: np.exp(-(k / 3.0) ** 2))
    s = np.stack([w, b]) * kept_mask(n, 2)[None]
    t = oracle_mod.tendency2d_strat(s, N2)
    kx = np.arange(n // 2 + 1)[None, :].astype(float)
    ky = np.fft.fftfreq(n, 1.0 / n)[:, None]
    k2 = kx ** 2 + ky ** 2
    k2[0, 0] = 1.0
    wgt = np.where(kx == 0, 1.0, 2.0) * kept_mask(n, 2)
    kin = np.sum(wgt * np.real(np.conj(s[0]) * t[0]) / k2)
    pot = np.sum(wgt * np.real(np.conj(s[1]) * t[1])) / N2
    scale = np.sum(wgt * np.abs(s[0] * t[0]) / k2) + np.sum(wgt * np.abs(s[1] * t[1])) / N2
    assert abs(kin + pot) <= 1e-13 * scale
    assert abs(kin) > 1e-3 * scale  # buoyancy really exchanges energy


def test_reduces_to_2d_solver(oracle_mod):
    n = 32
    w = I.tg_plus_noise_2d(n)
    s = np.stack([w, np.zeros_like(w)])
    t = oracle_mod.tendency2d_strat(s, 0.0)
    assert np.array_equal(t[0], oracle_mod.tendency2d(w))
    assert np.abs(t[1]).max() == 0.0
