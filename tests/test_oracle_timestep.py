"""Pins of the RK2 scheme and the CFL step (CPU only).

RK2 is the Lawson (integrating-factor) midpoint rule: second order on a
scalar ODE with closed form, exact on fields whose nonlinear term vanishes.
The CFL step is dt_n = min(dt_max, cfl (L/n) / max |u_c|) with the maximum of
the physical velocity, checked against numpy's own inverse FFT of the state."""
import numpy as np

from helpers import kept_mask
from paper_1807_01769_amd import inputs as I


def test_lawson_rk2_scalar_order2(oracle_mod):
    lam, y0, T = 2.0, 0.7, 1.0
    exact = lam / (1 + (lam / y0 - 1) * np.exp(lam * T))
    errs = [abs(oracle_mod.lawson_scalar2(lam, y0, T / m, m) - exact) for m in (16, 32, 64)]
    assert errs[0] < 1e-2
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.5
    assert oracle_mod.lawson_scalar2(lam, 0.0, 0.3, 3) == 0.0


def test_rk2_exact_decays(oracle_mod):
    u0 = I.abc_flow_3d(16)
    u, t = oracle_mod.step3d_ex(u0, 0.01, 0.2, 4, scheme=2)
    assert abs(t - 0.8) < 1e-15
    assert np.abs(u - u0 * np.exp(-0.01 * 0.8)).max() <= 1e-15
    w0 = I.taylor_green_2d(32)
    w, t = oracle_mod.step2d_ex(w0, 0.05, 0.1, 3, scheme=2)
    assert np.abs(w - w0 * np.exp(-0.05 * 2 * 0.3)).max() <= 1e-15


def test_rk4_ex_equals_step3d(oracle_mod):
    u0 = I.random_solenoidal_3d(16, seed=61)
    a = oracle_mod.step3d(u0, 0.01, 2e-3, 3, power=0.1)
    b, t = oracle_mod.step3d_ex(u0, 0.01, 2e-3, 3, power=0.1)
    assert np.array_equal(a, b) and abs(t - 6e-3) < 1e-18


def _numpy_umax3d(u, n):
    full = np.zeros((3, n, n, n // 2 + 1), np.complex128)
    full[:] = u * kept_mask(n, 3)[None]
    # numpy's irfftn divides by n^3; the state's inverse is unscaled
    phys = np.fft.irfftn(full, s=(n, n, n), axes=(1, 2, 3)) * n ** 3
    return np.abs(phys).max()


def test_cfl_step_size_3d(oracle_mod):
    n, cfl = 16, 0.5
    u0 = I.random_solenoidal_3d(n, seed=62)
    um = _numpy_umax3d(u0, n)
    assert abs(oracle_mod.umax(u0, 3) - um) <= 1e-13 * um
    dt = cfl * (2 * np.pi / n) / um
    u1, t = oracle_mod.step3d_ex(u0, 0.01, 1.0, 1, cfl=cfl)
    assert abs(t - dt) <= 1e-15 * dt
    ref = oracle_mod.step3d(u0, 0.01, dt, 1)
    assert np.array_equal(u1, ref)
    # two steps: the second step size comes from the new state
    u2, t2 = oracle_mod.step3d_ex(u0, 0.01, 1.0, 2, cfl=cfl)
    dt2 = cfl * (2 * np.pi / n) / _numpy_umax3d(u1, n)
    assert abs(t2 - (dt + dt2)) <= 1e-14 * t2
    # a CFL bound above dt_max: the fixed step
    u3, t3 = oracle_mod.step3d_ex(u0, 0.01, 1e-3, 3, cfl=100.0)
    assert abs(t3 - 3e-3) < 1e-18
    assert np.array_equal(u3, oracle_mod.step3d(u0, 0.01, 1e-3, 3))


def test_cfl_step_size_2d(oracle_mod):
    n, cfl = 32, 0.8
    w0 = I.random_vorticity_2d(n, 63, lambda k: k * np.exp(-(k / 4.0) ** 2))
    kx = np.arange(n // 2 + 1)[None, :].astype(float)
    ky = np.fft.fftfreq(n, 1.0 / n)[:, None]
    k2 = kx ** 2 + ky ** 2
    k2[0, 0] = 1.0
    wm = w0 * kept_mask(n, 2)
    u = np.fft.irfft2(1j * ky * wm / k2, s=(n, n)) * n * n
    v = np.fft.irfft2(-1j * kx * wm / k2, s=(n, n)) * n * n
    um = max(np.abs(u).max(), np.abs(v).max())
    assert abs(oracle_mod.umax(w0, 2) - um) <= 1e-13 * um
    w1, t = oracle_mod.step2d_ex(w0, 1e-3, 1.0, 1, scheme=2, cfl=cfl)
    assert abs(t - cfl * (2 * np.pi / n) / um) <= 1e-15 * t
