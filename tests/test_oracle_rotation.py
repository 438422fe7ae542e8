"""Pins of the rotating-frame step (CPU only).

A single helical mode (i k x h = |k| h, so u x w = 0) is an exact solution:
u(t) = exp(-nu k^2 t + i sigma t) h with sigma = f kz / |k|, the inertial wave
the integrating factor reproduces to rounding.  With f = 0 the step is the
plain one.  A random field integrated with the Coriolis term written out as
-P(f z x u) and classic RK4 (numpy, nu = 0) agrees at fourth order, which
fixes the sign and the projection."""
import numpy as np

from helpers import kept_mask, kmesh
from paper_1807_01769_amd import inputs as I


def _helical(n, m, amp):
    k = np.array(m, float)
    kh = k / np.linalg.norm(k)
    a = np.array([0.0, 0.0, 1.0]) if abs(kh[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    e1 = np.cross(kh, a)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(kh, e1)
    h = (e1 - 1j * e2) / np.sqrt(2)  # khat x h = i h => i k x h = -|k| h
    u = np.zeros((3, n, n, n // 2 + 1), np.complex128)
    u[:, m[2] % n, m[1] % n, m[0]] = amp * h
    return u, h, kh


def test_helical_mode_is_exact_inertial_wave(oracle_mod):
    n, nu, f, dt, steps = 16, 0.01, 3.0, 0.05, 20
    m = (2, 1, 3)
    u0, h, kh = _helical(n, m, 0.4)
    assert np.abs(oracle_mod.tendency3d(u0)).max() < 1e-15
    u = oracle_mod.step3d_rot(u0, nu, dt, f, steps)
    k2 = float(np.dot(m, m))
    sigma = f * m[2] / np.sqrt(k2)
    T = dt * steps
    # khat x h = i h, so E(t) h = exp(-nu k^2 t) (cos - i sin)(sigma t) h
    want = u0 * np.exp(-nu * k2 * T - 1j * sigma * T)
    assert np.abs(u - want).max() <= 1e-14
    assert abs(sigma * T) > 1.0  # several radians: the phase is really tested


def test_f_zero_is_the_plain_step(oracle_mod):
    u0 = I.random_solenoidal_3d(16, seed=101)
    a = oracle_mod.step3d_rot(u0, 0.01, 2e-3, 0.0, 3, power=0.2)
    b = oracle_mod.step3d(u0, 0.01, 2e-3, 3, power=0.2)
    assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max()


def test_coriolis_written_out_agrees(oracle_mod):
    n, f, dt, steps = 16, 2.0, 1e-3, 10
    u0 = I.random_solenoidal_3d(n, seed=102) * kept_mask(n, 3)[None]
    u0[:, 0, 0, 0] = [0.3, -0.2, 0.25]  # a mean flow (k2 := 1 below: P = I on it)
    kx, ky, kz = kmesh(n, 3)
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    k2[k2 == 0] = 1.0
    mask = kept_mask(n, 3)[None]

    def rhs(u):
        c = np.stack([-u[1], u[0], np.zeros_like(u[0])])  # z x u
        kc = (kx * c[0] + ky * c[1] + kz * c[2]) / k2
        pc = c - np.stack([kx, ky, kz]) * kc  # projection
        return (oracle_mod.tendency3d(u) - f * pc) * mask

    u = u0.copy()
    for _ in range(steps):
        a1 = rhs(u)
        a2 = rhs(u + 0.5 * dt * a1)
        a3 = rhs(u + 0.5 * dt * a2)
        a4 = rhs(u + dt * a3)
        u = u + dt / 6 * (a1 + 2 * a2 + 2 * a3 + a4)
    got = oracle_mod.step3d_rot(u0, 0.0, dt, f, steps)
    ref_norot = oracle_mod.step3d(u0, 0.0, dt, steps)
    err = np.abs(got - u).max() / np.abs(u).max()
    effect = np.abs(ref_norot - u).max() / np.abs(u).max()
    assert effect > 1e-3
    assert err < 1e-9, (err, effect)


def test_rk2_helical_and_f_zero(oracle_mod):
    n, nu, f, dt, steps = 16, 0.01, 3.0, 0.05, 20
    m = (2, 1, 3)
    u0, h, kh = _helical(n, m, 0.4)
    u = oracle_mod.step3d_rot(u0, nu, dt, f, steps, scheme=2)
    k2 = float(np.dot(m, m))
    T = dt * steps
    want = u0 * np.exp(-nu * k2 * T - 1j * f * m[2] / np.sqrt(k2) * T)
    assert np.abs(u - want).max() <= 1e-14
    r = I.random_solenoidal_3d(16, seed=103)
    a = oracle_mod.step3d_rot(r, 0.01, 2e-3, 0.0, 3, scheme=2)
    b, _ = oracle_mod.step3d_ex(r, 0.01, 2e-3, 3, scheme=2)
    assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max()


def _numpy_umax(u, n):
    # numpy's irfftn divides by n^3; the state's inverse is unscaled
    phys = np.fft.irfftn(u[:3] * kept_mask(n, 3)[None], s=(n, n, n), axes=(1, 2, 3)) * n ** 3
    return np.abs(phys).max()


def test_cfl_steps_rotating(oracle_mod):
    """Adaptive steps: each step's size from numpy's velocity maximum of the
    step's initial state, then the fixed-step rotating step with that size."""
    n, cfl, f = 16, 0.5, 3.0
    u0 = I.random_solenoidal_3d(n, seed=108)
    got, t = oracle_mod.step3d_rot(u0, 0.01, 1.0, f, 2, power=0.1, cfl=cfl, return_time=True)
    u, tt = u0.copy(), 0.0
    for _ in range(2):
        dt = cfl * (2 * np.pi / n) / _numpy_umax(u, n)
        u = oracle_mod.step3d_rot(u, 0.01, dt, f, 1, power=0.1)
        tt += dt
    assert abs(t - tt) <= 1e-14 * tt
    assert np.abs(got - u).max() <= 1e-13 * np.abs(u).max()
    # a CFL bound above the step: the fixed steps exactly
    fixed, t3 = oracle_mod.step3d_rot(u0, 0.01, 1e-3, f, 3, cfl=100.0, return_time=True)
    assert abs(t3 - 3e-3) < 1e-18
    assert np.array_equal(fixed, oracle_mod.step3d_rot(u0, 0.01, 1e-3, f, 3))
