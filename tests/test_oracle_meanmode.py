"""Pins of the mean mode (k = 0) in the 3D steps (CPU only).

A periodic pressure has no mean gradient, so the mean velocity U and mean
buoyancy B obey the unprojected linear terms: dU/dt = -f z x U + B z,
dB/dt = -N^2 U_z.  If u'(x, t) (with b') solves the equations with zero
mean, then U(t) + u'(x - X(t), t) solves them with the mean U(t), where
X(t) is the integral of U: the nonlinear terms see a uniform translation
(Galilean invariance), and the Coriolis and buoyancy terms of the mean
cancel against dU/dt.  In Fourier space the fluctuation only changes phase,
u'(k) exp(-i k.X(t)).  So a step of (mean + fluctuation) must equal the
closed-form mean plus the phase-shifted step of the fluctuation alone; the
time scheme breaks the symmetry only at fifth order in (k.U dt), far below
the tolerance here.  This fixes the mean-mode reading in the propagators and
the mean's part in the nonlinear terms independently of the oracle's code."""
import numpy as np
import pytest

from helpers import kmesh
from paper_1807_01769_amd import inputs as I


def mean_trajectory(U0, B0, f, N2, t):
    """Closed form of U(t), B(t) and X(t) = int_0^t U."""
    ux, uy, uz = U0
    c, s = np.cos(f * t), np.sin(f * t)
    U = np.array([c * ux + s * uy, c * uy - s * ux, 0.0])
    if f != 0:
        X = np.array([(ux * s + uy * (1 - c)) / f, (uy * s - ux * (1 - c)) / f, 0.0])
    else:
        X = np.array([ux * t, uy * t, 0.0])
    N = np.sqrt(N2)
    if N > 0:
        U[2] = uz * np.cos(N * t) + B0 * np.sin(N * t) / N
        B = B0 * np.cos(N * t) - N * uz * np.sin(N * t)
        X[2] = uz * np.sin(N * t) / N + B0 * (1 - np.cos(N * t)) / N2
    else:
        U[2] = uz + B0 * t
        B = B0
        X[2] = uz * t + B0 * t * t / 2
    return U, B, X


def shift(a, X, n):
    kx, ky, kz = kmesh(n, 3)
    return a * np.exp(-1j * (kx * X[0] + ky * X[1] + kz * X[2]))


def _run(oracle_mod, kind, f, N2, dt, steps):
    """(step of mean + fluctuation, closed-form mean + shifted step of the
    fluctuation, step of the fluctuation alone) after `steps` steps."""
    n, nu, power = 16, 0.01, 0.05
    U0, B0 = np.array([1.5, -1.0, 1.2]), 2.0
    u = I.random_solenoidal_3d(n, seed=301)
    if kind == "strat":
        s = np.concatenate([u, I.random_solenoidal_3d(n, seed=302)[2][None]])
        with_mean = s.copy()
        with_mean[:3, 0, 0, 0] = U0
        with_mean[3, 0, 0, 0] = B0
        got = oracle_mod.step3d_strat(with_mean, nu, dt, N2, steps, power=power, f=f)
        ref = oracle_mod.step3d_strat(s, nu, dt, N2, steps, power=power, f=f)
        bm = B0
    else:
        with_mean = u.copy()
        with_mean[:, 0, 0, 0] = U0
        if kind == "rot":
            got = oracle_mod.step3d_rot(with_mean, nu, dt, f, steps, power=power)
            ref = oracle_mod.step3d_rot(u, nu, dt, f, steps, power=power)
        else:
            got = oracle_mod.step3d(with_mean, nu, dt, steps, power=power)
            ref = oracle_mod.step3d(u, nu, dt, steps, power=power)
        bm = 0.0
    U, B, X = mean_trajectory(U0, bm, f, N2, dt * steps)
    want = shift(ref, X, n)
    want[:3, 0, 0, 0] = U
    if kind == "strat":
        want[3, 0, 0, 0] = B
    return got, want, ref


@pytest.mark.parametrize("kind,f,N2", [("plain", 0.0, 0.0), ("rot", 3.0, 0.0),
                                       ("strat", 0.0, 6.0), ("strat", 2.0, 6.0),
                                       ("strat", 2.5, 0.0)])
def test_mean_flow_translates_the_fluctuation(oracle_mod, kind, f, N2):
    got, want, ref = _run(oracle_mod, kind, f, N2, 2e-3, 20)
    scale = np.abs(want).max()
    # the mean really moves the fluctuation (phases up to ~0.3 rad)
    effect = np.abs(want[:, 1:] - ref[:, 1:]).max() / scale
    err = np.abs(got - want).max() / scale
    assert effect > 1e-2
    # the mean itself is the closed form to rounding
    assert np.abs(got[:, 0, 0, 0] - want[:, 0, 0, 0]).max() <= 1e-14
    # the rest agrees up to the time scheme's truncation: fourth order, so
    # halving the step (same end time) divides the difference by ~16
    got2, want2, _ = _run(oracle_mod, kind, f, N2, 1e-3, 40)
    err2 = np.abs(got2 - want2).max() / np.abs(want2).max()
    assert err <= 1e-9 and 12.0 <= err / err2 <= 20.0, (err, err2)
