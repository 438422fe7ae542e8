"""Pins of the 3D Boussinesq (stratified) oracle (CPU only).

* The closed-form propagator equals the matrix exponential (scipy) of the
  linear operator built from its definition, (u, b) -> (P[b z] - nu k^2 u,
  -N^2 uz - nu k^2 b), for random 4-vectors at every kept mode.
* The buoyancy flux equals numpy's transforms of the physical product u b and,
  for a uniform flow U, -i (k.U) b_hat; the velocity part is the 3D tendency;
  the nonlinear terms conserve kinetic energy and buoyancy variance.
* A plane internal gravity wave (velocity along the poloidal direction) is an
  exact solution: the nonlinear terms vanish and the step reproduces the wave
  of frequency N |k_h| / |k| to rounding (RK4 and RK2).
* With b = 0 and N^2 = 0 the step is the plain 3D step (RK4 and RK2).
* The linear terms written out and integrated with classic RK4 (numpy) agree
  at fourth order, which fixes their signs and the projection of b z."""
import numpy as np
import pytest
from scipy.linalg import expm

from helpers import kept_mask, kept_weight, kmesh
from paper_1807_01769_amd import inputs as I


def _state(n, seed, bscale=1.0):
    u = I.random_solenoidal_3d(n, seed=seed)
    b = I.random_solenoidal_3d(n, seed=seed + 1)[2] * bscale
    return np.concatenate([u, b[None]]) * kept_mask(n, 3)[None]


@pytest.mark.parametrize("N2", [0.0, 2.5, 40.0])
def test_propagator_is_matrix_exponential(oracle_mod, N2):
    n, nu, t = 8, 0.01, 0.7
    rng = np.random.default_rng(5)
    s = (rng.standard_normal((4, n, n, n // 2 + 1)) + 1j * rng.standard_normal((4, n, n, n // 2 + 1)))
    s *= kept_mask(n, 3)[None]
    got = oracle_mod.strat_propagate(s, nu, N2, t)
    kx, ky, kz = kmesh(n, 3)
    mask = kept_mask(n, 3)
    worst, scale = 0.0, 0.0
    for idx in zip(*np.nonzero(mask)):
        k = np.array([kx[idx], ky[idx], kz[idx]])
        k2 = k @ k
        # a periodic pressure has no mean gradient: nothing projects the mean
        P = np.eye(3) - np.outer(k, k) / k2 if k2 > 0 else np.eye(3)
        A = np.zeros((4, 4))
        A[:3, 3] = P @ np.array([0.0, 0.0, 1.0])
        A[3, 2] = -N2
        A -= nu * k2 * np.eye(4)
        want = expm(t * A) @ s[(slice(None),) + idx]
        worst = max(worst, np.abs(got[(slice(None),) + idx] - want).max())
        scale = max(scale, np.abs(want).max())
    assert worst <= 1e-14 * scale, (worst, scale)


def test_buoyancy_flux_matches_numpy_product(oracle_mod):
    n = 16
    s = _state(n, 31)
    out = oracle_mod.tendency3d_strat(s)
    assert np.abs(out[:3] - oracle_mod.tendency3d(s[:3])).max() == 0.0
    sh = (n, n, n)
    phys = [np.fft.irfftn(s[c], s=sh, axes=(0, 1, 2)) * n ** 3 for c in range(4)]
    kx, ky, kz = kmesh(n, 3)
    fl = [np.fft.rfftn(phys[c] * phys[3]) / n ** 3 for c in range(3)]
    want = -1j * (kx * fl[0] + ky * fl[1] + kz * fl[2])
    want *= kept_mask(n, 3)
    want[0, 0, 0] = 0
    assert np.abs(out[3] - want).max() <= 1e-13 * np.abs(want).max()


def test_uniform_flow_translates_buoyancy(oracle_mod):
    n = 16
    s = np.zeros((4, n, n, n // 2 + 1), np.complex128)
    U = np.array([0.3, -0.2, 0.5])
    s[:3, 0, 0, 0] = U
    s[3] = _state(n, 41)[3]
    out = oracle_mod.tendency3d_strat(s)
    kx, ky, kz = kmesh(n, 3)
    want = -1j * (kx * U[0] + ky * U[1] + kz * U[2]) * s[3]
    assert np.abs(out[3] - want).max() <= 1e-14 * np.abs(want).max()
    assert np.abs(out[:3]).max() <= 1e-15


def test_nonlinear_terms_conserve(oracle_mod):
    n = 16
    s = _state(n, 51)
    out = oracle_mod.tendency3d_strat(s)
    w = kept_weight(n, 3)
    ek = np.sum(w * np.real(np.conj(s[:3]) * out[:3]))
    eb = np.sum(w * np.real(np.conj(s[3]) * out[3]))
    scale = np.sum(w * np.abs(s) * np.abs(out))
    assert abs(ek) <= 1e-13 * scale and abs(eb) <= 1e-13 * scale


def _wave(n, m, A, B):
    k = np.array(m, float)
    kh = k / np.linalg.norm(k)
    q = np.array([0.0, 0.0, 1.0]) - kh * kh[2]
    ep = q / np.linalg.norm(q)
    s = np.zeros((4, n, n, n // 2 + 1), np.complex128)
    s[:3, m[2] % n, m[1] % n, m[0]] = A * ep
    s[3, m[2] % n, m[1] % n, m[0]] = B
    return s, ep, np.linalg.norm(q)


@pytest.mark.parametrize("scheme", [4, 2])
def test_plane_gravity_wave_is_exact(oracle_mod, scheme):
    n, nu, N2, dt, steps = 16, 0.01, 6.0, 0.05, 20
    m = (2, 1, 3)
    A, B = 0.3 - 0.1j, 0.2 + 0.4j
    s0, ep, g = _wave(n, m, A, B)
    assert np.abs(oracle_mod.tendency3d_strat(s0)).max() <= 1e-15
    got = oracle_mod.step3d_strat(s0, nu, dt, N2, steps, scheme=scheme)
    T, N = dt * steps, np.sqrt(N2)
    om = N * g
    d = np.exp(-nu * float(np.dot(m, m)) * T)
    sA = d * (A * np.cos(om * T) + B / N * np.sin(om * T))
    sB = d * (B * np.cos(om * T) - N * A * np.sin(om * T))
    want, _, _ = _wave(n, m, sA, sB)
    assert np.abs(got - want).max() <= 1e-14


@pytest.mark.parametrize("scheme", [4, 2])
def test_no_buoyancy_is_the_plain_step(oracle_mod, scheme):
    n = 16
    s = _state(n, 61)
    s[3] = 0
    got = oracle_mod.step3d_strat(s, 0.01, 2e-3, 0.0, 3, power=0.05, scheme=scheme)
    ref, _ = oracle_mod.step3d_ex(s[:3], 0.01, 2e-3, 3, scheme=scheme, power=0.05)
    assert np.abs(got[3]).max() == 0.0
    assert np.abs(got[:3] - ref).max() <= 1e-14 * np.abs(ref).max()


def test_linear_terms_written_out_agree(oracle_mod):
    n, N2, dt, steps = 16, 4.0, 1e-3, 10
    s0 = _state(n, 71)
    s0[:, 0, 0, 0] = [0.3, -0.2, 0.25, 0.4]  # a mean velocity and buoyancy (k2 := 1: P = I)
    kx, ky, kz = kmesh(n, 3)
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    k2[k2 == 0] = 1.0
    mask = kept_mask(n, 3)[None]

    def rhs(s):
        f = np.stack([np.zeros_like(s[3]), np.zeros_like(s[3]), s[3]])  # b z
        kf = (kx * f[0] + ky * f[1] + kz * f[2]) / k2
        pf = f - np.stack([kx, ky, kz]) * kf
        lin = np.concatenate([pf, (-N2 * s[2])[None]])
        return (oracle_mod.tendency3d_strat(s) + lin) * mask

    s = s0.copy()
    for _ in range(steps):
        a1 = rhs(s)
        a2 = rhs(s + 0.5 * dt * a1)
        a3 = rhs(s + 0.5 * dt * a2)
        a4 = rhs(s + dt * a3)
        s = s + dt / 6 * (a1 + 2 * a2 + 2 * a3 + a4)
    got = oracle_mod.step3d_strat(s0, 0.0, dt, N2, steps)
    plain = oracle_mod.step3d(s0[:3], 0.0, dt, steps)
    err = np.abs(got - s).max() / np.abs(s).max()
    effect = np.abs(plain - s[:3]).max() / np.abs(s).max()
    assert effect > 1e-3
    assert err < 1e-9, (err, effect)


def test_cfl_steps_stratified(oracle_mod):
    """Adaptive steps take their size from the velocity part only (numpy's
    maximum of the first three fields), then the fixed-step Boussinesq step."""
    n, cfl, N2 = 16, 0.5, 4.0
    s0 = _state(n, 81)
    got, t = oracle_mod.step3d_strat(s0, 0.01, 1.0, N2, 2, scheme=2, cfl=cfl, return_time=True)
    s, tt = s0.copy(), 0.0
    for _ in range(2):
        phys = np.fft.irfftn(s[:3] * kept_mask(n, 3)[None], s=(n, n, n), axes=(1, 2, 3)) * n ** 3
        dt = cfl * (2 * np.pi / n) / np.abs(phys).max()
        s = oracle_mod.step3d_strat(s, 0.01, dt, N2, 1, scheme=2)
        tt += dt
    assert abs(t - tt) <= 1e-14 * tt
    assert np.abs(got - s).max() <= 1e-13 * np.abs(s).max()
    fixed, t3 = oracle_mod.step3d_strat(s0, 0.01, 1e-3, N2, 3, cfl=100.0, return_time=True)
    assert abs(t3 - 3e-3) < 1e-18
    assert np.array_equal(fixed, oracle_mod.step3d_strat(s0, 0.01, 1e-3, N2, 3))


def _solenoidal_random(n, seed):
    """Random half-spectrum (u, b) with u projected to be solenoidal per mode."""
    rng = np.random.default_rng(seed)
    sh = (4, n, n, n // 2 + 1)
    s = (rng.standard_normal(sh) + 1j * rng.standard_normal(sh)) * kept_mask(n, 3)[None]
    kx, ky, kz = kmesh(n, 3)
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    k2[k2 == 0] = 1.0
    kd = (kx * s[0] + ky * s[1] + kz * s[2]) / k2
    s[0] -= kx * kd
    s[1] -= ky * kd
    s[2] -= kz * kd
    return s


@pytest.mark.parametrize("N2,f", [(2.5, 3.0), (0.0, 2.0), (40.0, 0.7)])
def test_rotating_stratified_propagator_is_matrix_exponential(oracle_mod, N2, f):
    """(u, b) -> (-f P(z x u) + P(b z) - nu k^2 u, -N^2 uz - nu k^2 b) on
    solenoidal velocities, exponentiated by scipy at every kept mode."""
    n, nu, t = 8, 0.01, 0.7
    s = _solenoidal_random(n, 11)
    got = oracle_mod.stratrot_propagate(s, nu, N2, f, t)
    kx, ky, kz = kmesh(n, 3)
    Z = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 0.0]])  # z x u
    worst, scale = 0.0, 0.0
    for idx in zip(*np.nonzero(kept_mask(n, 3))):
        k = np.array([kx[idx], ky[idx], kz[idx]])
        k2 = k @ k
        # the mean mode: no pressure gradient, so no projection
        P = np.eye(3) - np.outer(k, k) / k2 if k2 > 0 else np.eye(3)
        A = np.zeros((4, 4))
        A[:3, :3] = -f * P @ Z
        A[:3, 3] = P @ np.array([0.0, 0.0, 1.0])
        A[3, 2] = -N2
        A -= nu * k2 * np.eye(4)
        want = expm(t * A) @ s[(slice(None),) + idx]
        worst = max(worst, np.abs(got[(slice(None),) + idx] - want).max())
        scale = max(scale, np.abs(want).max())
    assert worst <= 1e-13 * scale, (worst, scale)


def test_rotating_stratified_reductions(oracle_mod):
    n = 16
    s = _solenoidal_random(n, 13)
    # f = 0: the stratified propagator
    a = oracle_mod.stratrot_propagate(s, 0.01, 2.5, 0.0, 0.3)
    b = oracle_mod.strat_propagate(s, 0.01, 2.5, 0.3)
    assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max()
    # N^2 = 0 and b = 0: the rotating step
    u = _state(n, 91)
    u[3] = 0
    got = oracle_mod.step3d_strat(u, 0.01, 2e-3, 0.0, 3, f=2.0, power=0.05)
    ref = oracle_mod.step3d_rot(u[:3], 0.01, 2e-3, 2.0, 3, power=0.05)
    assert np.abs(got[3]).max() == 0.0
    assert np.abs(got[:3] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_plane_inertia_gravity_wave_is_exact(oracle_mod):
    """A single solenoidal plane mode keeps the nonlinear terms zero, so the
    step is its propagator over the whole time (pinned above by expm)."""
    n, nu, N2, f, dt, steps = 16, 0.01, 6.0, 2.5, 0.05, 20
    m = (2, 1, 3)
    s0, ep, _ = _wave(n, m, 0.3 - 0.1j, 0.2 + 0.4j)
    k = np.array(m, float)
    e1 = np.cross(k / np.linalg.norm(k), [0.0, 0.0, 1.0])
    s0[:3, m[2], m[1], m[0]] += 0.25j * e1 / np.linalg.norm(e1)  # a toroidal part too
    assert np.abs(oracle_mod.tendency3d_strat(s0)).max() <= 1e-15
    got = oracle_mod.step3d_strat(s0, nu, dt, N2, steps, f=f)
    want = oracle_mod.stratrot_propagate(s0, nu, N2, f, dt * steps)
    assert np.abs(got - want).max() <= 1e-14


def test_rotating_stratified_written_out_agrees(oracle_mod):
    n, N2, f, dt, steps = 16, 4.0, 3.0, 1e-3, 10
    s0 = _state(n, 73)
    s0[:, 0, 0, 0] = [0.3, -0.2, 0.25, 0.4]  # a mean velocity and buoyancy (k2 := 1: P = I)
    kx, ky, kz = kmesh(n, 3)
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    k2[k2 == 0] = 1.0
    mask = kept_mask(n, 3)[None]

    def proj(v):
        kv = (kx * v[0] + ky * v[1] + kz * v[2]) / k2
        return v - np.stack([kx, ky, kz]) * kv

    def rhs(s):
        cor = np.stack([-s[1], s[0], np.zeros_like(s[0])])  # z x u
        buoy = np.stack([np.zeros_like(s[3]), np.zeros_like(s[3]), s[3]])
        lin = np.concatenate([proj(buoy - f * cor), (-N2 * s[2])[None]])
        return (oracle_mod.tendency3d_strat(s) + lin) * mask

    s = s0.copy()
    for _ in range(steps):
        a1 = rhs(s)
        a2 = rhs(s + 0.5 * dt * a1)
        a3 = rhs(s + 0.5 * dt * a2)
        a4 = rhs(s + dt * a3)
        s = s + dt / 6 * (a1 + 2 * a2 + 2 * a3 + a4)
    got = oracle_mod.step3d_strat(s0, 0.0, dt, N2, steps, f=f)
    nof = oracle_mod.step3d_strat(s0, 0.0, dt, N2, steps)
    err = np.abs(got - s).max() / np.abs(s).max()
    effect = np.abs(nof - s).max() / np.abs(s).max()
    assert effect > 1e-3
    assert err < 1e-9, (err, effect)
