"""Seeded synthetic initial states for the periodic-box Navier-Stokes step.

This module only *builds inputs*: it writes Fourier coefficients of initial
fields on the half spectrum.  It holds none of the solver's arithmetic (no
transform, no tendency, no time stepping) and imports neither the GPU library
nor the FP64 CPU reference, so both sides can be fed the very same arrays.

Conventions (shared with every consumer):

* domain [0, L)^d with L = 2*pi, so wavenumbers are integers m;
* a 3D spectral field is complex ``[3][N][N][N//2+1]`` indexed (component,
  kz, ky, kx); a 2D one is ``[N][N//2+1]`` indexed (ky, kx); kx is the
  contiguous half axis, ky and kz run in FFT order 0..N/2-1, -N/2..-1;
* forward transforms carry the 1/N^d factor, so the coefficient of
  exp(i k.x) is the value stored at k;
* the kept (alias-free) set is the cube 3|m_a| < N on every axis; every
  generator returns fields that vanish outside it, are Hermitian on the kx=0
  plane and have a zero mean mode;
* random draws use numpy's PCG64 ``default_rng(seed)``; draws are taken for
  all stored modes in C order (kz, ky, kx), then per mode the components and
  finally real before imaginary, so the stream does not depend on masks.

The shapes of the workloads follow the paper's benchmark setups (random-field
initial-value problems advanced with RK4, section "Performance", 2D and 3D
benchmarks) and the Taylor-Green closed forms used as exact checks.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "mode_numbers",
    "kept_cube",
    "taylor_green_2d",
    "taylor_green_3d",
    "abc_flow_3d",
    "random_vorticity_2d",
    "tg_plus_noise_2d",
    "random_solenoidal_3d",
    "broadband_solenoidal_3d",
    "broadband_vorticity_2d",
    "ensemble_sizes",
    "ensemble_vorticity",
]


def mode_numbers(n: int):
    """Integer mode numbers along a full axis (FFT order) and the half axis."""
    full = np.fft.fftfreq(n, d=1.0 / n).astype(np.int64)
    half = np.arange(n // 2 + 1, dtype=np.int64)
    return full, half


def kept_cube(n: int, ndim: int) -> np.ndarray:
    """Boolean support of the alias-free cube 3|m_a| < n on the half spectrum."""
    full, half = mode_numbers(n)
    kf = 3 * np.abs(full) < n
    kh = 3 * half < n
    if ndim == 2:
        return kf[:, None] & kh[None, :]
    return kf[:, None, None] & kf[None, :, None] & kh[None, None, :]


def _grids(n: int, ndim: int):
    full, half = mode_numbers(n)
    if ndim == 2:
        ky, kx = np.meshgrid(full, half, indexing="ij")
        return kx.astype(np.float64), ky.astype(np.float64)
    kz, ky, kx = np.meshgrid(full, full, half, indexing="ij")
    return kx.astype(np.float64), ky.astype(np.float64), kz.astype(np.float64)


def _hermitian_kx0(a: np.ndarray, ndim: int) -> None:
    """Make the kx = 0 plane (line in 2D) Hermitian in place; zero the mean."""
    n = a.shape[-2]
    if ndim == 2:
        for ky in range(1, n // 2):
            a[n - ky, 0] = np.conj(a[ky, 0])
        a[n // 2, 0] = 0.0
        a[0, 0] = 0.0
        return
    # a: [..., kz, ky, kx]; positive half of the plane = (ky > 0) or (ky == 0, kz > 0)
    plane = np.ascontiguousarray(a[..., 0])
    kz = np.arange(n)[:, None]
    ky = np.arange(n)[None, :]
    pos = ((ky >= 1) & (ky < n // 2)) | ((ky == 0) & (kz >= 1) & (kz < n // 2))
    sz, sy = np.nonzero(pos)
    plane[..., (-sz) % n, (-sy) % n] = np.conj(plane[..., sz, sy])
    # self-conjugate points other than the mean are Nyquist (outside the cube)
    plane[..., n // 2, :] = 0.0
    plane[..., :, n // 2] = 0.0
    plane[..., 0, 0] = 0.0
    a[..., 0] = plane


def taylor_green_2d(n: int) -> np.ndarray:
    """Coefficients of omega = 2 sin x sin y (velocity (sin x cos y, -cos x sin y))."""
    w = np.zeros((n, n // 2 + 1), np.complex128)
    w[1, 1] = -0.5
    w[n - 1, 1] = 0.5
    return w


def taylor_green_3d(n: int) -> np.ndarray:
    """Coefficients of u = (sin x cos y cos z, -cos x sin y cos z, 0)."""
    u = np.zeros((3, n, n, n // 2 + 1), np.complex128)
    for sy in (1, -1):
        for sz in (1, -1):
            u[0, sz % n, sy % n, 1] = -0.125j
            u[1, sz % n, sy % n, 1] = 0.125j * sy
    return u


def abc_flow_3d(n: int, a: float = 1.0, b: float = 1.0, c: float = 1.0) -> np.ndarray:
    """Arnold-Beltrami-Childress flow (curl u = u):
    u = (A sin z + C cos y, B sin x + A cos z, C sin y + B cos x)."""
    u = np.zeros((3, n, n, n // 2 + 1), np.complex128)
    # sin t = (e^{it} - e^{-it}) / 2i ; cos t = (e^{it} + e^{-it}) / 2
    # x-component: A sin z + C cos y
    u[0, 1, 0, 0] += a / 2j
    u[0, n - 1, 0, 0] += -a / 2j
    u[0, 0, 1, 0] += c / 2
    u[0, 0, n - 1, 0] += c / 2
    # y-component: B sin x + A cos z
    u[1, 0, 0, 1] += b / 2j
    u[1, 1, 0, 0] += a / 2
    u[1, n - 1, 0, 0] += a / 2
    # z-component: C sin y + B cos x
    u[2, 0, 1, 0] += c / 2j
    u[2, 0, n - 1, 0] += -c / 2j
    u[2, 0, 0, 1] += b / 2
    return u


def _shell(kx, ky, kz=None):
    k2 = kx * kx + ky * ky + (0.0 if kz is None else kz * kz)
    return np.floor(np.sqrt(k2) + 0.5).astype(np.int64), np.sqrt(k2)


def _half_weight(kx):
    return np.where(kx == 0, 1.0, 2.0)


def random_vorticity_2d(n: int, seed: int, shape_fn, kmin: float = 1.0,
                        kmax: float | None = None, energy: float = 1.0) -> np.ndarray:
    """Random-phase Gaussian vorticity whose shell energies follow ``shape_fn``.

    Energy per shell s (s = floor(|k| + 1/2)) is set to C*shape_fn(s) with C
    chosen so that the total 0.5*<|u|^2> equals ``energy``; the energy of a
    mode is 0.5*w*|omega|^2/|k|^2 (w = 1 on kx = 0, 2 elsewhere)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n // 2 + 1, 2))
    w = g[..., 0] + 1j * g[..., 1]
    kx, ky = _grids(n, 2)
    s, kmag = _shell(kx, ky)
    sup = kept_cube(n, 2) & (kmag >= kmin)
    if kmax is not None:
        sup &= kmag <= kmax
    w = np.where(sup, w, 0.0)
    _hermitian_kx0(w, 2)
    e_mode = 0.5 * _half_weight(kx) * np.abs(w) ** 2 / np.where(kmag > 0, kmag * kmag, 1.0)
    nb = int(s.max()) + 1
    e_shell = np.bincount(s.ravel(), weights=e_mode.ravel(), minlength=nb)
    target = np.array([shape_fn(float(q)) if q > 0 else 0.0 for q in range(nb)])
    target = np.where(e_shell > 0, target, 0.0)
    target *= energy / target.sum()
    scale = np.sqrt(np.where(e_shell > 0, target / np.where(e_shell > 0, e_shell, 1.0), 0.0))
    return w * scale[s]


def tg_plus_noise_2d(n: int, seed: int = 0, amplitude: float = 1e-2,
                     kmax: float = 4.0) -> np.ndarray:
    """Taylor-Green vorticity plus random-phase Gaussian noise on 1 <= |k| <= kmax,
    the noise scaled so that its rms vorticity equals ``amplitude``."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n // 2 + 1, 2))
    noise = g[..., 0] + 1j * g[..., 1]
    kx, ky = _grids(n, 2)
    kmag = np.sqrt(kx * kx + ky * ky)
    sup = kept_cube(n, 2) & (kmag >= 1.0) & (kmag <= kmax)
    noise = np.where(sup, noise, 0.0)
    _hermitian_kx0(noise, 2)
    rms = np.sqrt(np.sum(_half_weight(kx) * np.abs(noise) ** 2))
    return taylor_green_2d(n) + noise * (amplitude / rms)


def _craya_basis(kx, ky, kz):
    """Two orthonormal real vectors perpendicular to k (k != 0)."""
    k = np.stack([kx, ky, kz])
    kmag = np.sqrt(np.sum(k * k, axis=0))
    # e1 = k x z_hat / |k x z_hat|, or x_hat where k is parallel to z
    e1 = np.stack([ky, -kx, np.zeros_like(kx)])
    n1 = np.sqrt(np.sum(e1 * e1, axis=0))
    par = n1 == 0
    e1 = np.where(par, np.array([1.0, 0.0, 0.0])[:, None, None, None], e1 / np.where(par, 1.0, n1))
    # e2 = k x e1 / |k|
    e2 = np.stack([
        k[1] * e1[2] - k[2] * e1[1],
        k[2] * e1[0] - k[0] * e1[2],
        k[0] * e1[1] - k[1] * e1[0],
    ]) / np.where(kmag > 0, kmag, 1.0)
    return e1, e2


def random_solenoidal_3d(n: int, seed: int = 1, energy: float = 1.0,
                         shape_fn=lambda k: k ** 4 * np.exp(-2.0 * (k / 4.0) ** 2),
                         dtype=np.complex128) -> np.ndarray:
    """Random-phase solenoidal velocity with shell spectrum C*shape_fn(s), total
    energy 0.5*<|u|^2> = ``energy``.

    Per stored mode two complex Gaussians (a, b) are drawn and placed on two
    unit vectors orthogonal to k, so the field is divergence free by
    construction.  Planes of constant kz are generated one after the other
    (the random stream is the same as one draw over the whole array)."""
    rng = np.random.default_rng(seed)
    h = n // 2 + 1
    full, half = mode_numbers(n)
    kept_full = 3 * np.abs(full) < n
    ky, kx = np.meshgrid(full.astype(np.float64), half.astype(np.float64), indexing="ij")
    keep_plane = kept_full[:, None] & (3 * half < n)[None, :]
    # Craya basis: e1 = (ky, -kx, 0)/|k_perp| (x_hat on the kz axis) does not
    # depend on kz; e2 = k x e1 / |k|
    kp = np.sqrt(kx * kx + ky * ky)
    on_axis = kp == 0
    kps = np.where(on_axis, 1.0, kp)
    e1x = np.where(on_axis, 1.0, ky / kps)
    e1y = np.where(on_axis, 0.0, -kx / kps)
    u = np.zeros((3, n, n, h), np.complex128)
    ur = u.view(np.float64).reshape(3, n, n, h, 2)
    for iz in range(n):
        g = rng.standard_normal((n, h, 2, 2))
        if not kept_full[iz]:
            continue
        kz = float(full[iz])
        kmag = np.sqrt(kp * kp + kz * kz)
        sup = keep_plane & (kmag > 0)
        ik = np.where(sup, 1.0 / np.where(kmag > 0, kmag, 1.0), 0.0)
        f1x, f1y = e1x * sup, e1y * sup
        e2x = np.where(on_axis, 0.0, kz * kx / kps) * ik
        e2y = np.where(on_axis, kz, kz * ky / kps) * ik
        e2z = np.where(on_axis, 0.0, -kp) * ik
        for ri in range(2):  # real, imaginary
            ga, gb = g[..., 0, ri], g[..., 1, ri]
            ur[0, iz, :, :, ri] = ga * f1x + gb * e2x
            ur[1, iz, :, :, ri] = ga * f1y + gb * e2y
            ur[2, iz, :, :, ri] = gb * e2z
    _hermitian_kx0(u, 3)
    nb = int(np.floor(np.sqrt(3.0) * (n // 2) + 0.5)) + 2
    e_shell = np.zeros(nb)
    w = _half_weight(kx)
    for iz in range(n):
        if not kept_full[iz]:
            continue
        k2 = kx * kx + ky * ky + float(full[iz]) ** 2
        s = np.floor(np.sqrt(k2) + 0.5).astype(np.int64)
        e_mode = 0.5 * w * np.sum(np.abs(u[:, iz]) ** 2, axis=0)
        e_shell += np.bincount(s.ravel(), weights=e_mode.ravel(), minlength=nb)
    target = np.array([shape_fn(float(q)) if q > 0 else 0.0 for q in range(nb)])
    target = np.where(e_shell > 0, target, 0.0)
    target *= energy / target.sum()
    scale = np.sqrt(np.where(e_shell > 0, target / np.where(e_shell > 0, e_shell, 1.0), 0.0))
    out = np.empty((3, n, n, h), dtype)
    for iz in range(n):
        k2 = kx * kx + ky * ky + float(full[iz]) ** 2
        s = np.floor(np.sqrt(k2) + 0.5).astype(np.int64)
        out[:, iz] = u[:, iz] * scale[s][None]
    return out


def _broadband_rms(kmag, n):
    """Per-mode rms amplitude exp(-|m| / K) (K the largest kept mode): every
    kept mode carries signal, from 1 at the origin to exp(-sqrt(3)) at the
    corner of the kept cube (exp(-sqrt(2)) in 2D)."""
    return np.exp(-kmag / float((n - 1) // 3))


def broadband_solenoidal_3d(n: int, seed: int, energy: float = 1.0,
                            dtype=np.complex128) -> np.ndarray:
    """Random solenoidal velocity that fills the whole kept cube.

    Unlike the turbulence recipe (whose spectrum peaks at |k| ~ 4 and is
    negligible beyond |k| ~ 20), every kept mode gets two complex Gaussians on
    the two unit vectors orthogonal to k, scaled by a per-mode rms that decays
    only by exp(-|m| / K).  For checks that must see every tile of the kept
    cube, its faces, edges and corner.  Draw order as in the other
    generators; total energy 0.5*<|u|^2> = ``energy``."""
    rng = np.random.default_rng(seed)
    h = n // 2 + 1
    full, half = mode_numbers(n)
    kept_full = 3 * np.abs(full) < n
    ky, kx = np.meshgrid(full.astype(np.float64), half.astype(np.float64), indexing="ij")
    keep_plane = kept_full[:, None] & (3 * half < n)[None, :]
    kp = np.sqrt(kx * kx + ky * ky)
    on_axis = kp == 0
    kps = np.where(on_axis, 1.0, kp)
    e1x = np.where(on_axis, 1.0, ky / kps)
    e1y = np.where(on_axis, 0.0, -kx / kps)
    u = np.zeros((3, n, n, h), np.complex128)
    ur = u.view(np.float64).reshape(3, n, n, h, 2)
    for iz in range(n):
        g = rng.standard_normal((n, h, 2, 2))
        if not kept_full[iz]:
            continue
        kz = float(full[iz])
        kmag = np.sqrt(kp * kp + kz * kz)
        sup = keep_plane & (kmag > 0)
        ik = np.where(sup, 1.0 / np.where(kmag > 0, kmag, 1.0), 0.0)
        amp = _broadband_rms(kmag, n) * sup
        e2x = np.where(on_axis, 0.0, kz * kx / kps) * ik
        e2y = np.where(on_axis, kz, kz * ky / kps) * ik
        e2z = np.where(on_axis, 0.0, -kp) * ik
        for ri in range(2):
            ga, gb = g[..., 0, ri] * amp, g[..., 1, ri] * amp
            ur[0, iz, :, :, ri] = ga * e1x + gb * e2x
            ur[1, iz, :, :, ri] = ga * e1y + gb * e2y
            ur[2, iz, :, :, ri] = gb * e2z
    _hermitian_kx0(u, 3)
    w = _half_weight(kx)
    e = 0.0
    for iz in range(n):
        e += 0.5 * float(np.sum(w * np.sum(np.abs(u[:, iz]) ** 2, axis=0)))
    return (u * np.sqrt(energy / e)).astype(dtype)


def broadband_vorticity_2d(n: int, seed: int, energy: float = 1.0) -> np.ndarray:
    """Random vorticity that fills the whole kept square: complex Gaussian
    coefficients with per-mode rms exp(-|m| / K) (K the largest kept mode),
    total energy 0.5*<|u|^2> = ``energy``."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n // 2 + 1, 2))
    kx, ky = _grids(n, 2)
    kmag = np.sqrt(kx * kx + ky * ky)
    sup = kept_cube(n, 2) & (kmag > 0)
    w = np.where(sup, (g[..., 0] + 1j * g[..., 1]) * _broadband_rms(kmag, n), 0.0)
    _hermitian_kx0(w, 2)
    e = 0.5 * np.sum(_half_weight(kx) * np.abs(w) ** 2 / np.where(kmag > 0, kmag * kmag, 1.0))
    return w * np.sqrt(energy / e)


def ensemble_sizes(counts=((128, 128), (96, 256), (32, 512))):
    """Grid size of every run of the uneven 2D ensemble, in packing order."""
    out = []
    for cnt, n in counts:
        out += [n] * cnt
    return out


def ensemble_vorticity(r: int, n: int, energy: float = 1.0) -> np.ndarray:
    """Initial vorticity of ensemble run r: seed 1000 + r, E(k) ~ k exp(-(k/6)^2)."""
    return random_vorticity_2d(n, 1000 + r, lambda k: k * np.exp(-(k / 6.0) ** 2),
                               energy=energy)
