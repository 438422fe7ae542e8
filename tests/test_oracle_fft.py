"""Pins of the FP64 reference transforms (CPU only).

The transforms are the plain DFT (the paper's sim.oper "FFT, IFFT" operators,
section "Implementation and architecture"), so they are pinned to the DFT
written as an explicit exponent sum, to the round trip, to Parseval, to
single Fourier modes and, as a library cross-check, to numpy.fft."""
import numpy as np
import pytest

from helpers import brute_dft, half_weight

pytestmark = pytest.mark.filterwarnings("ignore")


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft1d_vs_bruteforce(oracle_mod, n, sign):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    got = oracle_mod.fft1d(x, sign)
    ref = brute_dft(x, sign)
    assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("shape", [(4, 8), (8, 4), (4, 4, 8), (2, 8, 4)])
def test_fftn_vs_bruteforce(oracle_mod, shape):
    rng = np.random.default_rng(7)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    got = oracle_mod.fftn(x, -1)
    ref = brute_dft(x, -1)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("ndim,n", [(1, 16), (2, 8), (2, 16), (3, 4), (3, 8)])
def test_rfftn_vs_bruteforce(oracle_mod, ndim, n):
    rng = np.random.default_rng(3)
    p = rng.standard_normal((n,) * ndim)
    got = oracle_mod.rfftn(p)
    ref = brute_dft(p, -1)[..., : n // 2 + 1] / n ** ndim
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("ndim,n", [(2, 8), (2, 32), (3, 8), (3, 16)])
def test_irfftn_vs_bruteforce(oracle_mod, ndim, n):
    """C2R of an arbitrary half spectrum equals the real part of the inverse
    DFT of its Hermitian completion (kx < 0 taken from the conjugate mirror)."""
    rng = np.random.default_rng(11)
    h = n // 2 + 1
    s = rng.standard_normal((n,) * (ndim - 1) + (h,)) + 1j * rng.standard_normal((n,) * (ndim - 1) + (h,))
    full = np.zeros((n,) * ndim, np.complex128)
    full[..., :h] = s
    for kx in range(h, n):
        mirror = s[..., n - kx]
        for ax in range(ndim - 1):
            mirror = np.roll(np.flip(mirror, axis=ax), 1, axis=ax)
        full[..., kx] = np.conj(mirror)
    ref = brute_dft(full, +1).real
    got = oracle_mod.irfftn(s)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("ndim,n", [(2, 64), (3, 16), (3, 32)])
def test_round_trip(oracle_mod, ndim, n):
    rng = np.random.default_rng(5)
    p = rng.standard_normal((n,) * ndim)
    back = oracle_mod.irfftn(oracle_mod.rfftn(p))
    assert np.abs(back - p).max() <= 1e-14 * max(1.0, np.log2(n)) * 4


@pytest.mark.parametrize("ndim,n", [(2, 32), (3, 16)])
def test_parseval(oracle_mod, ndim, n):
    rng = np.random.default_rng(9)
    p = rng.standard_normal((n,) * ndim)
    s = oracle_mod.rfftn(p)
    lhs = 0.5 * np.mean(p * p)
    rhs = 0.5 * np.sum(half_weight(n, ndim) * np.abs(s) ** 2)
    assert abs(lhs - rhs) <= 1e-14 * lhs * 10


@pytest.mark.parametrize("m", [(1, 0, 0), (0, 2, 0), (0, 0, 3), (2, -1, 3)])
def test_single_mode(oracle_mod, m):
    """cos(m.x) has coefficient 1/2 at +m and -m (stored as the conjugate
    mirror when kx = 0) and nothing else."""
    n = 16
    x = 2 * np.pi * np.arange(n) / n
    z, y, xx = np.meshgrid(x, x, x, indexing="ij")
    p = np.cos(m[0] * xx + m[1] * y + m[2] * z)
    s = oracle_mod.rfftn(p)
    ref = np.zeros_like(s)
    mx, my, mz = m
    if mx < 0 or (mx == 0 and (my < 0 or (my == 0 and mz < 0))):
        mx, my, mz = -mx, -my, -mz
    ref[mz % n, my % n, mx] += 0.5
    if mx == 0:
        ref[(-mz) % n, (-my) % n, 0] += 0.5
    assert np.abs(s - ref).max() <= 1e-15 * 20


@pytest.mark.parametrize("n", [16, 32, 64])
def test_vs_numpy_fft(oracle_mod, n):
    rng = np.random.default_rng(n)
    p = rng.standard_normal((n, n, n))
    s = oracle_mod.rfftn(p)
    ref = np.fft.rfftn(p) / n ** 3
    assert np.abs(s - ref).max() <= 1e-15 * np.abs(ref).max() * 50
    back = oracle_mod.irfftn(ref)
    assert np.abs(back - p).max() <= 1e-13


def test_dft_mode3d_vs_bruteforce(oracle_mod):
    n = 8
    rng = np.random.default_rng(2)
    p = rng.standard_normal((n, n, n))
    ref = brute_dft(p, -1) / n ** 3
    for m in [(0, 0, 0), (1, 0, 0), (0, 3, 0), (0, 0, 5), (2, -3, 1), (4, 4, -4), (3, 7, 2)]:
        got = oracle_mod.dft_mode3d(p, m)
        want = ref[m[2] % n, m[1] % n, m[0] % n]
        assert abs(got - want) <= 1e-14 * np.abs(ref).max() * 10
