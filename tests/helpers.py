"""Test-side helpers: brute-force definitions written independently of both
the FP64 reference and the GPU library (plain numpy loops and sums)."""
import numpy as np


def modes(n):
    return np.fft.fftfreq(n, d=1.0 / n).astype(np.int64)


def half_weight(n, ndim):
    """w = 1 on kx = 0 and kx = n/2, 2 elsewhere (half-spectrum Parseval)."""
    h = n // 2 + 1
    w = np.full(h, 2.0)
    w[0] = 1.0
    if n % 2 == 0:
        w[-1] = 1.0
    shape = (1,) * (ndim - 1) + (h,)
    return w.reshape(shape)


def kept_weight(n, ndim):
    """Half-spectrum weights restricted to the kept cube (kx = n/2 never kept)."""
    h = n // 2 + 1
    w = np.where(np.arange(h) == 0, 1.0, 2.0)
    return w.reshape((1,) * (ndim - 1) + (h,))


def kmesh(n, ndim):
    full = modes(n).astype(np.float64)
    half = np.arange(n // 2 + 1, dtype=np.float64)
    if ndim == 2:
        ky, kx = np.meshgrid(full, half, indexing="ij")
        return kx, ky
    kz, ky, kx = np.meshgrid(full, full, half, indexing="ij")
    return kx, ky, kz


def kept_mask(n, ndim):
    full = 3 * np.abs(modes(n)) < n
    half = 3 * np.arange(n // 2 + 1) < n
    if ndim == 2:
        return full[:, None] & half[None, :]
    return full[:, None, None] & full[None, :, None] & half[None, None, :]


def brute_dft(x, sign=-1):
    """O(n^2) DFT along every axis of an array, by explicit exponent sums."""
    out = np.asarray(x, dtype=np.complex128)
    for ax in range(out.ndim):
        n = out.shape[ax]
        j = np.arange(n)
        m = np.exp(sign * 2j * np.pi * np.outer(j, j) / n)
        out = np.moveaxis(np.tensordot(m, np.moveaxis(out, ax, 0), axes=(1, 0)), 0, ax)
    return out


def half_to_modes(a, n, ndim):
    """Dictionary {mode tuple (kx, ky[, kz]): value} of the full spectrum
    described by a half spectrum (Hermitian completion, kx < 0 from kx > 0)."""
    d = {}
    m = modes(n)
    if ndim == 2:
        for iy in range(n):
            for ix in range(n // 2 + 1):
                v = a[..., iy, ix]
                key = (ix, int(m[iy]))
                d[key] = v
                if ix > 0:
                    d[(-ix, int(-m[iy]))] = np.conj(v)
        return d
    for iz in range(n):
        for iy in range(n):
            for ix in range(n // 2 + 1):
                v = a[..., iz, iy, ix]
                key = (ix, int(m[iy]), int(m[iz]))
                d[key] = v
                if ix > 0:
                    d[(-ix, int(-m[iy]), int(-m[iz]))] = np.conj(v)
    return d


def rel_l2(a, b, w):
    return float(np.sqrt(np.sum(w * np.abs(a - b) ** 2) / np.sum(w * np.abs(b) ** 2)))
