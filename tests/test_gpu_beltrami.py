"""Exact Beltrami decay at full size.  A field whose Fourier modes all lie on
one shell |k| = k0 with positive helicity (i k x u = k0 u for every mode) has
vorticity k0 u, so u x w = 0 and the nonlinear term vanishes: an unforced step
multiplies every mode by exp(-nu k0^2 t) exactly.  This checks the fused passes
of 256^3 and 512^3 plans, FP64 (and FP32 at 512^3), at every mode against a
closed form, where a whole oracle step would be too costly.  In a frame
rotating about z each positive-helicity mode is an inertial wave (khat x h =
-i h, so the propagator multiplies it by exp(i f kz t / |k|)) and the field
stays Beltrami, so the rotating step is exact too."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fs():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1807_01769_amd import fs as _fs
    return _fs


def shell_modes(k0sq):
    """Integer vectors m with |m|^2 = k0sq and m_x >= 1 (stored columns with no
    Hermitian partner in the half spectrum)."""
    r = int(np.sqrt(k0sq))
    out = []
    for mx in range(1, r + 1):
        my = np.arange(-r, r + 1)
        rest = k0sq - mx * mx - my * my
        ok = rest >= 0
        for y, z2 in zip(my[ok], rest[ok]):
            z = int(round(np.sqrt(z2)))
            if z * z == z2:
                out.append((mx, int(y), z))
                if z:
                    out.append((mx, int(y), -z))
    return np.array(out)


def beltrami_field(n, k0sq, seed, dtype, device=False):
    """Positive-helicity modes h = e1 + i e2 (e1 ⟂ k, e2 = khat x e1), random
    complex amplitudes, on the shell |m|^2 = k0sq (device: the field is built
    as a device tensor, for sizes whose host copy would be slow)."""
    rng = np.random.default_rng(seed)
    ms = shell_modes(k0sq)
    k = ms.astype(np.float64)
    kh = k / np.linalg.norm(k, axis=1, keepdims=True)
    ref = np.where(np.abs(kh[:, 2:3]) < 0.9, [[0.0, 0.0, 1.0]], [[1.0, 0.0, 0.0]])
    e1 = np.cross(kh, ref)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(kh, e1)
    amp = (rng.standard_normal(len(ms)) + 1j * rng.standard_normal(len(ms))) / np.sqrt(len(ms))
    h = (e1 + 1j * e2) * amp[:, None]
    iz, iy, ix = ms[:, 2] % n, ms[:, 1] % n, ms[:, 0]
    if device:
        u = torch.zeros((3, n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
        hd = torch.from_numpy(h.astype(np.complex64)).cuda()
        ti, tj, tk = (torch.from_numpy(a).cuda() for a in (iz, iy, ix))
        for c in range(3):
            u[c, ti, tj, tk] = hd[:, c]
        return u, (iz, iy, ix), h
    u = np.zeros((3, n, n, n // 2 + 1), dtype)
    for c in range(3):
        u[c, iz, iy, ix] = h[:, c]
    return u, (iz, iy, ix), h


def test_beltrami_field_is_exact_eigenfield():
    """The construction itself (host only): i k x h = |k| h, k . h = 0."""
    _, _, h = beltrami_field(32, 50, 0, np.complex128)
    ms = shell_modes(50).astype(np.float64)
    assert len(ms) > 20
    assert np.abs(1j * np.cross(ms, h) - np.sqrt(50.0) * h).max() < 1e-13
    assert np.abs(np.einsum("ij,ij->i", ms, h)).max() < 1e-14


@pytest.mark.parametrize("n,k0sq,prec,f", [(256, 6254, "f64", 0.0), (512, 150 * 150, "f64", 0.0),
                                           (512, 150 * 150, "f32", 0.0),
                                           (256, 6254, "f64", 40.0), (512, 150 * 150, "f32", 40.0),
                                           (1024, 300 * 300, "f32", 40.0)])
def test_beltrami_decay_full_size(fs, n, k0sq, prec, f):
    print(f"case beltrami decay n={n} |m|^2={k0sq} {prec} rotation {f}", flush=True)
    nu, dt, steps = 2e-4, 1e-3, 5
    cd = np.complex128 if prec == "f64" else np.complex64
    u, idx, h = beltrami_field(n, k0sq, 7, cd, device=n > 512)
    nmodes = len(idx[0])
    plan = fs.Plan(n, precision=prec, nu=nu, dt=dt, rotation=f)
    d = u if n > 512 else torch.from_numpy(u).cuda()
    del u
    plan.step(d, steps)
    torch.cuda.synchronize()
    got = d[:, idx[0], idx[1], idx[2]].cpu().numpy().T.astype(np.complex128)  # [modes][3]
    d[:, idx[0], idx[1], idx[2]] = 0
    rest = torch.view_as_real(d).abs().max().item()
    t = dt * steps
    kz = shell_modes(k0sq)[:, 2].astype(np.float64)
    phase = np.exp(1j * f * kz / np.sqrt(k0sq) * t)[:, None]
    want = h.astype(cd).astype(np.complex128) * np.exp(-nu * k0sq * t) * phase
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"{nmodes} shell modes: rel err {err:.2e}; other modes {rest:.1e}", flush=True)
    # u x w vanishes only in exact arithmetic: its rounding, of order
    # eps k0 |u|^2 with |w| = k0 |u|, leaks into the modes off the shell at a
    # few 1e-6 of the largest amplitude in FP32 at k0 = 150 (a few 1e-14 in
    # FP64); the bound on that leak is the parity tolerance used elsewhere at
    # k0 = 150 and grows in proportion to k0 (k0 = 300 at 1024^3)
    tol = 1e-12 if prec == "f64" else 1e-5
    assert err <= tol
    assert rest <= tol * max(1.0, np.sqrt(k0sq) / 150.0) * np.abs(want).max()
    plan.close()
