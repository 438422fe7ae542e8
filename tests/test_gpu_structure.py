"""GPU parity of the longitudinal structure functions against the FP64
oracle (2D and 3D, FP32 and FP64, a Boussinesq state), and at 512^3 the
spectral identity <du_a^2>(r) = 2 sum w |u_a_hat|^2 (1 - cos(2 pi m_a r / n))
and <du> = 0, which hold at any size."""
import numpy as np
import pytest

from helpers import kept_mask, kept_weight
from paper_1807_01769_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fs():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1807_01769_amd import fs as _fs
    return _fs


def _check(got, ref, tol):
    gs, ga = (g.cpu().numpy() for g in got)
    rs, ra = ref
    scale = ra  # absolute moment of the same r and p
    assert np.all(np.abs(gs - rs) <= tol * scale), np.max(np.abs(gs - rs) / scale)
    assert np.all(np.abs(ga - ra) <= tol * scale), np.max(np.abs(ga - ra) / scale)


@pytest.mark.parametrize("ndim,n,prec", [(3, 32, "f32"), (3, 64, "f64"), (2, 128, "f32"),
                                         (2, 64, "f64")])
def test_structure_parity(fs, oracle_mod, ndim, n, prec):
    print(f"case structure {ndim}d n={n} {prec}", flush=True)
    cd = np.complex64 if prec == "f32" else np.complex128
    if ndim == 3:
        st = I.random_solenoidal_3d(n, seed=401, dtype=cd)
    else:
        st = I.random_vorticity_2d(n, 401, lambda k: k * np.exp(-(k / 8.0) ** 2)).astype(cd)
    r = [1, 2, 3, 5, 8, n // 4, n // 2, n - 1]
    plan = fs.Plan(n, ndim=ndim, precision=prec, nu=1e-3, dt=1e-3)
    got = plan.structure_functions(torch.from_numpy(st).cuda(), r, 8)
    ref = oracle_mod.structure(st.astype(np.complex128), ndim, r, 8)
    _check(got, ref, 3e-5 if prec == "f32" else 1e-11)
    again = plan.structure_functions(torch.from_numpy(st).cuda(), r, 8)
    assert torch.equal(got[0], again[0]) and torch.equal(got[1], again[1])
    plan.close()


def test_structure_boussinesq_state(fs, oracle_mod):
    n = 32
    u = I.random_solenoidal_3d(n, seed=403, dtype=np.complex64)
    b = I.random_solenoidal_3d(n, seed=404, dtype=np.complex64)[2]
    s = np.ascontiguousarray(np.concatenate([u, b[None]]))
    plan = fs.Plan(n, precision="f32", nu=1e-3, dt=1e-3, boussinesq=True, n2=1.0)
    got = plan.structure_functions(torch.from_numpy(s).cuda(), [1, 4, 16], 4)
    ref = oracle_mod.structure(u.astype(np.complex128), 3, [1, 4, 16], 4)
    _check(got, ref, 3e-5)
    plan.close()


def test_structure_512_spectral_identity(fs):
    n = 512
    print(f"case structure 3d n={n} f32 spectral identity", flush=True)
    u = I.random_solenoidal_3d(n, seed=1, dtype=np.complex64)
    r = [1, 4, 16, 64, 256]
    plan = fs.Plan(n, precision="f32", nu=2e-4, dt=1e-3)
    d = torch.from_numpy(u).cuda()
    sg, ab = (t.cpu().numpy() for t in plan.structure_functions(d, r, 2))
    plan.close()
    del d
    w = kept_weight(n, 3) * kept_mask(n, 3)
    want = np.zeros(len(r))
    for a in range(3):
        e = w * np.abs(u[a].astype(np.complex128)) ** 2
        # sum over the other axes first, then the cosine of axis a
        ax = 2 - a
        other = tuple(i for i in range(3) if i != ax)
        ea = e.sum(axis=other)
        m1 = np.arange(ea.shape[0])
        if ax != 2:
            m1 = np.where(m1 <= n // 2, m1, m1 - n)
        for j, rr in enumerate(r):
            want[j] += 2 * np.sum(ea * (1 - np.cos(2 * np.pi * m1 * rr / n))) / 3
    print("S2", ab[:, 1], "want", want, flush=True)
    assert np.all(np.abs(ab[:, 1] - want) <= 2e-5 * want)
    assert np.all(np.abs(sg[:, 1] - ab[:, 1]) <= 1e-12 * want)
    assert np.all(np.abs(sg[:, 0]) <= 1e-6 * np.sqrt(want))
