"""GPU parity of the rotating stratified 3D path (Boussinesq plan with a
rotation) against the FP64 oracle: forced RK4 / RK2 steps with the exact
propagator of Coriolis force, buoyancy force and stratification (1e-5 FP32,
1e-11 FP64 relative L2; graphs on and off), CFL-adaptive steps, the tendency
(which excludes the linear terms), and a plane inertia-gravity wave at 16^3
FP64 and at 512^3 FP32, checked against scipy's matrix exponential of the
mode's linear operator."""
import numpy as np
import pytest
from scipy.linalg import expm

from helpers import kept_weight, rel_l2
from paper_1807_01769_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fs():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1807_01769_amd import fs as _fs
    return _fs


def _state(n, seed, dtype):
    u = I.random_solenoidal_3d(n, seed=seed, dtype=dtype)
    b = I.random_solenoidal_3d(n, seed=seed + 1, dtype=dtype)[2]
    return np.ascontiguousarray(np.concatenate([u, b[None]]))


def _w4(n):
    return np.broadcast_to(kept_weight(n, 3)[None], (4, n, n, n // 2 + 1))


@pytest.mark.parametrize("n,prec,scheme,graphs", [(32, "f32", "rk4", True),
                                                  (64, "f32", "rk4", False),
                                                  (32, "f64", "rk4", True),
                                                  (32, "f32", "rk2", True),
                                                  (32, "f64", "rk2", False)])
def test_stratrot3d_steps(fs, oracle_mod, n, prec, scheme, graphs):
    print(f"case stratrot3d steps n={n} {prec} {scheme} graphs={graphs}", flush=True)
    cd = np.complex64 if prec == "f32" else np.complex128
    s = _state(n, 231, cd)
    nu, dt, N2, f, P = 2e-3, 4e-3, 4.0, 6.0, 0.05
    steps = 3
    plan = fs.Plan(n, precision=prec, nu=nu, dt=dt, forcing_power=P, boussinesq=True, n2=N2,
                   rotation=f, scheme=scheme, graphs=graphs)
    d = torch.from_numpy(s).cuda()
    plan.step(d, steps)
    got = d.cpu().numpy().astype(np.complex128)
    sc = 4 if scheme == "rk4" else 2
    s64 = s.astype(np.complex128)
    ref = oracle_mod.step3d_strat(s64, nu, dt, N2, steps, power=P, scheme=sc, f=f)
    nof = oracle_mod.step3d_strat(s64, nu, dt, N2, steps, power=P, scheme=sc)
    err = rel_l2(got, ref, _w4(n))
    effect = rel_l2(nof, ref, _w4(n))
    print(f"rel err {err:.2e}; rotation effect {effect:.2e}", flush=True)
    assert effect > 1e-3
    assert err <= (1e-5 if prec == "f32" else 1e-11)
    plan.close()


def test_stratrot3d_tendency_excludes_linear_terms(fs, oracle_mod):
    print("case stratrot3d tendency n=32 f64", flush=True)
    n = 32
    s = _state(n, 241, np.complex128)
    plan = fs.Plan(n, precision="f64", nu=1e-3, dt=1e-3, boussinesq=True, n2=4.0, rotation=3.0)
    got = plan.tendency(torch.from_numpy(s).cuda()).cpu().numpy()
    ref = oracle_mod.tendency3d_strat(s)
    err = rel_l2(got, ref, _w4(n))
    print(f"rel err {err:.2e}", flush=True)
    assert err <= 1e-12
    plan.close()


@pytest.mark.parametrize("prec,scheme", [("f32", "rk4"), ("f64", "rk2")])
def test_stratrot3d_cfl_steps(fs, oracle_mod, prec, scheme):
    print(f"case stratrot3d cfl n=32 {prec} {scheme}", flush=True)
    n, nu, dtmax, N2, f, cfl, steps = 32, 2e-3, 0.05, 4.0, 5.0, 0.4, 5
    cd = np.complex64 if prec == "f32" else np.complex128
    s = _state(n, 251, cd)
    plan = fs.Plan(n, nu=nu, dt=dtmax, precision=prec, forcing_power=0.05, boussinesq=True,
                   n2=N2, rotation=f, scheme=scheme, cfl=cfl)
    d = torch.from_numpy(s).cuda()
    plan.step(d, steps)
    t = float(plan.time()[0].item())
    got = d.cpu().numpy().astype(np.complex128)
    sc = 4 if scheme == "rk4" else 2
    ref, tr = oracle_mod.step3d_strat(s.astype(np.complex128), nu, dtmax, N2, steps, power=0.05,
                                      scheme=sc, cfl=cfl, return_time=True, f=f)
    err = rel_l2(got, ref, _w4(n))
    print(f"rel err {err:.2e}; time {t:.8f} vs {tr:.8f}", flush=True)
    assert tr < steps * dtmax * 0.9
    tol = 1e-5 if prec == "f32" else 1e-11
    assert err <= tol and abs(t - tr) <= tol * tr
    plan.close()


def _mode_operator(k, nu, N2, f):
    """The linear operator of one mode on (u, b): -f P(z x u) + P(b z) - nu k^2 u,
    -N^2 uz - nu k^2 b."""
    k = np.asarray(k, float)
    k2 = float(k @ k)
    P = np.eye(3) - np.outer(k, k) / k2
    Z = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    A = np.zeros((4, 4))
    A[:3, :3] = -f * P @ Z
    A[:3, 3] = P @ np.array([0.0, 0.0, 1.0])
    A[3, 2] = -N2
    return A - nu * k2 * np.eye(4)


def _plane_mode(m):
    """(u, b) of one solenoidal plane mode with toroidal and poloidal parts."""
    k = np.array(m, float)
    kh = k / np.linalg.norm(k)
    e1 = np.cross(kh, [0.0, 0.0, 1.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(kh, e1)
    return np.concatenate([(0.3 - 0.1j) * e2 + 0.25j * e1, [0.2 + 0.4j]])


def test_plane_inertia_gravity_wave_fp64(fs):
    n, nu, N2, f, dt, steps = 16, 0.01, 6.0, 2.5, 0.05, 20
    m = (2, 1, 3)
    w0 = _plane_mode(m)
    s = np.zeros((4, n, n, n // 2 + 1), np.complex128)
    s[:, m[2], m[1], m[0]] = w0
    plan = fs.Plan(n, nu=nu, dt=dt, precision="f64", boussinesq=True, n2=N2, rotation=f)
    d = torch.from_numpy(s).cuda()
    plan.step(d, steps)
    got = d.cpu().numpy()
    want = np.zeros_like(s)
    want[:, m[2], m[1], m[0]] = expm(dt * steps * _mode_operator(m, nu, N2, f)) @ w0
    err = np.abs(got - want).max()
    print(f"inertia-gravity wave 16^3 FP64: err {err:.2e}", flush=True)
    assert err <= 1e-13
    plan.close()


@pytest.mark.parametrize("n,f", [(512, 4.0), (1024, 4.0), (1024, 0.0)])
def test_plane_inertia_gravity_wave_full_size(fs, n, f):
    """The plane inertia-gravity wave through the 512^3 and 1024^3 FP32
    kernels (f = 0: the stratified propagator alone, at 1024^3 the
    1024-thread z pass without the stash)."""
    print(f"case plane inertia-gravity wave n={n} f={f}", flush=True)
    nu, N2, dt, steps = 2e-4, 9.0, 1e-3, 4
    m = (6, 2, -5)
    w0 = _plane_mode(m)
    d = torch.zeros((4, n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
    d[:, m[2] % n, m[1] % n, m[0]] = torch.from_numpy(w0.astype(np.complex64)).cuda()
    plan = fs.Plan(n, nu=nu, dt=dt, boussinesq=True, n2=N2, rotation=f)
    plan.step(d, steps)
    torch.cuda.synchronize()
    got = d[:, m[2] % n, m[1] % n, m[0]].cpu().numpy().astype(np.complex128)
    d[:, m[2] % n, m[1] % n, m[0]] = 0
    rest = torch.view_as_real(d).abs().max().item()
    want = expm(dt * steps * _mode_operator(m, nu, N2, f)) @ w0
    print(f"inertia-gravity wave {n}^3 f={f}: err {np.abs(got - want).max():.2e}, "
          f"other modes {rest:.1e}", flush=True)
    assert np.abs(got - want).max() <= 2e-6
    assert rest <= 1e-6
    plan.close()
