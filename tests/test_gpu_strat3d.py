"""GPU parity of the 3D Boussinesq (stratified) path against the FP64 oracle:
the nonlinear tendency (velocity and buoyancy flux), forced RK4 / RK2 steps
with the exact propagator of buoyancy force and stratification (1e-5 FP32,
1e-11 FP64 relative L2; graphs on and off), and an exact plane internal
gravity wave."""
import numpy as np
import pytest

from helpers import kept_mask, kept_weight, rel_l2
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


@pytest.mark.parametrize("n,prec", [(64, "f32"), (128, "f64")])
def test_strat3d_tendency(fs, oracle_mod, n, prec):
    print(f"case boussinesq3d tendency n={n} {prec}", flush=True)
    cd = np.complex64 if prec == "f32" else np.complex128
    s = _state(n, 201, cd)
    plan = fs.Plan(n, precision=prec, nu=1e-3, dt=1e-3, boussinesq=True, n2=4.0)
    got = plan.tendency(torch.from_numpy(s).cuda()).cpu().numpy().astype(np.complex128)
    ref = oracle_mod.tendency3d_strat(s.astype(np.complex128))
    err_u = rel_l2(got[:3], ref[:3], _w4(n)[:3])
    err_b = rel_l2(got[3], ref[3], _w4(n)[3])
    print(f"rel err u {err_u:.2e} b {err_b:.2e}", flush=True)
    tol = 1e-5 if prec == "f32" else 1e-12
    assert err_u <= tol and err_b <= tol
    # outside the kept set the tendency is zero
    assert np.abs(got * ~kept_mask(n, 3)[None]).max() == 0.0
    plan.close()


@pytest.mark.parametrize("n,prec,scheme,graphs", [(64, "f32", "rk4", True),
                                                  (64, "f32", "rk4", False),
                                                  (64, "f64", "rk4", True),
                                                  (32, "f32", "rk2", True),
                                                  (32, "f64", "rk2", False),
                                                  (128, "f32", "rk4", True)])
def test_strat3d_steps(fs, oracle_mod, n, prec, scheme, graphs):
    print(f"case boussinesq3d steps n={n} {prec} {scheme} graphs={graphs}", flush=True)
    cd = np.complex64 if prec == "f32" else np.complex128
    s = _state(n, 211, cd)
    nu, dt, N2, P = 2e-3, 4e-3, 4.0, 0.05
    steps = 3 if n < 128 else 1
    plan = fs.Plan(n, precision=prec, nu=nu, dt=dt, forcing_power=P, boussinesq=True, n2=N2,
                   scheme=scheme, graphs=graphs)
    d = torch.from_numpy(s).cuda()
    plan.step(d, steps)
    got = d.cpu().numpy().astype(np.complex128)
    sc = 4 if scheme == "rk4" else 2
    ref = oracle_mod.step3d_strat(s.astype(np.complex128), nu, dt, N2, steps, power=P, scheme=sc)
    plain, _ = oracle_mod.step3d_ex(s[:3].astype(np.complex128), nu, dt, steps, scheme=sc, power=P)
    err = rel_l2(got, ref, _w4(n))
    effect = rel_l2(plain, ref[:3], _w4(n)[:3])
    print(f"rel err {err:.2e}; buoyancy effect on u {effect:.2e}", flush=True)
    assert effect > 1e-3
    assert err <= (1e-5 if prec == "f32" else 1e-11)
    plan.close()


def test_plane_gravity_wave_fp64(fs):
    n, nu, N2, dt, steps = 16, 0.01, 6.0, 0.05, 20
    m = (2, 1, 3)
    k = np.array(m, float)
    kh = k / np.linalg.norm(k)
    q = np.array([0.0, 0.0, 1.0]) - kh * kh[2]
    g = np.linalg.norm(q)
    ep = q / g
    A, B = 0.3 - 0.1j, 0.2 + 0.4j
    s = np.zeros((4, n, n, n // 2 + 1), np.complex128)
    s[:3, m[2], m[1], m[0]] = A * ep
    s[3, m[2], m[1], m[0]] = B
    plan = fs.Plan(n, nu=nu, dt=dt, precision="f64", boussinesq=True, n2=N2)
    d = torch.from_numpy(s).cuda()
    plan.step(d, steps)
    got = d.cpu().numpy()
    T, N = dt * steps, np.sqrt(N2)
    om, dec = N * g, np.exp(-nu * float(k @ k) * T)
    want = np.zeros_like(s)
    want[:3, m[2], m[1], m[0]] = dec * (A * np.cos(om * T) + B / N * np.sin(om * T)) * ep
    want[3, m[2], m[1], m[0]] = dec * (B * np.cos(om * T) - N * A * np.sin(om * T))
    assert np.abs(got - want).max() <= 1e-13
    plan.close()


def test_plane_gravity_wave_512(fs):
    """The exact plane internal gravity wave through the 512^3 FP32 stratified
    kernels (seven-field x and z passes at full size)."""
    n, nu, N2, dt, steps = 512, 2e-4, 9.0, 1e-3, 4
    m = (6, 2, -5)
    k = np.array(m, float)
    kh = k / np.linalg.norm(k)
    q = np.array([0.0, 0.0, 1.0]) - kh * kh[2]
    g = np.linalg.norm(q)
    ep = q / g
    A, B = 0.3 - 0.1j, 0.2 + 0.4j
    s = np.zeros((4, n, n, n // 2 + 1), np.complex64)
    s[:3, m[2] % n, m[1] % n, m[0]] = A * ep
    s[3, m[2] % n, m[1] % n, m[0]] = B
    plan = fs.Plan(n, nu=nu, dt=dt, boussinesq=True, n2=N2)
    d = torch.from_numpy(s).cuda()
    del s
    plan.step(d, steps)
    got = d[:, m[2] % n, m[1] % n, m[0]].cpu().numpy().astype(np.complex128)
    d[:, m[2] % n, m[1] % n, m[0]] = 0
    rest = torch.view_as_real(d).abs().max().item()  # every other mode stays (rounding-) zero
    T, N = dt * steps, np.sqrt(N2)
    om, dec = N * g, np.exp(-nu * float(k @ k) * T)
    want = np.concatenate([dec * (A * np.cos(om * T) + B / N * np.sin(om * T)) * ep,
                           [dec * (B * np.cos(om * T) - N * A * np.sin(om * T))]])
    print(f"gravity wave 512^3: err {np.abs(got - want).max():.2e}, other modes {rest:.1e}",
          flush=True)
    assert np.abs(got - want).max() <= 2e-6
    assert rest <= 1e-6
    plan.close()


@pytest.mark.parametrize("prec,scheme", [("f32", "rk4"), ("f64", "rk2")])
def test_strat3d_cfl_steps(fs, oracle_mod, prec, scheme):
    """CFL-adaptive stratified steps: sizes from the velocity part's maximum,
    the exact buoyancy-stratification propagator at each size."""
    print(f"case boussinesq3d cfl n=32 {prec} {scheme}", flush=True)
    n, nu, dtmax, N2, cfl, steps = 32, 2e-3, 0.05, 4.0, 0.4, 5
    cd = np.complex64 if prec == "f32" else np.complex128
    s = _state(n, 221, cd)
    plan = fs.Plan(n, nu=nu, dt=dtmax, precision=prec, forcing_power=0.05, boussinesq=True,
                   n2=N2, scheme=scheme, cfl=cfl)
    d = torch.from_numpy(s).cuda()
    plan.step(d, steps)
    t = float(plan.time()[0].item())
    got = d.cpu().numpy().astype(np.complex128)
    sc = 4 if scheme == "rk4" else 2
    ref, tr = oracle_mod.step3d_strat(s.astype(np.complex128), nu, dtmax, N2, steps, power=0.05,
                                      scheme=sc, cfl=cfl, return_time=True)
    err = rel_l2(got, ref, _w4(n))
    print(f"rel err {err:.2e}; time {t:.8f} vs {tr:.8f}", flush=True)
    assert tr < steps * dtmax * 0.9
    tol = 1e-5 if prec == "f32" else 1e-11
    assert err <= tol and abs(t - tr) <= tol * tr
    plan.close()
