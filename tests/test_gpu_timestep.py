"""GPU parity of the RK2 scheme and the CFL-adaptive step against the FP64
oracle (same tolerances as the RK4 step: 1e-5 relative L2 in FP32, 1e-11 in
FP64; the adaptive step's size comes from an FP32 velocity maximum on the GPU,
so elapsed times agree to FP32 rounding)."""
import numpy as np
import pytest

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


def _run(fs, state, n, ndim, prec, steps, **kw):
    plan = fs.Plan(n, ndim=ndim, precision=prec, **kw)
    d = torch.from_numpy(state).cuda()
    plan.step(d, steps)
    t, dt = plan.time()
    out = d.cpu().numpy().astype(np.complex128), float(t.item()), float(dt.item())
    plan.close()
    return out


@pytest.mark.parametrize("prec,graphs", [("f32", True), ("f32", False), ("f64", True)])
def test_rk2_3d(fs, oracle_mod, prec, graphs):
    print(f"case rk2 3d n=32 {prec} graphs={graphs}", flush=True)
    n, nu, dt, steps = 32, 2e-3, 4e-3, 5
    cd = np.complex64 if prec == "f32" else np.complex128
    u = I.random_solenoidal_3d(n, seed=71, dtype=cd)
    got, t, _ = _run(fs, u, n, 3, prec, steps, nu=nu, dt=dt, forcing_power=0.05,
                     scheme="rk2", graphs=graphs)
    ref, tr = oracle_mod.step3d_ex(u.astype(np.complex128), nu, dt, steps, scheme=2, power=0.05)
    err = rel_l2(got, ref, kept_weight(n, 3)[None])
    print(f"rel err {err:.2e}", flush=True)
    assert err <= (1e-5 if prec == "f32" else 1e-11)
    assert abs(t - tr) <= 1e-12


def test_rk2_2d_fp64(fs, oracle_mod):
    n, nu, dt, steps = 64, 1e-3, 2e-3, 10
    w = I.tg_plus_noise_2d(n)
    got, _, _ = _run(fs, w, n, 2, "f64", steps, nu=nu, dt=dt, scheme="rk2")
    ref, _ = oracle_mod.step2d_ex(w, nu, dt, steps, scheme=2)
    assert rel_l2(got, ref, kept_weight(n, 2)) <= 1e-11


@pytest.mark.parametrize("prec,scheme,graphs", [("f32", "rk4", True), ("f32", "rk4", False),
                                                ("f64", "rk4", True), ("f32", "rk2", True)])
def test_cfl_3d(fs, oracle_mod, prec, scheme, graphs):
    print(f"case cfl 3d n=32 {prec} {scheme} graphs={graphs}", flush=True)
    n, nu, dtmax, cfl, steps = 32, 2e-3, 0.05, 0.4, 6
    cd = np.complex64 if prec == "f32" else np.complex128
    u = I.random_solenoidal_3d(n, seed=72, dtype=cd)
    got, t, last = _run(fs, u, n, 3, prec, steps, nu=nu, dt=dtmax, forcing_power=0.05,
                        scheme=scheme, cfl=cfl, graphs=graphs)
    ref, tr = oracle_mod.step3d_ex(u.astype(np.complex128), nu, dtmax, steps,
                                   scheme=4 if scheme == "rk4" else 2, cfl=cfl, power=0.05)
    err = rel_l2(got, ref, kept_weight(n, 3)[None])
    print(f"rel err {err:.2e}; time {t:.8f} vs {tr:.8f}; last dt {last:.3e}", flush=True)
    assert tr < steps * dtmax * 0.9  # the CFL bound is active
    tol = 1e-5 if prec == "f32" else 1e-11
    assert err <= tol
    assert abs(t - tr) <= tol * tr
    # the last step size is the CFL step of the state before it
    prev, _ = oracle_mod.step3d_ex(u.astype(np.complex128), nu, dtmax, steps - 1,
                                   scheme=4 if scheme == "rk4" else 2, cfl=cfl, power=0.05)
    want = cfl * (2 * np.pi / n) / oracle_mod.umax(prev, 3)
    assert abs(last - want) <= max(tol, 1e-6) * want


def test_cfl_2d_rk2_fp64(fs, oracle_mod):
    n, nu, dtmax, cfl, steps = 64, 1e-3, 0.1, 0.5, 8
    w = I.random_vorticity_2d(n, 73, lambda k: k * np.exp(-(k / 6.0) ** 2))
    got, t, _ = _run(fs, w, n, 2, "f64", steps, nu=nu, dt=dtmax, scheme="rk2", cfl=cfl)
    ref, tr = oracle_mod.step2d_ex(w, nu, dtmax, steps, scheme=2, cfl=cfl)
    assert tr < steps * dtmax * 0.9
    assert rel_l2(got, ref, kept_weight(n, 2)) <= 1e-11
    assert abs(t - tr) <= 1e-11 * tr


def test_time_of_fixed_steps(fs):
    plan = fs.Plan(32, nu=1e-3, dt=2.5e-3)
    d = torch.from_numpy(I.random_solenoidal_3d(32, seed=74, dtype=np.complex64)).cuda()
    plan.step(d, 3)
    plan.step(d, 4)
    t, dt = plan.time()
    assert abs(float(t.item()) - 7 * 2.5e-3) < 1e-15
    assert float(dt.item()) == np.float32(2.5e-3)
    plan.close()
