"""GPU checks of two boundary options: a caller-owned workspace gives the same
steps as the plan's own allocation (bitwise), and FS_CHECK_FINITE reports a
step that wrote non-finite values at the next call (3D and 2D) and leaves the
plan usable; without it the same input steps silently."""
import numpy as np
import pytest

from paper_1807_01769_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fs():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1807_01769_amd import fs as _fs
    return _fs


@pytest.mark.parametrize("ndim,n,prec", [(3, 64, "f32"), (2, 128, "f64")])
def test_caller_workspace(fs, ndim, n, prec):
    print(f"case caller workspace {ndim}d n={n} {prec}", flush=True)
    kw = dict(ndim=ndim, precision=prec)
    if ndim == 3:
        kw["forcing_power"] = 0.05
        st = I.random_solenoidal_3d(n, seed=501, dtype=np.complex64)
    else:
        st = I.random_vorticity_2d(n, 501, lambda k: k * np.exp(-(k / 6.0) ** 2))
    need = fs.Plan.required_bytes(n, **kw)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    own = fs.Plan(n, nu=1e-3, dt=2e-3, **kw)
    assert own.workspace_bytes() == need
    mine = fs.Plan(n, nu=1e-3, dt=2e-3, workspace=ws, **kw)
    assert mine.workspace_bytes() == need
    a = torch.from_numpy(st).cuda()
    b = a.clone()
    own.step(a, 4)
    mine.step(b, 4)
    assert torch.equal(a, b)
    with pytest.raises(fs.FsError):
        fs.Plan(n, nu=1e-3, dt=2e-3, workspace=ws[: need - 256], **kw)
    own.close()
    mine.close()


@pytest.mark.parametrize("ndim", [3, 2])
def test_check_finite(fs, ndim):
    print(f"case check finite {ndim}d", flush=True)
    n = 32
    if ndim == 3:
        st = I.random_solenoidal_3d(n, seed=503, dtype=np.complex64)
        bad = st.copy()
        bad[1, 2, 3, 4] = np.nan
    else:
        st = I.random_vorticity_2d(n, 503, lambda k: np.exp(-(k / 4.0) ** 2)).astype(np.complex64)
        bad = st.copy()
        bad[2, 3] = np.inf
    plan = fs.Plan(n, ndim=ndim, nu=1e-3, dt=1e-3, check_finite=True)
    good = torch.from_numpy(st).cuda()
    plan.step(good, 3)
    plan.step(good, 2)           # the clean steps report nothing
    d = torch.from_numpy(bad).cuda()
    plan.step(d, 2)              # enqueued; the next call reports it
    with pytest.raises(fs.FsError) as err:
        plan.step(d, 1)
    assert err.value.status == fs.FS_E_NONFINITE
    again = torch.from_numpy(st).cuda()
    plan.step(again, 3)          # the plan stays usable
    plan.step(again, 1)
    assert torch.isfinite(torch.view_as_real(again)).all()
    plan.close()
    # without the flag the same input steps silently
    quiet = fs.Plan(n, ndim=ndim, nu=1e-3, dt=1e-3)
    d = torch.from_numpy(bad).cuda()
    quiet.step(d, 2)
    quiet.step(d, 1)
    torch.cuda.synchronize()
    assert not torch.isfinite(torch.view_as_real(d)).all()
    quiet.close()
