"""The allocation-free diagnostics entry point (fs_energy_spectrum_static)
through the C ABI against the plan's fs_energy_spectrum on the same states:
two calls in a row, the second with a smaller input (they share the static
scratch), results bit for bit equal and within 1e-12 of the FP64 oracle; a
request beyond the static scratch is refused before anything is enqueued;
device memory is the same before and after the calls (nothing allocated)."""
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


def _plan_result(fs, a, ndim, n, prec):
    with fs.Plan(n, ndim=ndim, precision=prec, nu=1e-3, dt=1e-3) as p:
        spec, e, z = p.energy_spectrum(a)
        torch.cuda.synchronize()
        return spec.cpu().numpy(), float(e.item()), float(z.item())


@pytest.mark.parametrize("first,second", [((3, 64, "f32"), (3, 32, "f64")),
                                          ((3, 128, "f64"), (2, 64, "f32"))])
def test_static_spectrum_equals_plan_spectrum(fs, oracle_mod, first, second):
    print(f"case static spectrum {first} then {second}", flush=True)
    states = []
    for ndim, n, prec in (first, second):
        cd = np.complex64 if prec == "f32" else np.complex128
        a = (I.random_solenoidal_3d(n, seed=n) if ndim == 3 else I.ensemble_vorticity(2, n)).astype(cd)
        states.append((torch.from_numpy(a).cuda(), ndim, n, prec, a))
    refs = [_plan_result(fs, d, ndim, n, prec) for d, ndim, n, prec, _ in states]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    outs = []
    for d, ndim, n, prec, _ in states:   # two calls in a row, the second smaller
        spec, e, z = fs.energy_spectrum_static(d, ndim, n, prec)
        outs.append((spec, e, z))
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    for (spec, e, z), (rs, re_, rz), (_, ndim, n, prec, a) in zip(outs, refs, states):
        s = spec.cpu().numpy()
        assert np.array_equal(s, rs), np.abs(s - rs).max()
        assert float(e.item()) == re_ and float(z.item()) == rz
        os_, oe, oz = (oracle_mod.diag3d if ndim == 3 else oracle_mod.diag2d)(
            a.astype(np.complex128), len(s))
        assert abs(re_ - oe) <= 1e-12 * oe and abs(rz - oz) <= 1e-12 * oz
        assert np.abs(s - os_).max() <= 1e-12 * os_.max()
    # the outputs (48 bytes and the spectra) came from torch's cache, which
    # keeps its blocks; the library itself allocated nothing
    assert free0 - free1 <= 2 * 1024 * 1024


def test_static_spectrum_rejects_beyond_scratch(fs):
    print("case static spectrum beyond scratch", flush=True)
    d = torch.zeros((3, 32, 32, 17), dtype=torch.complex64, device="cuda")
    # n = 1024 in 3D: 1024 blocks of partial sums, nbins + 2 doubles each, beyond
    # the static scratch; refused before any launch (the pointers are not used)
    st = fs.lib.fs_energy_spectrum_static(3, 1024, 0, 6.283185307179586, d.data_ptr(),
                                          d.data_ptr(), 1024, None, None, None)
    assert st == -1
    assert "static scratch" in fs.lib.fs_last_error().decode()
    assert float(d.abs().max().item()) == 0.0
