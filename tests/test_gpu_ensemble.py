"""GPU parity of the uneven-size 2D ensemble: every run of the ensemble must
match the same run advanced alone (bitwise where the schedule is the same
arithmetic) and the FP64 oracle (2D step), on the graph and the direct path."""
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


def _rel(got, ref, n):
    w, m = kept_weight(n, 2), kept_mask(n, 2)
    return float(np.sqrt(np.sum(w * np.abs(np.where(m, got - ref, 0)) ** 2) /
                         np.sum(w * np.abs(np.where(m, ref, 0)) ** 2)))


@pytest.mark.parametrize("graphs,autotune", [(True, True), (False, False)])
def test_ensemble_matches_single_runs_and_oracle(fs, oracle_mod, graphs, autotune):
    print(f"case ensemble graphs={graphs} autotune={autotune}", flush=True)
    sizes = [128, 64, 256, 64, 512, 128, 256]
    nu, dt, steps = 1e-4, 5e-4, 6
    fields = [I.ensemble_vorticity(r, n).astype(np.complex64) for r, n in enumerate(sizes)]
    with fs.Ensemble(sizes, nu=nu, dt=dt, graphs=graphs, autotune=autotune) as ens:
        print("schedule", ens.schedule(), flush=True)
        st = ens.pack(fields)
        ens.step(st, steps)
        torch.cuda.synchronize()
        got = [ens.unpack(st, r).cpu().numpy() for r in range(len(sizes))]
    for r, n in enumerate(sizes):
        with fs.Plan(n, ndim=2, precision="f32", nu=nu, dt=dt) as p:
            s1 = torch.from_numpy(fields[r]).cuda()
            p.step(s1, steps)
            torch.cuda.synchronize()
            alone = s1.cpu().numpy()
        ref = oracle_mod.step2d(fields[r].astype(np.complex128), nu, dt, steps)
        e_alone = _rel(got[r].astype(np.complex128), alone.astype(np.complex128), n)
        e_ref = _rel(got[r].astype(np.complex128), ref, n)
        print(f"run {r} n={n}: vs alone {e_alone:.2e}, vs oracle {e_ref:.2e}", flush=True)
        assert e_alone <= 1e-6
        assert e_ref <= 1e-5


@pytest.mark.timeout(900)
def test_full_ensemble_200_steps(fs, oracle_mod):
    """The full configuration: 256 runs (128 at 128^2, 96 at 256^2, 32 at
    512^2), 200 RK4 steps in one graph launch; a stratified sample of more
    than 10 % of the runs -- every tenth run of each size class, and its last
    run -- against the FP64 oracle's 200 steps."""
    print("case full ensemble 256 runs, 200 steps", flush=True)
    nu, dt, steps = 1e-4, 5e-4, 200
    sizes = I.ensemble_sizes()
    fields = [I.ensemble_vorticity(r, n).astype(np.complex64) for r, n in enumerate(sizes)]
    with fs.Ensemble(sizes, nu=nu, dt=dt) as ens:
        st = ens.pack(fields)
        ens.step(st, steps)
        torch.cuda.synchronize()
        picks = sorted(set(list(range(0, 128, 10)) + [127] + list(range(128, 224, 10)) + [223] +
                           list(range(224, 256, 10)) + [255]))
        assert len(picks) >= 26
        got = {r: ens.unpack(st, r).cpu().numpy() for r in picks}
    for r in picks:
        n = sizes[r]
        ref = oracle_mod.step2d(fields[r].astype(np.complex128), nu, dt, steps)
        e = _rel(got[r].astype(np.complex128), ref, n)
        print(f"run {r} n={n}: 200 steps vs oracle {e:.2e}", flush=True)
        assert e <= 1e-5


@pytest.mark.parametrize("graphs,steps", [(True, 3), (False, 1), (False, 2)])
def test_resident_classes_match_class_batched(fs, graphs, steps):
    """Classes of 64 and 128 points a side are advanced block-resident (one
    block per run, its intermediate in LDS through all the steps of a call):
    every run must match the class-batched passes to rounding (the same
    operations in the same order; the compiler may contract multiply-adds
    differently in the two kernels), for classes of one run and of several,
    next to a class-batched 256^2 class; a run alone in its resident class
    must match the same run in a larger one bit for bit."""
    print(f"case resident vs class-batched graphs={graphs} steps={steps}", flush=True)
    sizes = [128, 64, 256, 128, 128, 64, 64, 64]
    nu, dt = 1e-4, 5e-4
    fields = [I.ensemble_vorticity(50 + r, n).astype(np.complex64) for r, n in enumerate(sizes)]
    out = {}
    for resident in (True, False):
        with fs.Ensemble(sizes, nu=nu, dt=dt, graphs=graphs, resident=resident) as ens:
            sch = ens.schedule()
            print("schedule", sch, flush=True)
            assert [c.get("resident", False) for c in sch] == [resident, resident, False]
            st = ens.pack(fields)
            ens.step(st, steps)
            torch.cuda.synchronize()
            out[resident] = st.cpu()
    assert torch.isfinite(torch.view_as_real(out[True])).all()
    offs = ens.offsets
    for r, n in enumerate(sizes):
        a = out[True][offs[r]:offs[r + 1]].numpy().reshape(n, n // 2 + 1).astype(np.complex128)
        b = out[False][offs[r]:offs[r + 1]].numpy().reshape(n, n // 2 + 1).astype(np.complex128)
        e = _rel(a, b, n)
        print(f"run {r} n={n}: resident vs class-batched {e:.2e}, max |diff| "
              f"{np.max(np.abs(a - b)):.2e}", flush=True)
        assert e <= 1e-6
        if n == 256:
            assert np.array_equal(a, b)  # the same kernels
    with fs.Ensemble([128], nu=nu, dt=dt, graphs=graphs) as ens:
        st = ens.pack(fields[:1])
        ens.step(st, steps)
        torch.cuda.synchronize()
        one = st.cpu()
    assert torch.equal(one, out[True][:one.numel()])
