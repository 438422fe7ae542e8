"""GPU parity of the learned-closure path against the FP64 oracle.

Samples: the cutoff is a copy (bit exact); gradients and subgrid stress are
FP32 transforms of O(|u|^2) products, compared to 1e-5 of the largest product
magnitude (FP32 transforms of 32^3..128^3 carry ~1e-6 relative error).

LES: the network runs on BF16 matrix cores with BF16 hidden activations, so
the stress term agrees with the oracle (evaluated on the same BF16 weights and
BF16-rounded features) to a few BF16 ulps: 2e-2 relative L2 on the closure's
contribution; the resolved part keeps the solver's FP32 tolerance."""
import numpy as np
import pytest

from helpers import kept_mask, modes
from paper_1807_01769_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 576, 640, 4736, 4800, 5184


@pytest.fixture(scope="module")
def fs():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1807_01769_amd import fs as _fs
    return _fs


def _bf16_weights(p):
    q = np.array(p, dtype=np.float64)
    for a, b in ((OFF_W1, OFF_B1), (OFF_W2, OFF_B2), (OFF_W3, OFF_B3)):
        q[a:b] = torch.tensor(q[a:b], dtype=torch.float32).to(torch.bfloat16).double().numpy()
    return q


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _flat_field(n, seed):
    # broad spectrum so that the subgrid stress is far from zero
    return I.random_solenoidal_3d(n, seed=seed, shape_fn=lambda k: k ** 2 * np.exp(-0.15 * k),
                                  dtype=np.complex64)


@pytest.mark.parametrize("nf,nc,filt", [(32, 16, "sharp"), (64, 32, "sharp"), (128, 16, "sharp"),
                                         (64, 32, "box"), (128, 16, "box")])
def test_samples_vs_oracle(fs, oracle_mod, nf, nc, filt):
    print(f"case closure samples nf={nf} nc={nc} {filt}", flush=True)
    u = _flat_field(nf, 40 + nf + nc)
    fine = fs.Plan(nf, nu=1e-3, dt=1e-3)
    coarse = fs.Plan(nc, nu=1e-3, dt=1e-3)
    cl = fs.Closure(fine, coarse, filter=filt)
    box = filt == "box"
    uc, A, tau = cl.samples(_dev(u))
    torch.cuda.synchronize()
    u64 = u.astype(np.complex128)
    want_uc = oracle_mod.cutoff3d(u64, nc, box=box)
    got_uc = uc.cpu().numpy().astype(np.complex128)
    if box:  # the gains are single-precision products of sines
        assert np.abs(got_uc - want_uc).max() <= 3e-7 * np.abs(want_uc).max()
        want_uc = got_uc
    else:
        assert np.array_equal(got_uc, want_uc)
    ref_A = oracle_mod.grad3d(want_uc).reshape(9, -1)
    ref_tau = oracle_mod.sgs_tau3d(u64, nc, box=box).reshape(6, -1)
    uphys = np.stack([oracle_mod.irfftn(u64[c]) for c in range(3)])
    scale = float(np.abs(uphys).max()) ** 2
    eA = np.abs(A.cpu().numpy() - ref_A).max() / np.abs(ref_A).max()
    eT = np.abs(tau.cpu().numpy() - ref_tau).max() / scale
    print(f"A max err {eA:.2e}, tau max err {eT:.2e} (|tau|max/|u|^2 "
          f"{np.abs(ref_tau).max() / scale:.2e})", flush=True)
    assert np.abs(ref_tau).max() > 1e-3 * scale  # a real subgrid stress
    assert eA <= 1e-5
    assert eT <= 1e-5
    # moments (FP64, fixed order) and standardised features / targets
    m = cl.moments(A, tau).cpu().numpy()
    want_m = np.concatenate([(A.double() ** 2).mean(1).cpu().numpy(),
                             (tau.double() ** 2).mean(1).cpu().numpy()])
    assert np.allclose(m, want_m, rtol=1e-12, atol=0)
    a_scale = float(np.sqrt(m[:9].mean()))
    ts = np.sqrt(m[9:]).astype(np.float32)
    x, t = cl.features(A, a_scale, tau, ts)
    inv = np.float32(1.0) / np.float32(a_scale)
    want_x = torch.zeros((nc ** 3, 16), dtype=torch.bfloat16)
    want_x[:, :9] = (A.cpu().t() * torch.tensor(inv)).to(torch.bfloat16)
    assert torch.equal(x.cpu(), want_x)
    inv_t = torch.tensor(np.float32(1.0) / ts)
    assert torch.equal(t.cpu(), tau.cpu().t() * inv_t[None, :])
    for o in (cl, coarse, fine):
        o.close()


def test_samples_of_band_limited_field_have_zero_stress(fs):
    nf, nc = 64, 16
    u = _flat_field(nf, 9).astype(np.complex128)
    kz, ky, kx = np.meshgrid(modes(nf), modes(nf), np.arange(nf // 2 + 1), indexing="ij")
    band = (np.abs(kx) <= 2) & (np.abs(ky) <= 2) & (np.abs(kz) <= 2)
    u = np.where(band[None], u, 0).astype(np.complex64)
    fine, coarse = fs.Plan(nf), fs.Plan(nc)
    cl = fs.Closure(fine, coarse)
    _, A, tau = cl.samples(_dev(u))
    torch.cuda.synchronize()
    uu = float(A.abs().max())
    assert float(tau.abs().max()) <= 1e-6 * max(uu, 1.0)
    # tr A = 0 (solenoidal)
    tr = (A[0] + A[4] + A[8]).abs().max().item()
    assert tr <= 1e-5 * uu
    for o in (cl, coarse, fine):
        o.close()


def test_les_without_model_is_the_plain_solver(fs):
    n = 32
    u = _dev(I.random_solenoidal_3d(n, seed=5, dtype=np.complex64))
    plan = fs.Plan(n, nu=2e-3, dt=4e-3, forcing_power=1e-2)
    les = fs.Les(plan, None)
    a, b = u.clone(), u.clone()
    plan.step(a, 3)
    les.step(b, 3)
    ta, tb = plan.tendency(u), les.tendency(u)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(ta, tb)
    les.close()
    plan.close()


def _linear_eddy_net():
    from test_oracle_closure import linear_eddy_net
    return linear_eddy_net(5190)


def test_les_eddy_viscosity_network(fs):
    """The exactly linear network gives tend - nu_e |k|^2 u (GPU only, BF16
    hidden activations: 2e-2 on the closure's contribution)."""
    n, nu_e, a = 32, 0.02, 1.0
    u = I.random_solenoidal_3d(n, seed=6, dtype=np.complex64)
    net = fs.Mlp()
    net.set_params(torch.from_numpy(_linear_eddy_net().astype(np.float32)))
    plan = fs.Plan(n, nu=1e-3, dt=2e-3)
    les = fs.Les(plan, net, a, [nu_e * a] * 6)
    ud = _dev(u)
    t_les = les.tendency(ud).cpu().numpy().astype(np.complex128)
    t_dns = plan.tendency(ud).cpu().numpy().astype(np.complex128)
    kz, ky, kx = np.meshgrid(modes(n), modes(n), np.arange(n // 2 + 1), indexing="ij")
    k2 = (kx ** 2 + ky ** 2 + kz ** 2)[None]
    want = -nu_e * k2 * u.astype(np.complex128) * kept_mask(n, 3)[None]
    err = _rel(t_les - t_dns, want)
    print(f"eddy-viscosity closure term rel err {err:.3e}", flush=True)
    assert err <= 2e-2
    les.close()
    plan.close()
    net.close()


def _random_net(fs, seed):
    rng = np.random.default_rng(seed)
    p = (rng.standard_normal(5190) * 0.3).astype(np.float32)
    net = fs.Mlp()
    net.set_params(torch.from_numpy(p))
    return net, _bf16_weights(p)


@pytest.mark.parametrize("clip", [0.0, 0.5])
def test_les_tendency_vs_oracle(fs, oracle_mod, clip):
    print(f"case LES tendency n=32 clip={clip}", flush=True)
    n = 32
    u = I.random_solenoidal_3d(n, seed=7, dtype=np.complex64)
    u64 = u.astype(np.complex128)
    net, p64 = _random_net(fs, 8)
    a_scale = float(np.sqrt(np.mean(oracle_mod.grad3d(u64) ** 2)))
    ts = np.array([0.05, 0.04, 0.03, 0.02, 0.03, 0.04], np.float32)
    plan = fs.Plan(n, nu=1e-3, dt=2e-3, forcing_power=1e-2)
    les = fs.Les(plan, net, a_scale, ts, clip)
    ud = _dev(u)
    t_gpu = les.tendency(ud).cpu().numpy().astype(np.complex128)
    alpha = oracle_mod.forcing_alpha3d(u64, 1e-2)
    ref = oracle_mod.les_tendency3d(u64, p64, np.float32(a_scale), ts.astype(np.float64), clip=clip,
                                    alpha=alpha)
    base = oracle_mod.tendency3d(u64, alpha=alpha)
    e_sgs = _rel(t_gpu - base, ref - base)
    e_all = _rel(t_gpu, ref)
    share = np.linalg.norm(ref - base) / np.linalg.norm(ref)
    print(f"closure term rel err {e_sgs:.3e}; total {e_all:.3e}; closure share {share:.3f}",
          flush=True)
    assert share > 1e-2
    assert e_sgs <= 2e-2
    assert e_all <= 1e-5 + 2e-2 * share
    les.close()
    plan.close()
    net.close()


def test_les_steps_vs_oracle(fs, oracle_mod):
    print("case LES 3 steps n=32 forced", flush=True)
    n, nu, dt, power, steps = 32, 2e-3, 4e-3, 1e-2, 3
    u = I.random_solenoidal_3d(n, seed=9, dtype=np.complex64)
    u64 = u.astype(np.complex128)
    net, p64 = _random_net(fs, 10)
    a_scale = float(np.sqrt(np.mean(oracle_mod.grad3d(u64) ** 2)))
    ts = np.full(6, 0.05, np.float32)
    plan = fs.Plan(n, nu=nu, dt=dt, forcing_power=power)
    les = fs.Les(plan, net, a_scale, ts, 1.0)
    ud = _dev(u)
    les.step(ud, steps)
    got = ud.cpu().numpy().astype(np.complex128)
    ref = oracle_mod.step3d_les(u64, nu, dt, steps, p64, np.float32(a_scale), ts.astype(np.float64),
                                clip=1.0, power=power)
    plain = oracle_mod.step3d(u64, nu, dt, steps, power=power)
    effect = _rel(ref, plain)
    err = _rel(got, ref)
    print(f"LES {steps} steps rel err {err:.3e}; closure effect {effect:.3e}", flush=True)
    assert effect > 1e-4
    assert err <= 1e-5 + 2e-2 * effect
    # replaying the captured step graph on another state pointer
    ud2 = _dev(u)
    les.step(ud2, steps)
    assert torch.equal(ud2, ud)
    les.close()
    plan.close()
    net.close()
