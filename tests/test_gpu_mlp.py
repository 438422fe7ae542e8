"""GPU parity of the closure network kernels (BF16 matrix cores, FP32
accumulate) against the FP64 oracle evaluated on the same BF16-rounded
weights and inputs.  The GPU also rounds hidden activations to BF16 between
layers, so agreement is to a few BF16 ulps (2^-8 relative): tolerance 2e-2
in relative L2."""
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


OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 576, 640, 4736, 4800, 5184


def _bf16_weights(p):
    """Round the weight matrices (not the biases) to BF16, as the kernels use them."""
    q = p.copy()
    for a, b in ((OFF_W1, OFF_B1), (OFF_W2, OFF_B2), (OFF_W3, OFF_B3)):
        q[a:b] = torch.tensor(q[a:b], dtype=torch.float32).to(torch.bfloat16).double().numpy()
    return q


def _setup(fs, P, seed):
    rng = np.random.default_rng(seed)
    net = fs.Mlp(seed=7)
    p = (rng.standard_normal(5190) * 0.25).astype(np.float32)
    net.set_params(torch.from_numpy(p))
    x = rng.standard_normal((P, 9)).astype(np.float32)
    xb = fs.bf16_features(x)
    x64 = xb[:, :9].double().cpu().numpy()
    t = rng.standard_normal((P, 6)).astype(np.float32)
    return net, p, xb, x64, t


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("P", [16, 1000, 4099])
def test_forward_vs_oracle(fs, oracle_mod, P):
    print(f"case mlp forward P={P}", flush=True)
    net, p, xb, x64, _ = _setup(fs, P, P)
    y = net.forward(xb)
    torch.cuda.synchronize()
    ref = oracle_mod.mlp_forward(_bf16_weights(p.astype(np.float64)), x64)
    err = _rel(y.double().cpu().numpy(), ref)
    print(f"forward rel err {err:.3e}", flush=True)
    assert err <= 2e-2
    net.close()


@pytest.mark.parametrize("P", [16, 3000])
def test_gradient_vs_oracle(fs, oracle_mod, P):
    print(f"case mlp gradient P={P}", flush=True)
    net, p, xb, x64, t = _setup(fs, P, 100 + P)
    g, loss = net.grad(xb, torch.from_numpy(t).cuda())
    g2, loss2 = net.grad(xb, torch.from_numpy(t).cuda())
    torch.cuda.synchronize()
    assert torch.equal(g, g2) and torch.equal(loss, loss2)  # deterministic
    rl, rg = oracle_mod.mlp_loss_grad(_bf16_weights(p.astype(np.float64)), x64, t.astype(np.float64))
    gg = g.double().cpu().numpy()
    print(f"loss {float(loss.cpu()):.6e} vs {rl:.6e}", flush=True)
    assert abs(float(loss.cpu()) - rl) <= 2e-2 * rl
    for name, a, b in (("W1", OFF_W1, OFF_B1), ("b1", OFF_B1, OFF_W2), ("W2", OFF_W2, OFF_B2),
                       ("b2", OFF_B2, OFF_W3), ("W3", OFF_W3, OFF_B3), ("b3", OFF_B3, 5190)):
        err = _rel(gg[a:b], rg[a:b])
        print(f"grad {name} rel err {err:.3e}", flush=True)
        assert err <= 2e-2, name
    net.close()


def test_adam_step_matches_oracle(fs, oracle_mod):
    print("case mlp adam", flush=True)
    net, p, xb, x64, t = _setup(fs, 512, 5)
    tt = torch.from_numpy(t).cuda()
    g, _ = net.grad(xb, tt)
    net.train_step(xb, tt, lr=1e-3)
    w1 = net.get_params()
    torch.cuda.synchronize()
    w = p.astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    oracle_mod.adam(w, m, v, g.double().cpu().numpy(), 1, lr=1e-3)
    assert np.abs(w1.double().cpu().numpy() - w).max() <= 1e-6
    net.close()


def test_training_reduces_loss(fs):
    print("case mlp training", flush=True)
    rng = np.random.default_rng(9)
    P = 8192
    x = rng.standard_normal((P, 9)).astype(np.float32)
    A = rng.standard_normal((9, 6)).astype(np.float32) * 0.5
    t = np.tanh(x @ A).astype(np.float32)
    net = fs.Mlp(seed=7)
    xb, tt = fs.bf16_features(x), torch.from_numpy(t).cuda()
    first = float(net.train_step(xb, tt, lr=3e-3).cpu())
    for _ in range(300):
        last = net.train_step(xb, tt, lr=3e-3)
    last = float(last.cpu())
    print(f"loss {first:.4f} -> {last:.4f}", flush=True)
    assert last < 0.2 * first
    net.close()
