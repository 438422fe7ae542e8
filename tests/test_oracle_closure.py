"""Pins of the FP64 reference closure pieces (CPU only): the sharp cutoff
filter, velocity gradients, subgrid stress, the MLP and its gradient, Adam,
and the LES tendency."""
import numpy as np
import pytest

from helpers import kept_mask, modes
from paper_1807_01769_amd import inputs as I


def test_cutoff_exact_and_idempotent(oracle_mod):
    nf, nc = 32, 16
    u = I.random_solenoidal_3d(nf, seed=21)
    c = oracle_mod.cutoff3d(u, nc)
    Kc = (nc - 1) // 3
    mf, mc = modes(nf), modes(nc)
    for iz in range(nc):
        for iy in range(nc):
            for ix in range(nc // 2 + 1):
                m = (mc[iz], mc[iy], ix)
                inside = max(abs(m[0]), abs(m[1]), m[2]) <= Kc
                want = u[:, m[0] % nf, m[1] % nf, ix] if inside else 0
                assert np.all(c[:, iz, iy, ix] == want)
    assert np.array_equal(oracle_mod.cutoff3d(c, nc), c)


def test_gradient_closed_form_and_trace(oracle_mod):
    n = 16
    A = oracle_mod.grad3d(I.taylor_green_3d(n))
    x = 2 * np.pi * np.arange(n) / n
    z, y, xx = np.meshgrid(x, x, x, indexing="ij")
    # u = (sin x cos y cos z, -cos x sin y cos z, 0)
    assert np.abs(A[0] - np.cos(xx) * np.cos(y) * np.cos(z)).max() < 1e-14
    assert np.abs(A[1] + np.sin(xx) * np.sin(y) * np.cos(z)).max() < 1e-14
    assert np.abs(A[2] + np.sin(xx) * np.cos(y) * np.sin(z)).max() < 1e-14
    assert np.abs(A[4] + np.cos(xx) * np.cos(y) * np.cos(z)).max() < 1e-14
    assert np.abs(A[6:]).max() < 1e-14
    R = oracle_mod.grad3d(I.random_solenoidal_3d(n, seed=5))
    assert np.abs(R[0] + R[4] + R[8]).max() < 1e-13 * np.abs(R).max()


def test_sgs_tau_zero_for_band_limited_field(oracle_mod):
    nf, nc = 32, 16
    u = I.random_solenoidal_3d(nf, seed=3)
    kz, ky, kx = np.meshgrid(modes(nf), modes(nf), np.arange(nf // 2 + 1), indexing="ij")
    band = (np.abs(kx) <= 2) & (np.abs(ky) <= 2) & (np.abs(kz) <= 2)
    u = np.where(band[None], u, 0)
    tau = oracle_mod.sgs_tau3d(u, nc)
    assert np.abs(tau).max() < 1e-15


def test_sgs_tau_matches_galerkin_definition(oracle_mod):
    """cutoff(u_i u_j) from the exact triad sum of the fine field, evaluated at
    the coarse points, minus the product of the filtered fields there, trace
    removed."""
    from test_oracle_ns import _convolve, _cube_from_half
    nf, nc = 16, 8
    Kf, Kc = (nf - 1) // 3, (nc - 1) // 3
    u = I.random_solenoidal_3d(nf, seed=4, shape_fn=lambda k: np.exp(-0.2 * k))
    tau = oracle_mod.sgs_tau3d(u, nc)
    uc = _cube_from_half(u, nf, 3)  # [3][x][y][z], modes -Kf..Kf
    x = 2 * np.pi * np.arange(nc) / nc
    z, y, xx = np.meshgrid(x, x, x, indexing="ij")

    def at_points(cube, K):  # sum of the cube's coefficients |m_a| <= Kc at the coarse points
        out = np.zeros((nc, nc, nc), np.complex128)
        for a in range(-Kc, Kc + 1):
            for b in range(-Kc, Kc + 1):
                for c in range(-Kc, Kc + 1):
                    v = cube[a + K, b + K, c + K]
                    if v != 0:
                        out += v * np.exp(1j * (a * xx + b * y + c * z))
        return out.real

    ubar = [at_points(uc[c], Kf) for c in range(3)]
    raw = []
    for (i, j) in oracle_mod.TAU_COMPONENTS:
        prod = _convolve(uc[i], uc[j], Kf, 3)  # modes -Kf..Kf of u_i u_j (exact)
        raw.append(at_points(prod, Kf) - ubar[i] * ubar[j])
    tr = (raw[0] + raw[1] + raw[2]) / 3.0
    for s in range(6):
        ref = raw[s] - (tr if s < 3 else 0.0)
        assert np.abs(tau[s] - ref).max() <= 1e-12 * np.abs(ref).max() + 1e-16


def test_mlp_gradient_matches_finite_differences(oracle_mod):
    rng = np.random.default_rng(0)
    npar = oracle_mod.mlp_nparams()
    assert npar == 5190
    p = rng.standard_normal(npar) * 0.3
    x = rng.standard_normal((7, 9))
    t = rng.standard_normal((7, 6))
    loss, g = oracle_mod.mlp_loss_grad(p, x, t)
    y = oracle_mod.mlp_forward(p, x)
    assert abs(loss - np.mean((y - t) ** 2)) <= 1e-14 * loss
    h = 1e-6
    for idx in list(rng.choice(npar, 40, replace=False)) + [0, 575, 576, 639, 640, 4799, 4800, 5183, 5189]:
        pp, pm = p.copy(), p.copy()
        pp[idx] += h
        pm[idx] -= h
        fd = (oracle_mod.mlp_loss_grad(pp, x, t)[0] - oracle_mod.mlp_loss_grad(pm, x, t)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-7 * max(1.0, abs(g[idx])) + 1e-9, idx


def test_adam_first_step_closed_form(oracle_mod):
    g = np.array([0.5, -2.0, 1e-3, -7.0])
    w = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    oracle_mod.adam(w, m, v, g, 1, lr=1e-2)
    # m_hat = g, v_hat = g^2: the step is lr * g / (|g| + eps)
    assert np.allclose(w, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=0)


def test_les_tendency_reductions(oracle_mod):
    n = 16
    u = I.random_solenoidal_3d(n, seed=8)
    zero = np.zeros((6, n, n, n))
    assert np.array_equal(oracle_mod.tendency3d_les(u, zero), oracle_mod.tendency3d(u))
    # isotropic stress is a pressure: projected away
    iso = np.zeros((6, n, n, n))
    rng = np.random.default_rng(1)
    iso[0] = iso[1] = iso[2] = rng.standard_normal((n, n, n))
    nz = np.zeros_like(u)
    assert np.abs(oracle_mod.tendency3d_les(nz, iso)).max() < 1e-15
    # tau_xy = sin y: -d_j tau_ij = (-cos y, 0, 0), already solenoidal
    x = 2 * np.pi * np.arange(n) / n
    z, y, xx = np.meshgrid(x, x, x, indexing="ij")
    t = np.zeros((6, n, n, n))
    t[3] = np.sin(y)
    got = oracle_mod.tendency3d_les(nz, t)
    ref = np.zeros_like(got)
    ref[0, 0, 1, 0] = -0.5
    ref[0, 0, n - 1, 0] = -0.5
    assert np.abs(got - ref).max() < 1e-15


# ---- LES with the network closure -------------------------------------------
def linear_eddy_net(npar):
    """Parameters of a network that is exactly linear, y = C x: the pair
    GELU(z) - GELU(-z) = z carries each feature through both hidden layers.
    C maps the standardised gradients to -(A + A^T) in xx, yy, zz, xy, xz, yz
    order, so with tau_scale = nu_e * a_scale the stress is the eddy-viscosity
    stress -nu_e (A + A^T)."""
    W1 = np.zeros((64, 9))
    W2 = np.zeros((64, 64))
    W3 = np.zeros((6, 64))
    for k in range(9):
        W1[2 * k, k], W1[2 * k + 1, k] = 1.0, -1.0
        W2[2 * k, 2 * k], W2[2 * k, 2 * k + 1] = 1.0, -1.0
        W2[2 * k + 1, 2 * k], W2[2 * k + 1, 2 * k + 1] = -1.0, 1.0
    Cm = np.zeros((6, 9))
    Cm[0, 0] = Cm[1, 4] = Cm[2, 8] = -2.0
    Cm[3, 1] = Cm[3, 3] = -1.0
    Cm[4, 2] = Cm[4, 6] = -1.0
    Cm[5, 5] = Cm[5, 7] = -1.0
    for k in range(9):
        W3[:, 2 * k], W3[:, 2 * k + 1] = Cm[:, k], -Cm[:, k]
    p = np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), W3.ravel(), np.zeros(6)])
    assert p.size == npar
    return p


def test_round_bf16_ties_and_torch(oracle_mod):
    import torch
    e = 2.0 ** -8
    cases = {1 + e: 1.0, 1 + 3 * e: 1 + 4 * e, 1 + e + 2.0 ** -20: 1 + 2 * e,
             -(1 + 3 * e): -(1 + 4 * e), 0.0: 0.0, 3.0: 3.0, 2.0 ** -30 * (1 + e): 2.0 ** -30}
    for x, want in cases.items():
        assert oracle_mod.round_bf16(x) == want, x
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-8, 8, 20000))).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(oracle_mod.round_bf16(x.astype(np.float64)), ref)


def test_linear_network_is_exactly_linear(oracle_mod):
    p = linear_eddy_net(oracle_mod.mlp_nparams())
    x = np.random.default_rng(0).standard_normal((50, 9)) * 3
    y = oracle_mod.mlp_forward(p, x)
    assert np.abs(y[:, 0] + 2 * x[:, 0]).max() < 1e-14 * 10
    assert np.abs(y[:, 3] + x[:, 1] + x[:, 3]).max() < 1e-14 * 10
    assert np.abs(y[:, 5] + x[:, 5] + x[:, 7]).max() < 1e-14 * 10


def test_les_tendency_eddy_viscosity_closed_form(oracle_mod):
    """-d_j tau_ij with tau = -nu_e (A + A^T) is nu_e lap u for a solenoidal u."""
    n, nu_e, a = 16, 0.03, 1.7
    u = I.random_solenoidal_3d(n, seed=12) * kept_mask(n, 3)[None]
    p = linear_eddy_net(oracle_mod.mlp_nparams())
    got = oracle_mod.les_tendency3d(u, p, a, [nu_e * a] * 6, bf16=False)
    base = oracle_mod.tendency3d(u)
    kz, ky, kx = np.meshgrid(modes(n), modes(n), np.arange(n // 2 + 1), indexing="ij")
    k2 = (kx ** 2 + ky ** 2 + kz ** 2).astype(np.float64)
    want = base - nu_e * k2[None] * u
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    # the same with forcing on: the forcing term is untouched by the closure
    alpha = 0.37
    got_f = oracle_mod.les_tendency3d(u, p, a, [nu_e * a] * 6, bf16=False, alpha=alpha)
    want_f = oracle_mod.tendency3d(u, alpha=alpha) - nu_e * k2[None] * u
    assert np.abs(got_f - want_f).max() <= 1e-13 * np.abs(want_f).max()


def test_les_step_eddy_viscosity_equals_higher_viscosity(oracle_mod):
    """LES with the eddy-viscosity network = DNS at nu + nu_e up to the
    scheme's error (the extra viscosity is explicit in one and exact in the
    other): over 5 steps the gap shrinks as dt^5, fourth order globally."""
    n, nu, nu_e, a = 16, 0.01, 0.02, 1.0
    u0 = I.random_solenoidal_3d(n, seed=13) * kept_mask(n, 3)[None]
    p = linear_eddy_net(oracle_mod.mlp_nparams())
    errs = []
    for dt in (2e-3, 4e-3):
        les = oracle_mod.step3d_les(u0, nu, dt, 5, p, a, [nu_e * a] * 6, bf16=False, power=1e-2)
        dns = oracle_mod.step3d(u0, nu + nu_e, dt, 5, power=1e-2)
        errs.append(np.linalg.norm(les - dns) / np.linalg.norm(dns))
    ref = oracle_mod.step3d(u0, nu, 4e-3, 5, power=1e-2)
    effect = np.linalg.norm(ref - dns) / np.linalg.norm(dns)
    assert effect > 1e-3          # the closure does something
    assert errs[0] < 2e-12, errs
    assert 25 < errs[1] / errs[0] < 40, errs


def test_les_step_null_and_isotropic_outputs(oracle_mod):
    n, nu, dt = 16, 0.01, 2e-3
    u0 = I.random_solenoidal_3d(n, seed=14) * kept_mask(n, 3)[None]
    npar = oracle_mod.mlp_nparams()
    rng = np.random.default_rng(2)
    p = rng.standard_normal(npar) * 0.2
    p[4800:5190] = 0.0           # W3 = 0, b3 = 0: zero stress
    ref = oracle_mod.step3d(u0, nu, dt, 3, power=1e-2)
    out = oracle_mod.step3d_les(u0, nu, dt, 3, p, 1.0, [1.0] * 6, power=1e-2)
    assert np.array_equal(out, ref)
    p[5184:5187] = 4.0           # b3 = (4, 4, 4, 0, 0, 0): a uniform pressure
    out = oracle_mod.step3d_les(u0, nu, dt, 3, p, 1.0, [0.5] * 6, power=1e-2)
    assert np.abs(out - ref).max() <= 1e-15 * np.abs(ref).max()


def test_les_tau_clip_and_scale(oracle_mod):
    n = 8
    u = I.random_solenoidal_3d(n, seed=15)
    p = np.zeros(oracle_mod.mlp_nparams())
    p[5184:5190] = [3.0, -3.0, 0.5, -0.25, 2.0, -0.999]
    ts = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    tau = oracle_mod.les_tau3d(u, p, 1.0, ts, clip=1.0)
    want = np.array([1.0, -1.0, 0.5, -0.25, 1.0, -0.999]) * ts
    assert np.array_equal(tau.reshape(6, -1), np.repeat(want[:, None], n ** 3, axis=1))


def _band_field(n, kmax, seed):
    """Random solenoidal spectral velocity with modes |m_a| <= kmax only."""
    u = I.random_solenoidal_3d(n, seed=seed)
    m = np.fft.fftfreq(n, 1.0 / n)
    keep = (np.abs(m)[:, None, None] <= kmax) & (np.abs(m)[None, :, None] <= kmax) & \
        (np.arange(n // 2 + 1)[None, None, :] <= kmax)
    return u * keep[None]


def _eval(uh, pts):
    """u(x) at arbitrary points from the half spectrum (weights 1 on kx = 0, 2 else)."""
    n = uh.shape[-2]
    m = np.fft.fftfreq(n, 1.0 / n)
    kz, ky, kx = np.meshgrid(m, m, np.arange(n // 2 + 1), indexing="ij")
    w = np.where(kx == 0, 1.0, 2.0)
    nz = np.nonzero(np.abs(uh).sum(axis=0) > 0)
    out = np.zeros((3, len(pts)))
    for c in range(3):
        coef = (w * uh[c])[nz]
        ph = np.exp(1j * (np.outer(pts[:, 0], kx[nz]) + np.outer(pts[:, 1], ky[nz]) +
                          np.outer(pts[:, 2], kz[nz])))
        out[c] = np.real(ph @ coef)
    return out


def _tophat(uh, x0, D, f):
    """Average of f(u) over the cube of side D centred at x0 (Gauss-Legendre, 12^3)."""
    g, wg = np.polynomial.legendre.leggauss(12)
    o = 0.5 * D * g
    pts = np.stack(np.meshgrid(o, o, o, indexing="ij"), -1).reshape(-1, 3)
    ww = np.einsum("i,j,k->ijk", wg, wg, wg).reshape(-1) / 8.0
    return f(_eval(uh, x0[None, :] + pts)) @ ww


def test_box_filter_is_the_tophat_average(oracle_mod):
    nf, nc = 32, 16                     # Kc = 5, box width D = 2 pi / 10
    Kc, D = 5, 2 * np.pi / 10
    u = _band_field(nf, Kc, 601)        # nothing beyond the cutoff
    ub = oracle_mod.cutoff3d(u, nc, box=True)
    phys = np.stack([np.fft.irfftn(ub[c], s=(nc,) * 3, axes=(0, 1, 2)) * nc ** 3
                     for c in range(3)])
    rng = np.random.default_rng(3)
    for _ in range(4):
        iz, iy, ix = rng.integers(0, nc, 3)
        x0 = 2 * np.pi * np.array([ix, iy, iz]) / nc
        want = _tophat(u, x0, D, lambda v: v)
        assert np.abs(phys[:, iz, iy, ix] - want).max() <= 1e-12 * np.abs(phys).max()


def test_box_filter_stress_is_the_tophat_covariance(oracle_mod):
    nf, nc = 32, 16
    D = 2 * np.pi / 10
    u = _band_field(nf, 2, 603)         # products reach |m| <= 4 < Kc: no cutoff loss
    tau = oracle_mod.sgs_tau3d(u, nc, box=True)
    rng = np.random.default_rng(4)
    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    for _ in range(3):
        iz, iy, ix = rng.integers(0, nc, 3)
        x0 = 2 * np.pi * np.array([ix, iy, iz]) / nc
        mean = _tophat(u, x0, D, lambda v: v)
        cov = np.array([_tophat(u, x0, D, lambda v, i=i, j=j: v[i] * v[j]) - mean[i] * mean[j]
                        for i, j in pairs])
        cov[:3] -= cov[:3].mean()
        assert np.abs(tau[:, iz, iy, ix] - cov).max() <= 1e-12 * np.abs(tau).max()
    # unlike the sharp cutoff, the box filter leaves a stress on band-limited fields
    assert np.abs(tau).max() > 1e-3 * np.abs(oracle_mod.sgs_tau3d(_band_field(nf, 8, 605), nc)).max()
