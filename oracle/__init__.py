"""FP64 CPU reference of the pseudo-spectral Navier-Stokes RK4 step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library (``paper_1807_01769_amd``): the C source ``fs_oracle.c`` is
compiled on its own with gcc and loaded here with ctypes.

Every function is the plain definition of an operation the paper names
(section "Implementation and architecture": FFT/IFFT, dealiasing, curl,
divergence operators and RK4 time stepping; section "CFD pseudo-spectral code
comparisons": the 3D step's tasks FFT, RK4, curl, vector product and
projection, with part of the linear terms treated exactly).

Pins (tests/test_oracle_*.py, all CPU):
  fft / rfftn / irfftn   brute-force DFT, round trip, Parseval, single modes,
                         numpy.fft cross-check
  dft_mode3d             brute-force DFT (every mode of a small cube)
  tendency3d             exact Galerkin triad sum (dealiasing), closed-form
                         Taylor-Green vorticity/product, energy and helicity
                         conservation at nu = 0, solenoidality, ABC flow N = 0
  tendency2d             Taylor-Green N = 0, triad sum, energy and enstrophy
                         conservation (enstrophy only when alias free)
  step2d / step3d        exact decaying Taylor-Green / ABC solutions, a scalar
                         ODE with closed form (order-4 convergence of the
                         Lawson scheme), energy budget dE/dt = -2 nu Z
  step*_ex (RK2, CFL)    order 2 of the Lawson midpoint rule on the scalar ODE,
                         exact decays, the CFL step from the physical velocity
                         maximum (checked against numpy's inverse FFT), the
                         fixed step when the CFL bound exceeds it
  forcing_alpha3d        injected power equals the prescribed power
  diag2d / diag3d        closed-form Taylor-Green energy, enstrophy and shell,
                         sum of the spectrum equals the energy
  tendency2d_strat /     single plane waves are exact nonlinear solutions
  step2d_strat           (internal gravity waves: closed-form oscillation at
                         N |kx| / |k| with viscous decay, fourth-order
                         convergence of the step to it); kinetic plus
                         potential energy conserved by the inviscid tendency;
                         N2 = 0, b = 0 reduces to the 2D solver
  step3d_rot             a single helical mode is an exact inertial wave
                         (frequency f kz / |k|, viscous decay) reproduced to
                         rounding; f = 0 reduces to step3d; the propagator is
                         orthogonal (energy kept at nu = 0, N = 0)
  spectra1d2d / 3d       single Fourier modes land in their bins with the
                         closed-form energy; every axis sums to the component
                         energy measured in physical space
  transfer2d / 3d        per-shell dE/dt at nu = 0 from centred differences of
                         the shell spectrum under the exact-in-time step
                         (fourth-order scheme); total 0 without forcing (and
                         2D enstrophy rate 0 when alias free), total = power
                         with forcing
  cutoff3d / grad3d      tr A = 0 for solenoidal fields, closed-form gradient
                         of Taylor-Green, cutoff idempotent and exact on kept
  sgs_tau3d              zero for band-limited fields (sharp cutoff), symmetric, traceless,
                         equals the triad definition on a small grid
  mlp_forward/loss_grad  central finite differences
  adam                   closed form of the first step (sign descent by lr)
  tendency3d_les         zero stress reduces to tendency3d; the stress term
                         alone equals the projected divergence
  round_bf16             ties-to-even cases, torch's bfloat16 conversion
  les_tendency3d         an exactly linear network (GELU(z) - GELU(-z) = z)
                         that outputs the eddy-viscosity stress
                         -nu_e (A + A^T) gives tendency3d - nu_e |k|^2 u
  step3d_les             that network reproduces step3d at nu + nu_e (to the
                         scheme's order); zero or isotropic output leaves
                         step3d unchanged
Beyond those pins, long nonlinear runs are "parity unpinned": the reference
and the GPU path are compared with each other only.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        vp, i, d = C.c_void_p, C.c_int, C.c_double
        L.or_fft1d.argtypes = [vp, i, i]
        L.or_fftn.argtypes = [vp, i, vp, i]
        L.or_rfftn.argtypes = [i, i, vp, vp]
        L.or_irfftn.argtypes = [i, i, vp, vp]
        L.or_tendency3d.argtypes = [i, d, vp, d, d, d, vp]
        L.or_tendency2d.argtypes = [i, d, vp, vp]
        L.or_forcing_alpha3d.argtypes = [i, d, vp, d, d, d]
        L.or_forcing_alpha3d.restype = d
        L.or_step3d.argtypes = [i, d, d, d, d, d, d, vp, i]
        L.or_step2d.argtypes = [i, d, d, d, vp, i]
        L.or_diag3d.argtypes = [i, d, vp, i, vp, vp, vp]
        L.or_diag2d.argtypes = [i, d, vp, i, vp, vp, vp]
        L.or_set_threads.argtypes = [i]
        L.or_get_threads.restype = i
        L.or_kept.argtypes = [i, i]
        L.or_kept.restype = i
        L.or_dft_mode3d.argtypes = [i, vp, i, i, i, vp, vp]
        L.or_lawson_scalar.argtypes = [d, d, d, i]
        L.or_cutoff3d.argtypes = [i, vp, i, i, vp]
        L.or_grad3d.argtypes = [i, d, vp, vp]
        L.or_sgs_tau3d.argtypes = [i, vp, i, i, vp]
        L.or_mlp_nparams.restype = i
        L.or_mlp_forward.argtypes = [vp, vp, C.c_int64, vp]
        L.or_mlp_loss_grad.argtypes = [vp, vp, vp, C.c_int64, vp]
        L.or_mlp_loss_grad.restype = d
        L.or_adam.argtypes = [vp, vp, vp, vp, i, i, d, d, d, d]
        L.or_tendency3d_les.argtypes = [i, d, vp, vp, vp]
        L.or_lawson_scalar.restype = d
        L.or_lawson_scalar2.argtypes = [d, d, d, i]
        L.or_lawson_scalar2.restype = d
        L.or_step3d_ex.argtypes = [i, d, d, d, d, d, d, i, d, vp, i, vp]
        L.or_step2d_ex.argtypes = [i, d, d, d, i, d, vp, i, vp]
        L.or_umax.argtypes = [i, i, d, vp]
        L.or_umax.restype = d
        L.or_spectra1d3d.argtypes = [i, vp, vp]
        L.or_tendency2d_strat.argtypes = [i, d, d, vp, vp]
        L.or_step3d_rot.argtypes = [i, d, d, d, d, d, d, d, i, d, vp, i, vp]
        L.or_strat_propagate.argtypes = [i, d, d, d, d, vp, vp]
        L.or_tendency3d_strat.argtypes = [i, d, vp, d, d, d, vp]
        L.or_step3d_strat.argtypes = [i, d, d, d, d, d, d, d, d, i, d, vp, i, vp]
        L.or_stratrot_propagate.argtypes = [i, d, d, d, d, d, vp, vp]
        L.or_tendency3d_modes.argtypes = [i, d, vp, i, vp, vp]
        L.or_structure.argtypes = [i, i, d, vp, i, vp, i, vp]
        L.or_step2d_strat.argtypes = [i, d, d, d, d, vp, i]
        L.or_spectra1d2d.argtypes = [i, d, vp, vp]
        L.or_transfer3d.argtypes = [i, d, vp, vp, i, vp, vp, vp]
        L.or_transfer2d.argtypes = [i, d, vp, vp, i, vp, vp, vp]
        L.or_round_bf16.argtypes = [d]
        L.or_round_bf16.restype = d
        L.or_round_bf16_array.argtypes = [vp, C.c_int64]
        L.or_les_tau3d.argtypes = [i, d, vp, vp, d, vp, d, i, vp]
        L.or_les_tendency3d.argtypes = [i, d, vp, d, d, d, vp, d, vp, d, i, vp]
        L.or_step3d_les.argtypes = [i, d, d, d, d, d, d, vp, d, vp, d, i, vp, i]
        _LIB = L
    return _LIB


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


def fft1d(x, sign=-1):
    """Unnormalised radix-2 DFT (sign -1 forward, +1 inverse)."""
    a = _c128(x).copy()
    lib().or_fft1d(_p(a), a.size, int(sign))
    return a


def fftn(x, sign=-1):
    a = _c128(x).copy()
    shape = np.array(a.shape, dtype=np.int32)
    lib().or_fftn(_p(a), a.ndim, shape.ctypes.data_as(C.c_void_p), int(sign))
    return a


def rfftn(phys):
    """Forward R2C over all axes of a real cube, scaled by 1/N^d."""
    p = np.ascontiguousarray(phys, dtype=np.float64)
    n, d = p.shape[0], p.ndim
    out = np.empty(p.shape[:-1] + (n // 2 + 1,), np.complex128)
    lib().or_rfftn(d, n, _p(p), _p(out))
    return out


def irfftn(spec):
    """Unscaled C2R over all axes (half spectrum -> real cube)."""
    s = _c128(spec)
    n, d = s.shape[0], s.ndim
    out = np.empty((n,) * d, np.float64)
    lib().or_irfftn(d, n, _p(s), _p(out))
    return out


def tendency3d(uh, L=2 * np.pi, alpha=0.0, kf_min=2.0, kf_max=3.0):
    u = _c128(uh)
    out = np.empty_like(u)
    lib().or_tendency3d(u.shape[1], float(L), _p(u), float(alpha), float(kf_min),
                        float(kf_max), _p(out))
    return out


def tendency2d(wh, L=2 * np.pi):
    w = _c128(wh)
    out = np.empty_like(w)
    lib().or_tendency2d(w.shape[0], float(L), _p(w), _p(out))
    return out


def forcing_alpha3d(uh, power, L=2 * np.pi, kf_min=2.0, kf_max=3.0):
    u = _c128(uh)
    return float(lib().or_forcing_alpha3d(u.shape[1], float(L), _p(u), float(power),
                                          float(kf_min), float(kf_max)))


def step3d(uh, nu, dt, nsteps, L=2 * np.pi, power=0.0, kf_min=2.0, kf_max=3.0):
    u = _c128(uh).copy()
    lib().or_step3d(u.shape[1], float(L), float(nu), float(dt), float(power),
                    float(kf_min), float(kf_max), _p(u), int(nsteps))
    return u


def step2d(wh, nu, dt, nsteps, L=2 * np.pi):
    w = _c128(wh).copy()
    lib().or_step2d(w.shape[0], float(L), float(nu), float(dt), _p(w), int(nsteps))
    return w


def step3d_ex(uh, nu, dt_max, nsteps, scheme=4, cfl=0.0, L=2 * np.pi, power=0.0, kf_min=2.0,
              kf_max=3.0):
    """(state after nsteps, elapsed time) with scheme 4 / 2 and optional CFL steps."""
    u = _c128(uh).copy()
    t = C.c_double(0.0)
    lib().or_step3d_ex(u.shape[1], float(L), float(nu), float(dt_max), float(power),
                       float(kf_min), float(kf_max), int(scheme), float(cfl), _p(u), int(nsteps),
                       C.byref(t))
    return u, t.value


def step2d_ex(wh, nu, dt_max, nsteps, scheme=4, cfl=0.0, L=2 * np.pi):
    w = _c128(wh).copy()
    t = C.c_double(0.0)
    lib().or_step2d_ex(w.shape[0], float(L), float(nu), float(dt_max), int(scheme), float(cfl),
                       _p(w), int(nsteps), C.byref(t))
    return w, t.value


def umax(state, ndim, L=2 * np.pi):
    s = _c128(state)
    n = s.shape[1] if ndim == 3 else s.shape[0]
    return float(lib().or_umax(int(ndim), n, float(L), _p(s)))


def lawson_scalar2(lam, y0, dt, nsteps):
    return float(lib().or_lawson_scalar2(float(lam), float(y0), float(dt), int(nsteps)))


def diag3d(uh, nbins, L=2 * np.pi):
    u = _c128(uh)
    spec = np.zeros(nbins, np.float64)
    e, z = C.c_double(), C.c_double()
    lib().or_diag3d(u.shape[1], float(L), _p(u), int(nbins), _p(spec), C.byref(e), C.byref(z))
    return spec, e.value, z.value


def diag2d(wh, nbins, L=2 * np.pi):
    w = _c128(wh)
    spec = np.zeros(nbins, np.float64)
    e, z = C.c_double(), C.c_double()
    lib().or_diag2d(w.shape[0], float(L), _p(w), int(nbins), _p(spec), C.byref(e), C.byref(z))
    return spec, e.value, z.value


def strat_propagate(s, nu, N2, t, L=2 * np.pi):
    """Exact propagator of viscosity, buoyancy force and stratification on a
    [4][n][n][n/2+1] state (kept modes; zero elsewhere)."""
    a = _c128(s)
    out = np.empty_like(a)
    lib().or_strat_propagate(a.shape[1], float(L), float(nu), float(N2), float(t), _p(a), _p(out))
    return out


def tendency3d_strat(s, L=2 * np.pi, alpha=0.0, kf_min=2.0, kf_max=3.0):
    """Nonlinear tendency of the 3D Boussinesq system (P[u x w] + forcing,
    -i k.(u b)^); the linear terms belong to the propagator."""
    a = _c128(s)
    out = np.empty_like(a)
    lib().or_tendency3d_strat(a.shape[1], float(L), _p(a), float(alpha), float(kf_min),
                              float(kf_max), _p(out))
    return out


def stratrot_propagate(s, nu, N2, f, t, L=2 * np.pi):
    """Exact propagator of viscosity, buoyancy, stratification and rotation
    (Coriolis parameter f about z) on a [4][n][n][n/2+1] state with
    solenoidal velocity."""
    a = _c128(s)
    out = np.empty_like(a)
    lib().or_stratrot_propagate(a.shape[1], float(L), float(nu), float(N2), float(f), float(t),
                                _p(a), _p(out))
    return out


def step3d_strat(s, nu, dt, N2, nsteps, L=2 * np.pi, power=0.0, kf_min=2.0, kf_max=3.0,
                 scheme=4, cfl=0.0, return_time=False, f=0.0):
    """Lawson RK4 (or RK2) of the 3D Boussinesq system (f != 0: in a frame
    rotating about z); cfl > 0: adaptive steps of at most dt (return_time:
    also the elapsed time)."""
    a = _c128(s).copy()
    t = C.c_double(0.0)
    lib().or_step3d_strat(a.shape[1], float(L), float(nu), float(dt), float(N2), float(f),
                          float(power),
                          float(kf_min), float(kf_max), int(scheme), float(cfl), _p(a),
                          int(nsteps), C.byref(t))
    return (a, t.value) if return_time else a


def structure(state, ndim, r, pmax, L=2 * np.pi):
    """Longitudinal structure functions: (signed[nr][pmax], absolute[nr][pmax])
    of the kept-mode velocity (2D: from the vorticity) for separations r (grid
    spacings), averaged over grid points and axes."""
    a = _c128(state)
    n = a.shape[-2]
    rr = np.ascontiguousarray(r, dtype=np.int32)
    out = np.zeros(2 * len(rr) * pmax)
    lib().or_structure(int(ndim), n, float(L), _p(a), len(rr), rr.ctypes.data, int(pmax), _p(out))
    out = out.reshape(2, len(rr), pmax)
    return out[0], out[1]


def tendency3d_modes(uh, modes, L=2 * np.pi):
    """The 3D tendency (no forcing) at the given modes (mx >= 0, my, mz) by the
    direct Galerkin triad sum; returns [len(modes)][3] complex."""
    u = _c128(uh)
    m = np.ascontiguousarray(np.asarray(modes, dtype=np.int32).reshape(-1, 3))
    out = np.zeros((m.shape[0], 3), np.complex128)
    lib().or_tendency3d_modes(u.shape[1], float(L), _p(u), m.shape[0], m.ctypes.data, _p(out))
    return out


def step3d_rot(uh, nu, dt, f, nsteps, L=2 * np.pi, power=0.0, kf_min=2.0, kf_max=3.0, scheme=4,
               cfl=0.0, return_time=False):
    """Lawson RK4 (or RK2) in a frame rotating about z (Coriolis -f z x u);
    cfl > 0: adaptive steps of at most dt (return_time: also the elapsed time)."""
    u = _c128(uh).copy()
    t = C.c_double(0.0)
    lib().or_step3d_rot(u.shape[1], float(L), float(nu), float(dt), float(f), float(power),
                        float(kf_min), float(kf_max), int(scheme), float(cfl), _p(u), int(nsteps),
                        C.byref(t))
    return (u, t.value) if return_time else u


def tendency2d_strat(s, N2, L=2 * np.pi):
    """Tendency of the 2D Boussinesq state [2][n][n/2+1] = (w_hat, b_hat)."""
    x = _c128(s)
    out = np.empty_like(x)
    lib().or_tendency2d_strat(x.shape[1], float(L), float(N2), _p(x), _p(out))
    return out


def step2d_strat(s, nu, dt, N2, nsteps, L=2 * np.pi):
    x = _c128(s).copy()
    lib().or_step2d_strat(x.shape[1], float(L), float(nu), float(dt), float(N2), _p(x), int(nsteps))
    return x


def spectra1d3d(uh):
    """[axis x,y,z][component][k = 0..K] energies binned by |m_axis|."""
    u = _c128(uh)
    n = u.shape[1]
    out = np.zeros((3, 3, (n - 1) // 3 + 1))
    lib().or_spectra1d3d(n, _p(u), _p(out))
    return out


def spectra1d2d(wh, L=2 * np.pi):
    """[axis x,y][velocity component u,v][k = 0..K]."""
    w = _c128(wh)
    n = w.shape[0]
    out = np.zeros((2, 2, (n - 1) // 3 + 1))
    lib().or_spectra1d2d(n, float(L), _p(w), _p(out))
    return out


def transfer3d(uh, nh, nbins, L=2 * np.pi):
    """(T[nbins], dE/dt, dZ/dt): shell sums of w Re(conj(u) . N)."""
    u, a = _c128(uh), _c128(nh)
    T = np.zeros(nbins)
    e, z = C.c_double(), C.c_double()
    lib().or_transfer3d(u.shape[1], float(L), _p(u), _p(a), int(nbins), _p(T), C.byref(e), C.byref(z))
    return T, e.value, z.value


def transfer2d(wh, nh, nbins, L=2 * np.pi):
    w, a = _c128(wh), _c128(nh)
    T = np.zeros(nbins)
    e, z = C.c_double(), C.c_double()
    lib().or_transfer2d(w.shape[0], float(L), _p(w), _p(a), int(nbins), _p(T), C.byref(e), C.byref(z))
    return T, e.value, z.value


def kept(m: int, n: int) -> bool:
    return bool(lib().or_kept(int(m), int(n)))


def lawson_scalar(lam, y0, dt, nsteps):
    """Lawson RK4 on y' = -lam y + y^2 (the scheme used by step2d/step3d)."""
    return float(lib().or_lawson_scalar(float(lam), float(y0), float(dt), int(nsteps)))


def dft_mode3d(phys, m):
    """Forward coefficient N^-3 sum u(x) exp(-i m.x) of one mode m = (mx, my, mz)."""
    p = np.ascontiguousarray(phys, dtype=np.float64)
    re, im = C.c_double(), C.c_double()
    lib().or_dft_mode3d(p.shape[0], _p(p), int(m[0]), int(m[1]), int(m[2]), C.byref(re), C.byref(im))
    return complex(re.value, im.value)


# ---- learned closure -------------------------------------------------------
TAU_COMPONENTS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def cutoff3d(fine, nc, box=False):
    """Sharp cube cutoff of a fine spectral field (or [3] stack) to the nc grid
    (box: after the box filter of width L / (2 Kc))."""
    f = _c128(fine)
    lead = f.shape[:-3]
    nf = f.shape[-3]
    ff = f.reshape((-1,) + f.shape[-3:])
    out = np.empty((ff.shape[0], nc, nc, nc // 2 + 1), np.complex128)
    for c in range(ff.shape[0]):
        fc = np.ascontiguousarray(ff[c])
        oc = np.empty((nc, nc, nc // 2 + 1), np.complex128)
        lib().or_cutoff3d(nf, _p(fc), nc, int(bool(box)), _p(oc))
        out[c] = oc
    return out.reshape(lead + (nc, nc, nc // 2 + 1))


def grad3d(uh, L=2 * np.pi):
    """A[3i+j] = d u_i/d x_j on the n^3 grid (9 real fields)."""
    u = _c128(uh)
    n = u.shape[1]
    A = np.empty((9, n, n, n), np.float64)
    lib().or_grad3d(n, float(L), _p(u), _p(A))
    return A


def sgs_tau3d(uf, nc, box=False):
    """Deviatoric subgrid stress on the nc grid from a fine spectral velocity
    (box: box filter of width L / (2 Kc), then the cutoff)."""
    u = _c128(uf)
    tau = np.empty((6, nc, nc, nc), np.float64)
    lib().or_sgs_tau3d(u.shape[1], _p(u), nc, int(bool(box)), _p(tau))
    return tau


def mlp_nparams():
    return int(lib().or_mlp_nparams())


def mlp_forward(params, x):
    p = np.ascontiguousarray(params, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty((xx.shape[0], 6), np.float64)
    lib().or_mlp_forward(_p(p), _p(xx), xx.shape[0], _p(y))
    return y


def mlp_loss_grad(params, x, t):
    p = np.ascontiguousarray(params, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    tt = np.ascontiguousarray(t, dtype=np.float64)
    g = np.empty(p.size, np.float64)
    loss = lib().or_mlp_loss_grad(_p(p), _p(xx), _p(tt), xx.shape[0], _p(g))
    return float(loss), g


def adam(w, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays w, m, v."""
    lib().or_adam(_p(w), _p(m), _p(v), _p(np.ascontiguousarray(g, dtype=np.float64)), w.size,
                  int(step), float(lr), float(b1), float(b2), float(eps))


def tendency3d_les(uh, tau, L=2 * np.pi):
    u = _c128(uh)
    t = np.ascontiguousarray(tau, dtype=np.float64)
    out = np.empty_like(u)
    lib().or_tendency3d_les(u.shape[1], float(L), _p(u), _p(t), _p(out))
    return out


def round_bf16(x):
    """Nearest BF16 value (8 significant bits, ties to even), as float64."""
    a = np.array(x, dtype=np.float64, copy=True, order="C")
    lib().or_round_bf16_array(_p(a), a.size)
    return a


def _net_args(params, a_scale, tau_scale):
    p = np.ascontiguousarray(params, dtype=np.float64)
    ts = np.ascontiguousarray(tau_scale, dtype=np.float64)
    assert p.size == mlp_nparams() and ts.size == 6 and a_scale > 0
    return p, ts


def les_tau3d(uh, params, a_scale, tau_scale, clip=0.0, bf16=True, L=2 * np.pi):
    """Network stress tau_s = clip(net(A / a_scale))_s * tau_scale[s], [6][n^3]."""
    u = _c128(uh)
    n = u.shape[1]
    p, ts = _net_args(params, a_scale, tau_scale)
    tau = np.empty((6, n, n, n), np.float64)
    lib().or_les_tau3d(n, float(L), _p(u), _p(p), float(a_scale), _p(ts), float(clip), int(bf16),
                       _p(tau))
    return tau


def les_tendency3d(uh, params, a_scale, tau_scale, clip=0.0, bf16=True, L=2 * np.pi,
                   alpha=0.0, kf_min=2.0, kf_max=3.0):
    u = _c128(uh)
    p, ts = _net_args(params, a_scale, tau_scale)
    out = np.empty_like(u)
    lib().or_les_tendency3d(u.shape[1], float(L), _p(u), float(alpha), float(kf_min),
                            float(kf_max), _p(p), float(a_scale), _p(ts), float(clip), int(bf16),
                            _p(out))
    return out


def step3d_les(uh, nu, dt, nsteps, params, a_scale, tau_scale, clip=0.0, bf16=True,
               L=2 * np.pi, power=0.0, kf_min=2.0, kf_max=3.0):
    u = _c128(uh).copy()
    p, ts = _net_args(params, a_scale, tau_scale)
    lib().or_step3d_les(u.shape[1], float(L), float(nu), float(dt), float(power), float(kf_min),
                        float(kf_max), _p(p), float(a_scale), _p(ts), float(clip), int(bf16),
                        _p(u), int(nsteps))
    return u
