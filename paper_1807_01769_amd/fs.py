"""ctypes binding of libfs.so (include/fs.h): argument marshalling only.

Every computation runs in the library's HIP kernels; torch supplies device
memory and the stream.  Importing this module fails loudly when the library
has not been built, and creating a plan fails when no HIP device is present.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FS_LIBRARY") or os.path.join(_HERE, "libfs.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_1807_01769_amd/build.py")

lib = C.CDLL(LIB_PATH)

FS_OK, FS_E_INVALID, FS_E_UNSUPPORTED, FS_E_NOMEM, FS_E_DEVICE, FS_E_NONFINITE = 0, -1, -2, -3, -4, -5
FS_F32, FS_F64 = 0, 1
FS_SCHEME_RK4, FS_SCHEME_RK2 = 0, 1
FS_NO_GRAPH, FS_PROFILE, FS_BOUSSINESQ, FS_CHECK_FINITE = 0x1, 0x2, 0x8, 0x10
FS_E_NONFINITE = -5
KERNEL_NAMES = ["p1", "y_inverse", "x_c2r_product_r2c", "y_forward", "z_stage",
                "forcing_alpha", "fill", "fft_only", "diagnostics"]


class Opts(C.Structure):
    _fields_ = [
        ("ndim", C.c_int),
        ("precision", C.c_int),
        ("stream", C.c_void_p),
        ("forcing_power", C.c_double),
        ("forcing_kmin", C.c_double),
        ("forcing_kmax", C.c_double),
        ("flags", C.c_uint),
        ("scheme", C.c_int),
        ("cfl", C.c_double),
        ("n2", C.c_double),
        ("rotation", C.c_double),
        ("workspace", C.c_void_p),
        ("workspace_bytes", C.c_size_t),
    ]


_vp, _i, _d = C.c_void_p, C.c_int, C.c_double
lib.fs_plan_opts_default.argtypes = [C.POINTER(Opts)]
lib.fs_plan_opts_default.restype = None
lib.fs_plan_create.argtypes = [C.POINTER(_vp), _i, _d, _d, _d, C.POINTER(Opts)]
lib.fs_plan_destroy.argtypes = [_vp]
lib.fs_plan_set_stream.argtypes = [_vp, _vp]
lib.fs_state_elems.argtypes = [_vp, C.POINTER(C.c_size_t)]
lib.fs_workspace_bytes.argtypes = [_vp, C.POINTER(C.c_size_t)]
lib.fs_plan_workspace_bytes.argtypes = [_i, C.POINTER(Opts), C.POINTER(C.c_size_t)]
lib.fs_spectrum_bins.argtypes = [_vp, C.POINTER(_i)]
lib.fs_fft_forward.argtypes = [_vp, _vp, _vp]
lib.fs_fft_inverse.argtypes = [_vp, _vp, _vp]
lib.fs_tendency.argtypes = [_vp, _vp, _vp]
lib.fs_step_rk4.argtypes = [_vp, _vp, _i]
lib.fs_energy_spectrum.argtypes = [_vp, _vp, _vp, _i, _vp, _vp]
lib.fs_energy_spectrum_static.argtypes = [_i, _i, _i, _d, _vp, _vp, _i, _vp, _vp, _vp]
lib.fs_energy_transfer.argtypes = [_vp, _vp, _vp, _vp, _vp, _i, _vp, _vp]
lib.fs_energy_spectra_1d.argtypes = [_vp, _vp, _vp]
lib.fs_structure_functions.argtypes = [_vp, _vp, _i, _vp, _i, _vp]
lib.fs_plan_time.argtypes = [_vp, _vp, _vp]
lib.fs_profile_read.argtypes = [_vp, C.POINTER(_d), C.POINTER(C.c_long), C.POINTER(C.c_char_p), _i]
lib.fs_status_str.argtypes = [_i]
lib.fs_status_str.restype = C.c_char_p
lib.fs_last_error.argtypes = []
lib.fs_last_error.restype = C.c_char_p
for _f in ("fs_plan_create", "fs_plan_destroy", "fs_plan_set_stream", "fs_state_elems",
           "fs_workspace_bytes", "fs_plan_workspace_bytes", "fs_spectrum_bins",
           "fs_fft_forward", "fs_fft_inverse",
           "fs_tendency", "fs_step_rk4", "fs_energy_spectrum", "fs_energy_transfer",
           "fs_energy_spectra_1d", "fs_structure_functions", "fs_plan_time",
           "fs_profile_read"):
    getattr(lib, _f).restype = _i


class FsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib.fs_last_error().decode()
        super().__init__(f"{where}: {lib.fs_status_str(status).decode()} ({msg})")


def _check(status: int, where: str) -> None:
    if status != FS_OK:
        raise FsError(status, where)


def _stream_ptr(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _opts(ndim=3, precision="f32", forcing_power=0.0, forcing_kmin=2.0, forcing_kmax=3.0,
          graphs=True, profile=False, scheme="rk4", cfl=0.0, boussinesq=False, n2=0.0,
          rotation=0.0, check_finite=False) -> Opts:
    o = Opts()
    lib.fs_plan_opts_default(C.byref(o))
    o.ndim = int(ndim)
    o.precision = FS_F32 if precision == "f32" else FS_F64
    o.forcing_power = float(forcing_power)
    o.forcing_kmin = float(forcing_kmin)
    o.forcing_kmax = float(forcing_kmax)
    o.flags = ((0 if graphs else FS_NO_GRAPH) | (FS_PROFILE if profile else 0) |
               (FS_BOUSSINESQ if boussinesq else 0) | (FS_CHECK_FINITE if check_finite else 0))
    o.n2 = float(n2)
    o.rotation = float(rotation)
    o.scheme = {"rk4": FS_SCHEME_RK4, "rk2": FS_SCHEME_RK2}[scheme]
    o.cfl = float(cfl)
    return o


def energy_spectrum_static(state: torch.Tensor, ndim: int, n: int, precision: str = "f32",
                           nbins: int | None = None, L: float = 2 * math.pi, stream=None):
    """fs_energy_spectrum_static: the plan-free, allocation-free diagnostics of
    a state (device tensors spectrum[nbins], energy[1], enstrophy[1], float64;
    the caller allocates them here, the library allocates nothing)."""
    cdt = {"f32": torch.complex64, "f64": torch.complex128}[precision]
    h = n // 2 + 1
    shape = (3, n, n, h) if ndim == 3 else (n, h)
    if tuple(state.shape) != shape or state.dtype != cdt or not state.is_cuda \
            or not state.is_contiguous():
        raise ValueError(f"state must be a contiguous {cdt} device tensor of shape {shape}")
    if nbins is None:
        K = (n - 1) // 3
        nbins = int(math.floor(math.sqrt(ndim) * K + 0.5)) + 1  # as fs_spectrum_bins
    spec = torch.empty(int(nbins), dtype=torch.float64, device=state.device)
    ez = torch.empty(2, dtype=torch.float64, device=state.device)
    _check(lib.fs_energy_spectrum_static(int(ndim), int(n), FS_F32 if precision == "f32" else FS_F64,
                                         float(L), state.data_ptr(), spec.data_ptr(), int(nbins),
                                         ez.data_ptr(), ez.data_ptr() + 8, _stream_ptr(stream)),
           "fs_energy_spectrum_static")
    return spec, ez[0:1], ez[1:2]


class Plan:
    """One solver configuration: grid n, box length L, viscosity nu, step dt."""

    def __init__(self, n: int, L: float = 2 * math.pi, nu: float = 0.0, dt: float = 1e-3,
                 ndim: int = 3, precision: str = "f32", stream=None, forcing_power: float = 0.0,
                 forcing_kmin: float = 2.0, forcing_kmax: float = 3.0, graphs: bool = True,
                 profile: bool = False, scheme: str = "rk4", cfl: float = 0.0,
                 boussinesq: bool = False, n2: float = 0.0, rotation: float = 0.0,
                 check_finite: bool = False, workspace: torch.Tensor | None = None):
        """workspace: optional device tensor of at least Plan.required_bytes(...)
        bytes that the plan uses instead of allocating (kept referenced by the
        plan); check_finite: report non-finite steps as FsError (FS_E_NONFINITE)
        at the next call."""
        if not torch.cuda.is_available():
            raise RuntimeError("paper_1807_01769_amd.fs needs a HIP device")
        self.n, self.L, self.nu, self.dt, self.ndim = int(n), float(L), float(nu), float(dt), int(ndim)
        self.precision = precision
        self.real_dtype = {"f32": torch.float32, "f64": torch.float64}[precision]
        self.complex_dtype = {"f32": torch.complex64, "f64": torch.complex128}[precision]
        self.stream = stream
        # the physics options, as given (what a checkpoint needs to rebuild the plan)
        self.options = {"n": self.n, "L": self.L, "nu": self.nu, "dt": self.dt,
                        "ndim": self.ndim, "precision": precision,
                        "forcing_power": float(forcing_power),
                        "forcing_kmin": float(forcing_kmin), "forcing_kmax": float(forcing_kmax),
                        "scheme": scheme, "cfl": float(cfl), "boussinesq": bool(boussinesq),
                        "n2": float(n2), "rotation": float(rotation)}
        o = _opts(ndim, precision, forcing_power, forcing_kmin, forcing_kmax, graphs, profile,
                  scheme, cfl, boussinesq, n2, rotation, check_finite)
        o.stream = _stream_ptr(stream)
        self._workspace = workspace
        if workspace is not None:
            if not workspace.is_cuda or not workspace.is_contiguous():
                raise ValueError("workspace must be a contiguous device tensor")
            o.workspace = workspace.data_ptr()
            o.workspace_bytes = workspace.numel() * workspace.element_size()
        self.nfield = (3 if self.ndim == 3 else 1) + (1 if boussinesq else 0)
        h = _vp()
        _check(lib.fs_plan_create(C.byref(h), self.n, self.L, self.nu, self.dt, C.byref(o)),
               "fs_plan_create")
        self._h = h

    # -- shapes ------------------------------------------------------------
    @property
    def state_shape(self):
        n = self.n
        if self.ndim == 3:
            return (self.nfield, n, n, n // 2 + 1)
        return (2, n, n // 2 + 1) if self.nfield == 2 else (n, n // 2 + 1)

    @property
    def field_shape(self):
        """Shape of one scalar spectral field (diagnostics act on the first)."""
        n = self.n
        return (3, n, n, n // 2 + 1) if self.ndim == 3 else (n, n // 2 + 1)

    @property
    def spec_shape(self):
        n = self.n
        return (n,) * (self.ndim - 1) + (n // 2 + 1,)

    @property
    def phys_shape(self):
        return (self.n,) * self.ndim

    @staticmethod
    def required_bytes(n: int, **opts) -> int:
        """Workspace bytes of a plan of size n with these options (keywords as
        for Plan), without creating it; needs no device."""
        o = _opts(**opts)
        b = C.c_size_t()
        _check(lib.fs_plan_workspace_bytes(int(n), C.byref(o), C.byref(b)),
               "fs_plan_workspace_bytes")
        return int(b.value)

    def workspace_bytes(self) -> int:
        b = C.c_size_t()
        _check(lib.fs_workspace_bytes(self._h, C.byref(b)), "fs_workspace_bytes")
        return int(b.value)

    def spectrum_bins(self) -> int:
        b = _i()
        _check(lib.fs_spectrum_bins(self._h, C.byref(b)), "fs_spectrum_bins")
        return int(b.value)

    def _arg(self, t: torch.Tensor, shape, dtype, name: str) -> int:
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a device tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t.data_ptr()

    def new_state(self) -> torch.Tensor:
        return torch.zeros(self.state_shape, dtype=self.complex_dtype, device="cuda")

    # -- entry points ------------------------------------------------------
    def fft_forward(self, phys: torch.Tensor, spec: torch.Tensor | None = None) -> torch.Tensor:
        if spec is None:
            spec = torch.empty(self.spec_shape, dtype=self.complex_dtype, device=phys.device)
        _check(lib.fs_fft_forward(self._h, self._arg(phys, self.phys_shape, self.real_dtype, "phys"),
                                  self._arg(spec, self.spec_shape, self.complex_dtype, "spec")),
               "fs_fft_forward")
        return spec

    def fft_inverse(self, spec: torch.Tensor, phys: torch.Tensor | None = None) -> torch.Tensor:
        if phys is None:
            phys = torch.empty(self.phys_shape, dtype=self.real_dtype, device=spec.device)
        _check(lib.fs_fft_inverse(self._h, self._arg(spec, self.spec_shape, self.complex_dtype, "spec"),
                                  self._arg(phys, self.phys_shape, self.real_dtype, "phys")),
               "fs_fft_inverse")
        return phys

    def tendency(self, state: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.state_shape, dtype=self.complex_dtype, device=state.device)
        _check(lib.fs_tendency(self._h, self._arg(state, self.state_shape, self.complex_dtype, "state"),
                               self._arg(out, self.state_shape, self.complex_dtype, "out")),
               "fs_tendency")
        return out

    def step(self, state: torch.Tensor, nsteps: int = 1) -> torch.Tensor:
        _check(lib.fs_step_rk4(self._h, self._arg(state, self.state_shape, self.complex_dtype, "state"),
                               int(nsteps)), "fs_step_rk4")
        return state

    def energy_spectrum(self, state: torch.Tensor, nbins: int | None = None):
        """Returns device tensors (spectrum[nbins], energy[1], enstrophy[1]) in float64."""
        nbins = self.spectrum_bins() if nbins is None else int(nbins)
        spec = torch.empty(nbins, dtype=torch.float64, device=state.device)
        ez = torch.empty(2, dtype=torch.float64, device=state.device)
        _check(lib.fs_energy_spectrum(self._h, self._arg(state, self.state_shape, self.complex_dtype, "state"),
                                      spec.data_ptr(), nbins, ez.data_ptr(), ez.data_ptr() + 8),
               "fs_energy_spectrum")
        return spec, ez[0:1], ez[1:2]

    def time(self):
        """Device float64 tensors (elapsed time, last step size)."""
        out = torch.empty(2, dtype=torch.float64, device="cuda")
        _check(lib.fs_plan_time(self._h, out.data_ptr(), out.data_ptr() + 8), "fs_plan_time")
        return out[0:1], out[1:2]

    def energy_spectra_1d(self, state: torch.Tensor) -> torch.Tensor:
        """Device float64 [axis][component][k = 0..K] energies binned by |m_axis|."""
        d, K = self.ndim, (self.n - 1) // 3
        out = torch.empty((d, d, K + 1), dtype=torch.float64, device=state.device)
        _check(lib.fs_energy_spectra_1d(
            self._h, self._arg(state, self.state_shape, self.complex_dtype, "state"),
            out.data_ptr()), "fs_energy_spectra_1d")
        return out

    def structure_functions(self, state: torch.Tensor, r, pmax: int = 6):
        """Longitudinal structure functions of the velocity for separations r
        (grid spacings): device float64 (signed[nr][pmax], absolute[nr][pmax])
        with signed[j][p-1] = <du^p> and absolute[j][p-1] = <|du|^p>."""
        rr = (C.c_int * len(r))(*[int(x) for x in r])
        out = torch.empty((2, len(r), int(pmax)), dtype=torch.float64, device=state.device)
        _check(lib.fs_structure_functions(
            self._h, self._arg(state, self.state_shape, self.complex_dtype, "state"), len(r),
            C.cast(rr, _vp), int(pmax), out.data_ptr()), "fs_structure_functions")
        return out[0], out[1]

    def energy_transfer(self, state: torch.Tensor, tend: torch.Tensor | None = None,
                        nbins: int | None = None):
        """Device float64 tensors (transfer[nbins], flux[nbins], energy_rate[1],
        enstrophy_rate[1]) of the tendency `tend` (default: fs_tendency of
        `state`); flux[s] = -sum_{s' <= s} transfer[s'] is the energy flux
        through shell s."""
        nbins = self.spectrum_bins() if nbins is None else int(nbins)
        if tend is None:
            tend = self.tendency(state)
        tr = torch.empty(nbins, dtype=torch.float64, device=state.device)
        fl = torch.empty(nbins, dtype=torch.float64, device=state.device)
        ez = torch.empty(2, dtype=torch.float64, device=state.device)
        _check(lib.fs_energy_transfer(
            self._h, self._arg(state, self.state_shape, self.complex_dtype, "state"),
            self._arg(tend, self.state_shape, self.complex_dtype, "tend"), tr.data_ptr(),
            fl.data_ptr(), nbins, ez.data_ptr(), ez.data_ptr() + 8), "fs_energy_transfer")
        return tr, fl, ez[0:1], ez[1:2]

    def profile_read(self) -> dict:
        """Per-kernel (total ms, launches) since the previous read (profile=True plans)."""
        nk = len(KERNEL_NAMES)
        ms = (_d * nk)()
        cnt = (C.c_long * nk)()
        _check(lib.fs_profile_read(self._h, ms, cnt, None, nk), "fs_profile_read")
        return {KERNEL_NAMES[k]: (ms[k], cnt[k]) for k in range(nk) if cnt[k] > 0}

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib.fs_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


FS_NO_AUTOTUNE = 0x4
FS_NO_RESIDENT = 0x20
lib.fs_ensemble_create.argtypes = [C.POINTER(_vp), _i, C.POINTER(_i), _d, _d, _d, C.POINTER(Opts)]
lib.fs_ensemble_offsets.argtypes = [_vp, C.POINTER(C.c_int64)]
lib.fs_ensemble_step_rk4.argtypes = [_vp, _vp, _i]
lib.fs_ensemble_schedule.argtypes = [_vp, _i, C.POINTER(_i), C.POINTER(_i), C.POINTER(_i),
                                     C.POINTER(_i), C.POINTER(_d), C.POINTER(_d)]
lib.fs_ensemble_destroy.argtypes = [_vp]
for _f in ("fs_ensemble_create", "fs_ensemble_offsets", "fs_ensemble_step_rk4",
           "fs_ensemble_schedule", "fs_ensemble_destroy"):
    getattr(lib, _f).restype = _i


class Ensemble:
    """Independent 2D FP32 runs of uneven sizes (64/128/256/512) advanced together."""

    def __init__(self, sizes, L: float = 2 * math.pi, nu: float = 0.0, dt: float = 1e-3,
                 stream=None, autotune: bool = True, graphs: bool = True,
                 resident: bool = True):
        if not torch.cuda.is_available():
            raise RuntimeError("paper_1807_01769_amd.fs needs a HIP device")
        self.sizes = [int(s) for s in sizes]
        o = Opts()
        lib.fs_plan_opts_default(C.byref(o))
        o.ndim = 2
        o.precision = FS_F32
        o.stream = _stream_ptr(stream)
        o.flags = ((0 if autotune else FS_NO_AUTOTUNE) | (0 if graphs else FS_NO_GRAPH) |
                   (0 if resident else FS_NO_RESIDENT))
        arr = (_i * len(self.sizes))(*self.sizes)
        h = _vp()
        _check(lib.fs_ensemble_create(C.byref(h), len(self.sizes), arr, float(L), float(nu),
                                      float(dt), C.byref(o)), "fs_ensemble_create")
        self._h = h
        off = (C.c_int64 * (len(self.sizes) + 1))()
        _check(lib.fs_ensemble_offsets(self._h, off), "fs_ensemble_offsets")
        self.offsets = [int(v) for v in off]

    def new_state(self) -> torch.Tensor:
        return torch.zeros(self.offsets[-1], dtype=torch.complex64, device="cuda")

    def pack(self, fields) -> torch.Tensor:
        """Packed device state from per-run [n][n/2+1] arrays (numpy or torch)."""
        st = self.new_state()
        for r, f in enumerate(fields):
            t = torch.as_tensor(f).to(torch.complex64).reshape(-1)
            st[self.offsets[r]:self.offsets[r + 1]] = t.to(st.device)
        return st

    def unpack(self, state: torch.Tensor, r: int) -> torch.Tensor:
        n = self.sizes[r]
        return state[self.offsets[r]:self.offsets[r + 1]].reshape(n, n // 2 + 1)

    def step(self, state: torch.Tensor, nsteps: int = 1) -> torch.Tensor:
        if not (state.is_cuda and state.dtype == torch.complex64 and state.is_contiguous()
                and state.numel() == self.offsets[-1]):
            raise ValueError("state must be a contiguous complex64 device tensor of the packed size")
        _check(lib.fs_ensemble_step_rk4(self._h, state.data_ptr(), int(nsteps)),
               "fs_ensemble_step_rk4")
        return state

    def schedule(self) -> list:
        out, c = [], 0
        while True:
            n, nr, yl, xr = _i(), _i(), _i(), _i()
            uy, ux = _d(), _d()
            st = lib.fs_ensemble_schedule(self._h, c, C.byref(n), C.byref(nr), C.byref(yl),
                                          C.byref(xr), C.byref(uy), C.byref(ux))
            if st != FS_OK:
                break
            if yl.value == 0:  # block-resident class
                out.append({"n": n.value, "runs": nr.value, "resident": True})
            else:
                out.append({"n": n.value, "runs": nr.value, "y_lines": yl.value,
                            "x_rowpairs": xr.value, "us_y": uy.value, "us_x": ux.value})
            c += 1
        return out

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib.fs_ensemble_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


lib.fs_mlp_create.argtypes = [C.POINTER(_vp), C.c_uint64, _vp]
lib.fs_mlp_destroy.argtypes = [_vp]
lib.fs_mlp_nparams.argtypes = [C.POINTER(_i)]
lib.fs_mlp_set_params.argtypes = [_vp, _vp]
lib.fs_mlp_get_params.argtypes = [_vp, _vp]
lib.fs_mlp_forward.argtypes = [_vp, _vp, _vp, C.c_int64]
lib.fs_mlp_grad.argtypes = [_vp, _vp, _vp, C.c_int64, _vp, _vp]
lib.fs_mlp_train_step.argtypes = [_vp, _vp, _vp, C.c_int64, C.c_float, _vp]
for _f in ("fs_mlp_create", "fs_mlp_destroy", "fs_mlp_nparams", "fs_mlp_set_params",
           "fs_mlp_get_params", "fs_mlp_forward", "fs_mlp_grad", "fs_mlp_train_step"):
    getattr(lib, _f).restype = _i


def bf16_features(x) -> torch.Tensor:
    """[P][9] float array -> device BF16 [P][16] feature tensor (zero padded)."""
    t = torch.as_tensor(x, dtype=torch.float32)
    out = torch.zeros((t.shape[0], 16), dtype=torch.bfloat16)
    out[:, :9] = t.to(torch.bfloat16)
    return out.cuda()


class Mlp:
    """The 9-64-64-6 GELU closure network on BF16 matrix cores."""

    def __init__(self, seed: int = 7, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("paper_1807_01769_amd.fs needs a HIP device")
        h = _vp()
        _check(lib.fs_mlp_create(C.byref(h), int(seed), _stream_ptr(stream)), "fs_mlp_create")
        self._h = h
        n = _i()
        _check(lib.fs_mlp_nparams(C.byref(n)), "fs_mlp_nparams")
        self.nparams = n.value

    def get_params(self) -> torch.Tensor:
        p = torch.empty(self.nparams, dtype=torch.float32, device="cuda")
        _check(lib.fs_mlp_get_params(self._h, p.data_ptr()), "fs_mlp_get_params")
        return p

    def set_params(self, p: torch.Tensor) -> None:
        p = p.to(device="cuda", dtype=torch.float32).contiguous()
        if p.numel() != self.nparams:
            raise ValueError("wrong parameter count")
        _check(lib.fs_mlp_set_params(self._h, p.data_ptr()), "fs_mlp_set_params")
        torch.cuda.synchronize()

    def _x(self, x):
        if not (x.is_cuda and x.dtype == torch.bfloat16 and x.dim() == 2 and x.shape[1] == 16
                and x.is_contiguous()):
            raise ValueError("features must be a contiguous device bfloat16 [P][16] tensor")
        return x.data_ptr()

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        y = torch.empty((x.shape[0], 6), dtype=torch.float32, device="cuda")
        _check(lib.fs_mlp_forward(self._h, self._x(x), y.data_ptr(), x.shape[0]), "fs_mlp_forward")
        return y

    def grad(self, x: torch.Tensor, t: torch.Tensor):
        t = t.contiguous()
        g = torch.empty(self.nparams, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float64, device="cuda")
        _check(lib.fs_mlp_grad(self._h, self._x(x), t.data_ptr(), x.shape[0], g.data_ptr(),
                               loss.data_ptr()), "fs_mlp_grad")
        return g, loss

    def train_step(self, x: torch.Tensor, t: torch.Tensor, lr: float = 1e-3) -> torch.Tensor:
        t = t.contiguous()
        loss = torch.empty(1, dtype=torch.float64, device="cuda")
        _check(lib.fs_mlp_train_step(self._h, self._x(x), t.data_ptr(), x.shape[0], float(lr),
                                     loss.data_ptr()), "fs_mlp_train_step")
        return loss

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib.fs_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- closure samples and LES -------------------------------------------------
lib.fs_closure_create.argtypes = [C.POINTER(_vp), _vp, _vp]
lib.fs_closure_destroy.argtypes = [_vp]
lib.fs_closure_set_filter.argtypes = [_vp, _i]
lib.fs_closure_samples.argtypes = [_vp, _vp, _vp, _vp, _vp]
lib.fs_closure_moments.argtypes = [_vp, _vp, _vp, _vp]
lib.fs_closure_features.argtypes = [_vp, _vp, _vp, C.c_float, C.POINTER(C.c_float), _vp, _vp]
lib.fs_les_create.argtypes = [C.POINTER(_vp), _vp, _vp, C.c_float, C.POINTER(C.c_float), C.c_float]
lib.fs_les_destroy.argtypes = [_vp]
lib.fs_les_tendency.argtypes = [_vp, _vp, _vp]
lib.fs_les_step_rk4.argtypes = [_vp, _vp, _i]
for _f in ("fs_closure_create", "fs_closure_destroy", "fs_closure_set_filter",
           "fs_closure_samples", "fs_closure_moments",
           "fs_closure_features", "fs_les_create", "fs_les_destroy", "fs_les_tendency",
           "fs_les_step_rk4"):
    getattr(lib, _f).restype = _i


def _six(v):
    v = [float(x) for x in v]
    if len(v) != 6:
        raise ValueError("six stress scales expected")
    return (C.c_float * 6)(*v)


class Closure:
    """Filtered-DNS samples: fine 3D f32 plan -> coarse 3D f32 plan."""

    def __init__(self, fine: Plan, coarse: Plan, filter: str = "sharp"):
        """filter: "sharp" (cube cutoff) or "box" (top-hat of width L / (2 Kc), then the cutoff)."""
        h = _vp()
        _check(lib.fs_closure_create(C.byref(h), fine._h, coarse._h), "fs_closure_create")
        self._h, self.fine, self.coarse = h, fine, coarse
        self.filter = filter
        _check(lib.fs_closure_set_filter(h, {"sharp": 0, "box": 1}[filter]), "fs_closure_set_filter")
        self.np = coarse.n ** 3

    def samples(self, fine_state: torch.Tensor):
        """-> (coarse_state [3][nc][nc][nc/2+1], A [9][nc^3], tau [6][nc^3]) device tensors."""
        c = self.coarse
        uc = torch.empty(c.state_shape, dtype=torch.complex64, device="cuda")
        A = torch.empty((9, self.np), dtype=torch.float32, device="cuda")
        tau = torch.empty((6, self.np), dtype=torch.float32, device="cuda")
        _check(lib.fs_closure_samples(
            self._h, self.fine._arg(fine_state, self.fine.state_shape, torch.complex64, "fine_state"),
            uc.data_ptr(), A.data_ptr(), tau.data_ptr()), "fs_closure_samples")
        return uc, A, tau

    def _field(self, t, rows, name):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
                and tuple(t.shape) == (rows, self.np)):
            raise ValueError(f"{name} must be a contiguous device float32 [{rows}][{self.np}] tensor")
        return t.data_ptr()

    def moments(self, A: torch.Tensor, tau: torch.Tensor) -> torch.Tensor:
        """Mean squares (float64 [15]): the 9 gradients then the 6 stresses."""
        m = torch.empty(15, dtype=torch.float64, device="cuda")
        _check(lib.fs_closure_moments(self._h, self._field(A, 9, "A"), self._field(tau, 6, "tau"),
                                      m.data_ptr()), "fs_closure_moments")
        return m

    def features(self, A: torch.Tensor, a_scale: float, tau: torch.Tensor | None = None,
                 tau_scale=None):
        """-> (x bf16 [nc^3][16], t float32 [nc^3][6] or None)."""
        x = torch.empty((self.np, 16), dtype=torch.bfloat16, device="cuda")
        t = None
        if tau is not None:
            t = torch.empty((self.np, 6), dtype=torch.float32, device="cuda")
        _check(lib.fs_closure_features(
            self._h, self._field(A, 9, "A"), None if tau is None else self._field(tau, 6, "tau"),
            float(a_scale), None if tau is None else _six(tau_scale), x.data_ptr(),
            None if t is None else t.data_ptr()), "fs_closure_features")
        return x, t

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib.fs_closure_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Les:
    """LES on a coarse 3D f32 plan with the network closure (model=None: no model)."""

    def __init__(self, plan: Plan, model: Mlp | None, a_scale: float = 1.0,
                 tau_scale=(1.0,) * 6, clip: float = 0.0):
        h = _vp()
        _check(lib.fs_les_create(C.byref(h), plan._h, None if model is None else model._h,
                                 float(a_scale), _six(tau_scale), float(clip)), "fs_les_create")
        self._h, self.plan, self.model = h, plan, model

    def tendency(self, state: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        p = self.plan
        if out is None:
            out = torch.empty(p.state_shape, dtype=p.complex_dtype, device="cuda")
        _check(lib.fs_les_tendency(self._h, p._arg(state, p.state_shape, p.complex_dtype, "state"),
                                   p._arg(out, p.state_shape, p.complex_dtype, "out")),
               "fs_les_tendency")
        return out

    def step(self, state: torch.Tensor, nsteps: int = 1) -> torch.Tensor:
        p = self.plan
        _check(lib.fs_les_step_rk4(self._h, p._arg(state, p.state_shape, p.complex_dtype, "state"),
                                   int(nsteps)), "fs_les_step_rk4")
        return state

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib.fs_les_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
