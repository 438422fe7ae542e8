"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/fs.h declares, and rejects bad arguments before touching a
device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fs.h")
LIB = os.path.join(ROOT, "paper_1807_01769_amd", "libfs.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libfs.so is not built (run paper_1807_01769_amd/build.py)")
    return C.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name


class Opts(C.Structure):
    _fields_ = [("ndim", C.c_int), ("precision", C.c_int), ("stream", C.c_void_p),
                ("forcing_power", C.c_double), ("forcing_kmin", C.c_double),
                ("forcing_kmax", C.c_double), ("flags", C.c_uint), ("scheme", C.c_int),
                ("cfl", C.c_double), ("n2", C.c_double), ("rotation", C.c_double),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t)]


def _create(lib, n, L, nu, dt, **kw):
    lib.fs_plan_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_double, C.c_double,
                                   C.c_double, C.POINTER(Opts)]
    lib.fs_plan_opts_default.argtypes = [C.POINTER(Opts)]
    o = Opts()
    lib.fs_plan_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    h = C.c_void_p()
    st = lib.fs_plan_create(C.byref(h), n, L, nu, dt, C.byref(o))
    return st, h


@pytest.mark.parametrize("args,kw,expect", [
    ((0, 6.28, 0.1, 0.01), {}, -1),
    ((-8, 6.28, 0.1, 0.01), {}, -1),
    ((48, 6.28, 0.1, 0.01), {}, -2),
    ((8, 6.28, 0.1, 0.01), {}, -2),
    ((2048, 6.28, 0.1, 0.01), {}, -2),
    ((64, 0.0, 0.1, 0.01), {}, -1),
    ((64, float("nan"), 0.1, 0.01), {}, -1),
    ((64, 6.28, -1.0, 0.01), {}, -1),
    ((64, 6.28, 0.1, 0.0), {}, -1),
    ((64, 6.28, 0.1, float("inf")), {}, -1),
    ((64, 6.28, 0.1, 0.01), {"ndim": 4}, -1),
    ((64, 6.28, 0.1, 0.01), {"precision": 7}, -1),
    ((64, 6.28, 0.1, 0.01), {"flags": 0x100}, -1),
    ((64, 6.28, 0.1, 0.01), {"forcing_power": -1.0}, -1),
    ((64, 6.28, 0.1, 0.01), {"forcing_power": 1.0, "ndim": 2}, -2),
    ((64, 6.28, 0.1, 0.01), {"forcing_power": 1.0, "forcing_kmin": 3.0, "forcing_kmax": 2.0}, -1),
    ((16, 6.28, 0.1, 0.01), {"forcing_power": 1.0, "forcing_kmin": 2.0, "forcing_kmax": 9.0}, -1),
    ((64, 6.28, 0.1, 0.01), {"forcing_power": 1.0, "forcing_kmin": 1.1, "forcing_kmax": 1.2}, -1),
    ((64, 6.28, 0.1, 0.01), {"forcing_power": 1.0, "forcing_kmin": 2.0, "forcing_kmax": 1e300}, -1),
    ((64, 6.28, 0.1, 0.01), {"scheme": 2}, -1),
    ((64, 6.28, 0.1, 0.01), {"scheme": -1}, -1),
    ((64, 6.28, 0.1, 0.01), {"cfl": -0.5}, -1),
    ((64, 6.28, 0.1, 0.01), {"cfl": float("nan")}, -1),
    ((64, 6.28, 0.1, 0.01), {"flags": 0x8, "rotation": 1.0, "ndim": 2}, -2),
    ((64, 6.28, 0.1, 0.01), {"flags": 0x8, "ndim": 2, "n2": -1.0}, -1),
    ((64, 6.28, 0.1, 0.01), {"flags": 0x20}, -1),
    ((64, 6.28, 0.1, 0.01), {"rotation": float("inf")}, -1),
    ((64, 6.28, 0.1, 0.01), {"rotation": 1.0, "ndim": 2}, -2),
    # a caller workspace that is too small or misaligned (checked before any device call)
    ((64, 6.28, 0.1, 0.01), {"workspace": 1 << 20, "workspace_bytes": 4096}, -1),
    ((64, 6.28, 0.1, 0.01), {"workspace": (1 << 40) + 16, "workspace_bytes": 1 << 40}, -1),
])
def test_create_validates_before_device(lib, args, kw, expect):
    st, h = _create(lib, *args, **kw)
    assert st == expect
    assert not h.value
    lib.fs_last_error.restype = C.c_char_p
    assert lib.fs_last_error()


def test_null_arguments(lib):
    lib.fs_plan_create.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_double, C.c_void_p]
    assert lib.fs_plan_create(None, 64, 6.28, 0.1, 0.01, None) == -1
    for fn, nargs in [("fs_step_rk4", 3), ("fs_tendency", 3), ("fs_fft_forward", 3),
                      ("fs_fft_inverse", 3), ("fs_energy_spectrum", 6), ("fs_plan_set_stream", 2),
                      ("fs_energy_transfer", 8), ("fs_energy_spectra_1d", 3), ("fs_plan_time", 3),
                      ("fs_structure_functions", 6),
                      ("fs_profile_read", 5)]:
        f = getattr(lib, fn)
        f.argtypes = [C.c_void_p] * nargs
        assert f(*([None] * nargs)) == -1, fn
    lib.fs_plan_destroy.argtypes = [C.c_void_p]
    assert lib.fs_plan_destroy(None) == 0


def test_status_strings(lib):
    lib.fs_status_str.restype = C.c_char_p
    assert lib.fs_status_str(0) == b"FS_OK"
    assert lib.fs_status_str(-2) == b"FS_E_UNSUPPORTED"
    assert lib.fs_status_str(-99) == b"FS_E_UNKNOWN"


def test_binding_imports_and_needs_device():
    from paper_1807_01769_amd import fs
    import torch
    if torch.cuda.is_available():
        pytest.skip("device present")
    with pytest.raises(RuntimeError):
        fs.Plan(16)


@pytest.mark.parametrize("nruns,sizes,kw,expect", [
    (0, [64], {}, -1),
    (1, [100], {}, -2),
    (2, [64, 32], {}, -2),
    (1, [64], {"precision": 1}, -2),
    (1, [64], {"ndim": 3}, -1),
    (1, [64], {"forcing_power": 1.0}, -2),
    (1, [64], {"flags": 0x2}, -1),
    (1, [64], {"flags": 0x10}, -1),
    (1, [64], {"scheme": 2}, -2),
    (1, [64], {"cfl": 0.5}, -2),
    (1, [64], {"rotation": 1.0}, -2),
    (1, [64], {"workspace": 1 << 20, "workspace_bytes": 1 << 30}, -2),
])
def test_ensemble_create_validates(lib, nruns, sizes, kw, expect):
    lib.fs_ensemble_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_int),
                                       C.c_double, C.c_double, C.c_double, C.POINTER(Opts)]
    lib.fs_plan_opts_default.argtypes = [C.POINTER(Opts)]
    o = Opts()
    lib.fs_plan_opts_default(C.byref(o))
    o.ndim = 2
    for k, v in kw.items():
        setattr(o, k, v)
    arr = (C.c_int * max(1, len(sizes)))(*sizes)
    h = C.c_void_p()
    assert lib.fs_ensemble_create(C.byref(h), nruns, arr, 6.28, 1e-3, 1e-3, C.byref(o)) == expect
    assert not h.value


def test_closure_and_les_null_arguments(lib):
    vp, f = C.c_void_p, C.c_float
    sigs = {
        "fs_closure_create": ([vp, vp, vp], (None, None, None)),
        "fs_closure_samples": ([vp] * 5, (None,) * 5),
        "fs_closure_moments": ([vp] * 4, (None,) * 4),
        "fs_closure_features": ([vp, vp, vp, f, vp, vp, vp], (None, None, None, 1.0, None, None, None)),
        "fs_les_create": ([vp, vp, vp, f, vp, f], (None, None, None, 1.0, None, 0.0)),
        "fs_les_tendency": ([vp] * 3, (None,) * 3),
        "fs_les_step_rk4": ([vp, vp, C.c_int], (None, None, 1)),
        "fs_mlp_create": ([vp, C.c_uint64, vp], (None, 1, None)),
        "fs_mlp_forward": ([vp, vp, vp, C.c_int64], (None, None, None, 16)),
        "fs_mlp_train_step": ([vp, vp, vp, C.c_int64, f, vp], (None, None, None, 16, 1e-3, None)),
    }
    for name, (argtypes, args) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = argtypes
        assert fn(*args) == -1, name
    for name in ("fs_closure_destroy", "fs_les_destroy", "fs_mlp_destroy"):
        fn = getattr(lib, name)
        fn.argtypes = [vp]
        assert fn(None) == 0, name


def test_opts_defaults(lib):
    lib.fs_plan_opts_default.argtypes = [C.POINTER(Opts)]
    o = Opts()
    o.scheme, o.cfl, o.n2, o.rotation = 7, 3.0, 1.0, 2.0
    o.workspace, o.workspace_bytes = 4096, 99
    lib.fs_plan_opts_default(C.byref(o))
    assert (o.ndim, o.precision, o.flags, o.scheme, o.cfl, o.n2, o.rotation) == \
        (3, 0, 0, 0, 0.0, 0.0, 0.0)
    assert not o.workspace and o.workspace_bytes == 0
    assert (o.forcing_power, o.forcing_kmin, o.forcing_kmax) == (0.0, 2.0, 3.0)


def _ws_bytes(lib, n, **kw):
    lib.fs_plan_workspace_bytes.argtypes = [C.c_int, C.POINTER(Opts), C.POINTER(C.c_size_t)]
    lib.fs_plan_opts_default.argtypes = [C.POINTER(Opts)]
    o = Opts()
    lib.fs_plan_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    b = C.c_size_t()
    st = lib.fs_plan_workspace_bytes(n, C.byref(o), C.byref(b))
    return st, b.value


def test_workspace_bytes_without_device(lib):
    st, b64 = _ws_bytes(lib, 64)
    assert st == 0 and b64 > 0
    _, b128 = _ws_bytes(lib, 128)
    _, b128d = _ws_bytes(lib, 128, precision=1)
    _, b128s = _ws_bytes(lib, 128, flags=0x8)
    _, b128_2d = _ws_bytes(lib, 128, ndim=2)
    # a 3D plan holds kept-mode workspaces of a few states plus fixed tables
    state = 3 * 128 * 128 * 65 * 8
    assert 2 * state < b128 < 16 * state
    assert b64 < b128 < b128d and b128 < b128s and b128_2d < b128 // 8
    assert b128 % 256 == 0
    # validated like fs_plan_create
    assert _ws_bytes(lib, 48)[0] == -2
    assert _ws_bytes(lib, 64, ndim=5)[0] == -1
    lib.fs_plan_workspace_bytes.argtypes = [C.c_int, C.c_void_p, C.c_void_p]
    assert lib.fs_plan_workspace_bytes(64, None, None) == -1
