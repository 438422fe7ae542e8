"""Checkpoint and resume of a solver run.

A checkpoint is two files: the spectral state as a raw ``.npy`` array (the
C ABI layout, complex64 or complex128 as the plan computes, written with
numpy's own format, no pickling) and a JSON sidecar holding what is needed
to continue the run exactly: the plan's physics options (n, L, nu, dt,
dimension, precision, forcing band and power, time scheme, CFL number,
buoyancy and rotation), the number of steps taken, the elapsed time and the
seed of the initial field.  The step kernels are deterministic and a fresh
plan carries no state between calls beyond the caller's array (the forcing
coefficient and adaptive step are recomputed from the state every step), so
resuming from a checkpoint reproduces an uninterrupted run bit for bit.
"""
from __future__ import annotations

import json
import os

import numpy as np

FORMAT = "fs-checkpoint-1"


def _paths(path: str):
    base = path[:-4] if path.endswith(".npy") else path
    return base + ".npy", base + ".json"


def save_arrays(path: str, state, meta: dict) -> tuple[str, str]:
    """Write a state (numpy array or tensor, any device) and its metadata."""
    arr = state.detach().cpu().numpy() if hasattr(state, "detach") else np.asarray(state)
    npy, js = _paths(path)
    np.save(npy, np.ascontiguousarray(arr), allow_pickle=False)
    meta = dict(meta)
    meta.update({"format": FORMAT, "shape": list(arr.shape), "dtype": str(arr.dtype),
                 "array": os.path.basename(npy)})
    with open(js, "w") as fh:
        json.dump(meta, fh, indent=1, sort_keys=True)
    return npy, js


def save(path: str, plan, state, step: int, seed: int | None = None,
         extra: dict | None = None) -> tuple[str, str]:
    """Checkpoint `state` of `plan` after `step` steps; the elapsed time is the
    plan's own (adaptive steps) plus the time the plan was resumed at."""
    import torch

    torch.cuda.synchronize()
    t = float(plan.time()[0].item()) + float(getattr(plan, "time_offset", 0.0))
    meta = {"plan": plan.options, "step": int(step), "time": t, "seed": seed,
            "extra": extra or {}}
    return save_arrays(path, state, meta)


def load_arrays(path: str):
    """(numpy state, metadata) of a checkpoint."""
    npy, js = _paths(path)
    with open(js) as fh:
        meta = json.load(fh)
    if meta.get("format") != FORMAT:
        raise ValueError(f"{js}: not a checkpoint of this format")
    arr = np.load(npy, allow_pickle=False)
    if list(arr.shape) != meta["shape"] or str(arr.dtype) != meta["dtype"]:
        raise ValueError(f"{npy}: array does not match its sidecar")
    return arr, meta


def resume(path: str, **plan_kw):
    """(plan, device state, metadata): a new plan with the checkpoint's physics
    options (plus `plan_kw`, e.g. graphs or stream) and the state on the
    current device.  plan.time_offset holds the checkpoint's elapsed time."""
    import torch

    from . import fs

    arr, meta = load_arrays(path)
    opts = dict(meta["plan"])
    n = opts.pop("n")
    plan = fs.Plan(n, **opts, **plan_kw)
    plan.time_offset = float(meta["time"])
    state = torch.from_numpy(arr).to("cuda")
    if tuple(state.shape) != tuple(plan.state_shape) or state.dtype != plan.complex_dtype:
        plan.close()
        raise ValueError("checkpoint state does not match the plan it describes")
    return plan, state, meta
