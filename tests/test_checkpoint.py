"""Checkpoint file format (CPU): the state round-trips bit for bit through
the .npy file and the sidecar describes it; a mismatched pair is refused."""
import json

import numpy as np
import pytest

from paper_1807_01769_amd import checkpoint as ck
from paper_1807_01769_amd import inputs as I


def test_round_trip_is_bitwise(tmp_path):
    u = I.random_solenoidal_3d(16, seed=3, dtype=np.complex64)
    meta = {"plan": {"n": 16, "nu": 1e-3}, "step": 7, "time": 0.007, "seed": 3, "extra": {}}
    npy, js = ck.save_arrays(str(tmp_path / "run"), u, meta)
    back, m = ck.load_arrays(npy)
    assert back.dtype == u.dtype and back.shape == u.shape
    assert np.array_equal(back.view(np.uint32), u.view(np.uint32))
    assert m["step"] == 7 and m["plan"]["n"] == 16 and m["format"] == ck.FORMAT


def test_mismatched_sidecar_is_refused(tmp_path):
    u = np.zeros((3, 8, 8, 5), np.complex128)
    npy, js = ck.save_arrays(str(tmp_path / "run"), u, {"plan": {}})
    meta = json.load(open(js))
    meta["shape"] = [3, 8, 8, 4]
    json.dump(meta, open(js, "w"))
    with pytest.raises(ValueError):
        ck.load_arrays(npy)
