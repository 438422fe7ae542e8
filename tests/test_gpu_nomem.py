"""Allocation failure: every object of the library makes its device (and, with
FS_CHECK_FINITE, pinned host) allocations at creation, and an allocation that
fails must make creation return FS_E_NOMEM and release whatever was already
allocated.  The failure is forced from the host by the library's test hook
(FS_TEST_FAIL_ALLOC = "k#tag": the k-th allocation after the variable took
that value fails); no kernel runs on the failing paths.  Device memory is
compared before and after each failed creation, and a creation right after
(hook cleared) must succeed."""
import os

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FS_E_NOMEM = -3
# a leak of the smallest workspace involved (the network's, ~1 MB) shows
# beyond this; the plans' and closures' workspaces are hundreds of MB
SLACK = 256 * 1024


@pytest.fixture(scope="module")
def fs():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1807_01769_amd import fs as _fs
    return _fs


def _free():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def _fails_cleanly(fs, make, k, tag):
    before = _free()
    os.environ["FS_TEST_FAIL_ALLOC"] = f"{k}#{tag}"
    try:
        with pytest.raises(fs.FsError) as e:
            make()
    finally:
        del os.environ["FS_TEST_FAIL_ALLOC"]
    assert e.value.status == FS_E_NOMEM, str(e.value)
    after = _free()
    print(f"{tag}: {e.value}; device memory {before - after} bytes lower after", flush=True)
    assert before - after <= SLACK
    obj = make()  # the hook is off: creation succeeds
    obj.close()


def test_plan_nomem(fs):
    print("case nomem plan", flush=True)
    _fails_cleanly(fs, lambda: fs.Plan(256, nu=1e-3, dt=1e-3), 1, "plan workspace")
    # the pinned flag of FS_CHECK_FINITE is the second allocation: the
    # workspace made before it must be returned
    _fails_cleanly(fs, lambda: fs.Plan(256, nu=1e-3, dt=1e-3, check_finite=True), 2,
                   "plan pinned flag")


def test_ensemble_mlp_nomem(fs):
    print("case nomem ensemble, network", flush=True)
    _fails_cleanly(fs, lambda: fs.Ensemble([128, 256, 256], nu=1e-4, dt=5e-4), 1, "ensemble")
    _fails_cleanly(fs, lambda: fs.Mlp(seed=7), 1, "network")


def test_closure_les_nomem(fs):
    print("case nomem closure, LES", flush=True)
    fine = fs.Plan(128, nu=1e-3, dt=1e-3)
    coarse = fs.Plan(32, nu=1e-3, dt=8e-3)
    net = fs.Mlp(seed=7)
    _fails_cleanly(fs, lambda: fs.Closure(fine, coarse), 1, "closure")
    _fails_cleanly(fs, lambda: fs.Les(coarse, net), 1, "les")
    for o in (net, coarse, fine):
        o.close()
