"""The allocation-free entry point (at_solve_noalloc) through the C ABI: calls
in a row, each on a smaller instance than the one before, each equal to
at_solve's result on the same input (bit for bit: scalars, best and final
routes, each mission's vehicle, the whole trace), and a solve too large for
the fixed workspace rejected before any launch."""
import ctypes as C

import numpy as np
import pytest

from gen.instances import m400_instance, small_instance, stress_instance
from helpers import gpu_to_np

pytestmark = pytest.mark.gpu

at = pytest.importorskip("paper_2002_11710_amd")


def _same(a, b, label):
    a, b = gpu_to_np(a), gpu_to_np(b)
    for k in ("status", "best_obj", "final_obj", "iters_done", "best_iter"):
        assert a[k] == b[k], (label, k, a[k], b[k])
    for k in ("route_off", "route_seq", "route_of", "final_off", "final_seq", "tr_move", "tr_delta",
              "tr_obj", "tr_flags"):
        assert np.array_equal(a[k], b[k]), (label, k)


def test_noalloc_equals_solve_on_shrinking_inputs():
    """The stress instance (HBM-resident schedule), then the 16x400 workload
    (multi-workgroup schedule), then the 3x12 workload (one workgroup): the
    fixed array keeps the previous call's contents, which no call may read."""
    runs = [(stress_instance(0), dict(tenure=25, iters=8), "256x10000 Tabu"),
            (m400_instance(0), dict(tenure=15, iters=1500), "16x400 Tabu"),
            (m400_instance(0), dict(variant=at.AT_NS, tenure=15, iters=5000), "16x400 NS"),
            (small_instance(0), dict(tenure=7, iters=500, restart_seed=3), "3x12 Tabu"),
            (small_instance(0), dict(variant=at.AT_NS, tenure=7, iters=500), "3x12 NS")]
    for inst, kw, label in runs:
        print(label, flush=True)
        dev = at.DeviceInstance.from_instance(inst)
        want = at.solve(dev, **kw)
        got = at.solve_noalloc(dev, **kw)
        assert want["status"] == 0 and want["iters_done"] > 0
        _same(want, got, label)


def test_noalloc_rejects_a_solve_beyond_the_fixed_workspace():
    """16 000 missions on 4300 locations need over 200 MiB of workspace: the call
    returns AT_ENOMEM from its host-side size check (the instance pointers are
    never dereferenced), and the next call still works."""
    L = at.lib()
    big = at._capi._Instance(4300, 0x1000, 16000, 0x2000, 0x3000, 300, 0x4000)
    pr = at._capi.make_params(tenure=25, iters=10)
    res = at._capi._Result()
    res.route_off, res.route_seq = 0x5000, 0x6000
    assert L.at_workspace_size(1, C.byref(big), C.byref(pr), 1) > (64 << 20)
    assert L.at_solve_noalloc(C.byref(big), C.byref(pr), None, C.byref(res)) == at.AT_ENOMEM
    assert b"64" in L.at_last_error() or b"67108864" in L.at_last_error()
    dev = at.DeviceInstance.from_instance(small_instance(0))
    _same(at.solve(dev, tenure=7, iters=50), at.solve_noalloc(dev, tenure=7, iters=50), "after rejection")
