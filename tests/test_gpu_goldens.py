"""Full-length parity with stored oracle results (tests/golden/, written by
tests/golden/make_goldens.py from the oracle alone): the 256 x 10000 stress
instance over its whole 1000-iteration budget (Tabu and neighbourhood search,
every trace record), a sample of the 4096-instance uneven batch solved in one
call with all its 32 768 solves, and a sample of the serving stream (its
largest request included) served through at_server_*."""
import json
import os
import sys

import numpy as np
import pytest

from gen.instances import batch_instance, batch_specs, make_instance, serve_specs, stress_instance
from helpers import gpu_to_np

pytestmark = pytest.mark.gpu

at = pytest.importorskip("paper_2002_11710_amd")

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLD)
import make_goldens as mg  # noqa: E402


def _load(name):
    path = os.path.join(GOLD, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} has not been written (tests/golden/make_goldens.py)")
    with open(path) as f:
        return json.load(f)


def _digest(g):
    """The GPU result in the golden file's form."""
    g = gpu_to_np(g)
    k = g["iters_done"]
    tm = g["tr_move"].view(np.uint32)[:k] if "tr_move" in g else None
    out = dict(best_obj=int(g["best_obj"]), final_obj=int(g["final_obj"]), iters_done=int(k),
               best_iter=int(g["best_iter"]),
               best_routes=mg.sha(g["route_off"], g["route_seq"]),
               best_route_of=mg.sha(g["route_of"]),
               final_routes=mg.sha(g["final_off"], g["final_seq"]))
    if tm is not None:
        out["trace"] = mg.sha(tm, g["tr_delta"][:k], g["tr_obj"][:k], g["tr_flags"][:k])
    return out, g


def _compare(want, g, label):
    got, raw = _digest(g)
    assert raw["status"] == 0, label
    if "tr_move" in want:
        k = want["iters_done"]
        tm = raw["tr_move"].view(np.uint32)[:k]
        diff = np.nonzero(tm != np.array(want["tr_move"], dtype=np.uint32))[0]
        assert diff.size == 0, (label, "first move mismatch at iteration", int(diff[0]) if diff.size else -1)
        assert np.array_equal(raw["tr_delta"][:k], want["tr_delta"]), label
        assert np.array_equal(raw["tr_obj"][:k], want["tr_obj"]), label
        assert np.array_equal(raw["tr_flags"][:k], want["tr_flags"]), label
    for key in ("iters_done", "best_obj", "final_obj", "best_iter", "best_routes", "best_route_of",
                "final_routes", "trace"):
        assert got[key] == want[key], (label, key, got[key], want[key])


@pytest.mark.parametrize("name,variant", [("stress_tabu.json", 0), ("stress_ns.json", 1)])
def test_stress_full_budget(name, variant):
    """256 vehicles x 10000 missions (1.5e8 moves per iteration, the HBM-resident
    schedule over the whole GPU), all 1000 iterations."""
    gold = _load(name)
    inst = stress_instance(0)
    print(f"stress {gold['variant']} 1000 iterations", flush=True)
    g = at.solve(at.DeviceInstance.from_instance(inst), variant=variant, tenure=25, iters=1000)
    _compare(gold["result"], g, gold["variant"])


def test_batch_sample_in_full_batch():
    """All 4096 instances x 8 restarts x 2000 iterations in one at_solve_batch
    call (the benchmark's launch configuration); every 64th instance, with its
    8 restarts, equals the oracle's result and trace."""
    gold = _load("batch_sample.json")
    n, stride, R = gold["n_instances"], gold["stride"], gold["restarts"]
    specs = batch_specs(n)
    sample = {row["instance"] for row in gold["solves"]}
    assert sample == set(range(0, n, stride))
    print(f"batch {n} x {R}", flush=True)
    devs = [at.DeviceInstance.from_instance(batch_instance(s)) for s in specs]
    params = [at._capi.make_params(at.AT_TABU, s["tenure"], s["iters"], True, s["seed"],
                                   s["index"] in sample) for s in specs]
    res = at.solve_batch(devs, params, R)
    assert all(r["status"] == 0 for r in res)
    for row in gold["solves"]:
        i, r = row["instance"], row["restart"]
        _compare(row["result"], res[i * R + r], f"instance {i} restart {r}")


def test_serving_sample():
    """The serving stream's first requests and its largest (M = 2000) served
    together through at_server_* with a slot limit, so requests are admitted
    while others run; each equals the oracle's solve."""
    gold = _load("serve_sample.json")
    specs = serve_specs(gold["n_requests"])
    rows = gold["requests"]
    print(f"serving {len(rows)} requests", flush=True)
    devs = {}
    for row in rows:
        s = specs[row["request"]]
        assert s["n_missions"] == row["n_missions"]
        devs[row["request"]] = at.DeviceInstance.from_instance(
            make_instance(s["seed"], s["n_fac"], s["n_bases"], s["n_vehicles"], s["n_missions"]))
    srv = at.Server(16 << 30, max_slots=4, chunk_iters=50)
    try:
        tickets = {srv.submit(devs[row["request"]], tenure=specs[row["request"]]["tenure"],
                              iters=specs[row["request"]]["iters"], trace=True): row for row in rows}
        pending = set(tickets)
        for _ in range(1000000):
            srv.progress()
            for t in list(pending):
                r = srv.poll(t)
                if r is not None:
                    pending.discard(t)
                    _compare(tickets[t]["result"], r, f"request {tickets[t]['request']}")
            if not pending:
                break
        assert not pending
    finally:
        srv.close()

