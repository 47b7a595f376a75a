"""Shared test helpers: run the oracle and the HIP path on the same seeded inputs
and compare them field by field."""
import numpy as np

import oracle


def oracle_problem(inst):
    return oracle.Problem.from_instance(inst)


def oracle_solve(inst, variant=0, tenure=None, iters=None, restart_seed=0, aspiration=1):
    P = oracle_problem(inst)
    r = P.solve(variant=variant, tenure=inst.tenure if tenure is None else tenure,
                iters=inst.iters if iters is None else iters, aspiration=aspiration,
                restart_seed=restart_seed)
    return P, r


def gpu_to_np(res):
    out = {}
    for k, v in res.items():
        if hasattr(v, "cpu"):
            out[k] = v.cpu().numpy()
        else:
            out[k] = v
    return out


def assert_same_result(o, g, label=""):
    """Bit-exact comparison of an oracle result dict and a GPU result dict."""
    g = gpu_to_np(g)
    assert g["status"] == 0, label
    assert g["iters_done"] == o["iters_done"], (label, g["iters_done"], o["iters_done"])
    if "tr_move" in g:
        k = o["iters_done"]
        tm = g["tr_move"].view(np.uint32)[:k]
        diff = np.nonzero(tm != o["tr_move"])[0]
        assert diff.size == 0, (label, "first trace mismatch at", int(diff[0]) if diff.size else -1,
                                tm[diff[:3]], o["tr_move"][diff[:3]])
        assert np.array_equal(g["tr_delta"][:k], o["tr_delta"]), label
        assert np.array_equal(g["tr_obj"][:k], o["tr_obj"]), label
        assert np.array_equal(g["tr_flags"][:k], o["tr_flags"]), label
    assert g["best_obj"] == o["best_obj"], (label, g["best_obj"], o["best_obj"])
    assert g["final_obj"] == o["final_obj"], (label, g["final_obj"], o["final_obj"])
    assert g["best_iter"] == o["best_iter"], (label, g["best_iter"], o["best_iter"])
    assert np.array_equal(g["route_off"], o["best_off"]), label
    assert np.array_equal(g["route_seq"], o["best_seq"]), label
    if "route_of" in g:
        assert np.array_equal(g["route_of"], route_of(o["best_off"], o["best_seq"])), label
    if "final_off" in g:
        assert np.array_equal(g["final_off"], o["final_off"]), label
        assert np.array_equal(g["final_seq"], o["final_seq"]), label


def route_of(off, seq):
    """Vehicle of every mission of a flattened solution (off: V+1, seq: M)."""
    off = np.asarray(off)
    out = np.empty(len(seq), dtype=np.int32)
    for v in range(len(off) - 1):
        out[np.asarray(seq[off[v]:off[v + 1]], dtype=np.int64)] = v
    return out
