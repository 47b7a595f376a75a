"""Write the stored expected results under tests/golden/ from the oracle alone.

Each file holds what the plain CPU oracle (oracle/) computes on a seeded
synthetic workload drawn by gen/instances.py; nothing here comes from the HIP
library.  The GPU parity tests compare the library's results with them.

  stress_tabu.json, stress_ns.json   256 vehicles x 10000 missions (2000
                                      facilities, 200 bases, seed 0), tenure 25,
                                      1000 iterations: Tabu search and
                                      neighbourhood search, full trace
  batch_sample.json                   every 64th instance of the 4096-instance
                                      uneven batch x 8 restarts x 2000 iterations
  serve_sample.json                   requests of the serving stream (M
                                      log-uniform in [10, 2000]), the largest
                                      one included, 1000 iterations each

Solves run on a thread pool (ctypes releases the GIL inside each oracle call).
Usage: python tests/golden/make_goldens.py [stress_tabu stress_ns batch serve] [--threads N]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from gen.instances import (batch_instance, batch_specs, make_instance, restart_seed,  # noqa: E402
                           serve_specs, stress_instance)

# the batch sample: instances 0, 64, 128, ... of the 4096-instance batch
BATCH_N, BATCH_STRIDE, BATCH_RESTARTS = 4096, 64, 8
# the serving sample: the first SERVE_FIRST requests of a SERVE_N-request stream
# plus its largest request
SERVE_N, SERVE_FIRST = 2000, 10


def sha(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).astype("<i8").tobytes())
    return h.hexdigest()


def route_of(off, seq):
    out = np.empty(len(seq), dtype=np.int64)
    for v in range(len(off) - 1):
        out[np.asarray(seq[off[v]:off[v + 1]], dtype=np.int64)] = v
    return out


def summary(r: dict, full_trace: bool) -> dict:
    """What a test compares: scalars, digests of the best and final routes (and
    of the best solution's vehicle per mission), the trace in full or as a
    digest."""
    out = dict(best_obj=int(r["best_obj"]), final_obj=int(r["final_obj"]),
               iters_done=int(r["iters_done"]), best_iter=int(r["best_iter"]),
               best_routes=sha(r["best_off"], r["best_seq"]),
               best_route_of=sha(route_of(r["best_off"], r["best_seq"])),
               final_routes=sha(r["final_off"], r["final_seq"]),
               trace=sha(r["tr_move"], r["tr_delta"], r["tr_obj"], r["tr_flags"]))
    if full_trace:
        out.update(tr_move=[int(x) for x in r["tr_move"]], tr_delta=[int(x) for x in r["tr_delta"]],
                   tr_obj=[int(x) for x in r["tr_obj"]], tr_flags=[int(x) for x in r["tr_flags"]])
    return out


def write(name: str, payload: dict):
    path = os.path.join(HERE, name)
    with open(path + ".tmp", "w") as f:
        json.dump(payload, f, indent=1)
        f.write("\n")
    os.replace(path + ".tmp", path)
    print("wrote", path, flush=True)


def stress(variant: int):
    inst = stress_instance(0)
    P = oracle.Problem.from_instance(inst)
    t0 = time.time()
    r = P.solve(variant=variant, tenure=25, iters=1000)
    name = "stress_tabu.json" if variant == 0 else "stress_ns.json"
    write(name, dict(workload="256 vehicles x 10000 missions, 200 bases, 2000 facilities, seed 0",
                     variant="tabu" if variant == 0 else "ns", tenure=25, iters=1000,
                     oracle_s=round(time.time() - t0, 1), result=summary(r, True)))


def batch(threads: int):
    specs = batch_specs(BATCH_N)[::BATCH_STRIDE]
    jobs = [(sp, rr) for sp in specs for rr in range(BATCH_RESTARTS)]
    probs = {sp["index"]: oracle.Problem.from_instance(batch_instance(sp)) for sp in specs}

    def one(job):
        sp, rr = job
        r = probs[sp["index"]].solve(variant=0, tenure=sp["tenure"], iters=sp["iters"],
                                     restart_seed=restart_seed(sp["seed"], rr))
        return dict(instance=sp["index"], restart=rr, result=summary(r, False))

    t0 = time.time()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        rows = list(ex.map(one, jobs))
    write("batch_sample.json", dict(workload=f"uneven batch of {BATCH_N} instances (stream seed 0), "
                                             f"every {BATCH_STRIDE}th instance x {BATCH_RESTARTS} restarts, "
                                             f"Tabu, 2000 iterations",
                                    n_instances=BATCH_N, stride=BATCH_STRIDE, restarts=BATCH_RESTARTS,
                                    oracle_s=round(time.time() - t0, 1), solves=rows))


def serve(threads: int):
    specs = serve_specs(SERVE_N)
    big = max(range(SERVE_N), key=lambda k: specs[k]["n_missions"])
    picks = list(range(SERVE_FIRST)) + ([big] if big >= SERVE_FIRST else [])

    def one(k):
        s = specs[k]
        inst = make_instance(s["seed"], s["n_fac"], s["n_bases"], s["n_vehicles"], s["n_missions"])
        r = oracle.Problem.from_instance(inst).solve(variant=0, tenure=s["tenure"], iters=s["iters"])
        return dict(request=k, n_missions=s["n_missions"], result=summary(r, False))

    t0 = time.time()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        rows = list(ex.map(one, sorted(picks, key=lambda k: -specs[k]["n_missions"])))
    rows.sort(key=lambda x: x["request"])
    write("serve_sample.json", dict(workload=f"serving stream (stream seed 1) of {SERVE_N} requests: the first "
                                             f"{SERVE_FIRST} and the largest, Tabu, tenure 15, 1000 iterations",
                                    n_requests=SERVE_N, oracle_s=round(time.time() - t0, 1), requests=rows))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*", default=["stress_tabu", "stress_ns", "batch", "serve"])
    ap.add_argument("--threads", type=int, default=max(1, (os.cpu_count() or 2) - 2))
    a = ap.parse_args()
    oracle.lib()
    for c in a.cases:
        if c == "stress_tabu":
            stress(0)
        elif c == "stress_ns":
            stress(1)
        elif c == "batch":
            batch(a.threads)
        elif c == "serve":
            serve(a.threads)
        else:
            raise SystemExit(f"unknown case {c}")


if __name__ == "__main__":
    main()
