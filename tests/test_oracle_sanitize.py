"""The oracles under AddressSanitizer and UndefinedBehaviorSanitizer: both C
files are built with -fsanitize=address,undefined into a temporary library,
which a child Python process (with the ASan runtime preloaded) drives through
every entry point on small instances: the unconstrained search (Tabu, NS,
seeded starts, every slot's key, deltas by definition and closed form, applied
moves) and the constrained one (feasibility, keys in both modes, Algorithm 1
with its repair, best form and sweep form).  Any sanitizer report fails the
test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r'''
import os, sys
sys.path.insert(0, os.environ["ROOT"])
import numpy as np
import oracle
oracle._LIB = os.environ["SAN_LIB"]
from gen.instances import fleet_instance, make_instance, small_instance

for inst in (small_instance(0), make_instance(5, 40, 3, 4, 30), make_instance(3, 12, 1, 1, 1),
             make_instance(4, 12, 2, 3, 0)):
    P = oracle.Problem.from_instance(inst)
    for variant in (oracle.TABU, oracle.NS):
        for seed in (0, 7):
            P.solve(variant=variant, tenure=5, iters=60, restart_seed=seed)
    if P.M:
        off, seq = P.greedy(3)
        tabu = np.full(P.M * P.V, -1, np.int32)
        cur = P.objective(off, seq)
        P.keys(off, seq, tabu, 0, cur, cur)
        for idx in range(0, P.n_slots, max(1, P.n_slots // 50)):
            ok, d0 = P.delta(off, seq, idx, 0)
            ok, d1 = P.delta(off, seq, idx, 1)
            if ok:
                P.apply(off, seq, idx)
for seed in range(4):
    inst = fleet_instance(seed, 10, n_fac=14, n_plane=1, n_heli=2, w_lo=3600, w_hi=12 * 3600)
    F = oracle.FleetProblem(oracle.travel(inst.lat, inst.lon, 300.0), oracle.travel(inst.lat, inst.lon, 500.0),
                            inst.pickup, inst.delivery, inst.deadline, inst.heli_only, inst.vehicle_loc,
                            inst.vehicle_type, inst.flight_limit, inst.horizon)
    try:
        off, seq, _ = F.greedy(0)
    except ValueError:
        continue
    ok, cur = F.feasible(off, seq)
    tabu = np.full(F.M * F.V, -1, np.int32)
    F.keys(off, seq, tabu, 0, cur, cur, mode=0)
    F.keys(off, seq, tabu, 0, cur, cur, mode=1)
    F.solve(variant=oracle.TABU, tenure=3, iters=40, restart_seed=seed)
    F.solve(variant=oracle.NS, iters=40)
    F.sweep(variant=oracle.TABU, tenure=3, restart_seed=seed + 1)
    F.sweep(variant=oracle.NS)
print("sanitized run ok")
'''


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracles_under_asan_and_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    src = [os.path.join(ROOT, "oracle", "atabu_oracle.c"), os.path.join(ROOT, "oracle", "fleet_oracle.c")]
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-std=c99", "-fPIC",
                    "-shared", "-o", lib, *src, "-lm"], check=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True,
                           text=True).stdout.strip()
    env = dict(os.environ, ROOT=ROOT, SAN_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", DRIVER], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "sanitized run ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
