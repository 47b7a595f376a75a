"""Autotuner for the schedules of small solves.

For size buckets of move slots per iteration it times uneven batches (drawn
from the batch size law of gen.instances) on the wave schedule (one wavefront
per solve) and on the one-workgroup schedule under every launch shape
(threads per workgroup x columns per work unit), keeps the fastest per bucket,
and writes csrc/tuned_table.h; rebuild the library afterwards
(paper_2002_11710_amd/build.py).  Every schedule and shape gives identical
results, so the table only changes speed.  Needs the GPU.

Usage: python -m paper_2002_11710_amd.autotune [--iters 200] [--per-bucket 512] [--restarts 4]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

BUCKETS = [(0, 2000), (2000, 4000), (4000, 12000), (12000, 30000), (30000, 60000),
           (60000, 100000), (100000, 1 << 62)]
SHAPES = [(b, c) for b in (256, 512, 1024) for c in (8, 16, 32)]


def slots(m, v):
    return m * (m + v) + m * (m - 1) // 2


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=200)
    ap.add_argument("--per-bucket", type=int, default=512)
    ap.add_argument("--restarts", type=int, default=4)
    ap.add_argument("--out", default=os.path.join(HERE, "csrc", "tuned_table.h"))
    args = ap.parse_args()
    import torch

    import paper_2002_11710_amd as at
    from gen.instances import batch_instance, batch_specs

    # enough solves per bucket (per-bucket x restarts, default 2048) to fill every CU
    # several times over, so the shape that maximises throughput wins
    specs = batch_specs(60000)
    rows = []
    for lo, hi in BUCKETS:
        pick = [s for s in specs if lo <= slots(s["n_missions"], s["n_vehicles"]) < hi]
        pick = pick[: args.per_bucket]
        if not pick:
            continue
        devs = [at.DeviceInstance.from_instance(batch_instance(s)) for s in pick]
        best = None
        timings = []
        # (1, 0, 0): the wave schedule; else one workgroup of `block` threads, `chunk` columns
        wave_fits = hi <= 30000
        for wave, block, chunk in ([(1, 0, 0)] if wave_fits else []) + [(0, b, c) for b, c in SHAPES]:
            params = [at._capi.make_params(at.AT_TABU, s["tenure"], args.iters, True, s["seed"],
                                           False, at.SCHED_WAVE if wave else at.SCHED_WG, 0, block,
                                           chunk) for s in pick]
            at.solve_batch(devs, params, args.restarts)
            torch.cuda.synchronize()
            # the launch's own duration (HIP events around the search), best of three
            dt = min(float(at.solve_batch(devs, params, args.restarts)[0]["search_ms"]) / 1000.0
                     for _ in range(3))
            print(json.dumps(dict(bucket=[lo, hi], wave=wave, block=block, chunk=chunk,
                                  s=round(dt, 4))), flush=True)
            timings.append((dt, wave, block, chunk))
            if best is None or dt < best[0]:
                best = (dt, wave, block, chunk)
        if best[1]:
            # the workgroup shape still applies to these sizes when the wave schedule
            # is not taken (serving): the fastest one
            wg = min((r for r in timings if r[1] == 0), key=lambda r: r[0])
            rows.append((hi, 1, wg[2], wg[3]))
        else:
            rows.append((hi, 0, best[2], best[3]))
    lines = ["// tuned_table.h -- default schedule and launch shape of small solves by move",
             "// slots per iteration (M*(M+V) + M*(M-1)/2).  Rows are tried in order; the",
             "// first row whose max_slots exceeds the solve's slots applies: wave = 1 gives",
             "// such solves one wavefront each (the wave schedule), else one workgroup of",
             "// `block` threads with swap units of `chunk` columns.",
             "// Written by paper_2002_11710_amd/autotune.py from timings on gfx950.",
             "#pragma once", "#include <cstdint>", "", "namespace at {",
             "struct TunedRow { int64_t max_slots; int wave; int block; int chunk; };",
             "static const TunedRow kTuned[] = {"]
    for hi, wv, b, c in rows:
        lim = "INT64_MAX" if hi >= (1 << 62) else str(hi)
        lines.append(f"    {{{lim}, {wv}, {b}, {c}}},")
    lines += ["};", "}  // namespace at", ""]
    with open(args.out, "w") as f:
        f.write("\n".join(lines))
    print("wrote", args.out)


if __name__ == "__main__":
    main()
