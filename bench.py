"""Benchmark: Tabu-search move evaluations per second at M = 400.

One step = the search hot path on the 16-vehicle x 400-mission workload
(10 bases, 120 facilities, seed 0): a Tabu search of 5000 iterations with
tenure 15 and a neighbourhood search on the same instance, each a greedy
start plus every iteration's relocate + swap evaluation, tabu mask, argmin
and apply, all in the HIP library.  The travel matrix (Eq (1)) is built on
the host once per instance (at_build_travel) and uploaded before timing
starts, so every input is resident in HBM; its host time and upload time are
reported beside the step.

value = valid moves scored per second over the whole step (245 400 per
iteration), whole GPU.  Also reported: Tabu iterations per second, the search
kernel's roofline (integer VALU work per launch over its HIP-event duration),
optionally the uneven-batch solves per second (--batch), and the oracle timed
on the host as the CPU baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch N] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# int32 VALU lane-operations per clock per CU (4 SIMDs x 16 lanes) x 256 CUs x 2.4 GHz
ALU_PEAK_OPS = 256 * 64 * 2.4e9
# algorithmic integer work per scored move: relocate = 2 address adds + 3 delta adds
# + 1 min-select; swap = 4 address adds + 5 delta adds + 1 min-select
OPS_RELOCATE, OPS_SWAP = 6, 10
# algorithmic LDS bytes per scored move in the one-workgroup (LDS-resident) kernel, a 16-bit
# gather counted as one 4-byte bank access: relocate = 2 travel gathers, swap = 4 travel
# gathers + the partner's tabu entry (records are wavefront broadcasts, not counted)
LDS_RELOCATE, LDS_SWAP = 8, 20
# travel-time reads a move's delta needs beyond the per-position records (2-byte
# gathers at data-dependent addresses): relocate 2, swap 4
GATHERS_RELOCATE, GATHERS_SWAP = 2, 4
# LDS bandwidth: 128 bytes per clock per CU x 256 CUs x 2.4 GHz
LDS_PEAK_BPS = 128 * 256 * 2.4e9
COUNTERS = os.path.join(ROOT, "profiles", "counters.txt")


def library_sha256():
    import hashlib

    import paper_2002_11710_amd._capi as capi
    with open(capi.lib_path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def profile_counters():
    """Per-dispatch counters of the committed rocprofv3 --pmc summary, if it was
    taken on the library that is loaded (same sha256); else None."""
    if not os.path.exists(COUNTERS):
        return None
    kv, kernels = {}, {}
    with open(COUNTERS) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = line.split()
            if w[0] == "kernel":
                kernels[w[1]] = {w[i]: float(w[i + 1]) for i in range(2, len(w) - 1, 2)}
            else:
                kv[w[0]] = w[1]
    if kv.get("lib_sha256") != library_sha256():
        return None
    kv["kernels"] = kernels
    return kv


def traffic_bytes(pc, kernel):
    """HBM bytes per dispatch: FETCH_SIZE and WRITE_SIZE (KiB) scaled by what the
    same counters read for a plain copy of known size."""
    if not pc or kernel not in pc["kernels"]:
        return None
    k = pc["kernels"][kernel]
    return 1024.0 * (k["fetch_kib"] * float(pc["copy_fetch_factor"])
                     + k["write_kib"] * float(pc["copy_write_factor"]))


def move_counts(M: int, V: int):
    """(valid relocates, swaps) scored per iteration."""
    return M * (M + V - 2), M * (M - 1) // 2


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=4096,
                    help="also time an uneven batch of this many instances x 8 restarts (0: skip)")
    ap.add_argument("--serve", type=str, default="200,400,inf",
                    help="also run the serving stream at these arrival rates (req/s, comma separated, "
                         "'inf': every request at time 0, the saturation throughput; empty: skip)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-plain", type=int, default=400,
                    help="requests of the stream also solved one at_solve at a time (the plain form)")
    ap.add_argument("--serve-chunk", type=int, default=250,
                    help="iterations per serving launch, at least, of a solve that runs on its own workgroups")
    ap.add_argument("--serve-slots", type=int, default=2048, help="concurrent solves in the server")
    ap.add_argument("--stress", type=int, default=1000,
                    help="also run the 256 x 10000 stress instance for this many iterations "
                         "(Tabu and NS; 0: skip)")
    ap.add_argument("--fleet", type=int, default=4096,
                    help="also run this many paper-scale instances of the constrained model x 8 "
                         "restarts (wave schedule; best form and sweep form; 0: skip)")
    ap.add_argument("--no-lds-peak", action="store_true", help="skip the LDS bandwidth probe")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain per-instance comparisons (profiling runs)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="first run a device-to-device copy of this many MiB (counter calibration)")
    ap.add_argument("--schedule", type=int, default=0)
    ap.add_argument("--groups", type=int, default=0)
    ap.add_argument("--sequential", action="store_true",
                    help="run the step's Tabu and NS solves as two at_solve calls, one after the other, "
                         "instead of one at_solve_batch call that runs them side by side")
    return ap.parse_args()


def lds_peak(strides=(1, 2, 4, 8, 16, 32, 64, 128)):
    """Measured LDS read bandwidth (conflict-free ds_read_b32 over the whole GPU)
    and the slowdown of each lane stride, from paper_2002_11710_amd/libldspeak.so."""
    import ctypes as C

    import torch
    path = os.path.join(ROOT, "paper_2002_11710_amd", "libldspeak.so")
    L = C.CDLL(path)
    L.ldspeak_run.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double),
                              C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    blocks = 2 * cus                      # two 64 KiB workgroups of 1024 threads per CU

    def run(iters, stride):
        ms, clk, wt = C.c_double(0), C.c_uint64(0), C.c_uint64(0)
        rc = L.ldspeak_run(blocks, iters, stride, C.byref(ms), C.byref(clk), C.byref(wt))
        if rc != 0:
            raise RuntimeError(f"ldspeak_run: HIP error {rc}")
        return ms.value, clk.value, wt.value

    iters = 40000
    ms, clk, wt = run(iters, 1)
    nbytes = blocks * 1024 * iters * 8 * 4       # 8 reads of 4 bytes per thread and iteration
    ghz = clk / (wt / 100e6) / 1e9 if wt else None
    out = {"bytes": nbytes, "ms": ms, "TBps": nbytes / (ms / 1000.0) / 1e12, "cus": cus,
           "shader_GHz": ghz,
           "B_per_clk_per_CU": (nbytes / (ms / 1000.0)) / (cus * ghz * 1e9) if ghz else None}
    base = run(2000, 1)[0]
    out["stride_slowdown"] = {str(s): run(2000, s)[0] / base for s in strides}
    # random 2-byte gathers (the travel reads of the move deltas)
    L.ldspeak_gather_run.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_uint64),
                                     C.POINTER(C.c_uint64)]
    ms2, clk2, wt2 = C.c_double(0), C.c_uint64(0), C.c_uint64(0)
    giters = 20000
    rc = L.ldspeak_gather_run(blocks, giters, C.byref(ms2), C.byref(clk2), C.byref(wt2))
    if rc != 0:
        raise RuntimeError(f"ldspeak_gather_run: HIP error {rc}")
    gathers = blocks * 1024 * giters * 8
    out["random_u16_gathers_per_s"] = gathers / (ms2.value / 1000.0)
    out["random_u16_GBps"] = 2 * gathers / (ms2.value / 1000.0) / 1e9
    if ghz:
        out["random_u16_wave_reads_per_clk_per_CU"] = gathers / 64 / (ms2.value / 1000.0) / (cus * ghz * 1e9)
    return out


def host_cpu():
    """(usable host threads, CPU model name) of the machine the bench runs on."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return n, model


def cpu_baseline(inst, budget_s=20.0):
    """The oracle (plain C, untuned) on the host, on bounded samples: the 16x400
    Tabu search on one thread (the headline figure), the 3x12 workload on one
    thread, a sample of the uneven batch on every usable host thread (one solve
    per thread at a time; ctypes releases the GIL during each oracle call), and
    a few iterations of the 256x10000 stress instance on one thread."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    from gen.instances import batch_instance, batch_specs, restart_seed, small_instance, stress_instance
    nthreads, model = host_cpu()
    P = oracle.Problem.from_instance(inst)
    rel, swp = move_counts(P.M, P.V)
    t0 = time.perf_counter()
    iters = 0
    # Tabu in slices until the budget is used (the full run is 5000 iterations)
    n = 500
    P.solve(variant=0, tenure=15, iters=n, trace=False)
    iters += n
    dt = time.perf_counter() - t0
    while dt < budget_s * 0.5 and iters < 5000:
        n2 = min(5000, 2 * n)
        t1 = time.perf_counter()
        P.solve(variant=0, tenure=15, iters=n2, trace=False)
        dt = time.perf_counter() - t1
        iters, n = n2, n2
    evals = iters * (rel + swp)
    out = dict(value=evals / dt, unit="move evals/s", cores=1, kind="oracle",
               sample=f"oracle Tabu search on the 16x400 workload, {iters} iterations "
                      f"(single thread, {dt:.2f} s)",
               host_threads=nthreads, cpu_model=model)
    # 3 x 12, 500 Tabu iterations, single thread
    s12 = small_instance(0)
    P12 = oracle.Problem.from_instance(s12)
    t1 = time.perf_counter()
    reps = 0
    while time.perf_counter() - t1 < 0.5:
        P12.solve(variant=0, tenure=7, iters=500, trace=False)
        reps += 1
    d12 = time.perf_counter() - t1
    r12, w12 = move_counts(12, 3)
    out["small_3x12"] = dict(solves_per_s=reps / d12, move_evals_per_s=reps * 500 * (r12 + w12) / d12,
                             cores=1, sample=f"{reps} Tabu solves of 500 iterations")
    # the uneven batch on every usable thread: instances 0..k-1, restart 0, 2000 iterations
    specs = batch_specs(4096)[:4 * nthreads]
    probs = [oracle.Problem.from_instance(batch_instance(sp)) for sp in specs]

    def one(k):
        sp = specs[k]
        probs[k].solve(variant=0, tenure=sp["tenure"], iters=sp["iters"],
                       restart_seed=restart_seed(sp["seed"], 0), trace=False)

    t1 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=nthreads) as ex:
        list(ex.map(one, range(len(specs))))
    db = time.perf_counter() - t1
    bev = sum(2000 * sum(move_counts(sp["n_missions"], sp["n_vehicles"])) for sp in specs)
    out["batch_all_threads"] = dict(solves_per_s=len(specs) / db, move_evals_per_s=bev / db,
                                    cores=nthreads,
                                    sample=f"first {len(specs)} instances of the uneven batch, "
                                           f"restart 0, 2000 iterations each, {db:.2f} s")
    # stress instance: a few Tabu iterations (greedy start included), single thread
    st = stress_instance(0)
    Ps = oracle.Problem.from_instance(st)
    k = 2
    t1 = time.perf_counter()
    Ps.solve(variant=0, tenure=25, iters=k, trace=False)
    ds = time.perf_counter() - t1
    rs, ws_ = move_counts(st.n_missions, st.n_vehicles)
    out["stress_capped"] = dict(move_evals_per_s=k * (rs + ws_) / ds, cores=1,
                                est_s_per_1000_iters=ds / k * 1000.0,
                                sample=f"{k} Tabu iterations of the 256x10000 instance ({ds:.2f} s, "
                                       f"greedy start included); the 1000-iteration time is "
                                       f"extrapolated linearly")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only; --gpus {args.gpus} is not supported (batches and "
              f"serving streams would shard by solve, one share per GPU, with no exchange)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2002_11710_amd as at
    from gen.instances import m400_instance

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # a plain copy of known size, run before the benchmark in the same process:
        # FETCH_SIZE / WRITE_SIZE of this kernel give the counter-to-bytes factor
        # used to scale the search kernel's counters
        n = args.copy_calibration << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty(n, dtype=torch.uint8, device="cuda")
        a.fill_(1)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    torch.zeros(1, device="cuda")
    torch.cuda.synchronize()   # the device context exists before anything is timed
    pc = profile_counters()
    inst = m400_instance(0)
    M, V, ITERS, TEN = inst.n_missions, inst.n_vehicles, 5000, 15
    # Eq (1) on the host (at_build_travel), once per instance, then uploaded: the
    # timed step starts with every input resident in HBM
    t0 = time.perf_counter()
    travel_host = at.build_travel(inst.lat, inst.lon)
    travel_host_ms = (time.perf_counter() - t0) * 1000.0
    t0 = time.perf_counter()
    travel = torch.as_tensor(travel_host).cuda()
    torch.cuda.synchronize()
    travel_upload_ms = (time.perf_counter() - t0) * 1000.0
    dev = at.DeviceInstance(travel, inst.pickup, inst.delivery, inst.vehicle_loc)
    L = at.lib()
    stream = torch.cuda.current_stream()

    import ctypes as C
    pr_tabu = at._capi.make_params(at.AT_TABU, TEN, ITERS, True, 0, True, args.schedule,
                                   args.groups)
    pr_ns = at._capi.make_params(at.AT_NS, TEN, ITERS, True, 0, True, args.schedule, args.groups)
    ci = dev.c_struct()
    out_t = at._capi._alloc_result(M, V, ITERS, True, "cuda")
    out_n = at._capi._alloc_result(M, V, ITERS, True, "cuda")
    sp = C.c_void_p(stream.cuda_stream)
    if args.sequential:
        # two calls on the stream: the Tabu solve, then the NS solve
        nbytes = int(L.at_workspace_size(1, C.byref(ci), C.byref(pr_tabu), 1))
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")

        def step():
            rt = at._capi._c_result(out_t)
            at._capi._check(L.at_solve(C.byref(ci), C.byref(pr_tabu), C.c_void_p(ws.data_ptr()),
                                       nbytes, sp, C.byref(rt)))
            rn = at._capi._c_result(out_n)
            at._capi._check(L.at_solve(C.byref(ci), C.byref(pr_ns), C.c_void_p(ws.data_ptr()),
                                       nbytes, sp, C.byref(rn)))
            return rt, rn, rt.search_ms + rn.search_ms, rt.search_ms
    else:
        # one call: the two solves side by side in one multi-workgroup launch, each
        # on its own workgroups
        ia = (at._capi._Instance * 2)(ci, ci)
        pa = (at._capi._Params * 2)(pr_tabu, pr_ns)
        nbytes = int(L.at_workspace_size(2, ia, pa, 1))
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")

        def step():
            res = (at._capi._Result * 2)(at._capi._c_result(out_t), at._capi._c_result(out_n))
            at._capi._check(L.at_solve_batch(2, ia, pa, 1, C.c_void_p(ws.data_ptr()), nbytes, sp, res))
            return res[0], res[1], res[0].search_ms, res[0].search_ms

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    launch_ms_l, tabu_ms_l, ns_iters = [], [], []
    for _ in range(args.steps):
        rt, rn, lms, tms = step()
        launch_ms_l.append(lms)
        tabu_ms_l.append(tms)
        ns_iters.append(rn.iters_done)
        assert rt.status == 0 and rn.status == 0
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1000.0 / args.steps
    rel, swp = move_counts(M, V)
    per_iter = rel + swp
    evals_per_step = per_iter * (ITERS + float(np.mean(ns_iters)))
    value = evals_per_step / (ms_per_step / 1000.0)
    # the step's search kernel: the algorithmic work of both solves over the HIP-event
    # time of the step's launches (one launch, or the two of the sequential form)
    launch_ms = float(np.mean(launch_ms_l))
    n_launch = 2 if args.sequential else 1
    it_all = ITERS + float(np.mean(ns_iters))
    ops = it_all * (rel * OPS_RELOCATE + swp * OPS_SWAP)
    achieved = ops / (launch_ms / 1000.0)
    lds_bytes = it_all * (rel * LDS_RELOCATE + swp * LDS_SWAP)
    line = {
        "metric": "move evals/s (M=400 Tabu + NS step)",
        "value": value,
        "unit": "move evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "16 vehicles x 400 missions, 10 bases, 120 facilities, seed 0; "
                               "Tabu 5000 iterations tenure 15 + neighbourhood search",
                   "moves_per_iter": per_iter, "iters": ITERS},
        "step_form": ("two at_solve calls (Tabu, then NS)" if args.sequential else
                      "one at_solve_batch call: the Tabu and NS solves side by side in one "
                      "multi-workgroup launch"),
        # the Tabu solve's launch (in the side-by-side form the step's launch, which
        # ends with the Tabu solve, the longer of the two)
        "tabu_iters_per_s": ITERS / (float(np.mean(tabu_ms_l)) / 1000.0),
        "search_ms_per_step": launch_ms,
        "ns_iters": float(np.mean(ns_iters)),
        "best_obj": int(rt.best_obj),
        "travel_host_ms": travel_host_ms,
        "travel_upload_ms": travel_upload_ms,
        "event_ms_per_step": ev0.elapsed_time(ev1) / args.steps,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK_OPS / 1e12,
                     "unit": "Tops/s", "frac": achieved / ALU_PEAK_OPS,
                     "traffic": traffic_bytes(pc, "k_search_multi"),
                     "kernel": ("k_search_multi (the Tabu and the NS launch of the step)" if args.sequential
                                else "k_search_multi (the step's launch: the Tabu and NS solves)"),
                     "avg_launch_ms": launch_ms / n_launch,
                     "lds_GBps": lds_bytes / (launch_ms / 1000.0) / 1e9},
    }
    if args.batch:
        line["batch"] = bench_batch(args.batch, plain=not args.no_plain)
        b = line["batch"]
        # the move-delta kernel at scale: LDS bytes over LDS bandwidth, with the
        # committed counters (LDS busy time and bank-conflict stalls) when they match
        lds = {"kernel": "k_search_wg (batch)", "achieved_GBps": b["lds_bytes_per_s"] / 1e9,
               "peak_GBps": LDS_PEAK_BPS / 1e9, "frac": b["lds_bytes_per_s"] / LDS_PEAK_BPS,
               "pmc_lds_busy_frac": None, "pmc_bank_conflict_frac": None, "pmc_valu_busy_frac": None,
               "traffic": traffic_bytes(pc, "k_search_wg")}
        if pc and "k_search_wg" in pc["kernels"]:
            k = pc["kernels"]["k_search_wg"]
            lds.update(pmc_lds_busy_frac=k.get("lds_busy"), pmc_bank_conflict_frac=k.get("bank_conflict"),
                       pmc_valu_busy_frac=k.get("valu_busy"))
        line["lds_roofline"] = lds
    if not args.no_lds_peak:
        # the LDS roofline's peak is the measured one (conflict-free ds_read_b32 over the
        # whole GPU, at the clock it ran at); the nominal 128 B/clk/CU at 2.4 GHz beside it
        line["lds_peak"] = lds_peak()
        if "lds_roofline" in line:
            pk = line["lds_peak"]["TBps"] * 1e12
            line["lds_roofline"].update(peak_GBps=pk / 1e9, frac=line["batch"]["lds_bytes_per_s"] / pk,
                                        peak_source="measured (ldspeak)",
                                        nominal_peak_GBps=LDS_PEAK_BPS / 1e9,
                                        frac_of_nominal=line["batch"]["lds_bytes_per_s"] / LDS_PEAK_BPS)
            # the bound of the access pattern: the travel reads are 2-byte gathers at
            # data-dependent addresses, whose bank conflicts cap them far below the
            # conflict-free peak; the probe measures that cap
            gp = line["lds_peak"]["random_u16_gathers_per_s"]
            line["lds_roofline"].update(travel_gathers_per_s=line["batch"]["travel_gathers_per_s"],
                                        random_gather_peak_per_s=gp,
                                        gather_frac=line["batch"]["travel_gathers_per_s"] / gp)
    if args.fleet:
        line["fleet"] = bench_fleet(args.fleet, plain=not args.no_plain)
    if args.stress:
        line["stress"] = bench_stress(args.stress)
    if args.serve:
        rates = [float(x) for x in args.serve.split(",")]
        line["serving"] = bench_serve_sweep(rates, args.serve_requests, chunk=args.serve_chunk,
                                            slots=args.serve_slots,
                                            plain=0 if args.no_plain else args.serve_plain)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(inst)
    print(json.dumps(line), flush=True)
    # Explicit teardown before the interpreter exits: the library's internal
    # streams, this run's device buffers and torch's cached device memory are
    # released while every runtime (and a profiler, if one is attached) is live,
    # so the exit-time destructors find nothing of this run left to free.
    at.shutdown()
    del ws, out_t, out_n, dev, travel
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def bench_batch(n_inst: int, restarts: int = 8, plain: bool = True):
    """Uneven batch: n_inst instances x restarts restarts, 2000 iterations each, one call."""
    import numpy as np
    import torch

    import paper_2002_11710_amd as at
    from gen.instances import batch_instance, batch_specs

    specs = batch_specs(n_inst)
    insts = [batch_instance(s) for s in specs]
    devs = [at.DeviceInstance.from_instance(i) for i in insts]
    params = [at._capi.make_params(at.AT_TABU, s["tenure"], s["iters"], True, s["seed"], False)
              for s in specs]
    res = at.solve_batch_flat(devs, params, restarts)   # warm-up; its buffers are reused
    ws = torch.empty(at.workspace_size(devs, params, restarts), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = at.solve_batch_flat(devs, params, restarts, ws=ws, bufs=res)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    evals = 0
    ops = 0
    lds = 0
    gathers = 0
    for s in specs:
        rel, swp = move_counts(s["n_missions"], s["n_vehicles"])
        evals += restarts * 2000 * (rel + swp)
        ops += restarts * 2000 * (rel * OPS_RELOCATE + swp * OPS_SWAP)
        lds += restarts * 2000 * (rel * LDS_RELOCATE + swp * LDS_SWAP)
        gathers += restarts * 2000 * (rel * GATHERS_RELOCATE + swp * GATHERS_SWAP)
    kms = float(res.search_ms[0])
    assert (res.status == 0).all()
    out = {"instances": n_inst, "restarts": restarts, "solves": n_inst * restarts,
           "wall_s": wall, "solves_per_s": n_inst * restarts / wall,
           "move_evals_per_s": evals / wall, "search_ms": kms,
           "alu_frac": ops / (kms / 1000.0) / ALU_PEAK_OPS,
           "lds_bytes_per_s": lds / (kms / 1000.0),
           "travel_gathers_per_s": gathers / (kms / 1000.0)}
    if not plain:
        return out
    # the plain per-instance form: one at_solve launch per (instance, restart), in
    # sequence on one stream, on a sample of the same solves (identical results)
    from gen.instances import restart_seed
    n_plain = min(res.n, 64)
    pairs = [(k // restarts, k % restarts) for k in range(n_plain)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [at.solve(devs[i], variant=at.AT_TABU, tenure=specs[i]["tenure"], iters=specs[i]["iters"],
                      restart_seed=restart_seed(specs[i]["seed"], r), trace=False) for i, r in pairs]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    for (i, r), p in zip(pairs, plain):
        k = i * restarts + r
        assert p["best_obj"] == res.best_obj[k] and torch.equal(p["route_seq"], res.route_seq(k))
    plain_work = sum(move_counts(specs[i]["n_missions"], specs[i]["n_vehicles"])[0]
                     + move_counts(specs[i]["n_missions"], specs[i]["n_vehicles"])[1] for i, _ in pairs)
    all_work = sum(restarts * sum(move_counts(s["n_missions"], s["n_vehicles"])) for s in specs)
    # plain solves/s for this batch's mix: the sample's move-eval rate applied to all solves
    plain_evals_per_s = plain_work * 2000 / t_plain
    plain_sps = plain_evals_per_s / (all_work * 2000 / res.n)
    out.update({"plain_sample_solves": n_plain, "plain_sample_s": t_plain,
                "plain_solves_per_s": plain_sps,
                "speedup_vs_plain": (n_inst * restarts / wall) / plain_sps})
    return out


def bench_fleet(n_inst: int, restarts: int = 8, iters: int = 2000, plain: bool = True):
    """The constrained model at the paper's scale (12-33 missions, 4 planes and 8
    helicopters, time limits, flight limit, helicopter-only missions): n_inst
    instances x restarts, Tabu in the best form (iters iterations) and the sweep
    form of Algorithms 2 (NS) and 3 (Tabu), each batch in one call on the wave
    schedule."""
    import torch

    import paper_2002_11710_amd as at
    from gen.instances import fleet_instance, fleet_specs, restart_seed

    specs = fleet_specs(n_inst)
    insts = [fleet_instance(s["seed"], s["n_missions"]) for s in specs]
    devs = [at.DeviceInstance(at.build_travel(i.lat, i.lon, i.speed_heli), i.pickup, i.delivery,
                              i.vehicle_loc, travel_plane=at.build_travel(i.lat, i.lon, i.speed_plane),
                              vehicle_type=i.vehicle_type, deadline=i.deadline, heli_only=i.heli_only,
                              flight_limit=i.flight_limit, horizon=i.horizon) for i in insts]
    out = {"instances": n_inst, "restarts": restarts, "solves": n_inst * restarts}

    def run(form, variant, n_it):
        params = [at._capi.make_params(variant, s["tenure"], n_it, True, s["seed"], False,
                                       form=form) for s in specs]
        res = at.solve_batch_flat(devs, params, restarts, allow_infeasible=True)
        ws = torch.empty(at.workspace_size(devs, params, restarts), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = at.solve_batch_flat(devs, params, restarts, ws=ws, allow_infeasible=True, bufs=res)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ok = res.status == 0
        assert ((res.status == 0) | (res.status == at.AT_EINFEAS)).all()
        return res, {"wall_s": wall, "solves_per_s": res.n / wall, "search_ms": float(res.search_ms[0]),
                     "infeasible_starts": int((~ok).sum()),
                     "mean_best_obj": float(res.best_obj[ok].mean()),
                     "iters_done_total": int(res.iters_done[ok].sum())}

    res, out["tabu_best"] = run(at.FORM_BEST, at.AT_TABU, iters)
    out["tabu_best"]["iters"] = iters
    slots = sum(restarts * iters * (s["n_missions"] * (s["n_missions"] + 12) + s["n_missions"] * (s["n_missions"] - 1) // 2)
                for s in specs)
    out["tabu_best"]["slot_evals_per_s"] = slots / out["tabu_best"]["wall_s"]
    _, out["ns_sweep"] = run(at.FORM_SWEEP, at.AT_NS, 100000)
    _, out["tabu_sweep"] = run(at.FORM_SWEEP, at.AT_TABU, 100000)
    if plain:
        # the plain per-instance form of the best-form batch: one at_solve per solve, in
        # sequence, on the first solves of the batch (identical results)
        n_p = min(res.n, 128)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(n_p):
            i, r = k // restarts, k % restarts
            try:
                p = at.solve(devs[i], variant=at.AT_TABU, tenure=specs[i]["tenure"], iters=iters,
                             restart_seed=restart_seed(specs[i]["seed"], r), trace=False)
                assert p["best_obj"] == res.best_obj[k] and torch.equal(p["route_seq"], res.route_seq(k))
            except at.AtError as e:
                assert e.code == at.AT_EINFEAS and res.status[k] == at.AT_EINFEAS
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        out["tabu_best"].update(plain_sample_solves=n_p, plain_sample_s=t_plain,
                                plain_solves_per_s=n_p / t_plain,
                                speedup_vs_plain=out["tabu_best"]["solves_per_s"] / (n_p / t_plain))
    return out


def bench_stress(iters: int):
    """256 vehicles x 10000 missions (2000 facilities, 200 bases), tenure 25:
    Tabu search and neighbourhood search on the HBM-resident schedule."""
    import torch

    import paper_2002_11710_amd as at
    from gen.instances import stress_instance

    inst = stress_instance(0)
    dev = at.DeviceInstance.from_instance(inst)
    rel, swp = move_counts(inst.n_missions, inst.n_vehicles)
    out = {"iters": iters, "moves_per_iter": rel + swp}
    for name, variant in (("tabu", at.AT_TABU), ("ns", at.AT_NS)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = at.solve(dev, variant=variant, tenure=25, iters=iters, trace=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        assert g["status"] == 0
        out[name] = {"best_obj": int(g["best_obj"]), "iters_done": int(g["iters_done"]),
                     "search_ms": float(g["search_ms"]), "wall_s": wall,
                     "move_evals_per_s": (rel + swp) * g["iters_done"] / (g["search_ms"] / 1000.0)}
    return out


def bench_serve_sweep(rates, n_req: int, chunk: int = 50, slots: int = 256, budget: int = 64 << 30,
                      plain: int = 0):
    """Open-loop Poisson streams of n_req requests through the continuous-batching
    server, one per arrival rate (inf: every request arrives at time 0, which
    measures the saturation throughput); latency = result on the host minus the
    scheduled arrival.  Instances are uploaded before any clock starts.  Then the
    plain per-request form on the stream's first `plain` requests, one at_solve
    each in arrival order, each result checked equal to the served one."""
    import numpy as np
    import torch

    import paper_2002_11710_amd as at
    from gen.instances import make_instance, poisson_arrivals, serve_specs

    specs = serve_specs(n_req)
    devs = [at.DeviceInstance.from_instance(make_instance(s["seed"], s["n_fac"], s["n_bases"],
                                                          s["n_vehicles"], s["n_missions"]))
            for s in specs]
    torch.cuda.synchronize()
    work = [sum(move_counts(s["n_missions"], s["n_vehicles"])) * s["iters"] for s in specs]
    out = {"requests_per_rate": n_req, "chunk_iters": chunk, "max_slots": slots,
           "hbm_budget_GiB": budget >> 30, "move_evals_per_stream": float(sum(work)), "rates": []}
    served = None
    for lam in rates:
        arrivals = (np.zeros(n_req) if lam == float("inf")
                    else poisson_arrivals(n_req, lam, stream_seed=2 + int(lam)))
        srv = at.Server(budget, max_slots=slots, chunk_iters=chunk)
        done, res = {}, {}
        submitted = 0
        tickets = {}
        t0 = time.perf_counter()
        while len(done) < n_req:
            now = time.perf_counter() - t0
            while submitted < n_req and arrivals[submitted] <= now:
                s = specs[submitted]
                tickets[srv.submit(devs[submitted], tenure=s["tenure"], iters=s["iters"],
                                   trace=False)] = submitted
                submitted += 1
            srv.progress()
            for tk in srv.completed():
                r = srv.poll(tk)
                k = tickets.pop(tk)
                assert r is not None and r["status"] == 0
                done[k] = time.perf_counter() - t0
                if k < plain:
                    res[k] = (int(r["best_obj"]), r["route_seq"].cpu())
            if not tickets and submitted < n_req:
                time.sleep(max(0.0, min(0.001, arrivals[submitted] - (time.perf_counter() - t0))))
        wall = time.perf_counter() - t0
        srv.close()
        lat = np.array([done[k] - arrivals[k] for k in range(n_req)]) * 1000.0
        out["rates"].append({"lambda_req_per_s": lam if lam != float("inf") else "inf",
                             "wall_s": wall, "solves_per_s": n_req / wall,
                             "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                             "max_ms": float(lat.max())})
        served = served or res
    sat = [r for r in out["rates"] if r["lambda_req_per_s"] == "inf"]
    if sat:
        out["saturation_solves_per_s"] = sat[0]["solves_per_s"]
    if plain:
        n_p = min(plain, n_req)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(n_p):
            s = specs[k]
            r = at.solve(devs[k], variant=at.AT_TABU, tenure=s["tenure"], iters=s["iters"], trace=False)
            assert r["status"] == 0
            assert int(r["best_obj"]) == served[k][0] and torch.equal(r["route_seq"].cpu(), served[k][1]), k
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t1
        share = sum(work[:n_p]) / sum(work)
        out.update({"plain_requests": n_p, "plain_s": t_plain, "plain_solves_per_s": n_p / t_plain,
                    "plain_share_of_stream_work": share,
                    "note": f"the plain form was timed on the stream's first {n_p} requests "
                            f"({share:.1%} of its move evaluations), every result equal to the served one"})
        if sat:
            out["speedup_vs_plain"] = sat[0]["solves_per_s"] / (n_p / t_plain)
    return out


if __name__ == "__main__":
    main()
