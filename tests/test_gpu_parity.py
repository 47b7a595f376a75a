"""Parity of the HIP path (through the C ABI) with the oracle, bit for bit.

Everything here is integer work (travel seconds, deltas, keys, objectives,
whole trajectories), so the bar is exact equality.  Inputs are the seeded
synthetic workloads of gen.instances.
"""
import numpy as np
import pytest

import oracle
from gen.instances import (batch_instance, batch_specs, brute_twin, m400_instance, make_instance,
                           restart_seed, small_instance, stress_instance)
from helpers import assert_same_result, gpu_to_np, oracle_solve

pytestmark = pytest.mark.gpu

at = pytest.importorskip("paper_2002_11710_amd")


def _dev(inst):
    return at.DeviceInstance.from_instance(inst)


# ------------------------------------------------------------------ Eq (1)

@pytest.mark.parametrize("maker", [small_instance, brute_twin, m400_instance, stress_instance])
def test_device_travel_matrix_bit_exact(maker):
    """The device variant of Eq (1) (at_build_travel_device) on the workloads."""
    inst = maker(0)
    T = at.build_travel_device(inst.lat, inst.lon).cpu().numpy()
    assert np.array_equal(T, oracle.travel(inst.lat, inst.lon))


def test_device_travel_matrix_batch_sample():
    for spec in batch_specs(64)[::8]:
        inst = batch_instance(spec)
        T = at.build_travel_device(inst.lat, inst.lon).cpu().numpy()
        assert np.array_equal(T, oracle.travel(inst.lat, inst.lon)), spec["index"]


# ------------------------------------------------------------------ keys of every slot

def _random_state(P, rng, tenure_span=6):
    M, V = P.M, P.V
    perm = rng.permutation(M).astype(np.int32)
    cuts = np.sort(rng.integers(0, M + 1, size=V - 1))
    off = np.concatenate([[0], cuts, [M]]).astype(np.int32)
    tabu = np.where(rng.random((M, V)) < 0.3, rng.integers(5, 5 + tenure_span, (M, V)), -1)
    return off, perm, tabu.astype(np.int32)


@pytest.mark.parametrize("shape", [(20, 2, 1, 1), (20, 2, 1, 2), (20, 3, 3, 12), (30, 2, 5, 70),
                                   (60, 4, 7, 130), (120, 10, 16, 400)])
@pytest.mark.parametrize("chunk", [4, 8, 32])
def test_every_slot_key(shape, chunk):
    F, B, V, M = shape
    inst = make_instance(7 + M, F, B, V, M)
    P = oracle.Problem.from_instance(inst)
    dev = _dev(inst)
    rng = np.random.default_rng(M * 31 + V)
    states = [(*P.greedy(0), np.full((M, V), -1, np.int32))]
    for _ in range(3):
        states.append(_random_state(P, rng))
    for k, (off, seq, tabu) in enumerate(states):
        cur = P.objective(off, seq)
        for best in (cur, cur - 50):
            for t in (0, 6, 9):
                want = P.keys(off, seq, tabu, t, cur, best)
                got, fast = at.debug_eval_moves(dev, off, seq, tabu, t, cur, best, chunk=chunk)
                bad = np.nonzero(got != want)[0]
                assert bad.size == 0, (shape, k, t, best - cur, bad[:5], got[bad[:5]], want[bad[:5]])
                assert fast == int(want.min()), (shape, k, t, best - cur, hex(fast), hex(int(want.min())))


@pytest.mark.parametrize("chunk", [4, 8, 32])
def test_every_slot_key_wide_entries(chunk):
    """Travel times above 65535 s (5 km/h): the compact block holds 32-bit
    entries, and every slot's key and the minimum still equal the oracle's."""
    inst = make_instance(211, 60, 4, 7, 130)
    P = oracle.Problem.from_instance(inst, speed_kmh=5.0)
    assert int(P.T.max()) > 65535
    dev = at.DeviceInstance.from_instance(inst, speed_kmh=5.0)
    rng = np.random.default_rng(5)
    states = [(*P.greedy(0), np.full((P.M, P.V), -1, np.int32)), _random_state(P, rng)]
    for k, (off, seq, tabu) in enumerate(states):
        cur = P.objective(off, seq)
        for best in (cur, cur - 5000):
            want = P.keys(off, seq, tabu, 6, cur, best)
            got, fast = at.debug_eval_moves(dev, off, seq, tabu, 6, cur, best, chunk=chunk)
            bad = np.nonzero(got != want)[0]
            assert bad.size == 0, (k, best - cur, bad[:5])
            assert fast == int(want.min()), (k, best - cur)


@pytest.mark.parametrize("sched,groups", [(1, 0), (2, 0), (2, 7), (3, 4)])
def test_wide_entries_trajectory(sched, groups):
    """32-bit travel entries (5 km/h) under the one-workgroup, multi-workgroup
    (its relocate units then keep per-route segments) and HBM-resident
    schedules: Tabu and NS trajectories equal the oracle's."""
    inst = make_instance(212, 200, 5, 6, 150)
    P = oracle.Problem.from_instance(inst, speed_kmh=5.0)
    assert int(P.T.max()) > 65535
    dev = at.DeviceInstance.from_instance(inst, speed_kmh=5.0)
    for variant in (at.AT_TABU, at.AT_NS):
        o = P.solve(variant=variant, tenure=9, iters=300)
        g = at.solve(dev, variant=variant, tenure=9, iters=300, schedule=sched, n_groups=groups)
        assert_same_result(o, g, f"wide entries schedule {sched} groups {groups} variant {variant}")


_LONG = {}


def _long_shift_case():
    """1500 missions on 3 vehicles (40 facilities, so the state still fits one
    workgroup's LDS): the oracle's Tabu trajectory, and how many of its relocates
    rewrite more than 512 flat positions, moving the mission up and down."""
    if not _LONG:
        inst = make_instance(1503, 40, 3, 3, 1500)
        P = oracle.Problem.from_instance(inst)
        o = P.solve(variant=oracle.TABU, tenure=7, iters=120)
        off, seq = P.greedy(0)
        R = P.M * (P.M + P.V)
        up = down = 0
        for idx in o["tr_move"]:
            if idx < R:
                m = int(idx) // (P.M + P.V)
                s = int(np.nonzero(seq == m)[0][0])
                off, seq = P.apply(off, seq, int(idx))
                q = int(np.nonzero(seq == m)[0][0])
                if abs(q - s) + 1 > 512:
                    up += q > s
                    down += q < s
            else:
                off, seq = P.apply(off, seq, int(idx))
        assert np.array_equal(seq, o["final_seq"]) and np.array_equal(off, o["final_off"])
        _LONG.update(inst=inst, o=o, up=up, down=down)
    return _LONG


@pytest.mark.parametrize("sched,groups", [(1, 0), (2, 0), (2, 3)])
def test_long_relocate_shifts_trajectory(sched, groups):
    """Relocates that shift more than 512 positions (the LDS schedules apply a
    move 512 positions at a time, in the direction of the shift): the trajectory
    still equals the oracle's on the one-workgroup and multi-workgroup schedules."""
    case = _long_shift_case()
    assert case["up"] >= 2 and case["down"] >= 2, (case["up"], case["down"])
    g = at.solve(_dev(case["inst"]), tenure=7, iters=120, schedule=sched, n_groups=groups)
    assert_same_result(case["o"], g, f"1500 missions sched {sched} groups {groups}")


# ------------------------------------------------------------------ whole trajectories

def test_small_workload_tabu_trajectory():
    inst = small_instance(0)
    P, o = oracle_solve(inst)
    g = at.solve(_dev(inst), tenure=inst.tenure, iters=inst.iters)
    assert_same_result(o, g, "3x12 tabu")


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_small_workload_seeds_and_ns(seed):
    inst = small_instance(seed)
    _, o = oracle_solve(inst, restart_seed=seed * 977)
    g = at.solve(_dev(inst), tenure=7, iters=500, restart_seed=seed * 977)
    assert_same_result(o, g, f"3x12 seed {seed}")
    _, o = oracle_solve(inst, variant=oracle.NS, iters=500)
    g = at.solve(_dev(inst), variant=at.AT_NS, iters=500)
    assert_same_result(o, g, f"3x12 NS seed {seed}")


def test_brute_twin_reaches_optimum_on_gpu():
    inst = brute_twin(0)
    _, o = oracle_solve(inst)
    g = at.solve(_dev(inst), tenure=7, iters=500)
    assert_same_result(o, g, "2x6")
    assert g["best_obj"] == 105168   # brute-force optimum of this instance (tests/test_oracle_search.py)


@pytest.mark.parametrize("sched,groups", [(1, 0), (2, 8), (2, 0)])
def test_m400_tabu_trajectory(sched, groups):
    inst = m400_instance(0)
    _, o = _m400_oracle(0)
    g = at.solve(_dev(inst), tenure=15, iters=5000, schedule=sched, n_groups=groups)
    assert_same_result(o, g, f"16x400 tabu sched {sched}/{groups}")


def test_m400_ns_trajectory():
    inst = m400_instance(0)
    _, o = _m400_oracle(1)
    for sched in (1, 2):
        g = at.solve(_dev(inst), variant=at.AT_NS, tenure=15, iters=5000, schedule=sched)
        assert_same_result(o, g, f"16x400 NS sched {sched}")


_M400 = {}


def _m400_oracle(variant):
    if variant not in _M400:
        _M400[variant] = oracle_solve(m400_instance(0), variant=variant, tenure=15, iters=5000)
    return _M400[variant]


def test_batch_matches_oracle_and_solo():
    specs = batch_specs(24)[::3]          # 8 uneven instances
    insts = [batch_instance(s) for s in specs]
    for s, inst in zip(specs, insts):
        inst.iters = 300
    devs = [_dev(i) for i in insts]
    params = [at._capi.make_params(at.AT_TABU, s["tenure"], 300, True, s["seed"], True)
              for s in specs]
    res = at.solve_batch(devs, params, n_restarts=2)
    for i, (s, inst) in enumerate(zip(specs, insts)):
        for r in range(2):
            _, o = oracle_solve(inst, tenure=s["tenure"], iters=300,
                                restart_seed=restart_seed(s["seed"], r))
            assert_same_result(o, res[i * 2 + r], f"batch {i} restart {r}")


def test_edge_cases():
    # no missions
    inst = make_instance(3, 10, 2, 3, 0)
    _, o = oracle_solve(inst, iters=5)
    g = at.solve(_dev(inst), tenure=3, iters=5)
    assert g["best_obj"] == 0 and g["iters_done"] == 5
    assert np.all(g["tr_move"].cpu().numpy().view(np.uint32) == 0xFFFFFFFF)
    # one mission, one vehicle: no move exists
    inst = make_instance(4, 10, 1, 1, 1)
    _, o = oracle_solve(inst, iters=4)
    g = at.solve(_dev(inst), tenure=3, iters=4)
    assert_same_result(o, g, "1x1")
    # one vehicle, ragged tile (M = 65)
    inst = make_instance(5, 40, 1, 1, 65)
    _, o = oracle_solve(inst, tenure=5, iters=60)
    g = at.solve(_dev(inst), tenure=5, iters=60)
    assert_same_result(o, g, "1x65")
    # tenure 0 and aspiration off
    inst = make_instance(6, 30, 3, 5, 40)
    _, o = oracle_solve(inst, tenure=0, iters=100)
    g = at.solve(_dev(inst), tenure=0, iters=100)
    assert_same_result(o, g, "tenure 0")
    _, o = oracle_solve(inst, tenure=9, iters=100, aspiration=0)
    g = at.solve(_dev(inst), tenure=9, iters=100, aspiration=False)
    assert_same_result(o, g, "no aspiration")


@pytest.mark.parametrize("sched,groups", [(2, 0), (2, 5), (3, 3)])
def test_cooperative_schedules_tenure_and_aspiration(sched, groups):
    """The multi-workgroup and HBM-resident schedules with tenure 0, a short
    tenure without aspiration and a longer one, on 40 vehicles for 120 missions
    (many empty routes, so relocate units span many vehicles)."""
    inst = make_instance(213, 90, 8, 40, 120)
    dev = _dev(inst)
    for tenure, asp in ((0, 1), (3, 0), (12, 1)):
        _, o = oracle_solve(inst, tenure=tenure, iters=200, aspiration=asp)
        g = at.solve(dev, tenure=tenure, iters=200, aspiration=bool(asp), schedule=sched, n_groups=groups)
        assert_same_result(o, g, f"schedule {sched} groups {groups} tenure {tenure} aspiration {asp}")


@pytest.mark.parametrize("sched,groups", [(1, 0), (2, 0), (2, 3), (3, 4)])
def test_all_tabu_fallback_every_schedule(sched, groups):
    """A tenure longer than the budget (300 over 400 iterations on 4 vehicles x
    36 missions) makes every move tabu for many iterations: the best blocked
    move is taken (trace flag bit 2) on every schedule, as in the oracle."""
    inst = make_instance(91, 40, 3, 4, 36)
    _, o = oracle_solve(inst, tenure=300, iters=400)
    assert int(np.count_nonzero(o["tr_flags"] & 4)) > 50
    g = at.solve(_dev(inst), tenure=300, iters=400, schedule=sched, n_groups=groups)
    assert_same_result(o, g, f"fallback schedule {sched} groups {groups}")


def test_bad_device_inputs_are_rejected():
    inst = small_instance(0)
    dev = _dev(inst)
    bad = at.DeviceInstance(dev.travel, dev.pickup, dev.pickup, dev.vehicle_loc)   # pickup == delivery
    with pytest.raises(at.AtError) as e:
        at.solve(bad, iters=3)
    assert e.value.code == at.AT_EINVAL
    T = dev.travel.clone()
    T[1, 2] = -5
    with pytest.raises(at.AtError) as e:
        at.solve(at.DeviceInstance(T, dev.pickup, dev.delivery, dev.vehicle_loc), iters=3)
    assert e.value.code == at.AT_ERANGE
    import torch
    p = dev.pickup.clone()
    p[0] = 10 ** 6
    with pytest.raises(at.AtError) as e:
        at.solve(at.DeviceInstance(dev.travel, p, dev.delivery, dev.vehicle_loc), iters=3)
    assert e.value.code == at.AT_EINVAL
    assert torch.cuda.is_available()


def test_determinism_repeated():
    inst = make_instance(11, 60, 4, 6, 90)
    dev = _dev(inst)
    first = at.solve(dev, tenure=9, iters=400)
    tm = first["tr_move"].cpu().numpy()
    for block, chunk in ((256, 8), (512, 16), (1024, 64), (512, 4)):
        g = at.solve(dev, tenure=9, iters=400, block=block, chunk=chunk, schedule=1)
        assert np.array_equal(g["tr_move"].cpu().numpy(), tm), (block, chunk)
    for groups in (2, 5):
        g = at.solve(dev, tenure=9, iters=400, schedule=2, n_groups=groups)
        assert np.array_equal(g["tr_move"].cpu().numpy(), tm), groups


# ------------------------------------------------------------------ HBM-resident schedule

@pytest.mark.parametrize("groups", [1, 4, 16])
def test_m400_global_schedule(groups):
    inst = m400_instance(0)
    _, o = _m400_oracle(0)
    g = at.solve(_dev(inst), tenure=15, iters=5000, schedule=at.SCHED_GLOBAL, n_groups=groups)
    assert_same_result(o, g, f"16x400 tabu global/{groups}")


def test_m400_global_schedule_ns():
    inst = m400_instance(0)
    _, o = _m400_oracle(1)
    g = at.solve(_dev(inst), variant=at.AT_NS, tenure=15, iters=5000, schedule=at.SCHED_GLOBAL,
                 n_groups=8)
    assert_same_result(o, g, "16x400 NS global")


def test_global_schedule_edge_cases():
    for (F, B, V, M, it) in ((10, 2, 3, 0, 4), (10, 1, 1, 1, 4), (40, 1, 1, 65, 40), (30, 3, 5, 40, 80)):
        inst = make_instance(21 + M, F, B, V, M)
        _, o = oracle_solve(inst, tenure=5, iters=it)
        g = at.solve(_dev(inst), tenure=5, iters=it, schedule=at.SCHED_GLOBAL, n_groups=3)
        assert_same_result(o, g, f"global {V}x{M}")


@pytest.mark.parametrize("groups", [1, 16, 64])
def test_global_schedule_short_routes(groups):
    """24 vehicles x 40 missions: a block of consecutive positions spans more
    routes than the eval stages tabu rows for (the rest read from HBM), and the
    group count sets the block size (8, 2 and 1 missions)."""
    inst = make_instance(77, 60, 6, 24, 40)
    for variant in (at.AT_TABU, at.AT_NS):
        _, o = oracle_solve(inst, variant=variant, tenure=5, iters=120)
        g = at.solve(_dev(inst), variant=variant, tenure=5, iters=120, schedule=at.SCHED_GLOBAL,
                     n_groups=groups)
        assert_same_result(o, g, f"global 24x40 variant {variant} groups {groups}")


@pytest.mark.parametrize("tenure,iters", [(0, 60), (1, 60), (40, 30), (80, 200), (300, 400)])
def test_global_schedule_tenure_edges(tenure, iters):
    """The HBM-resident schedule keeps its tabu state as a ring of the entries of
    the last min(tenure + 1, iterations) iterations: no tenure, tenure 1, a
    tenure beyond the budget (the ring never wraps), more active entries than
    the per-iteration list holds (tenure 80) and a ring longer than a
    workgroup's threads give the oracle's trajectories, tabu flags included."""
    inst = make_instance(91, 40, 3, 4, 36)
    for variant in (at.AT_TABU, at.AT_NS):
        _, o = oracle_solve(inst, variant=variant, tenure=tenure, iters=iters)
        g = at.solve(_dev(inst), variant=variant, tenure=tenure, iters=iters,
                     schedule=at.SCHED_GLOBAL, n_groups=4)
        assert_same_result(o, g, f"global tenure {tenure} iters {iters} variant {variant}")


@pytest.mark.parametrize("vehicles,seed,groups", [(16, 0, 4), (16, 5, 4), (16, 9, 1), (16, 3, 16),
                                                   (100, 0, 8), (100, 7, 8), (300, 0, 8), (300, 11, 2)])
def test_global_schedule_greedy_orders(vehicles, seed, groups):
    """The HBM-resident schedule's greedy start (per-vehicle state in registers up
    to 64, 128 and 256 vehicles, in LDS beyond) with the identity and seeded
    orders, at group counts that change its LDS budget: the oracle's whole
    trajectory from that start."""
    inst = m400_instance(0) if vehicles == 16 else make_instance(40 + vehicles, 150, 12, vehicles, 400)
    _, o = oracle_solve(inst, tenure=15, iters=60, restart_seed=seed)
    g = at.solve(_dev(inst), tenure=15, iters=60, restart_seed=seed, schedule=at.SCHED_GLOBAL,
                 n_groups=groups)
    assert_same_result(o, g, f"global greedy seed {seed} groups {groups}")


def test_stress_instance_prefix():
    """The 256-vehicle x 10000-mission instance: greedy start and the first
    iterations against the oracle (each oracle iteration scores 1.5e8 moves)."""
    inst = stress_instance(0)
    iters = 3
    _, o = oracle_solve(inst, tenure=25, iters=iters)
    g = at.solve(_dev(inst), tenure=25, iters=iters)
    assert_same_result(o, g, "256x10000 prefix")


def test_batch_mixed_schedules():
    """One batch call with instances too large for LDS (HBM-resident schedule,
    sharing a cooperative launch) and small ones (one workgroup each): every
    solve equals its oracle run."""
    insts = [make_instance(500 + k, 750, 13, 25, 500) for k in range(2)]
    insts += [make_instance(510 + k, 40, 3, 4, 25 + 5 * k) for k in range(4)]
    devs = [_dev(i) for i in insts]
    params = [at._capi.make_params(at.AT_TABU, 7, 50, True, 0, True) for _ in insts]
    res = at.solve_batch(devs, params, 2)
    from gen.instances import restart_seed
    for k, inst in enumerate(insts):
        for r in range(2):
            _, o = oracle_solve(inst, tenure=7, iters=50, restart_seed=restart_seed(0, r))
            assert_same_result(o, res[k * 2 + r], f"batch instance {k} restart {r}")


def test_global_shared_launch_partition():
    """More global-schedule solves than the launch can give their requested
    workgroups: the launch's groups are shared out (one each, then to the job that
    would finish last); each result equals the solve alone."""
    insts = [make_instance(600 + k, 60, 4, 6, 45 + 3 * k) for k in range(12)]
    devs = [_dev(i) for i in insts]
    params = [at._capi.make_params(at.AT_TABU, 5, 40, True, 0, True, at.SCHED_GLOBAL, 64) for _ in insts]
    res = at.solve_batch(devs, params, 1)
    for k, d in enumerate(devs):
        alone = at.solve(d, tenure=5, iters=40, schedule=at.SCHED_GLOBAL, n_groups=3)
        assert np.array_equal(gpu_to_np(res[k])["tr_move"], gpu_to_np(alone)["tr_move"]), k
        assert res[k]["best_obj"] == alone["best_obj"], k


def test_flat_batch_marshalling_equals_list():
    """solve_batch_flat (descriptors built as one numpy array, routes in flat
    tensors) gives the same results as solve_batch on the same batch."""
    specs = batch_specs(24)
    devs = [_dev(batch_instance(dict(s, iters=120))) for s in specs]
    params = [at._capi.make_params(at.AT_TABU, s["tenure"], 120, True, s["seed"], False) for s in specs]
    lst = at.solve_batch(devs, params, 3)
    flat = at.solve_batch_flat(devs, params, 3, final_routes=True)
    assert flat.n == len(lst)
    for k, r in enumerate(lst):
        r = gpu_to_np(r)
        for f in ("best_obj", "final_obj", "iters_done", "best_iter", "status"):
            assert getattr(flat, f)[k] == r[f], (k, f)
        assert np.array_equal(flat.route_off(k).cpu().numpy(), r["route_off"])
        assert np.array_equal(flat.route_seq(k).cpu().numpy(), r["route_seq"])
        assert np.array_equal(flat.route_of(k).cpu().numpy(), r["route_of"])
        assert np.array_equal(flat.final_off(k).cpu().numpy(), r["final_off"])
        assert np.array_equal(flat.final_seq(k).cpu().numpy(), r["final_seq"])


def test_small_batch_of_large_solves_shares_one_multi_launch():
    """A batch of a few large LDS-resident solves runs them side by side on the
    multi-workgroup schedule, each on its own workgroup range and slot set: the
    Tabu and NS solves of the 16 x 400 workload, and three restarts of one
    instance, each equal to its oracle run."""
    from gen.instances import restart_seed
    inst = m400_instance(0)
    dev = _dev(inst)
    params = [at._capi.make_params(at.AT_TABU, 15, 300, True, 0, True),
              at._capi.make_params(at.AT_NS, 15, 300, True, 0, True)]
    res = at.solve_batch([dev, dev], params, 1)
    for k, variant in enumerate((at.AT_TABU, at.AT_NS)):
        _, o = oracle_solve(inst, variant=variant, tenure=15, iters=300)
        assert_same_result(o, res[k], f"Tabu + NS batch, solve {k}")
    inst2 = make_instance(77, 450, 9, 18, 300)
    res = at.solve_batch([_dev(inst2)], [at._capi.make_params(at.AT_TABU, 9, 120, True, 41, True)], 3)
    for r in range(3):
        _, o = oracle_solve(inst2, tenure=9, iters=120, restart_seed=restart_seed(41, r))
        assert_same_result(o, res[r], f"restart batch, restart {r}")


def test_batch_of_many_large_solves_keeps_one_workgroup_each():
    """More large solves than one multi-workgroup launch takes: each keeps one
    workgroup, and equals the solve alone."""
    insts = [make_instance(900 + k, 300, 8, 12, 180) for k in range(9)]
    devs = [_dev(i) for i in insts]
    params = [at._capi.make_params(at.AT_TABU, 7, 25, True, 0, True) for _ in insts]
    res = at.solve_batch(devs, params, 1)
    for k, d in enumerate(devs):
        alone = at.solve(d, tenure=7, iters=25)
        assert np.array_equal(gpu_to_np(res[k])["tr_move"], gpu_to_np(alone)["tr_move"]), k
        assert res[k]["best_obj"] == alone["best_obj"], k


@pytest.mark.parametrize("sched,groups", [(1, 0), (2, 0), (2, 7)])
def test_half_width_units_ragged(sched, groups):
    """Units of 4 partners and 8 gaps (chunk 4) on a ragged size: 333 missions on
    11 vehicles (a last tile of 13 lanes, chunks that end inside a tile), Tabu and
    NS, on the one-workgroup and multi-workgroup schedules, equal to the oracle."""
    inst = make_instance(555, 250, 6, 11, 333)
    dev = _dev(inst)
    for variant in (0, 1):
        _, o = oracle_solve(inst, variant=variant, tenure=9, iters=300)
        g = at.solve(dev, variant=variant, tenure=9, iters=300, schedule=sched, n_groups=groups, chunk=4)
        assert_same_result(o, g, f"chunk 4 schedule {sched} groups {groups} variant {variant}")


def test_batch_of_eight_large_solves_shares_one_multi_launch():
    """Eight restarts of the 16 x 400 instance in one call: more half-width groups
    than the GPU holds at once, so the shared multi-workgroup launch takes
    8-partner units; every restart equals its oracle run."""
    from gen.instances import restart_seed
    inst = m400_instance(0)
    res = at.solve_batch([_dev(inst)], [at._capi.make_params(at.AT_TABU, 15, 60, True, 5, True)], 8)
    for r in range(8):
        _, o = oracle_solve(inst, tenure=15, iters=60, restart_seed=restart_seed(5, r))
        assert_same_result(o, res[r], f"eight-restart batch, restart {r}")


@pytest.mark.parametrize("sched,groups", [(1, 0), (2, 0), (2, 5)])
def test_relocates_across_many_routes(sched, groups):
    """130 vehicles for 200 missions: relocates between routes more than 64
    vehicles apart move more than one wavefront's worth of route offsets (and
    many routes stay empty), on both LDS-resident schedules, Tabu and NS, equal
    to the oracle."""
    inst = make_instance(731, 160, 10, 130, 200)
    dev = _dev(inst)
    for variant in (0, 1):
        _, o = oracle_solve(inst, variant=variant, tenure=11, iters=250)
        g = at.solve(dev, variant=variant, tenure=11, iters=250, schedule=sched, n_groups=groups)
        assert_same_result(o, g, f"130 vehicles schedule {sched} groups {groups} variant {variant}")
