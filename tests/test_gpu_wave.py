"""Parity of the wave schedule (one wavefront per solve) with the oracles, bit
for bit, through the C ABI: the unconstrained best-form search on small
instances and in batches, every slot's key of the constrained model, the
constrained best-form search (Tabu and NS), the sweep form of Algorithms 2-3,
and Algorithm 1 with its repair and its error report."""
import numpy as np
import pytest

import oracle
from gen.instances import (batch_instance, batch_specs, brute_twin, fleet_instance, fleet_specs,
                           make_instance, restart_seed, small_instance)
from helpers import assert_same_result, gpu_to_np, oracle_solve

pytestmark = pytest.mark.gpu

at = pytest.importorskip("paper_2002_11710_amd")


def fleet_problem(inst):
    return oracle.FleetProblem(oracle.travel(inst.lat, inst.lon, inst.speed_heli),
                               oracle.travel(inst.lat, inst.lon, inst.speed_plane), inst.pickup,
                               inst.delivery, inst.deadline, inst.heli_only, inst.vehicle_loc,
                               inst.vehicle_type, inst.flight_limit, inst.horizon)


def fleet_device(inst):
    return at.DeviceInstance(at.build_travel(inst.lat, inst.lon, inst.speed_heli), inst.pickup,
                             inst.delivery, inst.vehicle_loc,
                             travel_plane=at.build_travel(inst.lat, inst.lon, inst.speed_plane),
                             vehicle_type=inst.vehicle_type, deadline=inst.deadline,
                             heli_only=inst.heli_only, flight_limit=inst.flight_limit,
                             horizon=inst.horizon)


def _fleet_cases(n=64, min_m=0):
    out = []
    for sp in fleet_specs(n):
        if sp["n_missions"] >= min_m:
            out.append((sp, fleet_instance(sp["seed"], sp["n_missions"])))
    return out


def _feasible(F, seed=0):
    try:
        F.greedy(seed)
        return True
    except ValueError:
        return False


# ------------------------------------------------------------------ unconstrained, wave schedule

@pytest.mark.parametrize("maker", [lambda: small_instance(0), lambda: brute_twin(0),
                                   lambda: make_instance(5, 40, 3, 4, 30),
                                   lambda: make_instance(8, 100, 5, 12, 64),
                                   lambda: make_instance(13, 200, 6, 7, 130)])
def test_wave_unconstrained_trajectories(maker):
    inst = maker()
    dev = at.DeviceInstance.from_instance(inst)
    for variant, tenure, seed in ((at.AT_TABU, 7, 0), (at.AT_NS, 7, 0), (at.AT_TABU, 3, 17),
                                  (at.AT_TABU, 400, 0)):
        _, o = oracle_solve(inst, variant=variant, tenure=tenure, iters=250, restart_seed=seed)
        g = at.solve(dev, variant=variant, tenure=tenure, iters=250, restart_seed=seed,
                     schedule=at.SCHED_WAVE)
        assert_same_result(o, g, f"wave M={inst.n_missions} variant {variant} tenure {tenure} seed {seed}")


@pytest.mark.parametrize("maker", [lambda: small_instance(0), lambda: make_instance(8, 100, 5, 12, 64)])
def test_wave_generic_kernel_unconstrained(maker):
    """The wave kernel of the constrained model with every constraint switched
    off in substance (the plane matrix is the helicopter one, every vehicle a
    helicopter) runs the unconstrained search: equal to the oracle."""
    inst = maker()
    T = at.build_travel(inst.lat, inst.lon)
    dev = at.DeviceInstance(T, inst.pickup, inst.delivery, inst.vehicle_loc, travel_plane=T,
                            vehicle_type=np.zeros(inst.n_vehicles, np.int32))
    for variant, tenure, seed in ((at.AT_TABU, 7, 0), (at.AT_NS, 7, 0), (at.AT_TABU, 3, 17)):
        _, o = oracle_solve(inst, variant=variant, tenure=tenure, iters=200, restart_seed=seed)
        g = at.solve(dev, variant=variant, tenure=tenure, iters=200, restart_seed=seed)
        assert_same_result(o, g, f"generic wave M={inst.n_missions} variant {variant} seed {seed}")


def test_wave_unconstrained_keys():
    inst = make_instance(8, 100, 5, 12, 64)
    P = oracle.Problem.from_instance(inst)
    dev = at.DeviceInstance.from_instance(inst)
    rng = np.random.default_rng(3)
    off, seq = P.greedy(0)
    for _ in range(3):
        tabu = np.where(rng.random((P.M, P.V)) < 0.3, rng.integers(3, 9, (P.M, P.V)), -1).astype(np.int32)
        cur = P.objective(off, seq)
        for best in (cur, cur - 300):
            want = P.keys(off, seq, tabu, 5, cur, best)
            got, fast = at.debug_eval_moves(dev, off, seq, tabu, 5, cur, best, schedule=at.SCHED_WAVE)
            assert np.array_equal(got, want) and fast == int(want.min())
        perm = rng.permutation(P.M).astype(np.int32)
        cuts = np.sort(rng.integers(0, P.M + 1, size=P.V - 1))
        off, seq = np.concatenate([[0], cuts, [P.M]]).astype(np.int32), perm


def test_wave_unconstrained_batch():
    """A batch of small uneven instances x 4 restarts on the wave schedule in
    one call, each solve equal to the oracle's."""
    specs = [s for s in batch_specs(400) if s["n_missions"] <= 60][:24]
    insts = [batch_instance(dict(s, iters=150)) for s in specs]
    devs = [at.DeviceInstance.from_instance(i) for i in insts]
    params = [at._capi.make_params(at.AT_TABU, s["tenure"], 150, True, s["seed"], True, at.SCHED_WAVE)
              for s in specs]
    res = at.solve_batch(devs, params, 4)
    for i, (s, inst) in enumerate(zip(specs, insts)):
        for r in range(4):
            _, o = oracle_solve(inst, tenure=s["tenure"], iters=150, restart_seed=restart_seed(s["seed"], r))
            assert_same_result(o, res[i * 4 + r], f"batch instance {i} restart {r}")


# ------------------------------------------------------------------ constrained model

def _replay(F, r, seed=0):
    off, seq, _ = F.greedy(seed)
    P = oracle.Problem(F.T0, F.p, F.d, F.b)
    out = [(off, seq)]
    for mv in r["tr_move"]:
        if mv != oracle.NO_MOVE:
            off, seq = P.apply(off, seq, int(mv))
        out.append((off, seq))
    return out


def test_constrained_every_slot_key():
    """Every slot's key of the constrained model (delta, feasibility, tabu,
    aspiration) on states along an oracle trajectory, with random tabu tables."""
    cases = [(sp, inst) for sp, inst in _fleet_cases(64, 18) if _feasible(fleet_problem(inst))][:4]
    rng = np.random.default_rng(1)
    for sp, inst in cases:
        F = fleet_problem(inst)
        dev = fleet_device(inst)
        r = F.solve(variant=oracle.TABU, tenure=5, iters=30)
        for off, seq in _replay(F, r)[::6]:
            ok, cur = F.feasible(off, seq)
            assert ok
            tabu = np.where(rng.random((F.M, F.V)) < 0.3, rng.integers(0, 8, (F.M, F.V)), -1).astype(np.int32)
            for best in (cur, cur - 200):
                want = F.keys(off, seq, tabu, 3, cur, best)
                got, fast = at.debug_eval_moves(dev, off, seq, tabu, 3, cur, best)
                bad = np.nonzero(got != want)[0]
                assert bad.size == 0, (sp["index"], bad[:5], got[bad[:3]], want[bad[:3]])
                assert fast == int(want.min())


@pytest.mark.parametrize("variant", [at.AT_TABU, at.AT_NS])
def test_constrained_best_form_trajectories(variant):
    cases = _fleet_cases(40)
    n_ok = n_bad = 0
    for sp, inst in cases[:16]:
        F = fleet_problem(inst)
        dev = fleet_device(inst)
        for seed in (0, sp["seed"] % 1000 + 1):
            try:
                o = F.solve(variant=variant, tenure=sp["tenure"], iters=300, restart_seed=seed)
            except ValueError as e:
                with pytest.raises(at.AtError) as err:
                    at.solve(dev, variant=variant, tenure=sp["tenure"], iters=300, restart_seed=seed)
                assert err.value.code == at.AT_EINFEAS and e.args[0] == oracle.FO_EINFEAS
                n_bad += 1
                continue
            g = at.solve(dev, variant=variant, tenure=sp["tenure"], iters=300, restart_seed=seed)
            assert_same_result(o, g, f"fleet {sp['index']} seed {seed} variant {variant}")
            n_ok += 1
    assert n_ok >= 10 and n_bad >= 1


def test_constrained_batch_with_restarts_and_infeasible_starts():
    """40 paper-scale instances x 4 restarts in one call: every feasible solve
    equals the oracle's, every infeasible start reports AT_EINFEAS."""
    cases = _fleet_cases(40)
    devs = [fleet_device(inst) for _, inst in cases]
    params = [at._capi.make_params(at.AT_TABU, sp["tenure"], 200, True, sp["seed"], True)
              for sp, _ in cases]
    res = at.solve_batch(devs, params, 4, allow_infeasible=True)
    n_inf = 0
    for i, (sp, inst) in enumerate(cases):
        F = fleet_problem(inst)
        for r in range(4):
            seed = restart_seed(sp["seed"], r)
            g = res[i * 4 + r]
            try:
                o = F.solve(variant=oracle.TABU, tenure=sp["tenure"], iters=200, restart_seed=seed)
            except ValueError:
                assert g["status"] == at.AT_EINFEAS
                n_inf += 1
                continue
            assert_same_result(o, g, f"fleet batch {i} restart {r}")
    assert n_inf >= 1


# ------------------------------------------------------------------ the sweep form

def _same_sweep(o, g, label):
    g = gpu_to_np(g)
    assert g["status"] == 0, label
    k = o["iters_done"]
    assert g["iters_done"] == k, (label, g["iters_done"], k)
    assert np.array_equal(g["tr_move"].view(np.uint32)[:k], o["tr_move"]), label
    assert np.array_equal(g["tr_delta"][:k], o["tr_delta"]), label
    assert np.array_equal(g["tr_obj"][:k], o["tr_obj"]), label
    for key in ("best_obj", "final_obj", "best_iter"):
        assert g[key] == o[key], (label, key, g[key], o[key])
    assert np.array_equal(g["route_off"], o["best_off"]) and np.array_equal(g["route_seq"], o["best_seq"]), label
    assert np.array_equal(g["final_off"], o["final_off"]) and np.array_equal(g["final_seq"], o["final_seq"]), label


@pytest.mark.parametrize("variant,tenure", [(at.AT_NS, 0), (at.AT_TABU, 4), (at.AT_TABU, 1)])
def test_sweep_constrained(variant, tenure):
    n = 0
    for sp, inst in _fleet_cases(40)[:16]:
        F = fleet_problem(inst)
        if not _feasible(F):
            continue
        dev = fleet_device(inst)
        for seed in (0, 1 + sp["index"]):
            o = F.sweep(variant=variant, tenure=tenure, iters=5000, restart_seed=seed)
            g = at.solve(dev, variant=variant, tenure=tenure, iters=5000, restart_seed=seed,
                         form=at.FORM_SWEEP)
            _same_sweep(o, g, f"sweep fleet {sp['index']} seed {seed}")
            n += 1
    assert n >= 10


@pytest.mark.parametrize("maker", [lambda: small_instance(0), lambda: make_instance(5, 40, 3, 4, 30),
                                   lambda: make_instance(13, 200, 6, 7, 130)])
def test_sweep_unconstrained_and_budget(maker):
    inst = maker()
    P = oracle.Problem.from_instance(inst)
    F = oracle.FleetProblem.relaxed(P.T, P.p, P.d, P.b)
    dev = at.DeviceInstance.from_instance(inst)
    for variant, tenure, seed, iters in ((at.AT_NS, 0, 0, 100000), (at.AT_TABU, 5, 3, 100000),
                                         (at.AT_TABU, 5, 0, 17)):
        o = F.sweep(variant=variant, tenure=tenure, iters=iters, restart_seed=seed)
        g = at.solve(dev, variant=variant, tenure=tenure, iters=iters, restart_seed=seed,
                     form=at.FORM_SWEEP)
        _same_sweep(o, g, f"sweep M={inst.n_missions} variant {variant} seed {seed} budget {iters}")


# ------------------------------------------------------------------ Algorithm 1 repair

def test_greedy_repair_and_error_on_gpu():
    """Small instances where the plain append-only greedy gets stuck: the
    repaired start (one Algorithm 2 sweep, one more try) or the AT_EINFEAS
    report equals the oracle's."""
    saved = failed = 0
    for seed in range(400):
        inst = fleet_instance(seed, 10, n_fac=14, n_plane=1, n_heli=2, w_lo=3600, w_hi=12 * 3600)
        F = fleet_problem(inst)
        try:
            off, seq, rep = F.greedy(0)
        except ValueError:
            with pytest.raises(at.AtError) as err:
                at.solve(fleet_device(inst), tenure=3, iters=50)
            assert err.value.code == at.AT_EINFEAS
            failed += 1
            continue
        if rep == 0:
            continue
        o = F.solve(variant=oracle.TABU, tenure=3, iters=50)
        assert_same_result(o, at.solve(fleet_device(inst), tenure=3, iters=50), f"repair seed {seed}")
        saved += 1
        if saved >= 2 and failed >= 2:
            break
    assert saved >= 1 and failed >= 1


def test_wave_rejections():
    inst = fleet_instance(1, 12)
    dev = fleet_device(inst)
    with pytest.raises(at.AtError) as e:
        at.solve(dev, schedule=at.SCHED_WG)
    assert e.value.code == at.AT_EINVAL
    srv = at.Server(1 << 26, max_slots=2)
    try:
        with pytest.raises(at.AtError) as e:
            srv.submit(dev, tenure=3, iters=10)
        assert e.value.code == at.AT_EINVAL
    finally:
        srv.close()


def _nonmetric_dev(w_n):
    import test_oracle_fleet as tf
    F = tf._nonmetric(w_n)
    dev = at.DeviceInstance(F.T0, F.p, F.d, F.b, travel_plane=F.T1, vehicle_type=F.type,
                            deadline=F.w, heli_only=None, flight_limit=F.flight_limit,
                            horizon=F.horizon)
    return F, dev


def test_nonmetric_removal_and_ties():
    """Hand-built non-metric instance: a mission whose removal would make its
    route late stays (keys and sweep); three vehicles on one base give tied
    sweep candidates, resolved to the first vehicle as in the oracle."""
    off, seq = [0, 3, 5], [0, 1, 2, 3, 4]
    for w_n in (600, 6000):
        F, dev = _nonmetric_dev(w_n)
        cur = F.feasible(off, seq)[1]
        tabu = np.full((5, 2), -1, np.int32)
        want = F.keys(off, seq, tabu, 0, cur, cur)
        got, fast = at.debug_eval_moves(dev, off, seq, tabu, 0, cur, cur)
        assert np.array_equal(got, want) and fast == int(want.min())
        _same_sweep(F.sweep(variant=oracle.NS), at.solve(dev, variant=at.AT_NS, iters=1000,
                                                         form=at.FORM_SWEEP), f"non-metric {w_n}")
    for seed in range(4):
        inst = make_instance(40 + seed, 30, 1, 3, 14)
        P = oracle.Problem.from_instance(inst)
        F = oracle.FleetProblem.relaxed(P.T, P.p, P.d, P.b)
        dev = at.DeviceInstance.from_instance(inst)
        for rs in (0, 5):
            _same_sweep(F.sweep(variant=oracle.NS, restart_seed=rs),
                        at.solve(dev, variant=at.AT_NS, iters=100000, restart_seed=rs, form=at.FORM_SWEEP),
                        f"one-base sweep {seed} {rs}")
