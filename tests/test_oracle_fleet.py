"""Pins of the oracle of the constrained model and of the paper's own forms of
Algorithms 1-3 (oracle/fleet_oracle.c), each against something other than the
oracle itself:

* with every constraint off it reproduces the unconstrained oracle (itself
  pinned in test_oracle_*.py) bit for bit: greedy start, Tabu and NS
  trajectories;
* route feasibility and Eq (2) on hand-built routes at the boundary of each
  constraint (time limit with waiting, horizon, flight limit, helicopter-only
  missions, a plane's own matrix);
* the incremental evaluation of every slot equals the by-definition one (apply
  to a copy, re-check every route, recompute the objective) on states along
  trajectories, with random tabu tables;
* every state of a trajectory, rebuilt by applying its trace with the
  unconstrained oracle's plain list edits, is feasible and has the trace's
  objective; the neighbourhood search ends where no feasible move improves;
* the best solution is never below the feasible optimum found by enumerating
  every solution of tiny instances;
* Algorithm 1's order and placement on hand-built instances, and its repair
  (NEXT-3) against an independent Python greedy that gets stuck where the
  repair is needed;
* the sweep form (Algorithms 2-3 as printed) against an independent Python
  driver: pass and turn order (including the seeded permutation vectors),
  each turn's choice from by-definition keys (smallest strictly negative
  change, first in vehicle then position order), TabuList counters.
"""
import itertools

import numpy as np
import pytest

import oracle
from gen.instances import SplitMix64, fleet_instance, fleet_specs, make_instance, small_instance

NONE = np.uint64(0xFFFFFFFFFFFFFFFF)


def fleet_problem(inst):
    return oracle.FleetProblem(oracle.travel(inst.lat, inst.lon, inst.speed_heli),
                               oracle.travel(inst.lat, inst.lon, inst.speed_plane), inst.pickup,
                               inst.delivery, inst.deadline, inst.heli_only, inst.vehicle_loc,
                               inst.vehicle_type, inst.flight_limit, inst.horizon)


def feasible_specs(n=64, min_m=0):
    out = []
    for sp in fleet_specs(n):
        if sp["n_missions"] < min_m:
            continue
        F = fleet_problem(fleet_instance(sp["seed"], sp["n_missions"]))
        try:
            F.greedy(0)
        except ValueError:
            continue
        out.append(sp)
    return out


# ------------------------------------------------------------------ constraints off

@pytest.mark.parametrize("maker", [lambda: small_instance(0), lambda: make_instance(5, 40, 3, 4, 30),
                                   lambda: make_instance(9, 60, 2, 6, 45)])
@pytest.mark.parametrize("seed", [0, 11])
def test_relaxed_model_is_the_unconstrained_oracle(maker, seed):
    inst = maker()
    P = oracle.Problem.from_instance(inst)
    F = oracle.FleetProblem.relaxed(P.T, P.p, P.d, P.b)
    off, seq = P.greedy(seed)
    foff, fseq, rep = F.greedy(seed)
    assert rep == 0 and np.array_equal(off, foff) and np.array_equal(seq, fseq)
    for variant, tenure in ((oracle.TABU, 7), (oracle.TABU, 0), (oracle.NS, 7)):
        o = P.solve(variant=variant, tenure=tenure, iters=150, restart_seed=seed)
        f = F.solve(variant=variant, tenure=tenure, iters=150, restart_seed=seed)
        for k in ("best_obj", "final_obj", "iters_done", "best_iter"):
            assert o[k] == f[k], k
        for k in ("tr_move", "tr_delta", "tr_obj", "tr_flags", "best_off", "best_seq", "final_off",
                  "final_seq"):
            assert np.array_equal(o[k], f[k]), k


# ------------------------------------------------------------------ hand-built routes

def _toy(w0, w1, horizon, flight_limit, heli1=0, vtype=0):
    """Locations 0-3 facilities, 4 the base; mission 0 flies 0 -> 1, mission 1
    flies 2 -> 3.  Helicopter times below, plane times half of them."""
    T = np.array([[0, 100, 300, 400, 200],
                  [100, 0, 150, 350, 250],
                  [300, 150, 0, 120, 330],
                  [400, 350, 120, 0, 180],
                  [200, 250, 330, 180, 0]], dtype=np.int32)
    return oracle.FleetProblem(T, T // 2, [0, 2], [1, 3], [w0, w1], [0, heli1], [4], [vtype],
                               flight_limit, horizon)


def test_route_feasibility_boundaries():
    # route base -> m0 -> m1 -> base on a helicopter:
    # reach m0's delivery at 200 + 100 = 300; leave at w0; reach m1's delivery at
    # w0 + 150 + 120; back home at w1 + 180.  Flight 200+100+150+120+180 = 750.
    off, seq = [0, 2], [0, 1]
    w0, w1 = 300, 300 + 270
    ok, obj = _toy(w0, w1, w1 + 180, 750).feasible(off, seq)
    assert ok and obj == 750
    assert not _toy(w0 - 1, w1, w1 + 180, 750).feasible(off, seq)[0]        # too late for m0
    assert not _toy(w0, w1 - 1, w1 + 180, 750).feasible(off, seq)[0]        # too late for m1
    assert not _toy(w0, w1, w1 + 179, 750).feasible(off, seq)[0]            # home after the horizon
    assert not _toy(w0, w1, w1 + 180, 749).feasible(off, seq)[0]            # over the flight limit
    # waiting: leaving m0 at its limit (1000), not on arrival (300), decides m1
    assert _toy(1000, 1270, 1450, 750).feasible(off, seq)[0]
    assert not _toy(1000, 1269, 1450, 750).feasible(off, seq)[0]
    # a plane flies the half-time matrix: flight 375, m0 reached at 150
    ok, obj = _toy(150, 150 + 135, 150 + 135 + 90, 375, vtype=1).feasible(off, seq)
    assert ok and obj == 375
    assert not _toy(149, 300, 1000, 1000, vtype=1).feasible(off, seq)[0]
    # a helicopter-only mission may not go on the plane, may on a helicopter
    assert not _toy(2000, 4000, 9000, 9000, heli1=1, vtype=1).feasible(off, seq)[0]
    assert _toy(2000, 4000, 9000, 9000, heli1=1, vtype=0).feasible(off, seq)[0]
    # an empty route is feasible and flies nothing
    ok, obj = _toy(0, 0, 1, 1).feasible([0, 0], [])
    assert ok and obj == 0


def test_time_limits_order_the_route():
    """With waiting until each limit, m1 before m0 is infeasible when m1's limit
    is earlier than m0's arrival from it."""
    F = _toy(5000, 600, 90000, 90000)
    assert F.feasible([0, 2], [1, 0])[0]          # m1 first (limit 600), then m0
    assert not F.feasible([0, 2], [0, 1])[0]      # m0 leaves at 5000: m1 missed


# ------------------------------------------------------------------ keys and trajectories

def _replay_states(F, r, seed=0):
    """States along a best-form trajectory: the greedy start, then each traced
    move applied by the unconstrained oracle's list edits."""
    off, seq, _ = F.greedy(seed)
    P = oracle.Problem(F.T0, F.p, F.d, F.b)
    states = [(off, seq)]
    for mv in r["tr_move"]:
        if mv != oracle.NO_MOVE:
            off, seq = P.apply(off, seq, int(mv))
        states.append((off, seq))
    return states


@pytest.mark.parametrize("k", [0, 1, 2])
def test_incremental_keys_equal_definition(k):
    sp = feasible_specs(64, min_m=18)[k]
    F = fleet_problem(fleet_instance(sp["seed"], sp["n_missions"]))
    r = F.solve(variant=oracle.TABU, tenure=5, iters=40)
    rng = np.random.default_rng(k)
    for t, (off, seq) in enumerate(_replay_states(F, r)[::4]):
        ok, cur = F.feasible(off, seq)
        assert ok
        tabu = np.where(rng.random((F.M, F.V)) < 0.3, rng.integers(0, 8, (F.M, F.V)), -1).astype(np.int32)
        for best in (cur, cur - 100):
            k0 = F.keys(off, seq, tabu, 3, cur, best, mode=0)
            k1 = F.keys(off, seq, tabu, 3, cur, best, mode=1)
            bad = np.nonzero(k0 != k1)[0]
            assert bad.size == 0, (t, bad[:5])
            assert 0 < np.count_nonzero(k0 != NONE) < len(k0)


@pytest.mark.parametrize("variant", [oracle.TABU, oracle.NS])
def test_every_state_feasible_and_objective_traced(variant):
    for sp in feasible_specs(64, min_m=24)[:3]:
        F = fleet_problem(fleet_instance(sp["seed"], sp["n_missions"]))
        r = F.solve(variant=variant, tenure=5, iters=120, restart_seed=sp["seed"] % 7)
        states = _replay_states(F, r, seed=sp["seed"] % 7)
        objs = [F.feasible(o, s) for o, s in states]
        assert all(ok for ok, _ in objs)
        assert [c for _, c in objs[1:]] == list(r["tr_obj"])
        assert r["best_obj"] == min(c for _, c in objs)
        assert F.feasible(r["best_off"], r["best_seq"]) == (True, r["best_obj"])
        assert F.feasible(r["final_off"], r["final_seq"]) == (True, r["final_obj"])
        if variant == oracle.NS:
            off, seq = states[-1]
            cur = objs[-1][1]
            keys = F.keys(off, seq, np.full((F.M, F.V), -1, np.int32), 0, cur, cur, variant=1, mode=0)
            valid = keys[keys != NONE]
            deltas = ((valid >> np.uint64(32)) & np.uint64(0x7FFFFFFF)).astype(np.int64) - (1 << 30)
            assert deltas.min() >= 0


def _enumerate_optimum(F):
    """Smallest objective over every feasible solution (V = 2)."""
    assert F.V == 2
    best = None
    for perm in itertools.permutations(range(F.M)):
        for cut in range(F.M + 1):
            ok, obj = F.feasible([0, cut, F.M], list(perm))
            if ok and (best is None or obj < best):
                best = obj
    return best


def test_search_never_beats_the_enumerated_optimum():
    """Tiny instances (one plane, one helicopter, 6 missions) whose greedy start
    exists: Tabu and NS never beat the feasible optimum found by enumerating
    every solution, and Tabu reaches it on some of them."""
    checked = reached = 0
    for seed in range(1, 60):
        inst = fleet_instance(seed, 6, n_fac=12, n_plane=1, n_heli=1, w_lo=3600, w_hi=20 * 3600)
        F = fleet_problem(inst)
        try:
            F.greedy(0)
        except ValueError:
            continue
        opt = _enumerate_optimum(F)
        for variant in (oracle.TABU, oracle.NS):
            r = F.solve(variant=variant, tenure=3, iters=200)
            assert r["best_obj"] >= opt, seed
            reached += variant == oracle.TABU and r["best_obj"] == opt
        checked += 1
        if checked == 5:
            break
    assert checked == 5 and reached >= 1


# ------------------------------------------------------------------ Algorithm 1

def test_greedy_order_helicopter_only_first_then_by_limit():
    """One helicopter: the route is the greedy order itself: helicopter-only
    missions first, each group by time limit; a plane never takes a
    helicopter-only mission."""
    T = np.full((7, 7), 10, dtype=np.int32)
    np.fill_diagonal(T, 0)
    p, d = [0, 1, 2, 3, 4], [1, 2, 3, 4, 5]
    w = [5000, 1000, 3000, 2000, 4000]
    heli = [0, 1, 0, 1, 0]
    F = oracle.FleetProblem(T, T, p, d, w, heli, [6], [0], 10 ** 6, 10 ** 6)
    off, seq, rep = F.greedy(0)
    # helicopter-only 1 (1000), 3 (2000); then 2 (3000), 4 (4000), 0 (5000)
    assert list(seq) == [1, 3, 2, 4, 0] and rep == 0
    F2 = oracle.FleetProblem(T, T, p, d, w, heli, [6, 6], [1, 0], 10 ** 6, 10 ** 6)
    off2, seq2, _ = F2.greedy(0)
    on_plane = list(seq2[off2[0]:off2[1]])
    assert 1 not in on_plane and 3 not in on_plane


def _python_greedy_without_repair(F):
    """Algorithm 1 without its repair step, written independently: returns the
    first mission that fits no vehicle, or None."""
    T = [F.T0, F.T1]
    order = sorted(range(F.M), key=lambda m: (-int(F.heli[m]), int(F.w[m]), m))
    routes = [[] for _ in range(F.V)]
    for m in order:
        best = None
        for v in range(F.V):
            tv = T[int(F.type[v])]
            if F.heli[m] and F.type[v] == 1:
                continue
            last = routes[v][-1] if routes[v] else None
            x = F.b[v] if last is None else F.d[last]
            leave = 0 if last is None else F.w[last]
            svc = tv[F.p[m], F.d[m]]
            if leave + tv[x, F.p[m]] + svc > F.w[m] or F.w[m] + tv[F.d[m], F.b[v]] > F.horizon:
                continue
            cost = 0
            prev = F.b[v]
            for q in routes[v] + [m]:
                cost += tv[prev, F.p[q]] + tv[F.p[q], F.d[q]]
                prev = F.d[q]
            cost += tv[prev, F.b[v]]
            if cost > F.flight_limit:
                continue
            add = tv[x, F.p[m]] + svc + tv[F.d[m], F.b[v]] - tv[x, F.b[v]]
            if best is None or add < best[0]:
                best = (add, v)
        if best is None:
            return m
        routes[best[1]].append(m)
    return None


def _repair_cases():
    """Seeded small instances where the plain greedy gets stuck (found by a
    seeded scan): those the repair rescues and those it does not."""
    saved, failed = [], []
    for seed in range(400):
        inst = fleet_instance(seed, 10, n_fac=14, n_plane=1, n_heli=2, w_lo=3600, w_hi=12 * 3600)
        F = fleet_problem(inst)
        stuck = _python_greedy_without_repair(F)
        if stuck is None:
            continue
        try:
            off, seq, rep = F.greedy(0)
            saved.append((seed, F, stuck, off, seq, rep))
        except ValueError as e:
            failed.append((seed, F, stuck, e.args))
        if len(saved) >= 2 and len(failed) >= 2:
            break
    return saved, failed


def test_greedy_repair_and_error_report():
    saved, failed = _repair_cases()
    assert saved, "no instance the repair rescues"
    assert failed, "no instance where even the repaired greedy fails"
    for seed, F, stuck, off, seq, rep in saved:
        assert rep >= 1, seed
        assert sorted(seq) == list(range(F.M)) and F.feasible(off, seq)[0], seed
    for seed, F, stuck, args in failed:
        assert args[0] == oracle.FO_EINFEAS, seed
    # without any constraint nothing ever needs repair
    for seed, F, *_ in saved + failed:
        R = oracle.FleetProblem.relaxed(F.T0, F.p, F.d, F.b)
        assert R.greedy(0)[2] == 0


# ------------------------------------------------------------------ the sweep form

def _sweep_by_hand(F, variant, tenure, seed, max_turns=10 ** 6):
    """Algorithms 2-3 as printed, driven from Python: the oracle only scores
    moves by definition (fo_keys mode 0); the passes, the turn order, the
    choice rule and the TabuList are all here."""
    off, seq, _ = F.greedy(seed)
    off, seq = list(off), list(seq)
    P = oracle.Problem(F.T0, F.p, F.d, F.b)
    M, V = F.M, F.V
    NG = M + V
    rng = SplitMix64(seed) if seed else None
    ttl = {}
    moves, turns = [], 0

    def shuffle(a):
        for i in range(len(a) - 1, 0, -1):
            j = rng.next() % (i + 1)
            a[i], a[j] = a[j], a[i]

    while True:
        moved = 0
        vord = list(range(V))
        if rng:
            shuffle(vord)
        for i in vord:
            lst = seq[off[i]:off[i + 1]]
            if rng:
                shuffle(lst)
            for j in lst:
                if turns >= max_turns:
                    return moves, turns
                cur = F.feasible(off, seq)[1]
                keys = F.keys(off, seq, np.full((M, V), -1, np.int32), 0, cur, cur, variant=1, mode=0)
                own = next(v for v in range(V) if j in seq[off[v]:off[v + 1]])
                best = None
                for v in range(V):
                    if v == own or (variant == oracle.TABU and ttl.get((j, v), 0) > 0):
                        continue
                    for g in range(off[v + 1] - off[v] + 1):
                        G = off[v] + v + g
                        k = keys[j * NG + G]
                        if k == NONE:
                            continue
                        dl = int((int(k) >> 32) & 0x7FFFFFFF) - (1 << 30)
                        if dl < 0 and (best is None or dl < best[0]):
                            best = (dl, G)
                if best is not None:
                    off, seq = [list(x) for x in P.apply(off, seq, j * NG + best[1])]
                    moves.append((turns, j * NG + best[1], best[0]))
                    moved += 1
                    if variant == oracle.TABU:
                        ttl[(j, own)] = tenure
                if variant == oracle.TABU:
                    ttl = {e: c - 1 for e, c in ttl.items() if c > 1}
                turns += 1
        if moved == 0:
            return moves, turns


@pytest.mark.parametrize("variant,tenure,seed", [(oracle.NS, 0, 0), (oracle.TABU, 4, 0),
                                                 (oracle.TABU, 3, 77), (oracle.NS, 0, 5),
                                                 (oracle.TABU, 1, 9)])
def test_sweep_against_python_driver(variant, tenure, seed):
    for sp in feasible_specs(64, min_m=15)[:2]:
        F = fleet_problem(fleet_instance(sp["seed"], sp["n_missions"]))
        r = F.sweep(variant=variant, tenure=tenure, restart_seed=seed)
        moves, turns = _sweep_by_hand(F, variant, tenure, seed)
        assert r["iters_done"] == turns
        got = [(t, int(r["tr_move"][t]), int(r["tr_delta"][t])) for t in range(turns)
               if r["tr_move"][t] != oracle.NO_MOVE]
        assert got == moves
        assert r["best_iter"] == (moves[-1][0] if moves else -1)
        assert F.feasible(r["best_off"], r["best_seq"]) == (True, r["best_obj"])


def test_sweep_relaxed_and_tenure_one():
    """Without constraints the sweep runs on the unconstrained model; a TabuList
    counter of 1 expires in the turn that sets it, so Tabu equals NS."""
    inst = make_instance(5, 40, 3, 4, 30)
    P = oracle.Problem.from_instance(inst)
    F = oracle.FleetProblem.relaxed(P.T, P.p, P.d, P.b)
    for seed in (0, 3):
        a = F.sweep(variant=oracle.TABU, tenure=1, restart_seed=seed)
        b = F.sweep(variant=oracle.NS, restart_seed=seed)
        assert np.array_equal(a["tr_move"], b["tr_move"]) and a["best_obj"] == b["best_obj"]
        moves, turns = _sweep_by_hand(F, oracle.NS, 0, seed)
        assert turns == b["iters_done"]
        assert P.objective(b["best_off"], b["best_seq"]) == b["best_obj"]


def test_sweep_ties_go_to_the_first_vehicle():
    """Three vehicles on one base: a mission's moves into two empty routes cost
    the same, and the sweep keeps the first (lower vehicle) of equal
    candidates, as the Python driver does."""
    n_tied = 0
    for seed in range(6):
        inst = make_instance(40 + seed, 30, 1, 3, 14)
        P = oracle.Problem.from_instance(inst)
        F = oracle.FleetProblem.relaxed(P.T, P.p, P.d, P.b)
        for rs in (0, 5):
            r = F.sweep(variant=oracle.NS, restart_seed=rs)
            moves, turns = _sweep_by_hand(F, oracle.NS, 0, rs)
            got = [(t, int(r["tr_move"][t]), int(r["tr_delta"][t])) for t in range(r["iters_done"])
                   if r["tr_move"][t] != oracle.NO_MOVE]
            assert got == moves and turns == r["iters_done"]
            n_tied += len(moves)
    assert n_tied > 0


def _nonmetric(w_n):
    """Vehicle 0 flies a, j, n; vehicle 1 flies c, e; the matrix breaks the
    triangle inequality twice: a's delivery to n's pickup is slow (5000 s), so
    taking j out makes n late unless its limit allows it; c's delivery to e's
    pickup is slower still (9000 s), so putting j between c and e saves time."""
    L = 11    # missions a, j, n, c, e fly 0->1, 2->3, 4->5, 6->7, 8->9; base 10
    T = np.full((L, L), 50, dtype=np.int32)
    np.fill_diagonal(T, 0)
    T[1, 4] = 5000
    T[7, 8] = 9000
    T[5, 8] = 20000
    p, d = [0, 2, 4, 6, 8], [1, 3, 5, 7, 9]
    w = [200, 400, w_n, 290, 10000]
    return oracle.FleetProblem(T, T, p, d, w, None, [10, 10], [0, 0], 10 ** 6, 10 ** 6)


def test_taking_a_mission_out_must_leave_a_feasible_route():
    off, seq = [0, 3, 5], [0, 1, 2, 3, 4]
    tight, loose = _nonmetric(600), _nonmetric(6000)
    for F in (tight, loose):
        assert F.feasible(off, seq)[0]
    # relocate j (mission 1) between c and e: G = off[1] + 1 + 1 = 5
    slot = 1 * (5 + 2) + 5
    no_tabu = np.full((5, 2), -1, np.int32)
    for F, valid in ((tight, False), (loose, True)):
        cur = F.feasible(off, seq)[1]
        k0 = F.keys(off, seq, no_tabu, 0, cur, cur, mode=0)
        k1 = F.keys(off, seq, no_tabu, 0, cur, cur, mode=1)
        assert np.array_equal(k0, k1)
        assert (k0[slot] != NONE) == valid
        if valid:
            assert int((int(k0[slot]) >> 32) & 0x7FFFFFFF) - (1 << 30) < 0


def test_sweep_keeps_a_mission_whose_removal_breaks_its_route():
    """Algorithm 1 builds exactly a, j, n | c, e on the non-metric instance;
    the sweep's move of j between c and e saves 4000 s, but taking j out makes
    n late under the tight limit: j stays there, and moves under the loose one."""
    for w_n, moves_j in ((600, False), (6000, True)):
        F = _nonmetric(w_n)
        off, seq, rep = F.greedy(0)
        assert list(off) == [0, 3, 5] and list(seq) == [0, 1, 2, 3, 4] and rep == 0
        r = F.sweep(variant=oracle.NS)
        assert (r["tr_move"][1] == 1 * 7 + 5) == moves_j
        if moves_j:
            assert r["tr_delta"][1] == -4000
        moves, turns = _sweep_by_hand(F, oracle.NS, 0, 0)
        assert [(t, int(r["tr_move"][t])) for t in range(turns) if r["tr_move"][t] != oracle.NO_MOVE] == \
               [(t, m) for t, m, _ in moves]
