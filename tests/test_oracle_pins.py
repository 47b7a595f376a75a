"""Pins of the oracle parts that no optimum or recompute check reaches.

* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) in both the input generator and
  the oracle: the generator's published reference outputs.
* The greedy start (Algorithm 1 without its feasibility checks): a hand-worked
  shuffled order (Fisher-Yates driven by the published SplitMix64 outputs, read
  off a one-vehicle instance, whose route is exactly the order), a hand-computed
  instance on which the route's return leg decides the vehicle, and an exact tie
  that must go to the lowest vehicle.
* The tabu bookkeeping of one step (Algorithm 3's TabuList/TabuCounter read as
  an expiry table): after a move at iteration t with tenure k, exactly the
  entries (moved mission, vehicle it left) read t + k, for relocates and swaps,
  and nothing else changes; the neighbourhood search writes none.
* Which (mission, vehicle) entries make a slot tabu: relocate checks its target
  vehicle (its own route included); a swap checks each mission against the
  other's vehicle.
* Aspiration is strict: a tabu move whose objective would equal the best found
  stays blocked; one unit better is admitted.
* Trace flag bit 1 is set exactly when the applied move was tabu and admitted by
  aspiration; bit 2 exactly when every admissible move was tabu.
* The input range of the oracle is the key's: travel times below 2^27.
"""
import numpy as np
import pytest

import oracle
from gen.instances import SplitMix64, make_instance, small_instance

# Published SplitMix64 reference outputs.
SM_1234567 = [6457827717110365317, 3203168211198807973, 9817491932198370423,
              4593380528125082431, 16408922859458223821]
SM_0 = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_splitmix64_reference_outputs():
    assert oracle.splitmix64(1234567, 5) == SM_1234567
    assert oracle.splitmix64(0, 3) == SM_0
    g = SplitMix64(1234567)
    assert [g.next() for _ in range(5)] == SM_1234567
    g = SplitMix64(0)
    assert [g.next() for _ in range(3)] == SM_0


def _flat_T(n, entries, fill=1000):
    T = np.full((n, n), fill, dtype=np.int32)
    np.fill_diagonal(T, 0)
    for (i, j), v in entries.items():
        T[i, j] = v
    return T


def test_greedy_seeded_order_by_hand():
    """One vehicle: the greedy route is the mission order itself.  Fisher-Yates
    over 5 missions with SplitMix64(1234567): i = 4, 3, 2, 1 draws j = o_k mod
    (i + 1) from the published outputs o_1..o_4:
      o_1 mod 5 = 2 -> [0 1 4 3 2];  o_2 mod 4 = 1 -> [0 3 4 1 2];
      o_3 mod 3 = 0 -> [4 3 0 1 2];  o_4 mod 2 = 1 -> unchanged."""
    assert [SM_1234567[0] % 5, SM_1234567[1] % 4, SM_1234567[2] % 3, SM_1234567[3] % 2] == [2, 1, 0, 1]
    T = _flat_T(11, {})
    p = np.array([0, 2, 4, 6, 8], np.int32)
    d = p + 1
    P = oracle.Problem(T, p, d, np.array([10], np.int32))
    off, seq = P.greedy(1234567)
    assert off.tolist() == [0, 5]
    assert seq.tolist() == [4, 3, 0, 1, 2]
    off, seq = P.greedy(0)                 # seed 0: missions in id order
    assert seq.tolist() == [0, 1, 2, 3, 4]


def test_greedy_return_leg_decides_vehicle():
    """Locations 0-3 facilities, 4 = base of vehicle 0, 5 = base of vehicle 1.
    Mission 0 = 0 -> 1, mission 1 = 2 -> 3, taken in id order.
      mission 0: vehicle 0 adds 10 + 5 + 100 = 115, vehicle 1 adds 50 + 5 + 70 = 125
                 -> vehicle 0, whose route now ends 1 -> base (100 s);
      mission 1: vehicle 0 adds 20 + 7 + 30 - 100 = -43 (the old return leg is
                 no longer flown), vehicle 1 adds 15 + 7 + 15 = 37 -> vehicle 0.
    Without the "- old return leg" term vehicle 0 would add 57 and lose."""
    T = _flat_T(6, {(4, 0): 10, (0, 1): 5, (1, 4): 100, (5, 0): 50, (1, 5): 70,
                    (2, 3): 7, (1, 2): 20, (3, 4): 30, (5, 2): 15, (3, 5): 15})
    P = oracle.Problem(T, np.array([0, 2], np.int32), np.array([1, 3], np.int32),
                       np.array([4, 5], np.int32))
    off, seq = P.greedy(0)
    assert off.tolist() == [0, 2, 2] and seq.tolist() == [0, 1]
    assert P.objective(off, seq) == 10 + 5 + 20 + 7 + 30


def test_greedy_tie_goes_to_lowest_vehicle():
    """Two vehicles on the same base: every first mission costs both the same."""
    T = _flat_T(5, {(4, 0): 9, (0, 1): 4, (1, 4): 11, (4, 2): 3, (2, 3): 4, (3, 4): 3})
    P = oracle.Problem(T, np.array([0], np.int32), np.array([1], np.int32),
                       np.array([4, 4], np.int32))
    off, seq = P.greedy(0)
    assert off.tolist() == [0, 1, 1]
    # three vehicles, vehicles 1 and 2 on the same base and both cheaper than vehicle 0
    T = _flat_T(6, {(4, 0): 50, (0, 1): 4, (1, 4): 50, (5, 0): 8, (1, 5): 8})
    P = oracle.Problem(T, np.array([0], np.int32), np.array([1], np.int32),
                       np.array([4, 5, 5], np.int32))
    off, _ = P.greedy(0)
    assert off.tolist() == [0, 0, 1, 1]


# ---------------------------------------------------------------- move decoding

def _route_of(P, off, seq):
    ro = np.empty(P.M, np.int32)
    for v in range(P.V):
        ro[seq[off[v]:off[v + 1]]] = v
    return ro


def _slot(P, off, idx):
    """('reloc', m, v_dst) or ('swap', m1, m2) of a slot index: relocate slots are
    m*(M+V) + off[v] + v + g; swap slots of a < b follow in row order of a."""
    M, V = P.M, P.V
    R = M * (M + V)
    if idx < R:
        m, G = divmod(idx, M + V)
        for v in range(V):
            if off[v] + v <= G <= off[v + 1] + v:
                return ("reloc", m, v)
        raise AssertionError(idx)
    r = idx - R
    for a in range(M):
        row = M - 1 - a
        if r < row:
            return ("swap", a, a + 1 + r)
        r -= row
    raise AssertionError(idx)


def _dl(key):
    return ((int(key) >> 32) & 0x7FFFFFFF) - (1 << 30)


# ---------------------------------------------------------------- tabu bookkeeping

@pytest.mark.parametrize("tenure", [0, 3, 7])
def test_step_writes_exactly_the_left_vehicle_entries(tenure):
    inst = small_instance(0)
    P = oracle.Problem.from_instance(inst)
    st = oracle.new_state(P, *P.greedy(0))
    kinds = set()
    for t in range(250):
        before = st["tabu"].copy().reshape(P.M, P.V)
        ro = _route_of(P, st["off"], st["seq"])
        off0 = st["off"].copy()
        applied, (mv, dl, ob, fl) = P.step(st, tenure=tenure)
        after = st["tabu"].reshape(P.M, P.V)
        assert applied == 1
        kind, a, b = _slot(P, off0, mv)
        kinds.add(kind)
        want = before.copy()
        if kind == "reloc":
            want[a, ro[a]] = t + tenure
        else:
            want[a, ro[a]] = t + tenure
            want[b, ro[b]] = t + tenure
        assert np.array_equal(after, want), (t, kind, a, b)
        assert bool(fl & 1) == (kind == "swap")
    assert kinds == {"reloc", "swap"}


def test_ns_step_writes_no_tabu_entry():
    inst = small_instance(1)
    P = oracle.Problem.from_instance(inst)
    st = oracle.new_state(P, *P.greedy(0))
    for _ in range(20):
        applied, _ = P.step(st, variant=oracle.NS, tenure=7)
        if not applied:
            break
        assert np.all(st["tabu"] == -1)


def test_tabu_attribute_of_relocate_and_swap():
    inst = make_instance(31, 20, 3, 3, 9)
    P = oracle.Problem.from_instance(inst)
    off = np.array([0, 4, 4, 9], np.int32)              # one empty route
    seq = np.array([3, 8, 0, 5, 1, 7, 2, 6, 4], np.int32)
    cur = P.objective(off, seq)
    ro = _route_of(P, off, seq)
    low = cur - 10 ** 7                     # no move can aspirate
    free = P.keys(off, seq, np.full((P.M, P.V), -1, np.int32), 0, cur, low)
    assert not np.any((free != np.uint64(0xFFFFFFFFFFFFFFFF)) & (free >> np.uint64(63) == 1))
    checked = {"reloc_other": 0, "reloc_own": 0, "swap": 0}
    for idx in range(P.n_slots):
        if free[idx] == np.uint64(0xFFFFFFFFFFFFFFFF):
            continue
        kind, a, b = _slot(P, off, idx)
        if kind == "reloc":
            cases = [((a, b), True)] + [((a, v), False) for v in range(P.V) if v != b]
            cases += [((m, b), False) for m in range(P.M) if m != a]
            checked["reloc_own" if b == ro[a] else "reloc_other"] += 1
        else:
            if ro[a] == ro[b]:
                continue
            cases = [((a, ro[b]), True), ((b, ro[a]), True), ((a, ro[a]), False), ((b, ro[b]), False)]
            checked["swap"] += 1
        for (m, v), blocked in cases:
            tabu = np.full((P.M, P.V), -1, np.int32)
            tabu[m, v] = 4
            k = int(P.keys(off, seq, tabu, 2, cur, low)[idx])
            assert (k >> 63) == int(blocked), (idx, kind, a, b, m, v)
            assert (k & ~(1 << 63)) == int(free[idx])
    assert min(checked.values()) > 0, checked


def test_aspiration_is_strict():
    inst = make_instance(32, 20, 3, 3, 9)
    P = oracle.Problem.from_instance(inst)
    off, seq = P.greedy(0)
    cur = P.objective(off, seq)
    free = P.keys(off, seq, np.full((P.M, P.V), -1, np.int32), 0, cur, cur)
    tabu = np.full((P.M, P.V), 50, np.int32)
    valid = np.nonzero(free != np.uint64(0xFFFFFFFFFFFFFFFF))[0]
    R = P.M * (P.M + P.V)
    picks = [int(i) for i in valid if i < R][::17] + [int(i) for i in valid if i >= R][::7]
    assert any(i >= R for i in picks) and any(i < R for i in picks)
    for idx in picks:
        dl = _dl(free[idx])
        k_eq = int(P.keys(off, seq, tabu, 0, cur, cur + dl)[idx])
        k_gt = int(P.keys(off, seq, tabu, 0, cur, cur + dl + 1)[idx])
        assert k_eq >> 63 == 1, idx            # cur + delta == best: not strictly better
        assert k_gt >> 63 == 0, idx            # one second better than the best: admitted
        k_off = P.keys(off, seq, tabu, 0, cur, cur + dl + 1, aspiration=0)[idx]
        assert int(k_off) >> 63 == 1, idx      # aspiration off: stays blocked


def _tabu_entries(P, ro, kind, a, b):
    if kind == "reloc":
        return [(a, b)]
    return [(a, ro[b]), (b, ro[a])]


@pytest.mark.parametrize("seed", [33, 34, 35, 36])
def test_trace_flags_tabu_aspirated_and_fallback(seed):
    inst = make_instance(seed, 20, 3, 3, 9)
    P = oracle.Problem.from_instance(inst)
    off, seq = P.greedy(0)
    cur = P.objective(off, seq)
    ro = _route_of(P, off, seq)
    free = P.keys(off, seq, np.full((P.M, P.V), -1, np.int32), 0, cur, cur)
    k0 = int(free.min())
    idx0, dl0 = k0 & 0xFFFFFFFF, _dl(k0)
    assert dl0 < 0
    kind, a, b = _slot(P, off, idx0)
    swap_bit = 1 if kind == "swap" else 0
    # 1. nothing tabu: bit 1 clear
    st = oracle.new_state(P, off, seq)
    applied, (mv, dl, ob, fl) = P.step(st, tenure=5)
    assert (mv, fl) == (idx0, swap_bit)
    # 2. the best move tabu, best == cur: it improves on the best, so aspiration
    #    admits it and bit 1 is set
    st = oracle.new_state(P, off, seq)
    for (m, v) in _tabu_entries(P, ro, kind, a, b):
        st["tabu"][m * P.V + v] = 3
    applied, (mv, dl, ob, fl) = P.step(st, tenure=5)
    assert (mv, dl, fl) == (idx0, dl0, swap_bit | 2)
    # 3. the same with aspiration off: blocked, another (free) move is taken
    st = oracle.new_state(P, off, seq)
    for (m, v) in _tabu_entries(P, ro, kind, a, b):
        st["tabu"][m * P.V + v] = 3
    applied, (mv, dl, ob, fl) = P.step(st, tenure=5, aspiration=0)
    assert mv != idx0 and (fl & 6) == 0
    # 4. every entry tabu and the best far below: the best blocked move is the
    #    fallback; bit 2 set, bit 1 clear
    st = oracle.new_state(P, off, seq)
    st["tabu"][:] = 3
    st["best"] = cur - 10 ** 7
    applied, (mv, dl, ob, fl) = P.step(st, tenure=5)
    assert (mv, fl) == (idx0, swap_bit | 4)


def test_oracle_range_is_the_key_field():
    """Travel times up to 2^27 - 1 s (max T * 8 < 2^30) are accepted; 2^27 is not."""
    T = np.full((4, 4), (1 << 27) - 1, np.int32)
    np.fill_diagonal(T, 0)
    P = oracle.Problem(T, np.array([0, 1], np.int32), np.array([1, 2], np.int32),
                       np.array([3], np.int32))
    r = P.solve(tenure=1, iters=3)
    assert r["best_obj"] == P.objective(r["best_off"], r["best_seq"])
    T[0, 1] = 1 << 27
    P = oracle.Problem(T, np.array([0, 1], np.int32), np.array([1, 2], np.int32),
                       np.array([3], np.int32))
    with pytest.raises(ValueError):
        P.solve(tenure=1, iters=3)


def test_step_takes_smallest_definitional_delta_then_smallest_index():
    """Each step applies, among the admissible moves (not tabu, or strictly
    better than the best found), the one with the smallest cost change computed
    by definition (apply and recompute Eq (2)), ties to the smallest slot index;
    with two empty routes on each base, equal changes are common."""
    inst = make_instance(41, 20, 3, 6, 9)
    P = oracle.Problem.from_instance(inst)
    st = oracle.new_state(P, *P.greedy(0))
    tenure = 4
    ties = 0
    for t in range(40):
        off, seq = st["off"].copy(), st["seq"].copy()
        tabu = st["tabu"].reshape(P.M, P.V).copy()
        ro = _route_of(P, off, seq)
        cand_free, cand_all = [], []
        for idx in range(P.n_slots):
            valid, dl = P.delta(off, seq, idx, mode=0)
            if not valid:
                continue
            kind, a, b = _slot(P, off, idx)
            ent = [(a, b)] if kind == "reloc" else [(a, ro[b]), (b, ro[a])]
            is_tabu = any(tabu[m, v] >= t for m, v in ent)
            cand_all.append((dl, idx))
            if not is_tabu or st["cur"] + dl < st["best"]:
                cand_free.append((dl, idx))
        pool = cand_free or cand_all
        want = min(pool)
        ties += sum(1 for c in pool if c[0] == want[0]) > 1
        applied, (mv, dl, ob, fl) = P.step(st, tenure=tenure)
        assert (dl, mv) == want, t
        assert bool(fl & 4) == (not cand_free)
    assert ties >= 5, ties
