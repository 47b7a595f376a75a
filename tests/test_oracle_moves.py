"""Pins of the oracle's objective (Eq (2) on route lists), its move semantics
(relocate as in Figure 2, plus the swap move) and its move deltas.

Objective pins are explicit edge lists summed by hand; move pins are the
routes a move must produce, written out; the closed-form deltas are checked
against apply-and-recompute on every slot of random solutions, including
empty routes, one-mission routes, a single vehicle and adjacent swaps.
"""
import itertools

import numpy as np
import pytest

import oracle
from gen.instances import SplitMix64, small_instance


def _toy_T(L):
    T = np.zeros((L, L), dtype=np.int32)
    for i in range(L):
        for j in range(L):
            if i != j:
                T[i, j] = (i * 7 + j * 13 + i * j) % 50 + 1
    return T


def _toy():
    """6 facilities (0..5), bases 6 and 7; m0=(0,1), m1=(2,3), m2=(4,5)."""
    T = _toy_T(8)
    return oracle.Problem(T, [0, 2, 4], [1, 3, 5], [6, 7]), T


def test_objective_one_mission_by_hand():
    T = np.array([[0, 7, 3], [4, 0, 11], [5, 9, 0]], dtype=np.int32)
    P = oracle.Problem(T, [0], [1], [2])
    # base 2 -> pickup 0 (5) + loaded leg 0 -> 1 (7) + delivery 1 -> base 2 (11)
    assert P.objective([0, 1], [0]) == 23
    # with no missions nothing flies
    P0 = oracle.Problem(T, np.zeros(0, np.int32), np.zeros(0, np.int32), [2, 1])
    assert P0.objective([0, 0, 0], np.zeros(0, np.int32)) == 0


def test_objective_edge_list():
    P, T = _toy()
    # v0 (base 6): m0, m1 ; v1 (base 7): m2
    off, seq = [0, 2, 3], [0, 1, 2]
    edges = [(6, 0), (0, 1), (1, 2), (2, 3), (3, 6),     # base, m0 leg, d0->p1, m1 leg, d1->base
             (7, 4), (4, 5), (5, 7)]                     # base, m2 leg, d2->base
    assert P.objective(off, seq) == sum(int(T[a, b]) for a, b in edges)
    # an empty vehicle adds nothing
    assert P.objective([0, 3, 3], [0, 1, 2]) == sum(int(T[a, b]) for a, b in
        [(6, 0), (0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 6)])


def test_canonical_moves_by_hand():
    P, T = _toy()
    off, seq = [0, 2, 3], [0, 1, 2]          # v0: m0 m1 | v1: m2 ; M=3, V=2, M+V=5 gaps
    assert P.n_slots == 3 * 5 + 3
    # relocate m0 into v1 gap 1 (after m2): gap id = 2 + 1 + 1 = 4, slot 0*5 + 4
    o, s = P.apply(off, seq, 4)
    assert list(o) == [0, 1, 3] and list(s) == [1, 2, 0]
    # relocate m1 into v0 gap 0 (before m0): slot 1*5 + 0
    o, s = P.apply(off, seq, 5)
    assert list(o) == [0, 2, 3] and list(s) == [1, 0, 2]
    # relocate m0 to v0 gap 2 (after m1), same route, gap counted before removal: slot 0*5 + 2
    o, s = P.apply(off, seq, 2)
    assert list(o) == [0, 2, 3] and list(s) == [1, 0, 2]
    # m0 into its own gaps 0 and 1 changes nothing: not moves
    for idx in (0, 1):
        valid, _ = P.delta(off, seq, idx)
        assert not valid
    # m2 into v1 gaps 0/1 (its own) are not moves; into v0 gap 0 is slot 2*5 + 0
    assert not P.delta(off, seq, 2 * 5 + 3)[0] and not P.delta(off, seq, 2 * 5 + 4)[0]
    o, s = P.apply(off, seq, 10)
    assert list(o) == [0, 3, 3] and list(s) == [2, 0, 1]
    # swap (m0, m2): 15 + 0*3 - 0 + (2 - 0 - 1) = 16 ; swap (m0,m1) = 15 ; swap (m1,m2) = 17
    o, s = P.apply(off, seq, 16)
    assert list(o) == [0, 2, 3] and list(s) == [2, 1, 0]
    o, s = P.apply(off, seq, 15)
    assert list(s) == [1, 0, 2]
    o, s = P.apply(off, seq, 17)
    assert list(s) == [0, 2, 1]


def test_delta_by_hand():
    P, T = _toy()
    off, seq = [0, 2, 3], [0, 1, 2]
    base = P.objective(off, seq)
    # relocate m0 behind m2: v0 = [m1], v1 = [m2, m0]
    after = sum(int(T[a, b]) for a, b in [(6, 2), (2, 3), (3, 6),
                                          (7, 4), (4, 5), (5, 0), (0, 1), (1, 7)])
    assert P.delta(off, seq, 4, mode=1) == (True, after - base)
    assert P.delta(off, seq, 4, mode=0) == (True, after - base)
    # adjacent swap m0 <-> m1 on v0: 6 -> m1 -> m0 -> 6
    after = sum(int(T[a, b]) for a, b in [(6, 2), (2, 3), (3, 0), (0, 1), (1, 6),
                                          (7, 4), (4, 5), (5, 7)])
    assert P.delta(off, seq, 15, mode=1) == (True, after - base)


def _random_solution(rng, M, V, empty_bias=False):
    perm = list(range(M))
    for i in range(M - 1, 0, -1):
        j = rng.randint(i + 1)
        perm[i], perm[j] = perm[j], perm[i]
    cuts = sorted(rng.randint(M + 1) for _ in range(V - 1))
    if empty_bias and V > 1:
        cuts[0] = 0
    off = [0] + cuts + [M]
    return np.array(off, np.int32), np.array(perm, np.int32)


def _random_problem(rng, L, M, V):
    T = np.zeros((L, L), dtype=np.int32)
    for i in range(L):
        for j in range(L):
            if i != j:
                T[i, j] = 1 + rng.randint(1000)
    pairs = [(a, b) for a in range(L - V) for b in range(L - V) if a != b]
    pick = []
    for _ in range(M):
        pick.append(pairs.pop(rng.randint(len(pairs))))
    p = [a for a, _ in pick]
    d = [b for _, b in pick]
    b = [L - V + (v % V) for v in range(V)]
    return oracle.Problem(T, p, d, b)


@pytest.mark.parametrize("M,V", [(1, 1), (2, 1), (5, 1), (4, 3), (7, 2), (6, 4), (9, 3)])
def test_closed_form_equals_recompute_on_every_slot(M, V):
    rng = SplitMix64(1000 + 17 * M + V)
    P = _random_problem(rng, 14, M, V)
    for trial in range(6):
        off, seq = _random_solution(rng, M, V, empty_bias=(trial % 2 == 0))
        base = P.objective(off, seq)
        n_valid = 0
        for idx in range(P.n_slots):
            v1, d1 = P.delta(off, seq, idx, mode=1)
            v0, d0 = P.delta(off, seq, idx, mode=0)
            assert v0 == v1
            if v0:
                n_valid += 1
                assert d0 == d1, (M, V, trial, idx)
                o2, s2 = P.apply(off, seq, idx)
                assert P.objective(o2, s2) - base == d1
                # every mission still served exactly once, offsets consistent
                assert sorted(s2.tolist()) == list(range(M))
                assert o2[0] == 0 and o2[-1] == M and np.all(np.diff(o2) >= 0)
        # M(M+V) relocate slots minus 2 no-op gaps per mission, plus all swaps
        assert n_valid == M * (M + V - 2) + M * (M - 1) // 2


def test_keys_match_deltas_and_masks():
    inst = small_instance(0)
    P = oracle.Problem.from_instance(inst)
    off, seq = P.greedy(0)
    cur = P.objective(off, seq)
    tabu = np.full((P.M, P.V), -1, np.int32)
    keys = P.keys(off, seq, tabu, 0, cur, cur)
    assert keys.shape[0] == P.n_slots == 12 * 15 + 66
    for idx, k in enumerate(keys):
        valid, dl = P.delta(off, seq, idx, mode=0)
        if not valid:
            assert int(k) == 0xFFFFFFFFFFFFFFFF
            continue
        assert int(k) >> 63 == 0
        assert ((int(k) >> 32) & 0x7FFFFFFF) - (1 << 30) == dl
        assert int(k) & 0xFFFFFFFF == idx
