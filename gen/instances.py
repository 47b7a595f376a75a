"""Seeded synthetic instances for the air-ambulance scheduling problem.

This module produces INPUTS only: facility and base coordinates, missions as
(pickup, delivery) location pairs, and the vehicle -> base assignment.  It holds
none of the method's arithmetic (no travel times, no costs, no moves); the
oracle and the HIP path each compute those themselves from what this module
returns.

The paper (Section 5) uses real coordinates of air and health facilities that
are not available here, so every workload is a synthetic stand-in with the
structure of the paper's model (Section 3): F health facilities and B bases
drawn uniformly in a box of Northern Ontario / Manitoba (42-57 deg N,
75-95 deg W), M missions each a distinct ordered (pickup, delivery) pair of
different facilities, and V vehicles each parked at base (v mod B).

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): the state advances by the golden
gamma 0x9E3779B97F4A7C15 and each output is the state passed through the
variant-13 finaliser of MurmurHash3 (shifts 30/27/31).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15

LAT_LO, LAT_SPAN = 42.0, 15.0     # 42..57 deg N
LON_LO, LON_SPAN = -95.0, 20.0    # 95..75 deg W
SPEED_KMH = 260.0


class SplitMix64:
    """Sequential SplitMix64 stream (one 64-bit output per call)."""

    __slots__ = ("state",)

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + GAMMA) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def u01(self) -> float:
        """Uniform double in [0, 1) with 53 random bits."""
        return (self.next() >> 11) * (1.0 / 9007199254740992.0)

    def randint(self, n: int) -> int:
        """Integer in [0, n) by plain modulo (the bias is part of the recipe)."""
        return self.next() % n


@dataclass
class Instance:
    """One scheduling instance.

    Locations 0..F-1 are health facilities, F..F+B-1 are bases.
    """
    lat: np.ndarray            # float64 [F+B], degrees
    lon: np.ndarray            # float64 [F+B], degrees
    pickup: np.ndarray         # int32 [M], location ids < F
    delivery: np.ndarray       # int32 [M], location ids < F, != pickup
    vehicle_loc: np.ndarray    # int32 [V], base location ids
    n_fac: int
    n_bases: int
    seed: int
    tenure: int = 7
    iters: int = 500
    meta: dict = field(default_factory=dict)
    # the constrained model (None: unconstrained): per-mission time limit at the
    # delivery point (s) and helicopter-only flag, per-vehicle type (0
    # helicopter, 1 plane), the two speeds, flight limit and horizon (s)
    deadline: np.ndarray | None = None
    heli_only: np.ndarray | None = None
    vehicle_type: np.ndarray | None = None
    speed_heli: float = SPEED_KMH
    speed_plane: float = SPEED_KMH
    flight_limit: int = 0
    horizon: int = 0

    @property
    def n_locs(self) -> int:
        return self.n_fac + self.n_bases

    @property
    def n_missions(self) -> int:
        return int(self.pickup.shape[0])

    @property
    def n_vehicles(self) -> int:
        return int(self.vehicle_loc.shape[0])


def make_instance(seed: int, n_fac: int, n_bases: int, n_vehicles: int,
                  n_missions: int, tenure: int = 7, iters: int = 500) -> Instance:
    """Draw one instance from SplitMix64(seed).

    Draw order: F facilities (lat then lon each), then B bases the same way,
    then M missions by rejection (p = randint(F), d = randint(F) until p != d
    and the ordered pair is new).  Vehicle v sits at location F + (v mod B).
    """
    if n_fac < 2 or n_bases < 1 or n_vehicles < 1 or n_missions < 0:
        raise ValueError("need F >= 2, B >= 1, V >= 1, M >= 0")
    if n_missions > n_fac * (n_fac - 1):
        raise ValueError("more missions than distinct ordered facility pairs")
    rng = SplitMix64(seed)
    n_locs = n_fac + n_bases
    lat = np.empty(n_locs, dtype=np.float64)
    lon = np.empty(n_locs, dtype=np.float64)
    for i in range(n_locs):
        lat[i] = LAT_LO + LAT_SPAN * rng.u01()
        lon[i] = LON_LO + LON_SPAN * rng.u01()
    used = set()
    pick = np.empty(n_missions, dtype=np.int32)
    dlv = np.empty(n_missions, dtype=np.int32)
    for m in range(n_missions):
        while True:
            p = rng.randint(n_fac)
            d = rng.randint(n_fac)
            if p != d and (p, d) not in used:
                break
        used.add((p, d))
        pick[m] = p
        dlv[m] = d
    vloc = np.array([n_fac + (v % n_bases) for v in range(n_vehicles)], dtype=np.int32)
    return Instance(lat, lon, pick, dlv, vloc, n_fac, n_bases, seed, tenure, iters)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def small_instance(seed: int = 0) -> Instance:
    """3 bases x 1 vehicle each, 20 facilities, 12 missions; tenure 7, 500 iterations."""
    return make_instance(seed, 20, 3, 3, 12, tenure=7, iters=500)


def brute_twin(seed: int = 0) -> Instance:
    """2 bases x 1 vehicle, 20 facilities, 6 missions: small enough to enumerate."""
    return make_instance(seed, 20, 2, 2, 6, tenure=7, iters=500)


def m400_instance(seed: int = 0) -> Instance:
    """10 bases, 16 vehicles, 120 facilities, 400 missions; tenure 15, 5000 iterations."""
    return make_instance(seed, 120, 10, 16, 400, tenure=15, iters=5000)


def stress_instance(seed: int = 0) -> Instance:
    """200 bases, 256 vehicles, 2000 facilities, 10000 missions; tenure 25, 1000 iterations."""
    return make_instance(seed, 2000, 200, 256, 10000, tenure=25, iters=1000)


def batch_specs(n: int, stream_seed: int = 0):
    """Per-instance sizes of the uneven batch: a list of dicts, in stream order.

    From SplitMix64(stream_seed), per instance: M = 10 + randint(291),
    V = 2 + randint(23), B = 2 + randint(9), tenure = 7 + randint(9),
    inst_seed = next(); F = ceil(1.5 M).
    """
    rng = SplitMix64(stream_seed)
    out = []
    for k in range(n):
        m = 10 + rng.randint(291)
        v = 2 + rng.randint(23)
        b = 2 + rng.randint(9)
        ten = 7 + rng.randint(9)
        s = rng.next()
        out.append(dict(index=k, n_missions=m, n_vehicles=v, n_bases=b,
                        n_fac=(3 * m + 1) // 2, tenure=ten, seed=s, iters=2000))
    return out


def batch_instance(spec: dict) -> Instance:
    return make_instance(spec["seed"], spec["n_fac"], spec["n_bases"], spec["n_vehicles"],
                         spec["n_missions"], tenure=spec["tenure"], iters=spec["iters"])


def restart_seed(inst_seed: int, r: int) -> int:
    """Greedy-order seed of restart r: 0 (identity order) for r == 0, else inst_seed + r."""
    return 0 if r == 0 else (inst_seed + r) & MASK64


def serve_specs(n: int, stream_seed: int = 1):
    """Per-request sizes of the serving stream.

    From SplitMix64(stream_seed): M = clamp(llround(exp(ln 10 + u01 (ln 2000 - ln 10))),
    10, 2000), V = ceil(M/20), B = ceil(V/2), F = ceil(1.5 M), tenure 15,
    1000 iterations, inst_seed = next().
    """
    rng = SplitMix64(stream_seed)
    lo, hi = math.log(10.0), math.log(2000.0)
    out = []
    for k in range(n):
        x = math.exp(lo + rng.u01() * (hi - lo))
        m = int(math.floor(x + 0.5))
        m = min(max(m, 10), 2000)
        v = (m + 19) // 20
        b = (v + 1) // 2
        s = rng.next()
        out.append(dict(index=k, n_missions=m, n_vehicles=v, n_bases=b,
                        n_fac=(3 * m + 1) // 2, tenure=15, seed=s, iters=1000))
    return out


def poisson_arrivals(n: int, lam: float, stream_seed: int) -> np.ndarray:
    """n arrival times (seconds from 0) of a Poisson process of rate lam:
    gaps are -ln(1 - u01) / lam from SplitMix64(stream_seed)."""
    rng = SplitMix64(stream_seed)
    t = 0.0
    out = np.empty(n, dtype=np.float64)
    for i in range(n):
        t += -math.log(1.0 - rng.u01()) / lam
        out[i] = t
    return out


# ---------------------------------------------------------------------------
# The constrained model of the paper (Section 3)
# ---------------------------------------------------------------------------
HELI_KMH, PLANE_KMH = 300.0, 500.0        # rotary-wing and fixed-wing speeds
FLIGHT_LIMIT_S, HORIZON_S = 10 * 3600, 24 * 3600


FLEET_LAT_SPAN, FLEET_LON_SPAN = 4.0, 6.0   # the constrained workloads' region: 47-51 N, 91-85 W


def fleet_instance(seed: int, n_missions: int, n_fac: int = 40, n_plane: int = 4,
                   n_heli: int = 8, w_lo: int = 1 * 3600, w_hi: int = 23 * 3600,
                   heli_share: int = 4, tenure: int = 5, iters: int = 300) -> Instance:
    """An instance of the constrained model, drawn from SplitMix64(seed).

    As the paper's evaluation: one vehicle per base, the first n_plane bases
    hold planes (500 km/h), the other n_heli helicopters (300 km/h); a flight
    limit of 10 h and a 24 h horizon.  Points lie in a regional box of 4 x 6
    degrees (47-51 N, 91-85 W: a region one fleet serves in a day; the
    unconstrained workloads' larger box leaves most missions unreachable within
    these limits).  Draw order: F facilities and B bases (lat then lon each),
    M missions by rejection (as make_instance), then each mission's time limit
    at its delivery point, w = w_lo + randint(w_hi - w_lo + 1) seconds, then
    each mission's helicopter-only flag, randint(heli_share) == 0.
    """
    n_bases = n_plane + n_heli
    if n_fac < 2 or n_missions < 0 or n_missions > n_fac * (n_fac - 1):
        raise ValueError("need F >= 2 and at most F(F-1) missions")
    rng = SplitMix64(seed)
    n_locs = n_fac + n_bases
    lat = np.empty(n_locs, dtype=np.float64)
    lon = np.empty(n_locs, dtype=np.float64)
    for i in range(n_locs):
        lat[i] = 47.0 + FLEET_LAT_SPAN * rng.u01()
        lon[i] = -91.0 + FLEET_LON_SPAN * rng.u01()
    used = set()
    pick = np.empty(n_missions, dtype=np.int32)
    dlv = np.empty(n_missions, dtype=np.int32)
    for m in range(n_missions):
        while True:
            p = rng.randint(n_fac)
            d = rng.randint(n_fac)
            if p != d and (p, d) not in used:
                break
        used.add((p, d))
        pick[m] = p
        dlv[m] = d
    base = Instance(lat, lon, pick, dlv, np.zeros(0, dtype=np.int32), n_fac, n_bases, seed, tenure,
                    iters)
    w = np.array([w_lo + rng.randint(w_hi - w_lo + 1) for _ in range(n_missions)], dtype=np.int32)
    heli = np.array([1 if rng.randint(heli_share) == 0 else 0 for _ in range(n_missions)],
                    dtype=np.int32)
    base.vehicle_loc = np.array([n_fac + v for v in range(n_bases)], dtype=np.int32)
    base.vehicle_type = np.array([1 if v < n_plane else 0 for v in range(n_bases)], dtype=np.int32)
    base.deadline = w
    base.heli_only = heli
    base.speed_heli, base.speed_plane = HELI_KMH, PLANE_KMH
    base.flight_limit, base.horizon = FLIGHT_LIMIT_S, HORIZON_S
    return base


def fleet_specs(n: int, stream_seed: int = 3):
    """The paper-scale batch: per instance from SplitMix64(stream_seed),
    M = 12 + 3 * randint(8) (the paper's 12, 15, ..., 33 missions), 40
    facilities, 4 plane and 8 helicopter bases, tenure 5 + randint(5),
    inst_seed = next()."""
    rng = SplitMix64(stream_seed)
    out = []
    for k in range(n):
        m = 12 + 3 * rng.randint(8)
        ten = 5 + rng.randint(5)
        s = rng.next()
        out.append(dict(index=k, n_missions=m, tenure=ten, seed=s))
    return out
