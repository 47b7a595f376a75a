"""Python handle on the plain CPU oracle (atabu_oracle.c).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
implementation; `build()` compiles the C file with gcc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "atabu_oracle.c")
_SRC2 = os.path.join(_HERE, "fleet_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OR_OK, OR_EINVAL, OR_ERANGE, OR_ENOMEM = 0, -1, -2, -3
TABU, NS = 0, 1
NO_MOVE = 0xFFFFFFFF


def build(force: bool = True) -> str:
    """Compile the oracle into oracle/liboracle.so (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-Wall",
               "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, _SRC2, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Inst(C.Structure):
    _fields_ = [("L", C.c_int32), ("T", C.POINTER(C.c_int32)),
                ("M", C.c_int32), ("p", C.POINTER(C.c_int32)), ("d", C.POINTER(C.c_int32)),
                ("V", C.c_int32), ("b", C.POINTER(C.c_int32))]


class _Params(C.Structure):
    _fields_ = [("variant", C.c_int32), ("tenure", C.c_int32), ("max_iters", C.c_int32),
                ("aspiration", C.c_int32), ("restart_seed", C.c_uint64)]


class _FInst(C.Structure):
    _fields_ = [("L", C.c_int32), ("T0", C.POINTER(C.c_int32)), ("T1", C.POINTER(C.c_int32)),
                ("M", C.c_int32), ("p", C.POINTER(C.c_int32)), ("d", C.POINTER(C.c_int32)),
                ("w", C.POINTER(C.c_int32)), ("heli", C.POINTER(C.c_int32)),
                ("V", C.c_int32), ("b", C.POINTER(C.c_int32)), ("type", C.POINTER(C.c_int32)),
                ("flight_limit", C.c_int32), ("horizon", C.c_int32)]


class _FParams(C.Structure):
    _fields_ = [("variant", C.c_int32), ("tenure", C.c_int32), ("max_iters", C.c_int32),
                ("aspiration", C.c_int32), ("restart_seed", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                                                    os.path.getmtime(_SRC2)):
            build()
        L = C.CDLL(_LIB)
        i32p, i64p, u64p, u32p, u8p = (C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_uint64), C.POINTER(C.c_uint32),
                                       C.POINTER(C.c_uint8))
        L.or_travel.argtypes = [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                C.c_double, i32p]
        L.or_objective.argtypes = [C.POINTER(_Inst), i32p, i32p]
        L.or_objective.restype = C.c_int64
        L.or_greedy.argtypes = [C.POINTER(_Inst), C.c_uint64, i32p, i32p]
        L.or_delta.argtypes = [C.POINTER(_Inst), i32p, i32p, C.c_int64, C.c_int32, i32p]
        L.or_delta.restype = C.c_int64
        L.or_apply.argtypes = [C.POINTER(_Inst), i32p, i32p, C.c_int64]
        L.or_keys.argtypes = [C.POINTER(_Inst), i32p, i32p, i32p, C.c_int32, C.c_int64,
                              C.c_int64, C.POINTER(_Params), u64p]
        L.or_step.argtypes = [C.POINTER(_Inst), i32p, i32p, i32p, C.c_int32, i64p, i64p,
                              C.POINTER(_Params), u32p, i32p, i64p, u8p]
        L.or_solve.argtypes = [C.POINTER(_Inst), C.POINTER(_Params), i32p, i32p, i32p, i32p,
                               i64p, i64p, i32p, i32p, u32p, i32p, i64p, u8p]
        L.or_num_slots.argtypes = [C.c_int32, C.c_int32]
        L.or_num_slots.restype = C.c_int64
        L.or_splitmix64.argtypes = [C.c_uint64, C.c_int32, u64p]
        L.or_splitmix64.restype = None
        fi, fp = C.POINTER(_FInst), C.POINTER(_FParams)
        L.fo_keys.argtypes = [fi, i32p, i32p, i32p, C.c_int32, C.c_int64, C.c_int64, C.c_int32,
                              C.c_int32, C.c_int32, u64p]
        L.fo_feasible.argtypes = [fi, i32p, i32p, i64p]
        L.fo_greedy.argtypes = [fi, C.c_uint64, i32p, i32p, i32p, i32p]
        L.fo_solve_best.argtypes = [fi, fp, i32p, i32p, i32p, i32p, i64p, i64p, i32p, i32p, u32p,
                                    i32p, i64p, u8p, i32p]
        L.fo_solve_sweep.argtypes = [fi, fp, i32p, i32p, i64p, i32p, i32p, i32p, u32p, i32p, i64p,
                                     i32p]
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def splitmix64(seed: int, n: int) -> list:
    """The first n outputs of the oracle's SplitMix64(seed)."""
    out = np.empty(max(n, 1), dtype=np.uint64)
    lib().or_splitmix64(C.c_uint64(seed & ((1 << 64) - 1)), n, _ptr(out, C.c_uint64))
    return [int(x) for x in out[:n]]


def travel(lat, lon, speed_kmh: float = 260.0) -> np.ndarray:
    """Eq (1) travel-time matrix in integer seconds (FP64 haversine, R = 6371 km)."""
    lat = np.ascontiguousarray(lat, dtype=np.float64)
    lon = np.ascontiguousarray(lon, dtype=np.float64)
    n = lat.shape[0]
    out = np.empty((n, n), dtype=np.int32)
    rc = lib().or_travel(n, _ptr(lat, C.c_double), _ptr(lon, C.c_double), float(speed_kmh),
                         _ptr(out, C.c_int32))
    if rc != OR_OK:
        raise ValueError(f"or_travel rc={rc}")
    return out


class Problem:
    """An instance as the oracle sees it: travel matrix, missions, vehicle bases."""

    def __init__(self, T, pickup, delivery, vehicle_loc):
        self.T = np.ascontiguousarray(T, dtype=np.int32)
        self.p = np.ascontiguousarray(pickup, dtype=np.int32)
        self.d = np.ascontiguousarray(delivery, dtype=np.int32)
        self.b = np.ascontiguousarray(vehicle_loc, dtype=np.int32)
        self.L, self.M, self.V = self.T.shape[0], self.p.shape[0], self.b.shape[0]
        self._s = _Inst(self.L, _ptr(self.T, C.c_int32), self.M, _ptr(self.p, C.c_int32),
                        _ptr(self.d, C.c_int32), self.V, _ptr(self.b, C.c_int32))

    @classmethod
    def from_instance(cls, inst, speed_kmh: float = 260.0):
        return cls(travel(inst.lat, inst.lon, speed_kmh), inst.pickup, inst.delivery,
                   inst.vehicle_loc)

    @property
    def n_slots(self) -> int:
        return int(lib().or_num_slots(self.M, self.V))

    def objective(self, off, seq) -> int:
        off = np.ascontiguousarray(off, dtype=np.int32)
        seq = np.ascontiguousarray(seq, dtype=np.int32)
        return int(lib().or_objective(C.byref(self._s), _ptr(off, C.c_int32), _ptr(seq, C.c_int32)))

    def greedy(self, seed: int = 0):
        off = np.empty(self.V + 1, dtype=np.int32)
        seq = np.empty(max(self.M, 1), dtype=np.int32)
        rc = lib().or_greedy(C.byref(self._s), C.c_uint64(seed), _ptr(off, C.c_int32),
                             _ptr(seq, C.c_int32))
        if rc != OR_OK:
            raise ValueError(f"or_greedy rc={rc}")
        return off, seq[:self.M]

    def delta(self, off, seq, idx: int, mode: int = 1):
        """(valid, delta) of slot idx; mode 0 = by definition, 1 = closed form."""
        off = np.ascontiguousarray(off, dtype=np.int32)
        seq = np.ascontiguousarray(seq, dtype=np.int32)
        valid = C.c_int32(0)
        d = lib().or_delta(C.byref(self._s), _ptr(off, C.c_int32), _ptr(seq, C.c_int32),
                           C.c_int64(idx), mode, C.byref(valid))
        return bool(valid.value), int(d)

    def apply(self, off, seq, idx: int):
        off = np.array(off, dtype=np.int32)
        seq = np.array(seq, dtype=np.int32)
        rc = lib().or_apply(C.byref(self._s), _ptr(off, C.c_int32), _ptr(seq, C.c_int32),
                            C.c_int64(idx))
        if rc != OR_OK:
            raise ValueError(f"slot {idx} is not a move")
        return off, seq

    def keys(self, off, seq, tabu_until, t, cur, best, variant=TABU, aspiration=1):
        off = np.ascontiguousarray(off, dtype=np.int32)
        seq = np.ascontiguousarray(seq, dtype=np.int32)
        tabu = np.ascontiguousarray(tabu_until, dtype=np.int32).reshape(-1)
        out = np.empty(self.n_slots, dtype=np.uint64)
        pr = _Params(variant, 0, 0, aspiration, 0)
        rc = lib().or_keys(C.byref(self._s), _ptr(off, C.c_int32), _ptr(seq, C.c_int32),
                           _ptr(tabu, C.c_int32), t, cur, best, C.byref(pr),
                           _ptr(out, C.c_uint64))
        if rc != OR_OK:
            raise ValueError(f"or_keys rc={rc}")
        return out

    def step(self, state: dict, variant=TABU, tenure=7, aspiration=1):
        """One iteration on a state dict {off, seq, tabu, t, cur, best} (edited in place)."""
        cur = C.c_int64(state["cur"])
        best = C.c_int64(state["best"])
        mv, dl, ob, fl = C.c_uint32(0), C.c_int32(0), C.c_int64(0), C.c_uint8(0)
        pr = _Params(variant, tenure, 0, aspiration, 0)
        rc = lib().or_step(C.byref(self._s), _ptr(state["off"], C.c_int32),
                           _ptr(state["seq"], C.c_int32), _ptr(state["tabu"], C.c_int32),
                           state["t"], C.byref(cur), C.byref(best), C.byref(pr),
                           C.byref(mv), C.byref(dl), C.byref(ob), C.byref(fl))
        if rc < 0:
            raise ValueError(f"or_step rc={rc}")
        state["cur"], state["best"] = cur.value, best.value
        state["t"] += 1
        return rc, (mv.value, dl.value, ob.value, fl.value)

    def solve(self, variant=TABU, tenure=7, iters=500, aspiration=1, restart_seed=0,
              trace=True):
        M, V = self.M, self.V
        bo, bs = np.empty(V + 1, np.int32), np.empty(max(M, 1), np.int32)
        fo, fs = np.empty(V + 1, np.int32), np.empty(max(M, 1), np.int32)
        n = max(iters, 1)
        tm, td = np.empty(n, np.uint32), np.empty(n, np.int32)
        to, tf = np.empty(n, np.int64), np.empty(n, np.uint8)
        best, final = C.c_int64(0), C.c_int64(0)
        done, bi = C.c_int32(0), C.c_int32(0)
        pr = _Params(variant, tenure, iters, aspiration, C.c_uint64(restart_seed))
        args = [None, None, None, None]
        if trace:
            args = [_ptr(tm, C.c_uint32), _ptr(td, C.c_int32), _ptr(to, C.c_int64),
                    _ptr(tf, C.c_uint8)]
        rc = lib().or_solve(C.byref(self._s), C.byref(pr), _ptr(bo, C.c_int32),
                            _ptr(bs, C.c_int32), _ptr(fo, C.c_int32), _ptr(fs, C.c_int32),
                            C.byref(best), C.byref(final), C.byref(done), C.byref(bi), *args)
        if rc != OR_OK:
            raise ValueError(f"or_solve rc={rc}")
        k = done.value
        res = dict(best_off=bo, best_seq=bs[:M], final_off=fo, final_seq=fs[:M],
                   best_obj=best.value, final_obj=final.value, iters_done=k,
                   best_iter=bi.value)
        if trace:
            res.update(tr_move=tm[:k].copy(), tr_delta=td[:k].copy(), tr_obj=to[:k].copy(),
                       tr_flags=tf[:k].copy())
        return res


def new_state(prob: Problem, off, seq, cur=None):
    """A fresh search state (no tabu entries) on a flattened solution."""
    off = np.array(off, dtype=np.int32)
    seq = np.array(seq, dtype=np.int32)
    if cur is None:
        cur = prob.objective(off, seq)
    return dict(off=off, seq=seq, tabu=np.full(prob.M * prob.V, -1, dtype=np.int32), t=0,
                cur=cur, best=cur)


# ---------------------------------------------------------------------------
# The constrained model of Section 3 and the paper's forms of Algorithms 1-3
# (fleet_oracle.c)
# ---------------------------------------------------------------------------
FO_EINFEAS = -6
# no flight limit
NO_FLIGHT_LIMIT = 2 ** 31 - 1


class FleetProblem:
    """An instance of the constrained model: one travel matrix per vehicle type
    (0 helicopter, 1 plane), each mission's time limit at its delivery point and
    whether it is helicopter-only, each vehicle's type, the flight limit and the
    horizon (seconds)."""

    def __init__(self, T_heli, T_plane, pickup, delivery, deadline, heli_only, vehicle_loc,
                 vehicle_type, flight_limit=NO_FLIGHT_LIMIT, horizon=86400):
        """deadline None: no time limits and no horizon; heli_only None: none."""
        self.T0 = np.ascontiguousarray(T_heli, dtype=np.int32)
        self.T1 = np.ascontiguousarray(T_plane, dtype=np.int32)
        self.p = np.ascontiguousarray(pickup, dtype=np.int32)
        self.d = np.ascontiguousarray(delivery, dtype=np.int32)
        self.w = None if deadline is None else np.ascontiguousarray(deadline, dtype=np.int32)
        self.heli = None if heli_only is None else np.ascontiguousarray(heli_only, dtype=np.int32)
        self.b = np.ascontiguousarray(vehicle_loc, dtype=np.int32)
        self.type = np.ascontiguousarray(vehicle_type, dtype=np.int32)
        self.flight_limit, self.horizon = int(flight_limit), int(horizon)
        self.L, self.M, self.V = self.T0.shape[0], self.p.shape[0], self.b.shape[0]
        null = C.POINTER(C.c_int32)()
        self._s = _FInst(self.L, _ptr(self.T0, C.c_int32), _ptr(self.T1, C.c_int32), self.M,
                         _ptr(self.p, C.c_int32), _ptr(self.d, C.c_int32),
                         null if self.w is None else _ptr(self.w, C.c_int32),
                         null if self.heli is None else _ptr(self.heli, C.c_int32), self.V,
                         _ptr(self.b, C.c_int32), _ptr(self.type, C.c_int32), self.flight_limit,
                         self.horizon)

    @classmethod
    def relaxed(cls, T, pickup, delivery, vehicle_loc):
        """The unconstrained model as a special case: one matrix for both types,
        every vehicle a helicopter, no time limit, horizon or flight limit."""
        return cls(T, T, pickup, delivery, None, None, vehicle_loc, np.zeros(len(vehicle_loc)))

    @property
    def n_slots(self) -> int:
        return self.M * (self.M + self.V) + self.M * (self.M - 1) // 2

    def feasible(self, off, seq):
        off = np.ascontiguousarray(off, dtype=np.int32)
        seq = np.ascontiguousarray(seq, dtype=np.int32)
        obj = C.c_int64(0)
        ok = lib().fo_feasible(C.byref(self._s), _ptr(off, C.c_int32), _ptr(seq, C.c_int32), C.byref(obj))
        return bool(ok), int(obj.value)

    def keys(self, off, seq, tabu_until, t, cur, best, variant=TABU, aspiration=1, mode=1):
        off = np.ascontiguousarray(off, dtype=np.int32)
        seq = np.ascontiguousarray(seq, dtype=np.int32)
        tabu = np.ascontiguousarray(tabu_until, dtype=np.int32).reshape(-1)
        out = np.empty(max(self.n_slots, 1), dtype=np.uint64)
        rc = lib().fo_keys(C.byref(self._s), _ptr(off, C.c_int32), _ptr(seq, C.c_int32),
                           _ptr(tabu, C.c_int32), t, cur, best, variant, aspiration, mode,
                           _ptr(out, C.c_uint64))
        if rc != OR_OK:
            raise ValueError(f"fo_keys rc={rc}")
        return out[:self.n_slots]

    def greedy(self, seed: int = 0):
        """Algorithm 1: (off, seq, repairs) or raises ValueError(err, mission)."""
        off = np.empty(self.V + 1, dtype=np.int32)
        seq = np.empty(max(self.M, 1), dtype=np.int32)
        err, rep = C.c_int32(0), C.c_int32(0)
        rc = lib().fo_greedy(C.byref(self._s), C.c_uint64(seed), _ptr(off, C.c_int32),
                             _ptr(seq, C.c_int32), C.byref(err), C.byref(rep))
        if rc != OR_OK:
            raise ValueError(rc, err.value)
        return off, seq[:self.M], rep.value

    def solve(self, variant=TABU, tenure=7, iters=500, aspiration=1, restart_seed=0):
        """Algorithm 1, then the best-move Tabu search or neighbourhood search."""
        M, V = self.M, self.V
        bo, bs = np.empty(V + 1, np.int32), np.empty(max(M, 1), np.int32)
        fo_, fs = np.empty(V + 1, np.int32), np.empty(max(M, 1), np.int32)
        n = max(iters, 1)
        tm, td = np.empty(n, np.uint32), np.empty(n, np.int32)
        to, tf = np.empty(n, np.int64), np.empty(n, np.uint8)
        best, final = C.c_int64(0), C.c_int64(0)
        done, bi, err = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        pr = _FParams(variant, tenure, iters, aspiration, C.c_uint64(restart_seed))
        rc = lib().fo_solve_best(C.byref(self._s), C.byref(pr), _ptr(bo, C.c_int32),
                                 _ptr(bs, C.c_int32), _ptr(fo_, C.c_int32), _ptr(fs, C.c_int32),
                                 C.byref(best), C.byref(final), C.byref(done), C.byref(bi),
                                 _ptr(tm, C.c_uint32), _ptr(td, C.c_int32), _ptr(to, C.c_int64),
                                 _ptr(tf, C.c_uint8), C.byref(err))
        if rc != OR_OK:
            raise ValueError(rc, err.value)
        k = done.value
        return dict(best_off=bo, best_seq=bs[:M], final_off=fo_, final_seq=fs[:M],
                    best_obj=best.value, final_obj=final.value, iters_done=k, best_iter=bi.value,
                    tr_move=tm[:k].copy(), tr_delta=td[:k].copy(), tr_obj=to[:k].copy(),
                    tr_flags=tf[:k].copy())

    def sweep(self, variant=TABU, tenure=7, iters=100000, restart_seed=0):
        """Algorithm 1, then Algorithm 3 (variant 0) or 2 (variant 1) as printed."""
        M, V = self.M, self.V
        off, seq = np.empty(V + 1, np.int32), np.empty(max(M, 1), np.int32)
        n = max(iters, 1)
        tm, td, to = np.empty(n, np.uint32), np.empty(n, np.int32), np.empty(n, np.int64)
        obj = C.c_int64(0)
        done, bi, passes, err = C.c_int32(0), C.c_int32(0), C.c_int32(0), C.c_int32(0)
        pr = _FParams(variant, tenure, iters, 0, C.c_uint64(restart_seed))
        rc = lib().fo_solve_sweep(C.byref(self._s), C.byref(pr), _ptr(off, C.c_int32),
                                  _ptr(seq, C.c_int32), C.byref(obj), C.byref(done), C.byref(bi),
                                  C.byref(passes), _ptr(tm, C.c_uint32), _ptr(td, C.c_int32),
                                  _ptr(to, C.c_int64), C.byref(err))
        if rc != OR_OK:
            raise ValueError(rc, err.value)
        k = done.value
        return dict(best_off=off, best_seq=seq[:M], final_off=off, final_seq=seq[:M],
                    best_obj=obj.value, final_obj=obj.value, iters_done=k, best_iter=bi.value,
                    passes=passes.value, tr_move=tm[:k].copy(), tr_delta=td[:k].copy(),
                    tr_obj=to[:k].copy())
