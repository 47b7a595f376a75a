"""ctypes marshalling for libatabu.so; see include/atabu.h for the contract."""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

AT_OK, AT_EINVAL, AT_ERANGE, AT_ENOMEM, AT_EAGAIN, AT_EDEVICE, AT_EINFEAS = 0, -1, -2, -3, -4, -5, -6
AT_TABU, AT_NS = 0, 1
SCHED_AUTO, SCHED_WG, SCHED_MULTI, SCHED_GLOBAL, SCHED_WAVE = 0, 1, 2, 3, 4
FORM_BEST, FORM_SWEEP = 0, 1

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libatabu.so")

_EXPORTS = ("at_build_travel", "at_build_travel_device", "at_workspace_size", "at_solve",
            "at_solve_noalloc", "at_solve_batch", "at_debug_eval_moves", "at_server_create", "at_server_submit",
            "at_server_progress", "at_server_poll", "at_server_completed", "at_server_destroy", "at_shutdown",
            "at_last_error")


class AtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"atabu error {code}: {msg}")
        self.code = code


class _Instance(C.Structure):
    _fields_ = [("n_locs", C.c_int32), ("travel", C.c_void_p), ("n_missions", C.c_int32),
                ("pickup", C.c_void_p), ("delivery", C.c_void_p), ("n_vehicles", C.c_int32),
                ("vehicle_loc", C.c_void_p), ("travel_plane", C.c_void_p),
                ("vehicle_type", C.c_void_p), ("deadline", C.c_void_p), ("heli_only", C.c_void_p),
                ("flight_limit", C.c_int32), ("horizon", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("variant", C.c_int32), ("tenure", C.c_int32), ("max_iters", C.c_int32),
                ("aspiration", C.c_int32), ("restart_seed", C.c_uint64), ("trace", C.c_int32),
                ("schedule", C.c_int32), ("n_groups", C.c_int32), ("block", C.c_int32),
                ("chunk", C.c_int32), ("form", C.c_int32)]


class _Result(C.Structure):
    _fields_ = [("route_off", C.c_void_p), ("route_seq", C.c_void_p), ("route_of", C.c_void_p),
                ("final_off", C.c_void_p), ("final_seq", C.c_void_p), ("tr_move", C.c_void_p), ("tr_delta", C.c_void_p), ("tr_obj", C.c_void_p),
                ("tr_flags", C.c_void_p), ("best_obj", C.c_int64), ("final_obj", C.c_int64),
                ("iters_done", C.c_int32), ("best_iter", C.c_int32), ("status", C.c_int32),
                ("search_ms", C.c_float)]


_lib = None
_lock = threading.Lock()


def lib():
    """Load libatabu.so; raises if it has not been built (no fallback exists)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(lib_path):
                raise AtError(AT_EDEVICE, f"{lib_path} is missing: run paper_2002_11710_amd/build.py")
            # Load torch's HIP runtime first: the library then binds to the same
            # runtime (same SONAME) instead of pulling a second one into the process.
            import torch  # noqa: F401
            L = C.CDLL(lib_path)
            vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
            L.at_build_travel.argtypes = [i32, vp, vp, C.c_double, vp]
            L.at_build_travel_device.argtypes = [i32, vp, vp, C.c_double, vp, vp]
            L.at_workspace_size.argtypes = [i32, C.POINTER(_Instance), C.POINTER(_Params), i32]
            L.at_workspace_size.restype = C.c_size_t
            L.at_solve.argtypes = [C.POINTER(_Instance), C.POINTER(_Params), vp, C.c_size_t, vp,
                                   C.POINTER(_Result)]
            L.at_solve_noalloc.argtypes = [C.POINTER(_Instance), C.POINTER(_Params), vp,
                                           C.POINTER(_Result)]
            L.at_solve_batch.argtypes = [i32, C.POINTER(_Instance), C.POINTER(_Params), i32, vp,
                                         C.c_size_t, vp, C.POINTER(_Result)]
            L.at_debug_eval_moves.argtypes = [C.POINTER(_Instance), C.POINTER(_Params), vp, vp, vp,
                                              i32, i64, i64, vp, vp, C.c_size_t, vp]
            L.at_last_error.restype = C.c_char_p
            if hasattr(L, "at_server_create"):
                L.at_server_create.argtypes = [C.c_size_t, i32, i32, vp, C.POINTER(vp)]
                L.at_server_submit.argtypes = [vp, C.POINTER(_Instance), C.POINTER(_Params),
                                               C.POINTER(u64)]
                L.at_server_progress.argtypes = [vp, C.POINTER(i32)]
                L.at_server_poll.argtypes = [vp, u64, C.POINTER(_Result)]
                L.at_server_completed.argtypes = [vp, C.POINTER(u64), i32, C.POINTER(i32)]
                L.at_server_destroy.argtypes = [vp]
            _lib = L
    return _lib


def symbols():
    """Names of the C-ABI functions the loaded library exports."""
    L = lib()
    return [n for n in _EXPORTS if hasattr(L, n)]


def shutdown():
    """Release the library's internal streams (at_shutdown); see include/atabu.h."""
    if _lib is not None:
        _check(_lib.at_shutdown())


def _check(rc: int):
    if rc != AT_OK:
        msg = lib().at_last_error()
        raise AtError(rc, msg.decode() if msg else "")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise AtError(AT_EDEVICE, "no GPU visible to torch")
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def build_travel(lat, lon, speed_kmh: float = 260.0):
    """Eq (1) on the host (at_build_travel): (n, n) int32 seconds as a numpy array
    from FP64 latitudes and longitudes in degrees."""
    lat = np.ascontiguousarray(lat, dtype=np.float64)
    lon = np.ascontiguousarray(lon, dtype=np.float64)
    n = int(lat.shape[0])
    if lon.shape[0] != n:
        raise AtError(AT_EINVAL, "lat and lon differ in length")
    out = np.empty((n, n), dtype=np.int32)
    _check(lib().at_build_travel(n, lat.ctypes.data_as(C.c_void_p), lon.ctypes.data_as(C.c_void_p),
                                 float(speed_kmh), out.ctypes.data_as(C.c_void_p)))
    return out


def build_travel_device(lat, lon, speed_kmh: float = 260.0, stream=None):
    """Eq (1) on the device (at_build_travel_device): (n, n) int32 tensor."""
    torch = _torch()
    lat = torch.as_tensor(lat, dtype=torch.float64).contiguous().cuda()
    lon = torch.as_tensor(lon, dtype=torch.float64).contiguous().cuda()
    n = lat.shape[0]
    out = torch.empty((n, n), dtype=torch.int32, device=lat.device)
    _check(lib().at_build_travel_device(n, _dptr(lat), _dptr(lon), float(speed_kmh), _dptr(out),
                                        _stream_ptr(stream)))
    return out


class DeviceInstance:
    """An instance resident in HBM: travel matrix, missions, vehicle bases, and
    optionally the constrained model's fields (see at_instance in atabu.h):
    a plane travel matrix with each vehicle's type, each mission's time limit at
    its delivery point (with the horizon), helicopter-only flags and the flight
    limit."""

    def __init__(self, travel, pickup, delivery, vehicle_loc, travel_plane=None,
                 vehicle_type=None, deadline=None, heli_only=None, flight_limit=0, horizon=0):
        torch = _torch()

        def dev(x):
            return None if x is None else torch.as_tensor(x, dtype=torch.int32).contiguous().cuda()

        self.travel = dev(travel)
        self.pickup = dev(pickup)
        self.delivery = dev(delivery)
        self.vehicle_loc = dev(vehicle_loc)
        self.travel_plane = dev(travel_plane)
        self.vehicle_type = dev(vehicle_type)
        self.deadline = dev(deadline)
        self.heli_only = dev(heli_only)
        self.flight_limit = int(flight_limit)
        self.horizon = int(horizon)
        self.n_locs = int(self.travel.shape[0])
        self.n_missions = int(self.pickup.shape[0])
        self.n_vehicles = int(self.vehicle_loc.shape[0])

    @classmethod
    def from_coords(cls, lat, lon, pickup, delivery, vehicle_loc, speed_kmh=260.0):
        """Eq (1) on the host (at_build_travel), then the matrix is uploaded."""
        return cls(build_travel(lat, lon, speed_kmh), pickup, delivery, vehicle_loc)

    @classmethod
    def from_instance(cls, inst, speed_kmh=260.0):
        """From a gen.instances.Instance (coordinates, missions, vehicle bases)."""
        return cls.from_coords(inst.lat, inst.lon, inst.pickup, inst.delivery, inst.vehicle_loc,
                               speed_kmh)

    def c_struct(self) -> _Instance:
        def p(t):
            return t.data_ptr() if t is not None and t.numel() else None
        return _Instance(self.n_locs, self.travel.data_ptr(), self.n_missions,
                         p(self.pickup), p(self.delivery), self.n_vehicles,
                         self.vehicle_loc.data_ptr(), p(self.travel_plane), p(self.vehicle_type),
                         p(self.deadline), p(self.heli_only), self.flight_limit, self.horizon)


def make_params(variant=AT_TABU, tenure=7, iters=500, aspiration=True, restart_seed=0, trace=True,
                schedule=SCHED_AUTO, n_groups=0, block=0, chunk=0, form=FORM_BEST) -> _Params:
    return _Params(int(variant), int(tenure), int(iters), 1 if aspiration else 0,
                   C.c_uint64(int(restart_seed) & ((1 << 64) - 1)), 1 if trace else 0,
                   int(schedule), int(n_groups), int(block), int(chunk), int(form))


def _alloc_result(M: int, V: int, iters: int, trace: bool, device):
    torch = _torch()
    r = dict(route_off=torch.empty(V + 1, dtype=torch.int32, device=device),
             route_seq=torch.empty(max(M, 1), dtype=torch.int32, device=device),
             route_of=torch.empty(max(M, 1), dtype=torch.int32, device=device),
             final_off=torch.empty(V + 1, dtype=torch.int32, device=device),
             final_seq=torch.empty(max(M, 1), dtype=torch.int32, device=device))
    if trace:
        n = max(iters, 1)
        r.update(tr_move=torch.empty(n, dtype=torch.int32, device=device),
                 tr_delta=torch.empty(n, dtype=torch.int32, device=device),
                 tr_obj=torch.empty(n, dtype=torch.int64, device=device),
                 tr_flags=torch.empty(n, dtype=torch.uint8, device=device))
    return r


def _c_result(bufs) -> _Result:
    g = bufs.get
    return _Result(g("route_off").data_ptr(), g("route_seq").data_ptr(), g("route_of").data_ptr(),
                   g("final_off").data_ptr() if "final_off" in bufs else None,
                   g("final_seq").data_ptr() if "final_seq" in bufs else None,
                   g("tr_move").data_ptr() if "tr_move" in bufs else None,
                   g("tr_delta").data_ptr() if "tr_delta" in bufs else None,
                   g("tr_obj").data_ptr() if "tr_obj" in bufs else None,
                   g("tr_flags").data_ptr() if "tr_flags" in bufs else None, 0, 0, 0, 0, 0, 0.0)


def _finish(bufs, res: _Result, M: int):
    out = dict(bufs)
    out["route_seq"] = bufs["route_seq"][:M]
    out["route_of"] = bufs["route_of"][:M]
    if "final_seq" in bufs:
        out["final_seq"] = bufs["final_seq"][:M]
    k = res.iters_done
    for name in ("tr_move", "tr_delta", "tr_obj", "tr_flags"):
        if name in bufs:
            out[name] = bufs[name][:k]
    out.update(best_obj=res.best_obj, final_obj=res.final_obj, iters_done=res.iters_done,
               best_iter=res.best_iter, status=res.status, search_ms=res.search_ms)
    return out


def workspace_size(insts, params, n_restarts: int = 1) -> int:
    n = len(insts)
    ia = (_Instance * n)(*[i.c_struct() for i in insts])
    pa = (_Params * n)(*params)
    return int(lib().at_workspace_size(n, ia, pa, n_restarts))


def _workspace(nbytes: int, ws=None):
    torch = _torch()
    if ws is not None and ws.numel() >= nbytes:
        return ws
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")


def solve(inst: DeviceInstance, variant=AT_TABU, tenure=7, iters=500, aspiration=True,
          restart_seed=0, trace=True, schedule=SCHED_AUTO, n_groups=0, block=0, chunk=0,
          form=FORM_BEST, ws=None, stream=None, out=None):
    """One solve (at_solve).  Returns device tensors and host scalars."""
    pr = make_params(variant, tenure, iters, aspiration, restart_seed, trace, schedule, n_groups,
                     block, chunk, form)
    ci = inst.c_struct()
    nbytes = int(lib().at_workspace_size(1, C.byref(ci), C.byref(pr), 1))
    if nbytes == 0:
        _check(AT_EINVAL)
    ws = _workspace(nbytes, ws)
    bufs = out if out is not None else _alloc_result(inst.n_missions, inst.n_vehicles, iters,
                                                     trace, inst.travel.device)
    res = _c_result(bufs)
    _check(lib().at_solve(C.byref(ci), C.byref(pr), _dptr(ws), ws.numel(), _stream_ptr(stream),
                          C.byref(res)))
    return _finish(bufs, res, inst.n_missions)


def solve_noalloc(inst: DeviceInstance, variant=AT_TABU, tenure=7, iters=500, aspiration=True,
                  restart_seed=0, trace=True, schedule=SCHED_AUTO, n_groups=0, block=0, chunk=0,
                  stream=None, out=None):
    """One solve with the library's fixed workspace (at_solve_noalloc): the
    library allocates nothing; the result buffers are the caller's (`out`, as
    _alloc_result makes them, or allocated here)."""
    pr = make_params(variant, tenure, iters, aspiration, restart_seed, trace, schedule, n_groups,
                     block, chunk)
    ci = inst.c_struct()
    bufs = out if out is not None else _alloc_result(inst.n_missions, inst.n_vehicles, iters,
                                                     trace, inst.travel.device)
    res = _c_result(bufs)
    _check(lib().at_solve_noalloc(C.byref(ci), C.byref(pr), _stream_ptr(stream), C.byref(res)))
    return _finish(bufs, res, inst.n_missions)


def solve_batch(insts, params, n_restarts=1, ws=None, stream=None, outs=None,
                allow_infeasible=False):
    """n instances x n_restarts solves in one call (at_solve_batch).

    params: one _Params (make_params) per instance.  Returns a list in
    (instance, restart) order.  With allow_infeasible, a call whose only
    failures are starts Algorithm 1 could not build (AT_EINFEAS) returns the
    results, each with its own status."""
    n = len(insts)
    ia = (_Instance * n)(*[i.c_struct() for i in insts])
    pa = (_Params * n)(*params)
    nbytes = int(lib().at_workspace_size(n, ia, pa, n_restarts))
    if nbytes == 0:
        _check(AT_EINVAL)
    ws = _workspace(nbytes, ws)
    if outs is None:
        outs = []
        for i, inst in enumerate(insts):
            for _ in range(n_restarts):
                outs.append(_alloc_result(inst.n_missions, inst.n_vehicles, params[i].max_iters,
                                          bool(params[i].trace), inst.travel.device))
    ra = (_Result * len(outs))(*[_c_result(b) for b in outs])
    rc = lib().at_solve_batch(n, ia, pa, n_restarts, _dptr(ws), ws.numel(), _stream_ptr(stream), ra)
    if not (allow_infeasible and rc == AT_EINFEAS):
        _check(rc)
    return [_finish(outs[k], ra[k], insts[k // n_restarts].n_missions) for k in range(len(outs))]


class BatchResult:
    """Results of solve_batch_flat, solve k = (instance k // n_restarts, restart
    k % n_restarts): per-solve scalars as numpy arrays; the best routes of all
    solves in two flat device tensors (route_off of solve k at
    off_all[off_start[k]:off_start[k+1]], its route_seq at
    seq_all[seq_start[k]:seq_start[k+1]]), and optionally the final routes
    likewise."""

    def __init__(self, n, off_start, seq_start, bufs):
        self.n = n
        self.off_start, self.seq_start = off_start, seq_start
        self.off_all, self.seq_all, self.of_all = bufs["off"], bufs["seq"], bufs["of"]
        self.fin_off_all, self.fin_seq_all = bufs.get("fin_off"), bufs.get("fin_seq")

    def route_off(self, k):
        return self.off_all[int(self.off_start[k]):int(self.off_start[k + 1])]

    def route_seq(self, k):
        return self.seq_all[int(self.seq_start[k]):int(self.seq_start[k + 1])]

    def route_of(self, k):
        return self.of_all[int(self.seq_start[k]):int(self.seq_start[k + 1])]

    def final_off(self, k):
        return self.fin_off_all[int(self.off_start[k]):int(self.off_start[k + 1])]

    def final_seq(self, k):
        return self.fin_seq_all[int(self.seq_start[k]):int(self.seq_start[k + 1])]


def _result_dtype():
    names = [f[0] for f in _Result._fields_]
    kinds = {C.c_void_p: np.uint64, C.c_int64: np.int64, C.c_int32: np.int32, C.c_float: np.float32}
    return np.dtype({"names": names, "formats": [kinds[f[1]] for f in _Result._fields_],
                     "offsets": [getattr(_Result, n).offset for n in names],
                     "itemsize": C.sizeof(_Result)})


def solve_batch_flat(insts, params, n_restarts=1, ws=None, stream=None, final_routes=False,
                     allow_infeasible=False, bufs=None):
    """n instances x n_restarts solves in one call (at_solve_batch) without a
    trace, the result descriptors built as one numpy array: the marshalling of a
    batch of tens of thousands of solves costs milliseconds.  `bufs` (the
    BatchResult of an earlier call on the same instances and restart count)
    reuses its output tensors.  Returns a BatchResult."""
    torch = _torch()
    n = len(insts)
    ia = (_Instance * n)(*[i.c_struct() for i in insts])
    pa = (_Params * n)(*params)
    if any(p.trace for p in params):
        raise AtError(AT_EINVAL, "solve_batch_flat writes no trace")
    nbytes = int(lib().at_workspace_size(n, ia, pa, n_restarts))
    if nbytes == 0:
        _check(AT_EINVAL)
    ws = _workspace(nbytes, ws)
    V = np.repeat(np.array([i.n_vehicles for i in insts], dtype=np.int64), n_restarts)
    M = np.repeat(np.array([i.n_missions for i in insts], dtype=np.int64), n_restarts)
    off_start = np.concatenate([[0], np.cumsum(V + 1)])
    seq_start = np.concatenate([[0], np.cumsum(M)])
    dev = insts[0].travel.device
    if bufs is not None:
        b = dict(off=bufs.off_all, seq=bufs.seq_all, of=bufs.of_all)
        if final_routes:
            b.update(fin_off=bufs.fin_off_all, fin_seq=bufs.fin_seq_all)
    else:
        b = dict(off=torch.empty(int(off_start[-1]), dtype=torch.int32, device=dev),
                 seq=torch.empty(max(1, int(seq_start[-1])), dtype=torch.int32, device=dev),
                 of=torch.empty(max(1, int(seq_start[-1])), dtype=torch.int32, device=dev))
        if final_routes:
            b.update(fin_off=torch.empty_like(b["off"]), fin_seq=torch.empty_like(b["seq"]))
    k = len(V)
    ra = np.zeros(k, dtype=_result_dtype())
    ra["route_off"] = b["off"].data_ptr() + 4 * off_start[:-1].astype(np.uint64)
    ra["route_seq"] = b["seq"].data_ptr() + 4 * seq_start[:-1].astype(np.uint64)
    ra["route_of"] = b["of"].data_ptr() + 4 * seq_start[:-1].astype(np.uint64)
    if final_routes:
        ra["final_off"] = b["fin_off"].data_ptr() + 4 * off_start[:-1].astype(np.uint64)
        ra["final_seq"] = b["fin_seq"].data_ptr() + 4 * seq_start[:-1].astype(np.uint64)
    rc = lib().at_solve_batch(n, ia, pa, n_restarts, _dptr(ws), ws.numel(), _stream_ptr(stream),
                              ra.ctypes.data_as(C.POINTER(_Result)))
    if not (allow_infeasible and rc == AT_EINFEAS):
        _check(rc)
    out = BatchResult(k, off_start, seq_start, b)
    for f in ("best_obj", "final_obj", "iters_done", "best_iter", "status", "search_ms"):
        setattr(out, f, ra[f].copy())
    return out


def debug_eval_moves(inst: DeviceInstance, route_off, route_seq, tabu_until, t, cur, best,
                     variant=AT_TABU, aspiration=True, chunk=0, block=0, schedule=SCHED_AUTO,
                     ws=None, stream=None):
    """Every slot's 64-bit key for a state, as the search kernels compute it (uint64 numpy);
    schedule SCHED_WAVE (or a constrained instance) dumps the wave schedule's evaluation."""
    torch = _torch()
    M, V = inst.n_missions, inst.n_vehicles
    n = M * (M + V) + M * (M - 1) // 2
    pr = make_params(variant, 0, 0, aspiration, 0, False, schedule, 0, block, chunk)
    ci = inst.c_struct()
    nbytes = int(lib().at_workspace_size(1, C.byref(ci), C.byref(pr), 1))
    ws = _workspace(nbytes, ws)
    dev = inst.travel.device
    off = torch.as_tensor(np.asarray(route_off, dtype=np.int32)).to(dev)
    seq = torch.as_tensor(np.asarray(route_seq, dtype=np.int32)).to(dev)
    tab = torch.as_tensor(np.asarray(tabu_until, dtype=np.int32).reshape(-1)).to(dev)
    keys = torch.full((n + 1,), -1, dtype=torch.int64, device=dev)
    _check(lib().at_debug_eval_moves(C.byref(ci), C.byref(pr), _dptr(off), _dptr(seq), _dptr(tab),
                                     int(t), int(cur), int(best), _dptr(keys), _dptr(ws),
                                     ws.numel(), _stream_ptr(stream)))
    k = keys.cpu().numpy().view(np.uint64)
    return k[:n], int(k[n])


class Server:
    """Continuous-batching server (at_server_*)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 64, chunk_iters: int = 50,
                 stream=None):
        L = lib()
        if not hasattr(L, "at_server_create"):
            raise AtError(AT_EINVAL, "the loaded library has no server entry points")
        self._h = C.c_void_p()
        self._pending = {}
        _check(L.at_server_create(int(hbm_budget_bytes), int(max_slots), int(chunk_iters),
                                  _stream_ptr(stream), C.byref(self._h)))

    def submit(self, inst: DeviceInstance, **kw):
        pr = make_params(**kw)
        ticket = C.c_uint64(0)
        ci = inst.c_struct()
        _check(lib().at_server_submit(self._h, C.byref(ci), C.byref(pr), C.byref(ticket)))
        bufs = _alloc_result(inst.n_missions, inst.n_vehicles, pr.max_iters, bool(pr.trace),
                             inst.travel.device)
        # the instance's device arrays are read at admission: keep them alive until polled
        self._pending[ticket.value] = (bufs, inst.n_missions, inst)
        return ticket.value

    def progress(self) -> int:
        n = C.c_int32(0)
        _check(lib().at_server_progress(self._h, C.byref(n)))
        return n.value

    def poll(self, ticket: int):
        bufs, M, _inst = self._pending[ticket]
        res = _c_result(bufs)
        rc = lib().at_server_poll(self._h, C.c_uint64(ticket), C.byref(res))
        if rc == AT_EAGAIN:
            return None
        _check(rc)
        del self._pending[ticket]
        return _finish(bufs, res, M)

    def completed(self, capacity: int = 4096):
        """Tickets of requests that finished since the last call (at_server_completed)."""
        buf = (C.c_uint64 * capacity)()
        n = C.c_int32(0)
        _check(lib().at_server_completed(self._h, buf, int(capacity), C.byref(n)))
        return [int(buf[i]) for i in range(n.value)]

    def close(self):
        if self._h:
            _check(lib().at_server_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
