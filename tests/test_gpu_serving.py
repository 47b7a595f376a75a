"""Serving with continuous batching: every request's result is the same alone,
inside a mix of other requests, and under any chunking of its iterations, and
admission respects the memory budget and the slot count."""
import numpy as np
import pytest

from gen.instances import make_instance, serve_specs
from helpers import assert_same_result, gpu_to_np, oracle_solve

pytestmark = pytest.mark.gpu

at = pytest.importorskip("paper_2002_11710_amd")


def _dev(inst):
    return at.DeviceInstance.from_instance(inst)


def _drive(srv, tickets, limit=200000):
    out = {}
    for _ in range(limit):
        srv.progress()
        for t in list(tickets):
            r = srv.poll(t)
            if r is not None:
                out[t] = r
                tickets.remove(t)
        if not tickets:
            return out
    raise AssertionError("serving did not finish")


def _requests():
    reqs = []
    for k, (F, B, V, M) in enumerate(((30, 2, 3, 20), (60, 3, 5, 40), (90, 4, 8, 70), (20, 2, 2, 10),
                                      (150, 5, 10, 120), (45, 2, 4, 30))):
        inst = make_instance(300 + k, F, B, V, M)
        reqs.append((inst, dict(variant=at.AT_TABU if k % 3 else at.AT_NS, tenure=5 + k,
                                iters=150 + 10 * k, restart_seed=k * 31, trace=True)))
    return reqs


def _same(a, b, label):
    a, b = gpu_to_np(a), gpu_to_np(b)
    for k in ("best_obj", "final_obj", "iters_done", "best_iter", "status"):
        assert a[k] == b[k], (label, k, a[k], b[k])
    for k in ("route_off", "route_seq", "route_of", "final_off", "final_seq", "tr_move", "tr_delta",
              "tr_obj", "tr_flags"):
        assert np.array_equal(a[k], b[k]), (label, k)


@pytest.mark.parametrize("chunk", [1, 7, 64])
def test_mix_equals_alone(chunk):
    reqs = _requests()
    devs = [_dev(i) for i, _ in reqs]
    alone = [at.solve(d, **kw) for d, (_, kw) in zip(devs, reqs)]
    srv = at.Server(1 << 30, max_slots=4, chunk_iters=chunk)
    tickets = [srv.submit(d, **kw) for d, (_, kw) in zip(devs, reqs)]
    got = _drive(srv, list(tickets))
    for k, t in enumerate(tickets):
        _same(alone[k], got[t], f"request {k} chunk {chunk}")
    srv.close()


def test_mix_matches_oracle():
    reqs = _requests()[:3]
    srv = at.Server(1 << 28, max_slots=8, chunk_iters=13)
    tickets = [srv.submit(_dev(i), **kw) for i, kw in reqs]
    got = _drive(srv, list(tickets))
    for (inst, kw), t in zip(reqs, tickets):
        _, o = oracle_solve(inst, variant=kw["variant"], tenure=kw["tenure"], iters=kw["iters"],
                            restart_seed=kw["restart_seed"])
        assert_same_result(o, got[t], "served vs oracle")
    srv.close()


def test_budget_admission_and_late_arrivals():
    reqs = _requests()
    devs = [_dev(i) for i, _ in reqs]
    alone = [at.solve(d, **kw) for d, (_, kw) in zip(devs, reqs)]
    # two slots: the others wait until a resident solve finishes
    srv = at.Server(6 << 20, max_slots=2, chunk_iters=20)
    tickets = [srv.submit(devs[0], **reqs[0][1]), srv.submit(devs[1], **reqs[1][1])]
    got = {}
    srv.progress()
    # later arrivals join while the first ones are resident
    for k in range(2, len(reqs)):
        tickets.append(srv.submit(devs[k], **reqs[k][1]))
        srv.progress()
        for t in list(tickets):
            if t not in got:
                r = srv.poll(t)
                if r is not None:
                    got[t] = r
    rest = [t for t in tickets if t not in got]
    got.update(_drive(srv, rest))
    for k, t in enumerate(tickets):
        _same(alone[k], got[t], f"budgeted request {k}")
    srv.close()


def test_oversized_request_rejected():
    inst = make_instance(9, 1500, 25, 50, 1000)      # its compact travel block alone exceeds 4 MB
    srv = at.Server(2 << 20, max_slots=4, chunk_iters=10)
    with pytest.raises(at.AtError) as e:
        srv.submit(_dev(inst), iters=100, tenure=5)
    assert e.value.code == at.AT_ENOMEM
    srv.close()


def test_serving_stream_sample():
    """A few requests of the serving stream's size law, one of them large
    enough for the HBM-resident schedule."""
    specs = serve_specs(40)
    pick = sorted(specs, key=lambda s: s["n_missions"])
    chosen = [pick[0], pick[len(pick) // 2], pick[-1]]
    from gen.instances import make_instance as mk
    insts = [mk(s["seed"], s["n_fac"], s["n_bases"], s["n_vehicles"], s["n_missions"]) for s in chosen]
    devs = [_dev(i) for i in insts]
    kw = dict(tenure=15, iters=60, trace=True)
    alone = [at.solve(d, **kw) for d in devs]
    srv = at.Server(8 << 30, max_slots=16, chunk_iters=25)
    tickets = [srv.submit(d, **kw) for d in devs]
    got = _drive(srv, list(tickets))
    for k, t in enumerate(tickets):
        _same(alone[k], got[t], f"stream request M={chosen[k]['n_missions']}")
    srv.close()


def test_mix_with_hbm_resident_requests():
    """Requests too large for one workgroup's LDS (HBM-resident schedule, sharing
    one cooperative launch with per-request workgroup ranges) next to small
    ones: each result equals the request alone, under two chunkings."""
    big = [make_instance(400 + k, 750, 13, 25, 500) for k in range(2)]
    reqs = [(i, dict(variant=at.AT_TABU, tenure=9, iters=60, restart_seed=0, trace=True)) for i in big]
    reqs += _requests()[:3]
    devs = [_dev(i) for i, _ in reqs]
    alone = [at.solve(d, **kw) for d, (_, kw) in zip(devs, reqs)]
    for chunk in (5, 64):
        srv = at.Server(1 << 30, max_slots=8, chunk_iters=chunk)
        tickets = [srv.submit(d, **kw) for d, (_, kw) in zip(devs, reqs)]
        got = _drive(srv, list(tickets))
        for k, t in enumerate(tickets):
            _same(alone[k], got[t], f"request {k} chunk {chunk}")
        srv.close()
    _, o = oracle_solve(big[0], tenure=9, iters=60)
    assert_same_result(o, alone[0], "large request alone vs oracle")


def test_admission_batch_over_one_scatter_round():
    """300 requests admitted at once: more than one round of the admission
    scatter (256 requests) places their records.  Every request finishes, a
    sample equals the solve alone and two equal the oracle."""
    insts = [make_instance(900 + k, 12, 2, 2, 8 + k % 7) for k in range(300)]
    devs = [_dev(i) for i in insts]
    srv = at.Server(1 << 30, max_slots=320, chunk_iters=20)
    tickets = [srv.submit(d, tenure=3, iters=20, trace=True) for d in devs]
    got = _drive(srv, list(tickets))
    srv.close()
    for k in range(0, 300, 10):
        alone = at.solve(devs[k], tenure=3, iters=20, trace=True)
        _same(alone, got[tickets[k]], f"request {k} of 300")
    for k in (0, 299):
        _, o = oracle_solve(insts[k], tenure=3, iters=20)
        assert_same_result(o, got[tickets[k]], f"request {k} of 300 vs oracle")


def test_completed_lists_each_finished_ticket_once():
    """at_server_completed: every request appears once, only after it is done,
    and its poll then succeeds; a ticket polled before it is listed is not
    listed afterwards."""
    reqs = _requests()
    devs = [_dev(i) for i, _ in reqs]
    alone = [at.solve(d, **kw) for d, (_, kw) in zip(devs, reqs)]
    srv = at.Server(1 << 30, max_slots=3, chunk_iters=40)
    tickets = [srv.submit(d, **kw) for d, (_, kw) in zip(devs, reqs)]
    early = tickets[0]
    seen, got = [], {}
    for _ in range(200000):
        srv.progress()
        if early not in got:
            r = srv.poll(early)          # polled directly, without the list
            if r is not None:
                got[early] = r
        for t in srv.completed(capacity=2):
            assert t not in seen and t != early
            seen.append(t)
            r = srv.poll(t)
            assert r is not None
            got[t] = r
        if len(got) == len(tickets):
            break
    assert sorted(seen) == sorted(tickets[1:])
    assert srv.completed() == []
    for k, t in enumerate(tickets):
        _same(alone[k], got[t], f"request {k}")
    srv.close()


def test_mixed_tabu_widths_resume_in_chunks():
    """Resident solves of two tabu-entry widths (one budget above 2^16
    iterations) cannot share one grid: each launch then runs chunk_iters
    iterations of every solve, which resume from their saved state; every
    result equals the request alone."""
    reqs = _requests()[:4]
    reqs.append((make_instance(377, 20, 2, 2, 12), dict(variant=at.AT_TABU, tenure=6, iters=70000,
                                                         restart_seed=5, trace=True)))
    devs = [_dev(i) for i, _ in reqs]
    alone = [at.solve(d, **kw) for d, (_, kw) in zip(devs, reqs)]
    srv = at.Server(1 << 30, max_slots=8, chunk_iters=9)
    tickets = [srv.submit(d, **kw) for d, (_, kw) in zip(devs, reqs)]
    got = _drive(srv, list(tickets))
    for k, t in enumerate(tickets):
        _same(alone[k], got[t], f"request {k}")
    srv.close()


def test_many_short_hbm_resident_requests_share_the_queue():
    """Hundreds of short requests too large for one workgroup's LDS (HBM-resident)
    beside a long one: a launch cannot give each its own workgroups, so the short
    ones run to their end on the workers' queue while the long one keeps its own
    workgroups over several launches; every result equals the request alone, and
    two equal the oracle's."""
    big = make_instance(901, 1350, 23, 45, 900)
    reqs = [(big, dict(variant=at.AT_TABU, tenure=11, iters=200, restart_seed=3, trace=True))]
    for k in range(260):
        # 100 vehicles: the tabu table alone takes 60 KB of LDS, so the solve is HBM-resident
        inst = make_instance(5000 + k, 450, 10, 100, 300)
        reqs.append((inst, dict(variant=at.AT_TABU if k % 4 else at.AT_NS, tenure=7, iters=30,
                                restart_seed=k, trace=True)))
    devs = [_dev(i) for i, _ in reqs]
    alone = [at.solve(d, **kw) for d, (_, kw) in zip(devs, reqs)]
    srv = at.Server(8 << 30, max_slots=512, chunk_iters=25)
    tickets = [srv.submit(d, **kw) for d, (_, kw) in zip(devs, reqs)]
    got = _drive(srv, list(tickets))
    for k, t in enumerate(tickets):
        _same(alone[k], got[t], f"request {k}")
    srv.close()
    for k in (1, 2):
        inst, kw = reqs[k]
        _, o = oracle_solve(inst, variant=kw["variant"], tenure=kw["tenure"], iters=kw["iters"],
                            restart_seed=kw["restart_seed"])
        assert_same_result(o, alone[k], f"short HBM-resident request {k} vs oracle")
