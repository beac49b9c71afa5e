"""Serving on the GPU: every request's status, rounds and bounds must be
bitwise those of the same request run alone (prop_run on the same problem),
whatever else shares its problem's slots, under a budget small enough to
force queueing, slot reuse and reclaiming idle slot groups."""
import sys
import time

import numpy as np
import pytest
from bitwise import same_bits

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module")
def lib(torch_cuda):
    from paper_2009_07785_amd import binding

    return binding


@pytest.fixture(scope="module")
def pool(lib):
    insts = synth.config4_pool(count=6, scale=0.004)
    probs = [lib.Problem.from_instance(i) for i in insts]
    yield insts, probs
    for p in probs:
        p.close()


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def group_bytes(n):
    return 8 * 48 * max(n, 1)


def make_requests(insts, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for q in range(count):
        k = int(rng.integers(0, len(insts)))
        inst = insts[k]
        lb, ub = synth.request_bounds(inst, 50_000 + 97 * seed + q)
        max_rounds = int(rng.choice([1, 3, 100, 100, 100]))
        reqs.append((k, lb, ub, max_rounds))
    return reqs


def check_alone(probs, reqs, results):
    statuses = set()
    for (k, lb, ub, mr), (res, glb, gub) in zip(reqs, results):
        r1, lb1, ub1 = probs[k].run(lb, ub, mr)
        assert (res.status, res.rounds) == (r1.status, r1.rounds), (k, mr)
        statuses.add(r1.status)
        if r1.status != oracle.INFEASIBLE:
            assert same_bits(glb, lb1) and same_bits(gub, ub1), (k, mr)
    return statuses


def test_serving_burst_matches_alone(lib, pool):
    insts, probs = pool
    ns = [i.n for i in insts]
    say(f"pool n = {ns}, nnz = {[i.nnz for i in insts]}")
    reqs = make_requests(insts, 120, 1)
    # special requests: the root, a zero round limit, an empty input domain
    k0 = int(np.argmin(ns))
    inst = insts[k0]
    reqs.append((k0, inst.lb, inst.ub, 100))
    reqs.append((k0, inst.lb, inst.ub, 0))
    ivar = int(np.nonzero(inst.vartype == 1)[0][0])
    lb, ub = inst.lb.copy(), inst.ub.copy()
    lb[ivar], ub[ivar] = 3.0, 2.0
    reqs.append((k0, lb, ub, 100))
    # room for every problem's state plus two slot groups of the largest
    budget = 6 * (1 << 20) + 2 * group_bytes(max(ns))
    with lib.Server(budget, max_slots=16) as srv:
        ids = [srv.add_instance(p) for p in probs]
        assert ids == list(range(len(probs)))
        tickets = [srv.submit(k, lb, ub, mr) for k, lb, ub, mr in reqs]
        results = [srv.wait(t, ns[k], timeout_ms=60_000) for t, (k, *_) in zip(tickets, reqs)]
        assert all(r is not None for r in results)
        st = srv.stats()
    say(f"stats: {st}")
    assert st["completed"] == len(reqs) and st["queued"] == 0 and st["running"] == 0
    assert st["peak_device_bytes"] <= budget
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    statuses = check_alone(probs, reqs, results)
    assert {oracle.CONVERGED, oracle.INFEASIBLE, oracle.MAX_ROUNDS} <= statuses
    assert results[-2][0].status == oracle.MAX_ROUNDS and results[-2][0].rounds == 0
    assert results[-1][0].status == oracle.INFEASIBLE and results[-1][0].rounds == 0


def test_serving_staggered_arrivals(lib, pool):
    """Requests arrive while others run: they join running slot groups at
    round boundaries."""
    insts, probs = pool
    ns = [i.n for i in insts]
    reqs = make_requests(insts, 150, 2)
    budget = 1 << 30
    with lib.Server(budget, max_slots=64, rounds_per_step=1) as srv:
        for p in probs:
            srv.add_instance(p)
        tickets = []
        for q, (k, lb, ub, mr) in enumerate(reqs):
            tickets.append(srv.submit(k, lb, ub, mr))
            if q % 10 == 9:
                time.sleep(0.002)
        results = [srv.wait(t, ns[k], timeout_ms=60_000) for t, (k, *_) in zip(tickets, reqs)]
        st = srv.stats()
    assert all(r is not None for r in results)
    assert st["completed"] == len(reqs)
    check_alone(probs, reqs, results)


@pytest.mark.parametrize("rounds_per_step", [1, 3])
def test_serving_marked_matches_alone(lib, pool, rounds_per_step):
    """Marked rounds per group of slots: requests join running groups (each
    join forces its group's next round over every row), finish at different
    rounds and leave; every result stays bitwise that of the request run
    alone without marking, and the oracle's on a sample."""
    insts, probs = pool
    ns = [i.n for i in insts]
    reqs = make_requests(insts, 160, 3 + rounds_per_step)
    with lib.Server(1 << 30, max_slots=32, rounds_per_step=rounds_per_step,
                    marking=True) as srv:
        for p in probs:
            srv.add_instance(p)
        tickets = []
        for q, (k, lb, ub, mr) in enumerate(reqs):
            tickets.append(srv.submit(k, lb, ub, mr))
            if q % 7 == 6:
                time.sleep(0.002)
        results = [srv.wait(t, ns[k], timeout_ms=60_000) for t, (k, *_) in zip(tickets, reqs)]
        st = srv.stats()
    assert all(r is not None for r in results)
    assert st["completed"] == len(reqs)
    statuses = check_alone(probs, reqs, results)
    assert oracle.CONVERGED in statuses
    for (k, lb, ub, mr), (res, glb, gub) in list(zip(reqs, results))[:12]:
        ref = oracle.run(insts[k], lb, ub, mr)
        assert (res.status, res.rounds) == (ref.status, ref.rounds)
        if ref.status != oracle.INFEASIBLE:
            assert same_bits(glb, ref.lb) and same_bits(gub, ref.ub)


def test_serving_against_oracle(lib, pool):
    insts, probs = pool
    order = np.argsort([i.nnz for i in insts])[:2]
    reqs = []
    for k in order:
        for q in range(4):
            lb, ub = synth.request_bounds(insts[k], 70_000 + q)
            reqs.append((int(k), lb, ub, 100))
    with lib.Server(1 << 28, max_slots=8) as srv:
        for p in probs:
            srv.add_instance(p)
        tickets = [srv.submit(k, lb, ub, mr) for k, lb, ub, mr in reqs]
        for t, (k, lb, ub, mr) in zip(tickets, reqs):
            res, glb, gub = srv.wait(t, insts[k].n, timeout_ms=60_000)
            ref = oracle.run(insts[k], lb, ub, mr)
            assert (res.status, res.rounds) == (ref.status, ref.rounds)
            if ref.status != oracle.INFEASIBLE:
                assert same_bits(glb, ref.lb) and same_bits(gub, ref.ub)


def test_serving_errors_and_budget(lib, pool):
    insts, probs = pool
    k = int(np.argmax([i.n for i in insts]))
    inst, p = insts[k], probs[k]
    # per-problem state does not fit
    with lib.Server(1024) as srv:
        with pytest.raises(lib.PropError) as e:
            srv.add_instance(p)
        assert e.value.code == lib.ENOMEM
    # state fits, one slot group never does
    with lib.Server(group_bytes(inst.n) - 1, max_slots=8) as srv:
        i = srv.add_instance(p)
        with pytest.raises(lib.PropError) as e:
            srv.submit(i, inst.lb, inst.ub, 10)
        assert e.value.code == lib.ENOMEM
    with lib.Server(1 << 28, max_pending=2) as srv:
        i = srv.add_instance(p)
        bad = inst.lb.copy()
        bad[0] = np.nan
        with pytest.raises(lib.PropError) as e:
            srv.submit(i, bad, inst.ub, 10)
        assert e.value.code == lib.EINVAL
        with pytest.raises(lib.PropError) as e:
            srv.submit(7, inst.lb, inst.ub, 10)
        assert e.value.code == lib.EINVAL
        t1 = srv.submit(i, inst.lb, inst.ub, 100)
        t2 = srv.submit(i, inst.lb, inst.ub, 100)
        with pytest.raises(lib.PropError) as e:
            srv.submit(i, inst.lb, inst.ub, 100)
        assert e.value.code == lib.EBUSY
        a = srv.wait(t1, inst.n, timeout_ms=60_000)
        b = srv.wait(t2, inst.n, timeout_ms=60_000)
        assert a[0] == b[0] and same_bits(a[1], b[1]) and same_bits(a[2], b[2])
        with pytest.raises(lib.PropError):
            srv.poll(t1, inst.n)  # released
        t3 = srv.submit(i, inst.lb, inst.ub, 100)  # room again
        assert srv.wait(t3, inst.n, timeout_ms=60_000) is not None


def test_serving_completion_list_overflow(lib, pool):
    """More requests finish in one round than a step's completion list holds
    (512): the rest are reported in later rounds, none is lost or repeated."""
    insts, probs = pool
    k = int(np.argmin([i.n for i in insts]))
    inst = insts[k]
    with lib.Server(1 << 30, max_slots=1024, rounds_per_step=1) as srv:
        i = srv.add_instance(probs[k])
        # a zero round limit finishes every request at its start
        tickets = [srv.submit(i, inst.lb, inst.ub, 0) for _ in range(700)]
        tickets += [srv.submit(i, inst.lb, inst.ub, 1) for _ in range(300)]
        res = [srv.wait(t, inst.n, timeout_ms=60_000) for t in tickets]
        st = srv.stats()
    assert all(r is not None for r in res)
    assert [r[0].rounds for r in res] == [0] * 700 + [1] * 300
    assert all(r[0].status == oracle.MAX_ROUNDS for r in res[:700])
    assert st["completed"] == 1000 and st["running"] == 0
    ref = probs[k].run(inst.lb, inst.ub, 1)
    for r in res[700:]:
        assert (r[0].status, r[0].rounds) == (ref[0].status, ref[0].rounds)
        assert same_bits(r[1], ref[1]) and same_bits(r[2], ref[2])
