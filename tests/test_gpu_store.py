"""The single-precision bound store (prop_set_store(p, 32); the
mixed-precision variant of the paper's single-precision runs, Sec. 4.5):
FP64 arithmetic, bounds kept on the grid of zero, the infinities and the
normal singles, rounded outward at the input and at every commit.  Bar:
status, rounds and bounds bitwise those of the oracle's run with the same
store, on every round-loop driver, with marking and a parent; the store can
be switched back and forth on one problem; entry points that do not take it
refuse it."""
import numpy as np
import pytest
from bitwise import differing, same_bits

import oracle
import oracle_pins as pins
import synth

pytestmark = pytest.mark.gpu

LOOPS = ("persistent", "stream", "host", "graph", "graph_all")


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


def say(msg):
    print(msg, flush=True)


def same(tag, got, ref):
    res, lb, ub = got
    assert (res.status, res.rounds) == (ref.status, ref.rounds), (
        f"{tag}: {res.status}/{res.rounds} vs oracle {ref.status}/{ref.rounds}")
    if ref.status == oracle.INFEASIBLE:
        return
    for name, g, r in (("lb", lb, ref.lb), ("ub", ub, ref.ub)):
        bad = differing(g, r)
        assert bad.size == 0, f"{tag}: {name} differs at {bad.size} vars, first {bad[:5]}"


def on_grid(x):
    """Every value is 0, infinite, or a normal single."""
    x = np.asarray(x)
    fin = np.isfinite(x) & (x != 0)
    tiny = float(np.finfo(np.float32).tiny)
    big = float(np.finfo(np.float32).max)
    mag = np.abs(x[fin])
    if not np.all((mag >= tiny) & (mag <= big)):
        return False
    return bool(np.all(x[fin].astype(np.float32).astype(np.float64) == x[fin]))


def params_kw(params):
    if params is None:
        return {}
    return dict(eps_int=params.eps_int, cont_rel_tol=params.cont_rel_tol,
                feas_tol=params.feas_tol)


def check_all_loops(lib, inst, max_rounds=100, params=None, lb=None, ub=None):
    lb = inst.lb if lb is None else lb
    ub = inst.ub if ub is None else ub
    ref = oracle.run(inst, lb, ub, max_rounds, params, store=32)
    say(f"  {inst.name}: oracle (single-precision store) {oracle.STATUS_NAMES[ref.status]} "
        f"after {ref.rounds} rounds")
    with lib.Problem.from_instance(inst, **params_kw(params)) as p:
        p.set_store(32)
        for loop in LOOPS:
            p.set_loop(loop)
            got = p.run(lb, ub, max_rounds)
            same(f"{inst.name}/{loop}", got, ref)
            if ref.status != oracle.INFEASIBLE:
                assert on_grid(got[1]) and on_grid(got[2]), inst.name
    return ref


def test_closed_forms(lib):
    """Every hand-derived case, run with the single-precision store (the
    cases derived for it expect its values; the others must agree with the
    oracle's run under the same store)."""
    for c in pins.load_closed_forms():
        inst = pins.case_instance(c)
        ref = check_all_loops(lib, inst, c["max_rounds"], pins.case_params(c))
        if c.get("store", 64) == 32:
            e = c["expect"]
            assert (ref.status, ref.rounds) == (e["status"], e["rounds"]), c["name"]


@pytest.mark.parametrize("make", [lambda: synth.config0(), lambda: synth.layout_mix(0),
                                  lambda: synth.layout_mix(1), lambda: synth.code_edges(0),
                                  lambda: synth.config1(1)],
                         ids=["config0", "layout_mix0", "layout_mix1", "code_edges0", "config1"])
def test_instances(lib, make):
    """Chunks of every length class, long rows, hot variables, integer codes
    and continuous variables through the single-precision copies."""
    inst = make()
    ref = check_all_loops(lib, inst)
    assert ref.status == oracle.CONVERGED


def test_random_small(lib):
    """Tiny integer, mixed and continuous systems, with infinite bounds, and
    tolerance 0 so that gains smaller than a grid step occur."""
    for s in range(18):
        inst = synth.random_small(4000 + s, m=int(3 + s % 9), n=int(3 + s % 7), box=6,
                                  int_frac=[1.0, 0.5, 0.0][s % 3], inf_frac=0.2 * (s % 2))
        params = oracle.Params(cont_rel_tol=0.0) if s % 2 else None
        check_all_loops(lib, inst, 100, params)


def test_beyond_single_range(lib):
    """Bounds beyond the single-precision range become infinite, bounds below
    its smallest normal number go to zero or to that number, outward."""
    rng = np.random.default_rng(5)
    inst = synth.config0(4)
    lb, ub = inst.lb.copy(), inst.ub.copy()
    cont = np.nonzero(inst.vartype == 0)[0]
    pick = rng.choice(cont, size=40, replace=False)
    lb[pick[:10]] = -1e39
    ub[pick[10:20]] = 5e38
    lb[pick[20:30]] = 1e-40
    ub[pick[20:30]] = np.maximum(ub[pick[20:30]], 1.0)
    ub[pick[30:]] = -1e-41
    lb[pick[30:]] = np.minimum(lb[pick[30:]], -1.0)
    ref = check_all_loops(lib, inst, 100, None, lb, ub)
    assert ref.status in (oracle.CONVERGED, oracle.INFEASIBLE)


def test_marking_parent_and_switching(lib):
    """Marked rounds, a parent fixed point under the same store, and the
    store switched on one problem (captured rounds are redone): each run is
    the oracle's with the store it ran under."""
    import torch

    inst = synth.layout_mix(2)
    ref32 = oracle.run(inst, inst.lb, inst.ub, 100, store=32)
    ref64 = oracle.run(inst, inst.lb, inst.ub, 100)
    assert ref32.status == oracle.CONVERGED
    lbs, ubs = synth.branch_children(ref32.lb, ref32.ub, inst.vartype, 6, 19, 2)
    kids = [oracle.run(inst, lbs[k], ubs[k], 100, store=32) for k in range(6)]
    with lib.Problem.from_instance(inst) as p:
        p.set_loop("graph")
        same("graph/64", p.run(inst.lb, inst.ub, 100), ref64)
        p.set_store(32)
        same("graph/32", p.run(inst.lb, inst.ub, 100), ref32)
        p.set_store(64)
        same("graph/64 again", p.run(inst.lb, inst.ub, 100), ref64)
        p.set_store(32)
        p.set_marking(True)
        dev = torch.device("cuda:0")
        p.set_parent(torch.tensor(ref32.lb, dtype=torch.float64, device=dev),
                     torch.tensor(ref32.ub, dtype=torch.float64, device=dev))
        for loop in ("stream", "graph", "graph_all", "host"):
            p.set_loop(loop)
            for k in range(6):
                same(f"child{k}/marked+parent/{loop}", p.run(lbs[k], ubs[k], 100), kids[k])
            # the parent itself is a fixed point under this store
            res, lb, ub = p.run(ref32.lb, ref32.ub, 100)
            assert (res.status, res.rounds) == (oracle.CONVERGED, 1)
            assert same_bits(lb, ref32.lb) and same_bits(ub, ref32.ub)
        # switching the store clears the parent: a marked run is then a full one
        p.set_store(64)
        p.set_store(32)
        p.set_loop("stream")
        same("child0/marked, parent cleared", p.run(lbs[0], ubs[0], 100), kids[0])


def test_refusals(lib, torch_cuda):
    """Entry points that do not take the single-precision store refuse it;
    invalid stores are refused."""
    torch = torch_cuda
    inst = synth.config0()
    with lib.Problem.from_instance(inst) as p:
        for bad in (0, 16, 33, 128):
            with pytest.raises(lib.PropError) as ei:
                p.set_store(bad)
            assert ei.value.code == lib.EINVAL
        p.set_store(32)
        dev = torch.device("cuda:0")
        d_lb = torch.tensor(np.stack([inst.lb, inst.lb]), dtype=torch.float64, device=dev)
        d_ub = torch.tensor(np.stack([inst.ub, inst.ub]), dtype=torch.float64, device=dev)
        for call in (lambda: p.run_batch(np.stack([inst.lb]), np.stack([inst.ub]), 10),
                     lambda: p.run_batch_device(d_lb, d_ub, 10),
                     lambda: p.run_batch_device(d_lb, d_ub, 10, static=True)):
            with pytest.raises(lib.PropError) as ei:
                call()
            assert ei.value.code == lib.EINVAL
        srv = lib.Server(budget_bytes=1 << 28)
        try:
            with pytest.raises(lib.PropError) as ei:
                srv.add_instance(p)
            assert ei.value.code == lib.EINVAL
        finally:
            srv.close()
        # the problem still runs, and runs batches again with the FP64 store
        same("after refusals", p.run(inst.lb, inst.ub, 100),
             oracle.run(inst, inst.lb, inst.ub, 100, store=32))
        p.set_store(64)
        res = p.run_batch_device(d_lb, d_ub, 100)
        ref = oracle.run(inst, inst.lb, inst.ub, 100)
        assert all((r.status, r.rounds) == (ref.status, ref.rounds) for r in res)
    with lib.Problem.from_instance(inst, layout=1) as p:
        with pytest.raises(lib.PropError) as ei:
            p.set_store(32)
        assert ei.value.code == lib.EINVAL
