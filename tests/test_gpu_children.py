"""Marked rounds seeded from a parent fixed point (branch-and-bound children,
the paper's outlook in Sec. 5 with the marking of Algorithm 1): the
children's single and batched runs with marked rounds and a parent are
bitwise the unmarked runs, which are bitwise the oracle's, whatever the
round-loop driver; batches compact as children finish."""
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


def say(msg):
    print(msg, flush=True)


def same(tag, res, lb, ub, ref):
    assert (res.status, res.rounds) == (ref.status, ref.rounds), (
        f"{tag}: {res.status}/{res.rounds} vs oracle {ref.status}/{ref.rounds}")
    if ref.status != oracle.INFEASIBLE:
        assert same_bits(lb, ref.lb) and same_bits(ub, ref.ub), tag


CASES = [("config0", lambda: synth.config0(), 8, 1),
         ("layout_mix", lambda: synth.layout_mix(0), 6, 2),
         ("code_edges", lambda: synth.code_edges(1), 6, 3)]


def _setup(lib, torch, inst, count, per_child, seed):
    parent = oracle.run(inst, inst.lb, inst.ub, 100)
    assert parent.status == oracle.CONVERGED
    lbs, ubs = synth.branch_children(parent.lb, parent.ub, inst.vartype, count, seed, per_child)
    refs = [oracle.run(inst, lbs[k], ubs[k], 100) for k in range(count)]
    dev = torch.device("cuda:0")
    d_plb = torch.tensor(parent.lb, dtype=torch.float64, device=dev)
    d_pub = torch.tensor(parent.ub, dtype=torch.float64, device=dev)
    return parent, lbs, ubs, refs, d_plb, d_pub


@pytest.mark.parametrize("name,make,count,per_child", CASES)
def test_children_single_runs(lib, torch_cuda, name, make, count, per_child):
    inst = make()
    parent, lbs, ubs, refs, d_plb, d_pub = _setup(lib, torch_cuda, inst, count, per_child, 61)
    say(f"{inst.name}: parent {parent.rounds} rounds; children statuses "
        f"{sorted({oracle.STATUS_NAMES[r.status] for r in refs})}, rounds "
        f"{[r.rounds for r in refs]}")
    with lib.Problem.from_instance(inst) as p:
        # the GPU's own root run is the same fixed point
        res, lb, ub = p.run(inst.lb, inst.ub, 100)
        same(f"{inst.name}/root", res, lb, ub, parent)
        for k in range(count):
            res, lb, ub = p.run(lbs[k], ubs[k], 100)
            same(f"{inst.name}/child{k}/unmarked", res, lb, ub, refs[k])
        p.set_marking(True)
        p.set_parent(d_plb, d_pub)
        for loop in ("stream", "graph", "graph_all", "host"):
            p.set_loop(loop)
            for k in range(count):
                res, lb, ub = p.run(lbs[k], ubs[k], 100)
                same(f"{inst.name}/child{k}/marked+parent/{loop}", res, lb, ub, refs[k])
        # the parent itself: round 1 processes no row and nothing changes
        p.set_loop("stream")
        res, lb, ub = p.run(parent.lb, parent.ub, 100)
        assert (res.status, res.rounds) == (oracle.CONVERGED, 1)
        assert same_bits(lb, parent.lb) and same_bits(ub, parent.ub)
        # persistent driver: parent and marking ignored, same results
        p.set_loop("persistent")
        res, lb, ub = p.run(lbs[0], ubs[0], 100)
        same(f"{inst.name}/child0/persistent", res, lb, ub, refs[0])
        p.set_loop("stream")
        p.set_parent(None, None)
        for k in range(count):
            res, lb, ub = p.run(lbs[k], ubs[k], 100)
            same(f"{inst.name}/child{k}/marked", res, lb, ub, refs[k])


@pytest.mark.parametrize("name,make,count,per_child", CASES)
def test_children_batches(lib, torch_cuda, name, make, count, per_child):
    torch = torch_cuda
    inst = make()
    # three groups of 8 children: nodes finish at different rounds, so the
    # batch compacts, after which every group processes every row once
    count = 24
    parent, lbs, ubs, refs, d_plb, d_pub = _setup(lib, torch, inst, count, per_child, 73)
    dev = torch.device("cuda:0")
    with lib.Problem.from_instance(inst) as p:
        for marking, parent_set, loop in ((False, False, "stream"), (True, True, "stream"),
                                          (True, True, "graph"), (True, False, "stream")):
            p.set_marking(marking)
            p.set_parent(d_plb, d_pub) if parent_set else p.set_parent(None, None)
            p.set_loop(loop)
            d_lb = torch.tensor(lbs, dtype=torch.float64, device=dev)
            d_ub = torch.tensor(ubs, dtype=torch.float64, device=dev)
            res = p.run_batch_device(d_lb, d_ub, 100)
            torch.cuda.synchronize()
            lb, ub = d_lb.cpu().numpy(), d_ub.cpu().numpy()
            tag = f"{inst.name}/batch marking={marking} parent={parent_set} {loop}"
            say(f"  {tag}")
            for k in range(count):
                same(f"{tag}/node{k}", res[k], lb[k], ub[k], refs[k])


def test_parent_rejects_invalid_bounds(lib, torch_cuda):
    torch = torch_cuda
    inst = synth.config0()
    with lib.Problem.from_instance(inst) as p:
        bad = torch.tensor(inst.lb, dtype=torch.float64, device="cuda:0")
        bad[3] = float("nan")
        ub = torch.tensor(inst.ub, dtype=torch.float64, device="cuda:0")
        with pytest.raises(lib.PropError) as ei:
            p.set_parent(bad, ub)
        assert ei.value.code == lib.EINVAL
        # the parent stays cleared: a marked run processes every row
        p.set_marking(True)
        ref = oracle.run(inst, inst.lb, inst.ub, 100)
        res, lb, ub2 = p.run(inst.lb, inst.ub, 100)
        same("config0/after-bad-parent", res, lb, ub2, ref)
