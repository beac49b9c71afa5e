"""Exactly rounded activities on the GPU (Def. 1, read as the exact sum of
the products rounded once): rows whose sums sit on or next to a rounding
boundary, or cancel to a small remainder, through every lanes-per-row
class, long-row segments, every round-loop driver, batches (node-parallel
lanes and the few-node loop) and the serving engine.  Every result must be
bitwise the oracle's."""
import numpy as np
import pytest
from bitwise import differing, same_bits

import oracle
import synth

pytestmark = pytest.mark.gpu

LOOPS = ("stream", "persistent", "host", "graph", "graph_all")
# every chunk layout, and the nnz-split waves
LAYOUTS = (dict(steps=4), dict(steps=8), dict(steps=16), dict(layout=1))


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
    assert (res.status, res.rounds) == (ref.status, ref.rounds), (tag, res.status, res.rounds,
                                                                  ref.status, ref.rounds)
    if ref.status == oracle.INFEASIBLE:
        return
    bad_l = differing(lb, ref.lb)
    bad_u = differing(ub, ref.ub)
    assert bad_l.size == 0 and bad_u.size == 0, (tag, bad_l[:5], bad_u[:5])


def test_counterexample_row(lib):
    """x1 + x2 + x3 <= 2^53 + 4, l = (2^53, 1, 2^-60): u = (2^53 + 2, 3, 2)."""
    two53 = 2.0**53
    inst = synth.from_rows([[(0, 1.0), (1, 1.0), (2, 1.0)]], [-np.inf], [two53 + 4],
                           [two53, 1.0, 2.0**-60], [np.inf] * 3, [0, 0, 0], n=3)
    ref = oracle.run(inst, inst.lb, inst.ub, 100)
    assert same_bits(ref.ub, [two53 + 2, 3.0, 2.0])
    for kw in LAYOUTS:
        with lib.Problem.from_instance(inst, **kw) as p:
            for loop in LOOPS:
                p.set_loop(loop)
                res, lb, ub = p.run(inst.lb, inst.ub, 100)
                same(f"{kw} {loop}", res, lb, ub, ref)


@pytest.mark.parametrize("seed,tiny", [(0, False), (1, False), (2, True)])
def test_hard_sums_all_layouts(lib, seed, tiny):
    inst = synth.hard_sums(seed, tiny=tiny)
    ref = oracle.run(inst, inst.lb, inst.ub, 100)
    say(f"  {inst.name}: oracle {oracle.STATUS_NAMES[ref.status]} after {ref.rounds} rounds, "
        f"{int(np.sum(ref.ub != inst.ub))} upper bounds tightened")
    assert ref.status == oracle.CONVERGED
    for kw in LAYOUTS:
        with lib.Problem.from_instance(inst, **kw) as p:
            for loop in LOOPS:
                p.set_loop(loop)
                say(f"  {inst.name} {kw} loop={loop}")
                res, lb, ub = p.run(inst.lb, inst.ub, 100)
                same(f"{inst.name} {kw} {loop}", res, lb, ub, ref)


@pytest.mark.parametrize("nodes", [1, 2, 3, 8, 11])
def test_hard_sums_batched(lib, torch_cuda, nodes):
    """1-2 active nodes run the single-run shape per node, 3+ node-parallel
    lanes; node k gets the root bounds, or, for odd k, a copy with the
    padding variables' upper bounds halved (a different sum for some rows)."""
    torch = torch_cuda
    inst = synth.hard_sums(3, tiny=(nodes == 11))
    lbs = np.stack([inst.lb] * nodes)
    ubs = np.stack([inst.ub] * nodes)
    pad = (inst.lb == 0.0) & (inst.ub == 1.0)
    for k in range(1, nodes, 2):
        ubs[k, pad] = 0.5
    refs = [oracle.run(inst, lbs[k], ubs[k], 100) for k in range(nodes)]
    for steps in (4, 16):
        with lib.Problem.from_instance(inst, steps=steps) as p:
            for loop in ("stream", "graph"):
                p.set_loop(loop)
                say(f"  batch of {nodes} steps={steps} loop={loop}")
                d_lb = torch.tensor(lbs, dtype=torch.float64, device="cuda")
                d_ub = torch.tensor(ubs, dtype=torch.float64, device="cuda")
                res = p.run_batch_device(d_lb, d_ub, 100)
                glb, gub = d_lb.cpu().numpy(), d_ub.cpu().numpy()
                for k in range(nodes):
                    same(f"node {k}", res[k], glb[k], gub[k], refs[k])


def test_hard_sums_serving(lib):
    inst = synth.hard_sums(4)
    ref = oracle.run(inst, inst.lb, inst.ub, 50)
    with lib.Problem.from_instance(inst) as p:
        with lib.Server(1 << 30, max_slots=16) as srv:
            srv.add_instance(p)
            tickets = [srv.submit(0, inst.lb, inst.ub, 50) for _ in range(5)]
            for t in tickets:
                res, lb, ub = srv.wait(t, inst.n, timeout_ms=60_000)
                same("serving", res, lb, ub, ref)
