"""A seeded sweep over the options of a single run: power-law matrices of
three sizes, root and node bounds, every layout step count, both layouts,
both bound stores, marked and unmarked rounds, every round-loop driver.
Each run is compared bit for bit with the oracle's run under the same
store (status, rounds, bounds)."""
import itertools

import pytest
from bitwise import differing

import oracle
import synth

pytestmark = pytest.mark.gpu

LOOPS = ("stream", "graph", "graph_all", "host", "persistent")
SIZES = (3_000, 12_000, 40_000)


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
def matrices():
    return {m: synth.config3_matrix(m, m // 2) for m in SIZES}


def cases():
    out = []
    combos = itertools.product(SIZES, (4, 8, 16), (0, 1), (64, 32), (False, True))
    for q, (m, steps, layout, store, marking) in enumerate(combos):
        if layout == 1 and store == 32:
            continue  # the nnz-split layout keeps the FP64 store
        out.append((q, m, steps, layout, store, marking))
    return out


@pytest.mark.parametrize("q,m,steps,layout,store,marking", cases(),
                         ids=lambda v: str(v))
def test_sweep(lib, matrices, q, m, steps, layout, store, marking):
    inst = matrices[m]
    if q % 3 == 0:
        lb, ub = inst.lb, inst.ub
    else:
        lb, ub = synth.node_bounds(inst, 90_000 + q, frac_hi=0.08, only_int=q % 2 == 0)
    ref = oracle.run(inst, lb, ub, 100, store=store)
    loop = LOOPS[q % len(LOOPS)]
    print(f"case {q}: m={m} steps={steps} layout={layout} store={store} marking={marking} "
          f"loop={loop}: oracle {oracle.STATUS_NAMES[ref.status]} after {ref.rounds} rounds",
          flush=True)
    with lib.Problem.from_instance(inst, steps=steps, layout=layout) as p:
        p.set_store(store)
        p.set_marking(marking)
        p.set_loop(loop)
        res, glb, gub = p.run(lb, ub, 100)
        assert (res.status, res.rounds) == (ref.status, ref.rounds)
        if ref.status != oracle.INFEASIBLE:
            for name, g, r in (("lb", glb, ref.lb), ("ub", gub, ref.ub)):
                bad = differing(g, r)
                assert bad.size == 0, f"{name} differs at {bad.size} variables, first {bad[:5]}"
        # a round limit inside the run, on the next driver
        p.set_loop(LOOPS[(q + 1) % len(LOOPS)])
        k = max(1, ref.rounds // 2)
        part = oracle.run(inst, lb, ub, k, store=store)
        res2, lb2, ub2 = p.run(lb, ub, k)
        assert (res2.status, res2.rounds) == (part.status, part.rounds)
        if part.status != oracle.INFEASIBLE:
            assert differing(lb2, part.lb).size == 0 and differing(ub2, part.ub).size == 0
