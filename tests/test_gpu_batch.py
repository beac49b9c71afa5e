"""Batched nodes on the GPU: every node of a batch must give bitwise the
status, rounds and bounds of its own single run (and therefore of the
oracle, checked directly on the smaller cases)."""
import hashlib
import json
import os

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


def node_set(inst, count, seed0, frac_hi=0.05, only_int=True):
    lbs = np.empty((count, inst.n))
    ubs = np.empty((count, inst.n))
    for k in range(count):
        lbs[k], ubs[k] = synth.node_bounds(inst, seed0 + k, frac_hi=frac_hi, only_int=only_int)
    return lbs, ubs


def run_batch(torch, p, lbs, ubs, max_rounds=100):
    d_lb = torch.tensor(lbs, dtype=torch.float64, device="cuda")
    d_ub = torch.tensor(ubs, dtype=torch.float64, device="cuda")
    res = p.run_batch_device(d_lb, d_ub, max_rounds)
    return res, d_lb.cpu().numpy(), d_ub.cpu().numpy()


def check_batch_vs_single(torch, lib, inst, lbs, ubs, max_rounds=100, with_oracle=False):
    with lib.Problem.from_instance(inst) as p:
        res, blb, bub = run_batch(torch, p, lbs, ubs, max_rounds)
        # the graph drivers replay captured rounds (graph-all: every replay
        # queued up front, no compaction): the same results, twice each
        for loop in ("graph", "graph_all"):
            p.set_loop(loop)
            for _ in range(2):
                gres, glb, gub = run_batch(torch, p, lbs, ubs, max_rounds)
                assert [(r.status, r.rounds) for r in gres] == [(r.status, r.rounds) for r in res]
                assert same_bits(glb, blb) and same_bits(gub, bub)
        p.set_loop("stream")
        statuses = set()
        for k in range(lbs.shape[0]):
            r1, lb1, ub1 = p.run(lbs[k], ubs[k], max_rounds)
            assert (res[k].status, res[k].rounds) == (r1.status, r1.rounds), (inst.name, k)
            statuses.add(r1.status)
            if r1.status != oracle.INFEASIBLE:
                assert same_bits(blb[k], lb1) and same_bits(bub[k], ub1), (inst.name, k)
            if with_oracle:
                ref = oracle.run(inst, lbs[k], ubs[k], max_rounds)
                assert (ref.status, ref.rounds) == (r1.status, r1.rounds), (inst.name, k)
                if ref.status != oracle.INFEASIBLE:
                    assert same_bits(ref.lb, lb1) and same_bits(ref.ub, ub1)
    return statuses


def test_batch_config0(torch_cuda, lib):
    inst = synth.config0()
    lbs, ubs = node_set(inst, 20, 11_000, frac_hi=0.2)
    statuses = check_batch_vs_single(torch_cuda, lib, inst, lbs, ubs, with_oracle=True)
    assert oracle.CONVERGED in statuses


def test_batch_ragged_group_and_long_rows(torch_cuda, lib):
    """13 nodes (not a multiple of the 8-node group), rows of every class."""
    inst = synth.layout_mix(1)
    lbs, ubs = node_set(inst, 13, 12_000, frac_hi=0.1, only_int=False)
    check_batch_vs_single(torch_cuda, lib, inst, lbs, ubs, with_oracle=True)


def test_batch_mixed_outcomes(torch_cuda, lib):
    """Nodes that converge, hit the round limit and are infeasible at rounds
    0 and 1, all in one batch."""
    inst = synth.config0(1)
    lbs, ubs = node_set(inst, 9, 13_000, frac_hi=0.3)
    # node 0: the root; node 1: an empty input domain
    lbs[0], ubs[0] = inst.lb, inst.ub
    ivar = int(np.nonzero(inst.vartype == 1)[0][0])
    lbs[1][ivar], ubs[1][ivar] = 5.0, 4.0
    statuses = check_batch_vs_single(torch_cuda, lib, inst, lbs, ubs, max_rounds=3)
    assert oracle.MAX_ROUNDS in statuses and oracle.INFEASIBLE in statuses


def test_batch_medium(torch_cuda, lib):
    inst = synth.config3_matrix(100_000, 50_000)
    lbs, ubs = node_set(inst, 37, 14_000)
    check_batch_vs_single(torch_cuda, lib, inst, lbs, ubs)


def test_batch_reuse_and_invalid(torch_cuda, lib):
    torch = torch_cuda
    inst = synth.config0(2)
    lbs, ubs = node_set(inst, 16, 15_000)
    with lib.Problem.from_instance(inst) as p:
        a, alb, aub = run_batch(torch, p, lbs, ubs)
        b, blb, bub = run_batch(torch, p, lbs[:5], ubs[:5])  # smaller batch, same workspace
        for k in range(5):
            assert (a[k].status, a[k].rounds) == (b[k].status, b[k].rounds)
            assert same_bits(alb[k], blb[k]) and same_bits(aub[k], bub[k])
        bad = lbs.copy()
        bad[3, 7] = np.nan
        with pytest.raises(lib.PropError) as e:
            run_batch(torch, p, bad, ubs)
        assert e.value.code == lib.EINVAL
        c, clb, cub = run_batch(torch, p, lbs, ubs)  # still usable
        assert [(r.status, r.rounds) for r in c] == [(r.status, r.rounds) for r in a]


def test_batch_compaction(torch_cuda, lib):
    """Nodes that finish at different rounds: every third of 40 nodes (five
    groups) has an empty domain at round 0, so the 26 others fit in four
    groups and the driver compacts the batch at its first look at the
    active count, and again as nodes converge.  Every node still gives its
    own single run's results (and the oracle's), with the stream driver and
    with the graph driver (which continues with plain launches after a
    compaction)."""
    inst = synth.config0(3)
    lbs, ubs = node_set(inst, 40, 17_000, frac_hi=0.2)
    ivar = int(np.nonzero(inst.vartype == 1)[0][0])
    for k in range(0, 40, 3):
        lbs[k][ivar], ubs[k][ivar] = 5.0, 4.0
    statuses = check_batch_vs_single(torch_cuda, lib, inst, lbs, ubs, with_oracle=True)
    assert {oracle.CONVERGED, oracle.INFEASIBLE} <= statuses
    # a round limit that stops the survivors mid-run, after a compaction
    check_batch_vs_single(torch_cuda, lib, inst, lbs, ubs, max_rounds=9)
    # an invalid bound in one node of a batch that compacts: the call
    # reports it, and the problem stays usable
    bad = lbs.copy()
    bad[5, 3] = np.nan
    with lib.Problem.from_instance(inst) as p:
        with pytest.raises(lib.PropError) as e:
            run_batch(torch_cuda, p, bad, ubs)
        assert e.value.code == lib.EINVAL
        res, blb, bub = run_batch(torch_cuda, p, lbs, ubs)
        for k in (1, 2, 39):
            r1, lb1, ub1 = p.run(lbs[k], ubs[k], 100)
            assert (res[k].status, res[k].rounds) == (r1.status, r1.rounds)
            if r1.status != oracle.INFEASIBLE:
                assert same_bits(blb[k], lb1) and same_bits(bub[k], ub1)


def test_batch_host_arrays(torch_cuda, lib):
    """prop_run_batch on host arrays equals prop_run_batch_device, also after
    a larger batch has grown the staging (a smaller call reuses it)."""
    torch = torch_cuda
    inst = synth.layout_mix(2)
    lbs, ubs = node_set(inst, 19, 16_000, frac_hi=0.1, only_int=False)
    with lib.Problem.from_instance(inst) as p:
        dev, dlb, dub = run_batch(torch, p, lbs, ubs)
        for count in (19, 6):
            res, hlb, hub = p.run_batch(lbs[:count], ubs[:count])
            assert [(r.status, r.rounds) for r in res] == \
                [(r.status, r.rounds) for r in dev[:count]]
            for k in range(count):
                if res[k].status != oracle.INFEASIBLE:
                    assert same_bits(hlb[k], dlb[k]) and same_bits(hub[k], dub[k]), k
        with pytest.raises(ValueError):
            p.run_batch(lbs[:, :-1], ubs[:, :-1])


@pytest.fixture(scope="module")
def config3(lib):
    inst = synth.cached("config3", synth.config3_matrix)
    lbs, ubs = synth.config3_nodes(inst, 256)
    return inst, lbs, ubs


def _golden_nodes():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "config3_nodes.json")
    with open(path) as f:
        return json.load(f)["nodes"]


def bounds_sha(lb, ub):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(lb, dtype="<f8").tobytes())
    h.update(np.ascontiguousarray(ub, dtype="<f8").tobytes())
    return h.hexdigest()


def test_batch_config3_256_nodes(torch_cuda, lib, config3):
    """The 256 nodes of the 1,000,000 x 500,000 instance in one batch: each
    node bitwise equal to its own single run.  Eight nodes against the
    oracle's full runs (tests/golden/config3_nodes.json: status, rounds and
    the bounds' SHA-256 after every round): the batch's final state, and
    every round of the node's single run (max_rounds = r)."""
    torch = torch_cuda
    inst, lbs, ubs = config3
    gold = _golden_nodes()
    with lib.Problem.from_instance(inst) as p:
        res, blb, bub = run_batch(torch, p, lbs, ubs, 100)
        statuses = set()
        for k in range(256):
            r1, lb1, ub1 = p.run(lbs[k], ubs[k], 100)
            assert (res[k].status, res[k].rounds) == (r1.status, r1.rounds), k
            statuses.add(r1.status)
            if r1.status != oracle.INFEASIBLE:
                assert same_bits(blb[k], lb1) and same_bits(bub[k], ub1), k
        assert {oracle.CONVERGED, oracle.INFEASIBLE} <= statuses
        for key, g in gold.items():
            k = int(key)
            R = g["rounds"]
            assert (res[k].status, res[k].rounds) == (g["status"], R), k
            if g["status"] != oracle.INFEASIBLE:
                assert bounds_sha(blb[k], bub[k]) == g["sha"][R], k
            # every round before the last (infeasible nodes: bounds of the
            # final round are unspecified)
            last = R if g["status"] != oracle.INFEASIBLE else R - 1
            for r in range(1, last + 1):
                rr, lb_r, ub_r = p.run(lbs[k], ubs[k], r)
                assert bounds_sha(lb_r, ub_r) == g["sha"][r], f"node {k}: round {r} differs"
