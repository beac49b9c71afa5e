"""The allocation-free batch entry point (prop_run_batch_device_static)
against prop_run_batch_device, through the C ABI: status, rounds and bounds
bitwise equal on two calls in a row (the second with a smaller input, so
the fixed workspace holds a larger call's leftovers), and the size limit."""
import numpy as np
import pytest
from bitwise import same_bits

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


def _nodes(inst, count, seed0):
    lbs, ubs = [], []
    for k in range(count):
        lb, ub = synth.node_bounds(inst, seed0 + k)
        lbs.append(lb)
        ubs.append(ub)
    return np.stack(lbs), np.stack(ubs)


def _compare(lib, torch, prob, lbs, ubs, tag):
    dev = torch.device("cuda:0")
    outs = []
    for static in (False, True):
        d_lb = torch.tensor(lbs, dtype=torch.float64, device=dev)
        d_ub = torch.tensor(ubs, dtype=torch.float64, device=dev)
        res = prob.run_batch_device(d_lb, d_ub, 100, static=static)
        torch.cuda.synchronize()
        outs.append((res, d_lb.cpu().numpy(), d_ub.cpu().numpy()))
    (r0, l0, u0), (r1, l1, u1) = outs
    assert [(r.status, r.rounds) for r in r0] == [(r.status, r.rounds) for r in r1], tag
    for k, r in enumerate(r0):
        if r.status != lib.INFEASIBLE:
            assert same_bits(l0[k], l1[k]) and same_bits(u0[k], u1[k]), (tag, k)
    print(f"{tag}: {len(r0)} nodes, statuses "
          f"{sorted({lib.STATUS_NAMES[r.status] for r in r0})}, rounds up to "
          f"{max(r.rounds for r in r0)}", flush=True)
    return r0


def test_static_matches_batch_two_calls(lib, torch_cuda):
    torch = torch_cuda
    # power-law rows (long rows in segments) and hot variables
    big = synth.config3_matrix(50_000, 25_000)
    with lib.Problem.from_instance(big) as p:
        lbs, ubs = _nodes(big, 19, 31_000)
        res = _compare(lib, torch, p, lbs, ubs, "powerlaw 19 nodes")
        assert any(r.status == lib.CONVERGED for r in res)
        # second call, smaller: fewer nodes of the same problem
        lbs, ubs = _nodes(big, 5, 32_000)
        _compare(lib, torch, p, lbs, ubs, "powerlaw 5 nodes")
    # and a smaller problem after that
    small = synth.config0()
    with lib.Problem.from_instance(small) as p:
        lbs, ubs = _nodes(small, 3, 33_000)
        _compare(lib, torch, p, lbs, ubs, "config0 3 nodes")


def test_static_rejects_oversized_workspace(lib, torch_cuda):
    torch = torch_cuda
    n = 300_000  # one group of 8 nodes: 32 * n * 8 bytes > 64 MiB
    inst = synth.from_rows([[(0, 1.0), (1, 1.0)]], [-np.inf], [1.0], np.zeros(n), np.ones(n),
                           np.ones(n, dtype=np.uint8), n=n)
    with lib.Problem.from_instance(inst) as p:
        d_lb = torch.zeros((1, n), dtype=torch.float64, device="cuda:0")
        d_ub = torch.ones((1, n), dtype=torch.float64, device="cuda:0")
        with pytest.raises(lib.PropError) as ei:
            p.run_batch_device(d_lb, d_ub, 10, static=True)
        assert ei.value.code == lib.EINVAL and "fixed array" in str(ei.value)
        # the problem stays usable, and the ordinary entry point runs it
        res = p.run_batch_device(d_lb, d_ub, 10)
        assert res[0].status == lib.CONVERGED
